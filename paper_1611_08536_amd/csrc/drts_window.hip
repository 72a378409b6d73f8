// Windowed measurement (Eq. 27 with a window of several steps): a sensor's
// reading is the per-step detector sum filtered by the sensor's impulse
// response, M_d(t) = sum_j taps[d][j] m_d(t - tap0 - j), computed on the
// device from a solver's FP64 detector series.
//
// The series are stored per step as a scaled value and a power-of-two
// exponent (value * 2^exp2[s]), so terms of different steps are brought to a
// common exponent first: the largest exponent among the steps a reading
// combines, so that every term is scaled down (never overflows) and the
// reading is returned as (value, exponent) like the series.  Terms are added
// in ascending tap order; each reading is one thread's sequential sum.
#include <algorithm>
#include <cmath>
#include <vector>

#include "drts_internal.h"

namespace drts {

__global__ void __launch_bounds__(256) detector_window(WindowArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_out = a.count * a.n_det * a.n_rhs;
    if (i >= n_out) return;
    const int k = (int)(i % a.n_rhs);
    const int d = (int)((i / a.n_rhs) % a.n_det);
    const int64_t t = a.first + i / ((int64_t)a.n_rhs * a.n_det);
    const double *h = a.taps + (int64_t)d * a.n_taps;
    // common exponent: the largest among the contributing steps
    bool any = false;
    int32_t E = 0;
    for (int j = 0; j < a.n_taps; ++j) {
        const int64_t s = t - a.tap0 - j;
        if (s < 0 || s >= a.t_done || h[j] == 0.0) continue;
        const int32_t e = a.ser_exp[s * a.n_rhs + k];
        E = any ? max(E, e) : e;
        any = true;
    }
    double acc = 0.0;
    for (int j = 0; j < a.n_taps; ++j) {
        const int64_t s = t - a.tap0 - j;
        if (s < 0 || s >= a.t_done || h[j] == 0.0) continue;
        const double m = a.ser_det[(s * a.n_det + d) * a.n_rhs + k];
        acc += h[j] * ldexp(m, a.ser_exp[s * a.n_rhs + k] - E);
    }
    a.out[i] = acc;
    a.out_exp[i] = E;
}

hipError_t launch_detector_window(const WindowArgs &a, hipStream_t stream)
{
    const int64_t n_out = a.count * a.n_det * a.n_rhs;
    if (n_out == 0) return hipSuccess;
    hipLaunchKernelGGL(detector_window, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace drts
