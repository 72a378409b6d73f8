"""The oracle's pins catch plausible mistakes.

Each case copies the oracle package (oracle/drts_oracle.c and
oracle/__init__.py), plants one mistake of the kind the pins are meant to
catch (a dropped term, a wrong sign, a transposed index, an off-by-one range,
a wrong coefficient, a wrong operand), and runs tests/test_oracle_pins.py and
tests/test_oracle_pins_lebedev.py against the copy in a subprocess (the copy
builds its own library with the oracle's compiler flags): the pin suite must
fail.  A control case copies the package unchanged and must pass.  Only the copy is changed; the oracle itself
is never modified."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

C_SRC, PY_SRC = "drts_oracle.c", "__init__.py"

# (name, file of the oracle, text, planted replacement)
MUTANTS = [
    ("hg_sign", C_SRC, "double q = 1.0 + g * g - 2.0 * g * cs;", "double q = 1.0 + g * g + 2.0 * g * cs;"),
    # (p[m][n] is symmetric, so transposing the normalisation sum changes
    # nothing; the block itself is not: its normalisation differs per column)
    ("block_transposed", C_SRC, "C[m * NDIR + n] = (m != n)", "C[n * NDIR + m] = (m != n)"),
    ("forward_term_dropped", C_SRC, "alpha * (P0 + S[n][n])", "alpha * (S[n][n])"),
    ("absorption_coefficient", C_SRC, "double alpha = exp(-mu_a * h);", "double alpha = exp(-mu_s * h);"),
    ("fresnel_average", C_SRC, "R = 0.5 * (rs * rs + rp * rp);", "R = rs * rs;"),
    ("specular_factor", C_SRC, "r[i] = s[i] - (2.0 * cos_i) * N[i];", "r[i] = s[i] - cos_i * N[i];"),
    ("escaped_off_by_one", C_SRC, "for (int64_t r = D; r < R; ++r)\n            esc += y[r];",
     "for (int64_t r = D + 1; r < R; ++r)\n            esc += y[r];"),
    ("pulse_window", C_SRC, "double hi = erfc(((double)(t + 1) * dt_s - tc) / k);",
     "double hi = erfc(((double)(t + 2) * dt_s - tc) / k);"),
    ("rescale_sign", C_SRC, "y[r] = ldexp(y[r], E - En);", "y[r] = ldexp(y[r], En - E);"),
    ("absorbed_weight", C_SRC, "absorbed += A->absorb_of_voxel[v] * sv;", "absorbed += sv;"),
    # detector sums of Eq. (27)
    ("detector_reads_previous_state", C_SRC, "det[n_det * t + det_id[i]] += det_F[i] * y[det_row[i]];",
     "det[n_det * t + det_id[i]] += det_F[i] * x[det_row[i]];"),
    ("detector_weight_dropped", C_SRC, "det[n_det * t + det_id[i]] += det_F[i] * y[det_row[i]];",
     "det[n_det * t + det_id[i]] += y[det_row[i]];"),
    ("detector_state_row_for_escape", PY_SRC, "r = A.rows_of(st, d.escape)", "r = A.rows_of(st, False)"),
    # interface normal of the sphere: at the first voxel's centre, not the step midpoint
    ("sphere_normal_at_voxel_centre", C_SRC,
     "double P[3] = {(double)x + 0.5 + 0.5 * (double)e[0],\n"
     "                       (double)y + 0.5 + 0.5 * (double)e[1],\n"
     "                       (double)z + 0.5 + 0.5 * (double)e[2]};",
     "double P[3] = {(double)x + 0.5, (double)y + 0.5, (double)z + 0.5};"),
    # tied snap directions: the lowest index takes everything
    ("snap_ties_to_lowest", C_SRC, "if (or_dot3(s, target) >= best - 1e-12) out[k++] = d;",
     "if (or_dot3(s, target) >= best - 1e-12 && k == 0) out[k++] = d;"),
    # several scatterings per step (Eq. (4)): Poisson weight without 1/i,
    # the kernel power never advancing past G^2, the remaining probability
    # dropped, the medium's order not reaching the assembly
    ("poisson_factorial_dropped", C_SRC, "Pi = (Pi * lam) / (double)i;", "Pi = Pi * lam;"),
    ("kernel_power_stuck", C_SRC, "acc += G[m][k] * Gi[k][n];", "acc += G[m][k] * G[k][n];"),
    ("remaining_probability_dropped", C_SRC, "w = 1.0 - seen;", "w = 0.0 * seen;"),
    ("medium_order_ignored", PY_SRC, 'st.scatter_order = getattr(medium, "scatter_order", 1)',
     "st.scatter_order = 1"),
    # windowed measurement (Eq. (27)): response applied backwards in time,
    # delay of the response with the wrong sign
    ("window_response_reversed", PY_SRC, "s = t - tap0 - j", "s = t - tap0 + j"),
    ("window_delay_sign", PY_SRC, "s = t - tap0 - j", "s = t + tap0 - j"),
    # Lebedev-86 with the weights of Eq. (18)-(19): distance to the line
    # instead of the segment, the weight ramp inverted, the kernel without the
    # rule's solid-angle weights, offsets applied with the wrong sign, escape
    # weights counted as one, two digits of a generator value of the rule swapped
    ("leb_segment_as_line", C_SRC, "if (t > 1.0) t = 1.0;", ""),
    ("leb_weight_ramp_inverted", C_SRC, "raw[cnt] = 1.0 - d;", "raw[cnt] = d;"),
    ("leb_kernel_without_solid_angle", C_SRC, "p[m] = wq[m] * or_hg(g, cs);", "p[m] = or_hg(g, cs);"),
    ("leb_offset_sign", C_SRC, "int ux = x + o[0], uy = y + o[1], uz = z + o[2];",
     "int ux = x - o[0], uy = y - o[1], uz = z - o[2];"),
    ("leb_escape_weight", C_SRC, "esc += L->st->w[e];\n                            any_out = 1;",
     "esc += 1.0;\n                            any_out = 1;"),
    ("leb_generator_value", C_SRC, "0.6943540066026664", "0.6943450066026664"),
    ("leb_step_time_one_voxel", PY_SRC, 'dt = dt_seconds(med.h_mm * getattr(med, "c_dt", 1.0), workload.n_ref)',
     "dt = dt_seconds(med.h_mm, workload.n_ref)"),
    # crossing within the step (Sec. 4.2): the fraction in the wrong medium,
    # the absorption difference reversed, the tangential landing dropped, the
    # sphere's other root
    ("substep_fraction_swapped", C_SRC, "Tr = Tr * exp(-(mua2 - mua1) * ((1.0 - f) * M->h_mm));",
     "Tr = Tr * exp(-(mua2 - mua1) * (f * M->h_mm));"),
    ("substep_absorption_sign", C_SRC, "Tr = Tr * exp(-(mua2 - mua1) * ((1.0 - f) * M->h_mm));",
     "Tr = Tr * exp(-(mua1 - mua2) * ((1.0 - f) * M->h_mm));"),
    ("substep_no_tangential_landing", C_SRC,
     "vr = (int64_t)tx + (int64_t)M->nx * ((int64_t)ty + (int64_t)M->ny * z);", "vr = v;"),
    ("substep_sphere_root", C_SRC, "double s = (c <= 0.0) ? (-b + q) / (2.0 * a) : (-b - q) / (2.0 * a);",
     "double s = (c <= 0.0) ? (-b - q) / (2.0 * a) : (-b + q) / (2.0 * a);"),
    # dither key with row and column swapped
    ("dither_key_swapped", C_SRC, "uint64_t key = ((uint64_t)r << 32) ^ (uint64_t)(uint32_t)A->col[j];",
     "uint64_t key = ((uint64_t)(uint32_t)A->col[j] << 32) ^ (uint64_t)r;"),
]


def _copy(tmp_path, fname=None, old=None, new=None):
    dst = tmp_path / "pkg" / "oracle"
    dst.mkdir(parents=True)
    for f in (C_SRC, PY_SRC):
        shutil.copy(os.path.join(ORACLE, f), dst / f)
    if fname is not None:
        text = (dst / fname).read_text()
        assert text.count(old) == 1, (fname, old)
        (dst / fname).write_text(text.replace(old, new))
    return str(tmp_path / "pkg")


def _pins(pkg):
    env = dict(os.environ, DRTS_ORACLE_COPY=pkg)
    return subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                           os.path.join(ROOT, "tests", "test_oracle_pins_lebedev.py"),
                           "-x", "-q", "-p", "no:cacheprovider"], cwd=ROOT, env=env,
                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)


def test_unchanged_copy_passes_the_pins(tmp_path):
    r = _pins(_copy(tmp_path))
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name,fname,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, fname, old, new):
    r = _pins(_copy(tmp_path, fname, old, new))
    assert r.returncode != 0, "%s passed every pin:\n%s" % (name, r.stdout[-2000:])
