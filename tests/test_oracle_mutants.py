"""The oracle's pins catch plausible mistakes.

Each case copies oracle/drts_oracle.c, plants one mistake of the kind the
pins are meant to catch (a dropped term, a wrong sign, a transposed index,
an off-by-one range, a wrong coefficient), builds the copy with the
oracle's own compiler flags and runs tests/test_oracle_pins.py against it in
a subprocess: the pin suite must fail.  A control case builds the copy
unchanged and must pass.  Only the copy is changed; the oracle itself is
never modified."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "drts_oracle.c")

# (name, text of the oracle, planted replacement)
MUTANTS = [
    ("hg_sign", "double q = 1.0 + g * g - 2.0 * g * cs;", "double q = 1.0 + g * g + 2.0 * g * cs;"),
    # (p[m][n] is symmetric, so transposing the normalisation sum changes
    # nothing; the block itself is not: its normalisation differs per column)
    ("block_transposed", "C[m * NDIR + n] = (m != n)", "C[n * NDIR + m] = (m != n)"),
    ("forward_term_dropped", "alpha * (P0 + Ps * G)", "alpha * (Ps * G)"),
    ("absorption_coefficient", "double alpha = exp(-mu_a * h);", "double alpha = exp(-mu_s * h);"),
    ("fresnel_average", "R = 0.5 * (rs * rs + rp * rp);", "R = rs * rs;"),
    ("specular_factor", "r[i] = s[i] - (2.0 * cos_i) * N[i];", "r[i] = s[i] - cos_i * N[i];"),
    ("escaped_off_by_one", "for (int64_t r = D; r < R; ++r)\n            esc += y[r];",
     "for (int64_t r = D + 1; r < R; ++r)\n            esc += y[r];"),
    ("pulse_window", "double hi = erfc(((double)(t + 1) * dt_s - tc) / k);",
     "double hi = erfc(((double)(t + 2) * dt_s - tc) / k);"),
    ("rescale_sign", "y[r] = ldexp(y[r], E - En);", "y[r] = ldexp(y[r], En - E);"),
    ("absorbed_weight", "absorbed += A->absorb_of_voxel[v] * sv;", "absorbed += sv;"),
]


def _build(tmp_path, text):
    src = tmp_path / "drts_oracle.c"
    src.write_text(text)
    lib = tmp_path / "_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-o", str(lib), str(src), "-lm"])
    return str(lib)


def _pins(lib):
    env = dict(os.environ, DRTS_ORACLE_LIB=lib)
    return subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                           "-x", "-q", "-p", "no:cacheprovider"], cwd=ROOT, env=env,
                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)


def test_unchanged_copy_passes_the_pins(tmp_path):
    r = _pins(_build(tmp_path, open(SRC).read()))
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, name
    r = _pins(_build(tmp_path, text.replace(old, new)))
    assert r.returncode != 0, "%s passed every pin:\n%s" % (name, r.stdout[-2000:])
