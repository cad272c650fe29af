"""The oracle pins must catch plausible mistakes.  Each case compiles a copy of
oracle.c with one planted error (CPU only) and checks that the pin suite
fails against it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = {
    "gradient_sign": ("double d1 = -2.0 * alpha * ipow(x, a + 1);",
                      "double d1 = 2.0 * alpha * ipow(x, a + 1);"),
    "laplacian_dropped_term": ("+ 4.0 * alpha * alpha * ipow(x, a + 2);", ";"),
    "laplacian_wrong_factor": ("(double)(2 * a + 1)", "(double)(2 * a)"),
    "inverse_transposed": ("s += X[c * n + e] * G[(q * n + e) * n + c] * cscale[c];",
                           "s += X[e * n + c] * G[(q * n + e) * n + c] * cscale[c];"),
    "pivot_sign_dropped": ("if (d < 0) sg = -sg;", ";"),
    "column_scale_dropped": ("*logabs = la + colexp_sum * log(2.0);", "*logabs = la;"),
    "wrong_spin_ratio": ("double x = term * rd[e * 4 + q];", "double x = term * rt_u[e * 4 + q];"),
    # the error scales (denominators of every parity gate)
    "error_scale_psi_inflated": ("aabs[0] += fabs(term);", "aabs[0] += 1000.0 * fabs(term);"),
    "error_scale_psi_coef_only": ("aabs[0] += fabs(term);",
                                  "aabs[0] += fabs(c[k]);"),
    "error_scale_grad_inflated": ("aabs[1 + e * 4 + q] += fabs(x);",
                                  "aabs[1 + e * 4 + q] += 1000.0 * fabs(x);"),
    "error_scale_grad_dn_dropped": ("aabs[1 + (n_up + e) * 4 + q] += fabs(x);", ";"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", ["unmutated_control"] + sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    """The control build (no change) must pass the pins through the same
    harness, so a failure of a mutant is the pins' doing."""
    src = open(SRC).read()
    if name != "unmutated_control":
        old, new = MUTATIONS[name]
        assert src.count(old) == 1, name
        src = src.replace(old, new)
    mut_c = tmp_path / "oracle_mut.c"
    mut_c.write_text(src)
    so = tmp_path / "liboracle_mut.so"
    chain_c = os.path.join(ROOT, "oracle", "sm_chain.c")  # the rest of the oracle library
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", str(mut_c), chain_c,
                           "-o", str(so), "-lm"])
    env = dict(os.environ, MDET_ORACLE_LIB_OVERRIDE=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    if name == "unmutated_control":
        assert r.returncode == 0, r.stdout[-2000:]
    else:
        assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"
