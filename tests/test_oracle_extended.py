"""The extended-precision reference (oracle/extended.py) against the FP64
oracle: two independent evaluations of Eq. (1) and Eq. (nabla) (Sec. 2.3)
that must agree to FP64 rounding on well-conditioned walkers, and whose
agreement on the drawn-order stress case shows the oracle's own accuracy
there."""
import numpy as np

import oracle
from oracle.extended import evaluate_extended
from gen.workloads import make_config
from parity_util import scaled_errors


def test_extended_matches_oracle_default_orbitals():
    wl = make_config(2)
    R = wl.R[:4]
    ref = evaluate_extended(wl, R)
    o = oracle.evaluate(wl, R, n_threads=4)
    ep, eg = scaled_errors(ref, o.sign, o.logabs, o.gl)
    assert ep.max() < 1e-13 and eg.max() < 1e-12


def test_oracle_accurate_on_drawn_order():
    """Orbitals in drawn order (near-singular reference determinants): the
    FP64 oracle stays within 1e-11 of the extended-precision evaluation."""
    wl = make_config(3, n_walk=4, raw_orbital_order=True)
    ref = evaluate_extended(wl, wl.R)
    o = oracle.evaluate(wl, wl.R, n_threads=4)
    ep, eg = scaled_errors(ref, o.sign, o.logabs, o.gl)
    assert ep.max() < 1e-11 and eg.max() < 1e-11
