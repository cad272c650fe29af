"""Norm-based truncation of the expansion (Sec. 3): the oracle against the
paper's identity and closed forms, and the library bit for bit against the
oracle (CPU; the library entry point needs no GPU)."""
import math

import numpy as np
import pytest

from gen.workloads import encode, make_config
from oracle import truncation as tr

mdet = pytest.importorskip("paper_1510_00730_amd")


def test_norm_decomposition_identity():
    """sum_i N_i^up = sum_j N_j^dn = 1 (the decomposition of the norm)."""
    wl = make_config(3)
    _, ru, rd, total = tr.spin_norms(wl.det_up, wl.det_dn, wl.c)
    assert abs(math.fsum(ru.values()) - 1.0) < 1e-13
    assert abs(math.fsum(rd.values()) - 1.0) < 1e-13
    assert abs(total - math.fsum(float(x) ** 2 for x in wl.c)) < 1e-13


def test_separable_coefficients_closed_form():
    """c_ij = a_i b_j on the full grid: N_i^up = a_i^2 / sum a^2 exactly."""
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=6), rng.normal(size=5)
    ups = [encode([[0, 1 + i]], 1)[0] for i in range(6)]
    dns = [encode([[0, 1 + j]], 1)[0] for j in range(5)]
    det_up = np.array([ups[i] for i in range(6) for j in range(5)], dtype=np.uint64)
    det_dn = np.array([dns[j] for i in range(6) for j in range(5)], dtype=np.uint64)
    c = np.array([a[i] * b[j] for i in range(6) for j in range(5)])
    per_k, ru, rd, _ = tr.spin_norms(det_up, det_dn, c)
    for i in range(6):
        assert abs(ru[tuple(int(x) for x in ups[i])] - a[i] ** 2 / np.sum(a ** 2)) < 1e-14
    for j in range(5):
        assert abs(rd[tuple(int(x) for x in dns[j])] - b[j] ** 2 / np.sum(b ** 2)) < 1e-14


def hand_example():
    A, B, C = encode([[0, 1], [0, 2], [1, 2]], 1)
    X, Y = encode([[0, 1], [0, 3]], 1)
    det_up = np.array([A, A, B, C, B], dtype=np.uint64)
    det_dn = np.array([X, Y, X, Y, Y], dtype=np.uint64)
    c = np.array([0.8, 0.4, 0.3, 0.1, 0.2])
    return det_up, det_dn, c


@pytest.mark.parametrize("eps,mask,counts", [
    # N^up: A 0.80/0.94, B 0.13/0.94, C 0.01/0.94; N^dn: X 0.73/0.94, Y 0.21/0.94
    (0.05, [1, 1, 1, 0, 1], (4, 2, 2)),
    (0.2, [1, 1, 0, 0, 0], (2, 1, 2)),
    (0.5, [1, 0, 0, 0, 0], (1, 1, 1)),
    (0.0, [1, 1, 1, 1, 1], (5, 3, 2)),
    (1.0, [0, 0, 0, 0, 0], (0, 0, 0)),
])
def test_hand_example(eps, mask, counts):
    det_up, det_dn, c = hand_example()
    keep, nk, nu, nd = tr.norm_truncation(det_up, det_dn, c, eps)
    assert keep.astype(int).tolist() == mask and (nk, nu, nd) == counts
    k2, nk2, nu2, nd2 = mdet.norm_truncation(det_up, det_dn, c, eps)
    assert k2.astype(int).tolist() == mask and (nk2, nu2, nd2) == counts


@pytest.mark.parametrize("cid", [1, 2, 3])
def test_library_matches_oracle_bit_exact(cid):
    wl = make_config(cid)
    for eps_up, eps_dn in ((1e-2, 1e-2), (1e-4, 1e-5), (1e-6, 1e-6), (1e-8, 0.0)):
        ref = tr.norm_truncation(wl.det_up, wl.det_dn, wl.c, eps_up, eps_dn)
        got = mdet.norm_truncation(wl.det_up, wl.det_dn, wl.c, eps_up, eps_dn)
        assert np.array_equal(ref[0], got[0]) and ref[1:] == got[1:], (cid, eps_up, eps_dn)


def test_errors():
    det_up, det_dn, c = hand_example()
    with pytest.raises(mdet.MdetError):
        mdet.norm_truncation(det_up, det_dn, c, -1.0)
    with pytest.raises(mdet.MdetError):
        mdet.norm_truncation(det_up, det_dn, np.zeros_like(c), 0.1)
