"""The paper's Sherman-Morrison chain (Sec. 2.2) on the CPU, pinned against
the textbook determinant (Leibniz), the Cauchy-Binet closed form, the direct
LU of the oracle, and counts that follow from the bit strings alone."""
import math

import numpy as np
import pytest

import oracle
from gen.workloads import make_config
from oracle import brute, preprocess

from test_oracle_pins import _cauchy_binet_case


def _chain_degrees(uniq):
    """Sum over consecutive distinct determinants of their excitation degree."""
    tot = 0
    for a, b in zip(uniq[:-1], uniq[1:]):
        tot += sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)) // 2
    return tot


def _lists(wl):
    idx = preprocess.index_expansion(wl.det_up, wl.det_dn, wl.c)
    return idx["uniq_up"], idx["uniq_dn"]


def _close(a, b, tol_l, tol_g):
    assert np.array_equal(a.sign, b.sign)
    assert np.max(np.abs(a.logabs - b.logabs)) < tol_l
    assert np.max(np.abs(a.gl - b.gl) / (1.0 + np.abs(b.gl))) < tol_g


def test_tiny_vs_leibniz():
    wl = make_config(1)
    res = oracle.sm_evaluate(wl, n_threads=2)
    for w in range(wl.n_walk):
        psi, grad = brute.psi_brute(wl, wl.R[w])
        assert res.sign[w] == np.sign(psi)
        assert abs(res.logabs[w] - math.log(abs(psi))) < 1e-10
        np.testing.assert_allclose(res.gl[w], grad / psi, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("shape", [(8, 4, 3, 3), (12, 6, 5, 2)])
def test_cauchy_binet_full_ci(shape):
    """Full CI with c_IJ = det B_up[I] det B_dn[J]: the chain visits every
    subset of the orbitals and must reproduce det(Phi B_up) det(Phi B_dn)."""
    n_mo, n_up, n_dn, W = shape
    wl, Bu, Bd = _cauchy_binet_case(n_mo, n_up, n_dn, W, seed=n_mo)
    res = oracle.sm_evaluate(wl, n_threads=2)
    for w in range(W):
        orb = np.array([oracle.orbitals(wl, wl.R[w, e]) for e in range(wl.n_elec)])
        Mu = orb[:n_up, 0, :] @ Bu
        Md = orb[n_up:, 0, :] @ Bd
        psi = np.linalg.det(Mu) * np.linalg.det(Md)
        assert res.sign[w] == np.sign(psi)
        assert abs(res.logabs[w] - math.log(abs(psi))) < 1e-8
        # grad~_e Psi / Psi of a product of two determinants: row-replacement ratios
        iu, idn = np.linalg.inv(Mu), np.linalg.inv(Md)
        for e in range(n_up):
            for q in range(4):
                ref = (orb[e, 1 + q, :] @ Bu) @ iu[:, e]
                assert abs(res.gl[w, e, q] - ref) < 1e-7 * (1 + abs(ref))
        for e in range(n_dn):
            for q in range(4):
                ref = (orb[n_up + e, 1 + q, :] @ Bd) @ idn[:, e]
                assert abs(res.gl[w, n_up + e, q] - ref) < 1e-7 * (1 + abs(ref))


@pytest.mark.parametrize("cid", [1, 2])
def test_zero_threshold_counts(cid):
    """With no ratio rejected, every walker factorises once per spin and
    substitutes exactly the excitation degree between consecutive entries."""
    wl = make_config(cid, n_walk=16)
    uu, ud = _lists(wl)
    res = oracle.sm_evaluate(wl, threshold=0.0, n_threads=4)
    W = wl.n_walk
    assert res.n_inv == 2 * W and res.n_fail == 0
    assert res.n_subst == W * (_chain_degrees(uu) + _chain_degrees(ud))
    _close(res, oracle.evaluate(wl, max_degree=None, n_threads=4), 1e-6, 1e-5)


@pytest.mark.parametrize("cid", [1, 2])
def test_infinite_threshold_is_direct(cid):
    """Every substitution rejected: each determinant is factorised from
    scratch and the result is the direct LU's."""
    wl = make_config(cid, n_walk=16)
    uu, ud = _lists(wl)
    res = oracle.sm_evaluate(wl, threshold=np.inf, n_threads=4)
    W = wl.n_walk
    assert res.n_subst == 0 and res.n_inv == W * (len(uu) + len(ud))
    assert res.n_fail == W * (_chain_degrees(uu) + _chain_degrees(ud))
    _close(res, oracle.evaluate(wl, max_degree=None, n_threads=4), 1e-11, 1e-10)


@pytest.mark.parametrize("cid", [1, 2])
def test_default_threshold_matches_direct(cid):
    """The paper's 1e-3 rule on the small workloads: chain error stays small."""
    wl = make_config(cid, n_walk=64)
    res = oracle.sm_evaluate(wl, n_threads=4)
    ref = oracle.evaluate(wl, max_degree=None, n_threads=4)
    _close(res, ref, 1e-8, 1e-7)
    W = wl.n_walk
    uu, ud = _lists(wl)
    assert res.n_inv >= 2 * W
    # the retry rule never drops a substitution: done + abandoned cover the chain
    assert res.n_subst <= W * (_chain_degrees(uu) + _chain_degrees(ud))


def test_chain_counts_single_walker_additive():
    """Counters are per-walker sums: one batch equals the sum of its halves."""
    wl = make_config(2, n_walk=8)
    a = oracle.sm_evaluate(wl, R=wl.R[:4], n_threads=2)
    b = oracle.sm_evaluate(wl, R=wl.R[4:], n_threads=2)
    c = oracle.sm_evaluate(wl, n_threads=3)
    assert (a.n_subst + b.n_subst, a.n_inv + b.n_inv, a.n_fail + b.n_fail) == \
        (c.n_subst, c.n_inv, c.n_fail)
    np.testing.assert_array_equal(np.concatenate([a.logabs, b.logabs]), c.logabs)
