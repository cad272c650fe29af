"""Separate orbitals for the down electrons (the generalisation of Eq. (1)
the paper mentions in Sec. 2): the oracle against the Cauchy-Binet closed
form and brute force, and the library's host-side entry point."""
import numpy as np
import pytest

import oracle
from gen.workloads import make_config, with_down_orbitals
from oracle import brute

from test_oracle_pins import _cauchy_binet_case


def test_equal_sets_reproduce_the_common_set_bit_for_bit():
    wl = make_config(2, n_walk=16)
    same = with_down_orbitals(wl)
    same.alpha_dn, same.coef_dn = wl.alpha.copy(), wl.coef.copy()
    a = oracle.evaluate(wl, n_threads=4)
    b = oracle.evaluate(same, n_threads=4)
    assert np.array_equal(a.logabs, b.logabs) and np.array_equal(a.gl, b.gl)
    c = oracle.sm_evaluate(wl, n_threads=4)
    d = oracle.sm_evaluate(same, n_threads=4)
    assert np.array_equal(c.logabs, d.logabs) and np.array_equal(c.gl, d.gl)


def test_different_sets_change_only_the_down_determinants():
    wl = make_config(1)
    two = with_down_orbitals(wl)
    a = oracle.evaluate(wl, n_threads=2)
    b = oracle.evaluate(two, n_threads=2)
    assert not np.allclose(a.logabs, b.logabs)
    for w in range(wl.n_walk):
        psi, grad = brute.psi_brute(two, two.R[w])
        assert b.sign[w] == np.sign(psi)
        assert abs(b.logabs[w] - np.log(abs(psi))) < 1e-10
        np.testing.assert_allclose(b.gl[w], grad / psi, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("shape", [(8, 4, 3, 3), (12, 6, 5, 2)])
def test_cauchy_binet_with_two_sets(shape):
    """sum_{I,J} detB_up[I] detB_dn[J] D_I D_J = det(Phi_up B_up) det(Phi^dn_dn B_dn)."""
    n_mo, n_up, n_dn, W = shape
    wl, Bu, Bd = _cauchy_binet_case(n_mo, n_up, n_dn, W, seed=n_mo)
    wl = with_down_orbitals(wl, seed=n_mo + 1)
    res = oracle.evaluate(wl, n_threads=4)
    chain = oracle.sm_evaluate(wl, n_threads=4)
    for w in range(W):
        sgn, logabs = 1.0, 0.0
        gl = np.zeros((wl.n_elec, 4))
        for sp, e0, n, B in ((0, 0, n_up, Bu), (1, n_up, n_dn, Bd)):
            orb = np.array([oracle.orbitals(wl, wl.R[w, e], spin=sp) for e in range(e0, e0 + n)])
            Pm = orb[:, 0, :] @ B
            s, l = np.linalg.slogdet(Pm)
            sgn *= s
            logabs += l
            Pinv = np.linalg.inv(Pm)
            for q in range(4):
                gl[e0:e0 + n, q] = np.einsum("ce,ec->e", Pinv, orb[:, 1 + q, :] @ B)
        for r, tol in ((res, 1e-10), (chain, 1e-7)):
            assert r.sign[w] == sgn
            assert abs(r.logabs[w] - logabs) < tol * (1 + abs(logabs))
            np.testing.assert_allclose(r.gl[w], gl, rtol=0, atol=tol * (1 + np.abs(gl).max()))


def test_library_accepts_and_checks_a_down_set():
    mdet = pytest.importorskip("paper_1510_00730_amd")
    wl = with_down_orbitals(make_config(1))
    ev = mdet.Evaluator(device=-1)
    ev.load_workload(wl)
    with pytest.raises(mdet.MdetError):
        ev.init_orbitals_dn(wl.pow_abc_dn, -wl.alpha_dn, wl.coef_dn)  # exponents must be > 0
