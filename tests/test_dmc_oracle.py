"""Slater-Jastrow trial function and fixed-node DMC on the CPU oracle, pinned
against finite differences, the cusp conditions, the resampling invariant of
the comb, and the exact ground-state energy of the helium atom (a nodeless
ground state, so fixed-node DMC is exact up to time-step and population
bias)."""
import math

import numpy as np
import pytest

import oracle
from gen.workloads import make_config, make_helium
from oracle import dmc, vmc

PARAMS = (1.0, -2.0, 1.0)


def _fd_jastrow(R, n_up, params, h=1e-4):
    W, N, _ = R.shape
    g = np.zeros((W, N, 3))
    lap = np.zeros((W, N))
    J0 = dmc.jastrow(R, n_up, *params)[0]
    for e in range(N):
        for ax in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[:, e, ax] += h
            Rm[:, e, ax] -= h
            Jp = dmc.jastrow(Rp, n_up, *params)[0]
            Jm = dmc.jastrow(Rm, n_up, *params)[0]
            g[:, e, ax] = (Jp - Jm) / (2 * h)
            lap[:, e] += (Jp - 2 * J0 + Jm) / (h * h)
    return g, lap


@pytest.mark.parametrize("params", [(1.0, -2.0, 1.0), (0.3, 0.0, 1.0), (2.5, -5.0, 0.2)])
def test_jastrow_derivatives_by_finite_differences(params):
    wl = make_config(1)
    J, g, lap = dmc.jastrow(wl.R, wl.n_up, *params)
    gf, lf = _fd_jastrow(wl.R, wl.n_up, params)
    np.testing.assert_allclose(g, gf, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(lap, lf, rtol=1e-4, atol=1e-4)


def test_cusp_conditions():
    """dJ/dr_ij at coalescence: 1/2 for opposite spins, 1/4 for equal spins;
    the nuclear term's slope at the nucleus is a_en."""
    for n_up, a in ((2, 0.25), (1, 0.5)):  # two electrons, equal or opposite spins
        R = np.zeros((1, 2, 3))
        R[0, 0] = [0.3, -0.2, 0.1]
        h = 1e-7
        R[0, 1] = R[0, 0] + np.array([h, 0, 0])
        J1 = dmc.jastrow(R, n_up, 1.3, 0.0, 1.0)[0][0]
        R[0, 1] = R[0, 0] + np.array([2 * h, 0, 0])
        J2 = dmc.jastrow(R, n_up, 1.3, 0.0, 1.0)[0][0]
        assert abs((J2 - J1) / h - a) < 1e-5
    R = np.zeros((1, 2, 3))
    R[0, 1] = [0.0, 1e4, 0.0]  # far away, perpendicular to the displacement
    R[0, 0] = [1e-7, 0, 0]
    J1 = dmc.jastrow(R, 1, 1.0, -2.0, 0.7)[0][0]
    R[0, 0] = [2e-7, 0, 0]
    J2 = dmc.jastrow(R, 1, 1.0, -2.0, 0.7)[0][0]
    assert abs((J2 - J1) / 1e-7 - (-2.0)) < 1e-5


def test_slater_jastrow_product_rule_by_finite_differences():
    """grad ln Psi_T and lap Psi_T / Psi_T against differences of ln|Psi_T|."""
    wl = make_config(1)
    R = wl.R[:3]
    s, la, gl = dmc.trial(wl, R, PARAMS)
    h = 1e-4
    for e in range(wl.n_elec):
        lapfd = np.zeros(R.shape[0])
        for ax in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[:, e, ax] += h
            Rm[:, e, ax] -= h
            lp = dmc.trial(wl, Rp, PARAMS)[1]
            lm = dmc.trial(wl, Rm, PARAMS)[1]
            d1 = (lp - lm) / (2 * h)
            d2 = (lp - 2 * la + lm) / (h * h)
            np.testing.assert_allclose(gl[:, e, ax], d1, rtol=1e-5, atol=1e-6)
            lapfd += d2 + d1 * d1
        np.testing.assert_allclose(gl[:, e, 3], lapfd, rtol=1e-3, atol=1e-3)


def test_comb_copies_each_walker_floor_or_ceil_of_its_share():
    rng = np.random.default_rng(0)
    for trial in range(20):
        W = int(rng.integers(1, 300))
        w = rng.exponential(size=W) * (rng.random(W) < 0.8)
        if w.sum() == 0:
            continue
        u = rng.random()
        idx = dmc.comb(w, u)
        assert idx.shape == (W,) and np.all(np.diff(idx) >= 0)
        counts = np.bincount(idx, minlength=W)
        share = W * w / w.sum()
        assert np.all(counts >= np.floor(share) - 1e-9) and np.all(counts <= np.ceil(share) + 1e-9)
        assert np.all(counts[w == 0] == 0)


def test_helium_fixed_node_dmc_reaches_the_exact_energy():
    """He ground state -2.903724 hartree; fixed-node DMC is exact for it."""
    W, steps, tau = 512, 2000, 0.02
    wl = make_helium(W, seed=1)
    rng = np.random.default_rng(5)
    s, la, gl = dmc.trial(wl, wl.R, PARAMS)
    st = dict(R=wl.R.copy(), sign=s, logabs=la, gl=gl, elocal=vmc.local_energy(wl.R, gl, 2.0),
              weight=np.ones(W))
    e_vmc = float(np.mean(st["elocal"]))
    es = []
    for k in range(steps):
        et = np.mean(es[50:]) if k > 60 else -2.9
        st, sums, acc = dmc.dmc_step(wl, st, tau, et, 2.0, rng.standard_normal((W, 2, 3)),
                                     rng.random(W), rng.random(), PARAMS)
        es.append(sums[1] / sums[0])
    es = np.array(es[steps // 4:])
    nb = 20
    b = es[: len(es) // nb * nb].reshape(nb, -1).mean(axis=1)
    e, err = es.mean(), b.std(ddof=1) / math.sqrt(nb)
    assert abs(e - (-2.903724)) < 4 * err + 0.005, (e, err)
    assert e < e_vmc - 0.02, (e, e_vmc)
