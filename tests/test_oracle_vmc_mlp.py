"""Pins of the oracle's random numbers, MLP proposal and VMC step: published
known answers, closed forms, finite differences and sampling statistics."""
import math
import os

import numpy as np
import pytest

from oracle import mlp, rng, vmc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = [int(x, 16) for x in line.split()]
        out = rng.philox4x32_10(f[0:4], f[4:6])
        assert [int(x) for x in out] == f[6:10]


def test_uniform_and_normal_statistics():
    u = rng.uniforms(7, 1, 3, 400_000)
    assert 0.0 < u.min() and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / u.size)
    z = rng.normals(7, 2, 3, 400_000)
    assert abs(z.mean()) < 4 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4 * math.sqrt(2 / z.size)
    k = np.mean(z ** 4)
    assert abs(k - 3.0) < 0.05
    # different streams / steps give different numbers
    assert not np.array_equal(rng.normals(7, 2, 3, 16), rng.normals(7, 2, 4, 16))


def _params(n_in, n_hid, n_out, seed=0, scale=0.3):
    r = np.random.default_rng(seed)
    return r.normal(0, scale, mlp.n_params(n_in, n_hid, n_out))


def test_mlp_backward_finite_differences():
    n_in, n_hid, n_out, B = 6, 5, 8, 7
    p = _params(n_in, n_hid, n_out, 1)
    r = np.random.default_rng(2)
    X = r.normal(size=(B, n_in))
    dO = r.normal(size=(B, n_out))
    o, cache = mlp.forward(p, X, n_hid, n_out)
    gp, gX = mlp.backward(p, cache, dO, n_hid, n_out)
    f = lambda pp, XX: np.sum(dO * mlp.forward(pp, XX, n_hid, n_out)[0])
    h = 1e-6
    for i in r.choice(p.size, 20, replace=False):
        e = np.zeros_like(p); e[i] = h
        fd = (f(p + e, X) - f(p - e, X)) / (2 * h)
        assert abs(fd - gp[i]) < 1e-7 * (1 + abs(fd))
    for (b, j) in [(0, 0), (3, 5), (6, 2)]:
        e = np.zeros_like(X); e[b, j] = h
        fd = (f(p, X + e) - f(p, X - e)) / (2 * h)
        assert abs(fd - gX[b, j]) < 1e-7 * (1 + abs(fd))


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    new, m, v = mlp.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # bias-corrected first step: lr * g / (|g| + eps)
    np.testing.assert_allclose(new, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def _gaussian_psi(alpha):
    def fn(R):
        lp = -alpha * np.sum(R * R, axis=(1, 2))
        return lp, -2.0 * alpha * R
    return fn


def test_coulomb_potential_closed_form_and_gradient():
    # two electrons on the x axis at 1 and 3 around charge 2: V = -2 (1 + 1/3) + 1/2
    R = np.array([[[1.0, 0.0, 0.0], [3.0, 0.0, 0.0]]])
    V, g = mlp.coulomb_potential(R, 2.0)
    assert abs(V[0] - (-2.0 * (1 + 1 / 3) + 0.5)) < 1e-15
    # dV/dx1 = 2 x1/|x1|^3 - (x1 - x2)/|x1 - x2|^3 = 2 + 1/4, dV/dx2 = 2/9 - 1/4
    assert abs(g[0, 0, 0] - (2.0 + 0.25)) < 1e-14 and abs(g[0, 1, 0] - (2.0 / 9 - 0.25)) < 1e-14
    # finite differences on a random configuration
    rng = np.random.default_rng(7)
    R = rng.normal(0, 1.5, (2, 5, 3))
    V, g = mlp.coulomb_potential(R, 3.0)
    h = 1e-6
    for (b, e, ax) in ((0, 1, 2), (1, 4, 0), (1, 0, 1)):
        Rp, Rm = R.copy(), R.copy()
        Rp[b, e, ax] += h
        Rm[b, e, ax] -= h
        fd = (mlp.coulomb_potential(Rp, 3.0)[0][b] - mlp.coulomb_potential(Rm, 3.0)[0][b]) / (2 * h)
        assert abs(fd - g[b, e, ax]) < 1e-6 * (1 + abs(fd))


@pytest.mark.parametrize("jump_ref,objective", [(0.0, 0), (0.7, 0), (0.0, 1)])
def test_esjd_gradient_finite_differences(jump_ref, objective):
    N, n_hid, B = 3, 6, 5
    n_in, n_out = 3 * N, 4 * N
    p = _params(n_in, n_hid, n_out, 3, scale=0.2)
    r = np.random.default_rng(4)
    R = r.normal(0, 1.0, (B, N, 3))
    xi = r.normal(0, 1.0, (B, N, 3))
    psi = _gaussian_psi(0.4)
    lR = psi(R)[0]
    kw = dict(jump_ref=jump_ref, objective=objective, Z=3.0)
    loss, g, info = mlp.esjd_loss_and_grad(p, R, xi, lR, psi, n_hid, **kw)
    assert np.all(np.abs(info["ell"]) > 1e-3)      # no walker on the min(1, .) kink
    # the objective itself, written out
    if objective == 0:
        c = 1.0 if jump_ref <= 0 else 1.0 / (np.sum(R * R, axis=2) + jump_ref ** 2)
        J = info["A"] * np.sum(c * np.sum((info["Rp"] - R) ** 2, axis=2), axis=1)
    else:
        J = info["A"] * (mlp.coulomb_potential(info["Rp"], 3.0)[0]
                         - mlp.coulomb_potential(R, 3.0)[0]) ** 2
    assert abs(loss + J.mean()) < 1e-14 * abs(loss)
    h = 1e-6
    for i in r.choice(p.size, 25, replace=False):
        e = np.zeros_like(p); e[i] = h
        lp = mlp.esjd_loss_and_grad(p + e, R, xi, lR, psi, n_hid, **kw)[0]
        lm = mlp.esjd_loss_and_grad(p - e, R, xi, lR, psi, n_hid, **kw)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) < 2e-6 * (1 + abs(fd)), (i, fd, g[i])


def test_local_energy_closed_forms():
    # hydrogen-like 1s: Psi = exp(-Z r): grad = -Z r_hat, lap/Psi = Z^2 - 2Z/r -> E_L = -Z^2/2
    Z = 3.0
    R = np.array([[[0.3, -0.4, 1.2]]])
    r = np.linalg.norm(R[0, 0])
    gl = np.zeros((1, 1, 4))
    gl[0, 0, :3] = -Z * R[0, 0] / r
    gl[0, 0, 3] = Z * Z - 2 * Z / r
    assert abs(vmc.local_energy(R, gl, Z)[0] + Z * Z / 2) < 1e-13
    # two electrons, flat Psi, no nucleus: E_L = 1/|r1 - r2|
    R2 = np.array([[[0.0, 0.0, 0.0], [0.6, 0.8, 0.0]]]) + 5.0
    assert abs(vmc.local_energy(R2, np.zeros((1, 2, 4)), 0.0)[0] - 1.0) < 1e-14


@pytest.mark.parametrize("proposal,step", [(0, 0.6), (1, 0.3)])
def test_metropolis_samples_the_square_of_psi(proposal, step):
    """Psi = exp(-a r^2) -> |Psi|^2 gives <x^2> = 1/(4a) per coordinate."""
    a, N, W = 0.5, 2, 4000
    rr = np.random.default_rng(11)
    R = rr.normal(0, 1.0, (W, N, 3))

    def state(R):
        lp = -a * np.sum(R * R, axis=(1, 2))
        gl = np.zeros(R.shape[:2] + (4,))
        gl[:, :, :3] = -2 * a * R
        return lp, gl

    la, gl = state(R)
    acc = []
    x2 = []
    for it in range(400):
        xi = rr.normal(size=R.shape)
        Rp = vmc.propose(R, gl, xi, proposal, step)
        lap, glp = state(Rp)
        ell = vmc.log_accept(R, Rp, la, lap, gl, glp, proposal, step)
        u = rr.random(W)
        ok = np.log(u) < ell
        R = np.where(ok[:, None, None], Rp, R)
        la = np.where(ok, lap, la)
        gl = np.where(ok[:, None, None], glp, gl)
        acc.append(ok.mean())
        if it >= 100:
            x2.append(np.mean(R * R))
    x2 = np.array(x2)
    # blocks of 50 steps for the error bar
    blocks = x2.reshape(-1, 50).mean(axis=1)
    err = blocks.std(ddof=1) / math.sqrt(blocks.size)
    assert abs(x2.mean() - 1 / (4 * a)) < 4 * err + 2e-3
    assert 0.2 < np.mean(acc) < 0.99


def test_tau_int_walkers_ar1():
    """tau_int of a walker average from per-walker autocovariances, against
    the closed form (1 + phi) / (1 - phi) of AR(1) chains."""
    import torch
    from paper_1510_00730_amd.vmc import tau_int_walkers
    rng = np.random.default_rng(3)
    for phi in (0.0, 0.5, 0.9):
        n, W = 4000, 256
        x = np.zeros((n, W))
        z = rng.normal(size=(n, W))
        x[0] = z[0] / np.sqrt(1 - phi * phi)
        for t in range(1, n):
            x[t] = phi * x[t - 1] + z[t]
        tau = tau_int_walkers(torch.as_tensor(x))
        exact = (1 + phi) / (1 - phi)
        assert abs(tau - exact) < 0.08 * exact + 0.05, (phi, tau, exact)
