"""FP64 reference of the Slater-Jastrow trial function and of one
fixed-node diffusion Monte Carlo step.

TEST INFRASTRUCTURE ONLY.

Jastrow prefactor (the paper omits it from its algorithm and points to
standard O(N^2) techniques, Sec. 1): Psi_T = exp(J) Psi with
    J = sum_{i<j} u_ij(r_ij) + sum_i v(r_i),
    u_ij(r) = a_ij r / (1 + b_ee r),  a_ij = 1/2 (opposite spins), 1/4 (equal),
    v(r)    = a_en r / (1 + b_en r).
Product rule for the trial function's outputs, per electron e:
    grad ln Psi_T = grad J + grad Psi / Psi,
    lap Psi_T / Psi_T = lap J + |grad J|^2 + 2 grad J . grad Psi / Psi + lap Psi / Psi.

Fixed-node DMC step (importance sampled, drift-diffusion move with
Metropolis-Hastings acceptance, no node crossing), branching weight
w exp(-tau ((E_L + E_L')/2 - E_T)), then fixed-size resampling with the comb
(systematic resampling): new walker j copies the first walker whose
cumulative weight exceeds (j + u) sum w / W.
"""
from __future__ import annotations

import numpy as np

from . import vmc


def jastrow(R, n_up, b_ee, a_en, b_en):
    """J [W], grad J [W][N][3], lap J [W][N] for walkers R [W][N][3]."""
    R = np.asarray(R, dtype=np.float64)
    W, N, _ = R.shape
    J = np.zeros(W)
    g = np.zeros((W, N, 3))
    lap = np.zeros((W, N))
    for i in range(N):
        if a_en != 0.0:
            ri = np.linalg.norm(R[:, i], axis=1)
            s = 1.0 / (1.0 + b_en * ri)
            J += a_en * ri * s
            du = a_en * s * s
            g[:, i] += (du / ri)[:, None] * R[:, i]
            lap[:, i] += -2.0 * a_en * b_en * s ** 3 + 2.0 * du / ri
        for j in range(N):
            if j == i:
                continue
            a = 0.25 if (i < n_up) == (j < n_up) else 0.5
            d = R[:, i] - R[:, j]
            r = np.linalg.norm(d, axis=1)
            s = 1.0 / (1.0 + b_ee * r)
            if j > i:
                J += a * r * s
            du = a * s * s
            g[:, i] += (du / r)[:, None] * d
            lap[:, i] += -2.0 * a * b_ee * s ** 3 + 2.0 * du / r
    return J, g, lap


def apply_jastrow(R, n_up, params, logabs, gl):
    """Slater-Jastrow outputs from the expansion's (nodes left unchanged)."""
    b_ee, a_en, b_en = params
    J, gJ, lJ = jastrow(R, n_up, b_ee, a_en, b_en)
    logabs = np.array(logabs, dtype=np.float64)
    gl = np.array(gl, dtype=np.float64)
    live = np.isfinite(logabs)
    gd = gl[:, :, :3].copy()
    lap = gl[:, :, 3] + lJ + np.sum(gJ * gJ, axis=2) + 2.0 * np.sum(gJ * gd, axis=2)
    gl[live, :, 3] = lap[live]
    gl[live, :, :3] = gd[live] + gJ[live]
    logabs[live] += J[live]
    return logabs, gl


def trial(wl, R, params):
    """(sign, ln|Psi_T|, [grad ln Psi_T, lap Psi_T/Psi_T]) from the oracle's expansion."""
    from . import evaluate
    res = evaluate(wl, R, max_degree=None)
    if params is None:
        return res.sign, res.logabs, res.gl
    la, gl = apply_jastrow(R, wl.n_up, params, res.logabs, res.gl)
    return res.sign, la, gl


def comb(weights, u):
    """Indices of the walkers kept by the comb (systematic resampling)."""
    w = np.asarray(weights, dtype=np.float64)
    W = w.shape[0]
    tot = float(np.sum(w))
    if not tot > 0.0:
        return np.arange(W)
    cum = np.cumsum(w)
    x = (np.arange(W) + u) * (tot / W)
    return np.searchsorted(cum, x, side="right")


def dmc_step(wl, state, tau, e_trial, Z, noise, uniform, comb_u, params):
    """One step; state = dict(R, sign, logabs, gl, elocal, weight) (arrays over
    walkers).  Returns (new state, sums [4], accepted [W])."""
    R, sign, la, gl = state["R"], state["sign"], state["logabs"], state["gl"]
    e_old = state["elocal"]
    Rp = vmc.propose(R, gl, noise, 1, tau)
    sp, lap, glp = trial(wl, Rp, params)
    ell = vmc.log_accept(R, Rp, la, lap, gl, glp, 1, tau)
    acc = np.zeros(R.shape[0], dtype=bool)
    for w in range(R.shape[0]):
        if sp[w] == 0.0 or sp[w] != sign[w]:
            acc[w] = False
        elif sign[w] == 0.0:
            acc[w] = True
        else:
            acc[w] = np.log(uniform[w]) < ell[w]
    R = np.where(acc[:, None, None], Rp, R)
    gl = np.where(acc[:, None, None], glp, gl)
    sign = np.where(acc, sp, sign)
    la = np.where(acc, lap, la)
    e_new = vmc.local_energy(R, gl, Z)
    e_new = np.where(sign == 0.0, np.nan, e_new)
    ok = np.isfinite(e_old) & np.isfinite(e_new)
    x = np.where(ok, state["weight"] * np.exp(-tau * (0.5 * (e_old + e_new) - e_trial)), 0.0)
    sums = np.array([np.sum(x), np.sum(np.where(np.isfinite(e_new), x * e_new, 0.0)),
                     np.sum(x * x), float(np.sum(acc))])
    idx = comb(x, comb_u)
    new = dict(R=R[idx], sign=sign[idx], logabs=la[idx], gl=gl[idx], elocal=e_new[idx],
               weight=np.ones(R.shape[0]))
    return new, sums, acc
