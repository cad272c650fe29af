"""FP64 reference of one variational Monte Carlo step and the local energy.

TEST INFRASTRUCTURE ONLY.

A VMC step (all electrons moved, the paper's Monte Carlo step of Sec. 4)
with a proposal R' from R, then the Metropolis-Hastings test
    accept  iff  u < min(1, |Psi(R')/Psi(R)|^2 q(R|R') / q(R'|R))  and Psi(R') != 0,
done in logs.  Proposals: Gaussian R' = R + step xi (symmetric q), or
drift-diffusion R' = R + tau F(R) + sqrt(tau) xi with F = grad ln|Psi| and
ln q(R'|R) = -|R' - R - tau F(R)|^2 / (2 tau) + const.
Local energy for a point nucleus of charge Z at the origin (atomic units):
    E_L = -1/2 sum_e lap_e Psi / Psi - Z sum_e 1/|r_e| + sum_{e<f} 1/|r_e - r_f|.
"""
from __future__ import annotations

import numpy as np


def local_energy(R, gl, Z):
    kin = -0.5 * np.sum(gl[:, :, 3], axis=1)
    ven = -Z * np.sum(1.0 / np.linalg.norm(R, axis=2), axis=1)
    diff = R[:, :, None, :] - R[:, None, :, :]
    dist = np.linalg.norm(diff, axis=3)
    iu = np.triu_indices(R.shape[1], 1)
    vee = np.sum(1.0 / dist[:, iu[0], iu[1]], axis=1)
    return kin + ven + vee


def propose(R, gl, xi, proposal, step):
    if proposal == 0:
        return R + step * xi
    return R + step * gl[:, :, :3] + np.sqrt(step) * xi


def log_accept(R, Rp, la, lap, gl, glp, proposal, step):
    """ln of the acceptance ratio (before the min with 0)."""
    ell = 2.0 * (lap - la)
    if proposal == 1:
        fwd = Rp - R - step * gl[:, :, :3]
        rev = R - Rp - step * glp[:, :, :3]
        ell += (np.sum(fwd * fwd, axis=(1, 2)) - np.sum(rev * rev, axis=(1, 2))) / (2.0 * step)
    return ell
