"""Brute-force references for tiny inputs.

TEST INFRASTRUCTURE ONLY.

* Leibniz determinant (sum over permutations) for n <= 6, the textbook
  definition, used to check the oracle's LU determinants and its derivative
  ratios through the row-replacement identity grad~_e D = det(S with row e
  replaced by the derivative row).
* Eq. (1) by brute force: loop over the products, Leibniz per determinant,
  together with the sums of the absolute values of its terms (the error
  scales S_Psi = sum_k |c_k D_up D_dn| and, per electron and component,
  S_grad = sum_k |c_k grad~(D_up D_dn)|, over the terms of Eq. (1) and of
  Eq. (nabla), Sec. 2.3).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import orbitals as _orbitals
from .preprocess import occupied


def perm_sign(p) -> int:
    s = 1
    p = list(p)
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            s = -s
    return s


def leibniz(S) -> float:
    n = len(S)
    tot = 0.0
    for p in itertools.permutations(range(n)):
        prod = float(perm_sign(p))
        for i in range(n):
            prod *= S[i][p[i]]
        tot += prod
    return tot


def det_and_grad(S, G):
    """Leibniz det and grad~_e D for every row e (G: [4][n][n])."""
    n = len(S)
    D = leibniz(S)
    g = np.zeros((n, 4))
    for e in range(n):
        for q in range(4):
            Sr = [list(row) for row in S]
            Sr[e] = list(G[q][e])
            g[e, q] = leibniz(Sr)
    return D, g


def psi_brute(wl, Rw, with_abs=False):
    """Psi and grad~Psi (unnormalised, FP64, no scaling) by Eq. (1) with Leibniz.

    With ``with_abs`` also S_Psi and S_grad [N][4], the sums of the absolute
    values of the terms of Psi and of each component of grad~Psi."""
    N = wl.n_up + wl.n_dn
    orb = np.array([_orbitals(wl, Rw[e], spin=int(e >= wl.n_up)) for e in range(N)])  # [N][5][M]
    cache = {}

    def spin_det(words, e0, n):
        key = (tuple(int(x) for x in words), e0)
        if key not in cache:
            o = occupied(words)
            S = orb[e0:e0 + n, 0, :][:, o]
            G = orb[e0:e0 + n, 1:, :].transpose(1, 0, 2)[:, :, o]
            cache[key] = det_and_grad(S.tolist(), G.tolist())
        return cache[key]

    psi = 0.0
    grad = np.zeros((N, 4))
    s_psi = 0.0
    s_grad = np.zeros((N, 4))
    for k in range(wl.n_det):
        Du, gu = spin_det(wl.det_up[k], 0, wl.n_up)
        Dd, gd = spin_det(wl.det_dn[k], wl.n_up, wl.n_dn)
        psi += wl.c[k] * Du * Dd
        grad[:wl.n_up] += wl.c[k] * gu * Dd
        grad[wl.n_up:] += wl.c[k] * Du * gd
        # product rule: an up electron's derivative only touches D_up
        s_psi += abs(wl.c[k] * Du * Dd)
        s_grad[:wl.n_up] += np.abs(wl.c[k] * gu * Dd)
        s_grad[wl.n_up:] += np.abs(wl.c[k] * Du * gd)
    if with_abs:
        return psi, grad, s_psi, s_grad
    return psi, grad


def n_choose(m, n):
    return math.comb(m, n)
