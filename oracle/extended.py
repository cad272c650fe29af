"""Extended-precision reference for a few walkers.

TEST INFRASTRUCTURE ONLY.

Eq. (1) and the derivative ratios of Eq. (nabla) (Sec. 2.3) evaluated in
x87 extended precision (numpy ``longdouble``, 64-bit significand): the
orbital values come from the oracle in FP64, every distinct spin
determinant's matrix is inverted by Gauss-Jordan elimination with partial
pivoting, its determinant is the signed product of the pivots, and the
derivative ratios follow from the row-replacement identity
grad~_e D / D = sum_c (S^-1)_{c e} grad~ phi_{occ(c)}(r_e).  It serves to
judge which of two FP64 evaluations is the more accurate where they
disagree (ill-conditioned determinants), not as the parity reference.
"""
from __future__ import annotations

import numpy as np

from . import Result, evaluate
from . import orbitals as _orbitals
from .preprocess import index_expansion, occupied

LD = np.longdouble


def _gj_inverse_det(A):
    """Batched inverse and determinant of A [B][n][n] in longdouble."""
    B, n, _ = A.shape
    A = A.copy()
    inv = np.broadcast_to(np.eye(n, dtype=LD), (B, n, n)).copy()
    det = np.ones(B, dtype=LD)
    b = np.arange(B)
    for j in range(n):
        p = j + np.argmax(np.abs(A[:, j:, j]), axis=1)
        rj, rp = A[b, j].copy(), A[b, p].copy()
        A[b, j], A[b, p] = rp, rj
        ij, ip = inv[b, j].copy(), inv[b, p].copy()
        inv[b, j], inv[b, p] = ip, ij
        det = np.where(p != j, -det, det)
        piv = A[:, j, j].copy()
        det = det * piv
        A[:, j, :] /= piv[:, None]
        inv[:, j, :] /= piv[:, None]
        for i in range(n):
            if i != j:
                f = A[:, i, j][:, None].copy()
                A[:, i, :] -= f * A[:, j, :]
                inv[:, i, :] -= f * inv[:, j, :]
    return inv, det


def _spin_terms(phi, occ):
    """phi [n][5][M] of the spin's electrons, occ [U][n] -> determinants [U]
    and derivative ratios [U][n][4]."""
    S = np.transpose(phi[:, 0, :][:, occ], (1, 0, 2))           # [U][e][c]
    inv, det = _gj_inverse_det(S)                                # [U][c][e]
    ratio = np.zeros((occ.shape[0], phi.shape[0], 4), dtype=LD)
    for q in range(4):
        G = np.transpose(phi[:, 1 + q, :][:, occ], (1, 0, 2))   # [U][e][c]
        ratio[:, :, q] = np.einsum("uce,uec->ue", inv, G)
    return det, ratio


def evaluate_extended(wl, R, rows=None):
    """Result (sign, logabs, gl in FP64 after the extended computation) for
    the walkers ``rows`` of R, every product of the expansion taken (no
    per-walker degree limits); the error scales rs_psi, rs_gl are the FP64
    oracle's (magnitudes only)."""
    rows = list(range(R.shape[0])) if rows is None else list(rows)
    ix = index_expansion(wl.det_up, wl.det_dn, wl.c)
    occ_up = np.array([occupied(d) for d in ix["uniq_up"]])
    occ_dn = np.array([occupied(d) for d in ix["uniq_dn"]])
    i, j, c = ix["row_i"], ix["col_j"], ix["val"].astype(LD)
    n_up, N = wl.n_up, wl.n_up + wl.n_dn
    W = len(rows)
    sign, logabs, gl = np.zeros(W), np.zeros(W), np.zeros((W, N, 4))
    for k, r in enumerate(rows):
        phi = np.array([_orbitals(wl, R[r, e], 0 if e < n_up else 1) for e in range(N)]).astype(LD)
        Du, ru = _spin_terms(phi[:n_up], occ_up)
        Dd, rd = _spin_terms(phi[n_up:], occ_dn)
        t = c * Du[i] * Dd[j]
        psi = t.sum()
        g = np.zeros((N, 4), dtype=LD)
        g[:n_up] = np.einsum("k,keq->eq", t, ru[i]) / psi
        g[n_up:] = np.einsum("k,keq->eq", t, rd[j]) / psi
        sign[k] = 1.0 if psi > 0 else -1.0
        logabs[k] = float(np.log(np.abs(psi)))
        gl[k] = g.astype(np.float64)
    o = evaluate(wl, R[rows], max_degree=None)
    return Result(sign, logabs, gl, o.rs_psi, o.rs_gl)
