"""Truncation schemes of the CI expansion (Sec. 3), written from the paper.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this module; the
library's own implementation (mdet_norm_truncation) is compared with it bit
for bit.

Norm-based scheme (Sec. 3, the decomposition of the norm): with
N = sum_ij C_ij^2 = sum_k c_k^2, the contribution of up determinant i is
N_i^up = sum_j C_ij^2 (likewise N_j^dn = sum_i C_ij^2), and
sum_i N_i^up = sum_j N_j^dn = N.  Spin determinants with a contribution at
or below their threshold are removed, with every product holding them.
Reading: contributions are taken relative to N (the paper's wavefunctions
are normalised), sums run over the products in input order in FP64.

Standard scheme (the one the paper compares against): products with
|c_k| <= eps are removed.
"""
from __future__ import annotations

import numpy as np


def _rows(dets: np.ndarray):
    d = np.asarray(dets, dtype=np.uint64)
    if d.ndim == 1:
        d = d[:, None]
    return [tuple(int(x) for x in row) for row in d]


def spin_norms(det_up, det_dn, c):
    """Per product k: (N^up of its up determinant, N^dn of its down
    determinant), each divided by N; plus the dicts {det: contribution / N}
    and N itself."""
    up, dn = _rows(det_up), _rows(det_dn)
    c = np.asarray(c, dtype=np.float64)
    total = 0.0
    nu: dict = {}
    nd: dict = {}
    for k in range(len(c)):          # input order, plain FP64 sums
        c2 = float(c[k]) * float(c[k])
        total += c2
        nu[up[k]] = nu.get(up[k], 0.0) + c2
        nd[dn[k]] = nd.get(dn[k], 0.0) + c2
    rel_u = {key: v / total for key, v in nu.items()}
    rel_d = {key: v / total for key, v in nd.items()}
    per_k = np.array([[rel_u[up[k]], rel_d[dn[k]]] for k in range(len(c))])
    return per_k, rel_u, rel_d, total


def norm_truncation(det_up, det_dn, c, eps_up, eps_dn=None):
    """Keep mask of the norm-based scheme and the numbers of kept products,
    distinct up and distinct down determinants."""
    eps_dn = eps_up if eps_dn is None else eps_dn
    per_k, _, _, _ = spin_norms(det_up, det_dn, c)
    keep = (per_k[:, 0] > eps_up) & (per_k[:, 1] > eps_dn)
    up, dn = _rows(det_up), _rows(det_dn)
    n_up = len({up[k] for k in range(len(keep)) if keep[k]})
    n_dn = len({dn[k] for k in range(len(keep)) if keep[k]})
    return keep, int(keep.sum()), n_up, n_dn


def coefficient_truncation(det_up, det_dn, c, eps):
    """The standard scheme: keep products with |c_k| > eps."""
    c = np.asarray(c, dtype=np.float64)
    keep = np.abs(c) > eps
    up, dn = _rows(det_up), _rows(det_dn)
    n_up = len({up[k] for k in range(len(keep)) if keep[k]})
    n_dn = len({dn[k] for k in range(len(keep)) if keep[k]})
    return keep, int(keep.sum()), n_up, n_dn
