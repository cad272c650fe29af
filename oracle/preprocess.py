"""Pre-processing of the CI expansion (Sec. 2.1), written plainly in Python.

TEST INFRASTRUCTURE ONLY (the product library has its own C++ version; the
two are compared bit for bit).

Steps, in the paper's order:
  1. Encoding: a spin determinant is n_int 64-bit words, bit b of word w set
     iff orbital 64*w+b is occupied (worked example of Sec. 2.1).
  2. Sort key omega = xor of the n_int words (Eq. (comp)); the shift by -2^63
     only emulates unsigned order in a signed language, so the order used here
     is the plain unsigned value.  Distinct determinants may share omega when
     n_int >= 2; the paper leaves their order open, and the reading taken here
     breaks ties by the words from the last to the first, unsigned.
  3. Duplicates removed -> the distinct spin lists (N_det^up, N_det^dn).
  4. Every product is located in both lists (binary search) and the sparse C
     is kept in coordinate form ordered by the key U*j + i (the paper's
     1-based U*(j-1)+i), i.e. column by column.
The reference spin determinants are those of the product with the largest
|c_k| (the earliest one on ties).
"""
from __future__ import annotations

import bisect

import numpy as np


def words_to_ints(det: np.ndarray) -> list:
    """uint64 [n][n_int] -> list of tuples of Python ints."""
    return [tuple(int(x) for x in row) for row in np.asarray(det, dtype=np.uint64)]


def omega(words) -> int:
    """Eq. (comp) without the signed shift: xor of all words, as unsigned."""
    k = 0
    for x in words:
        k ^= int(x)
    return k


def sort_key(words):
    return (omega(words),) + tuple(int(x) for x in reversed(words))


def occupied(words) -> list:
    """Decode a bit string into its ascending 0-based occupied orbitals."""
    out = []
    for w, x in enumerate(words):
        x = int(x)
        b = 0
        while x:
            if x & 1:
                out.append(64 * w + b)
            x >>= 1
            b += 1
    return out


def distinct_sorted(dets) -> list:
    return sorted(set(dets), key=sort_key)


def index_expansion(det_up, det_dn, c):
    """Return the paper's indexing of the expansion as a dict of arrays."""
    ups = words_to_ints(det_up)
    dns = words_to_ints(det_dn)
    uu = distinct_sorted(ups)
    ud = distinct_sorted(dns)
    ku = [sort_key(d) for d in uu]
    kd = [sort_key(d) for d in ud]
    U, V = len(uu), len(ud)
    n_det = len(ups)
    rows = np.empty(n_det, dtype=np.int64)
    cols = np.empty(n_det, dtype=np.int64)
    for k in range(n_det):
        i = bisect.bisect_left(ku, sort_key(ups[k]))
        j = bisect.bisect_left(kd, sort_key(dns[k]))
        assert uu[i] == ups[k] and ud[j] == dns[k]
        rows[k], cols[k] = i, j
    key = U * cols + rows
    order = np.argsort(key, kind="stable")
    c = np.asarray(c, dtype=np.float64)
    kref = int(np.argmax(np.abs(c)))          # first maximum
    n_int = len(ups[0])
    return dict(
        uniq_up=np.array(uu, dtype=np.uint64).reshape(U, n_int),
        uniq_dn=np.array(ud, dtype=np.uint64).reshape(V, n_int),
        row_i=rows[order].astype(np.int32),
        col_j=cols[order].astype(np.int32),
        val=c[order],
        src_pos=order.astype(np.int64),
        key=key[order],
        ref_up=int(rows[kref]),
        ref_dn=int(cols[kref]),
    )
