"""Pins of the oracle's pre-processing (Sec. 2.1) against the paper's worked
examples and against invariants of the ordering rule."""
import itertools
import math
import os

import numpy as np

from gen.workloads import encode, make_config, make_custom
from oracle import preprocess as pp

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                out.append(line.split())
    return out


def test_encoding_worked_example():
    # Sec. 2.1: HF of Cl = (511, 255); excitation MO 7 -> 12 on both spins = (2495, 2239)
    for label, up1, dn1, dec_up, dec_dn, bin_up, bin_dn in _rows("encoding_cl.txt"):
        up = [int(x) - 1 for x in up1.split(",")]
        dn = [int(x) - 1 for x in dn1.split(",")]
        wu = encode([up], 1)[0]
        wd = encode([dn], 1)[0]
        assert int(wu[0]) == int(dec_up) and int(wd[0]) == int(dec_dn), label
        assert format(int(wu[0]), "b") == bin_up and format(int(wd[0]), "b") == bin_dn
        # the oracle's decoder inverts the encoding
        assert pp.occupied(wu) == up and pp.occupied(wd) == dn


def test_table1_ordering():
    # Table 1: the 70 four-in-eight determinants sorted by Eq. (comp)
    dets = [tuple(c) for c in itertools.combinations(range(8), 4)]
    rng = np.random.default_rng(0)
    rng.shuffle(dets)
    words = encode(dets, 1)
    ordered = pp.distinct_sorted(pp.words_to_ints(words))
    assert len(ordered) == 70
    for idx, dec, binary, occ in _rows("table1_ordering.txt"):
        w = ordered[int(idx) - 1]
        assert int(w[0]) == int(dec)
        assert format(int(w[0]), "08b") == binary
        assert "".join(str(m + 1) for m in pp.occupied(w)) == occ


def test_omega_is_xor_of_words_and_ties_broken_by_high_word():
    # two determinants with equal omega in two words are ordered by word 1 then word 0
    a = (0b1011, 0b0110)
    b = (0b1101, 0b0000)   # xor: 0b1101 for both
    c = (0b0000, 0b1101)
    assert pp.omega(a) == pp.omega(b) == pp.omega(c) == 0b1101
    got = pp.distinct_sorted([c, a, b])
    assert got == [b, a, c]


def test_unsigned_order_of_high_bit():
    # the -2^63 shift of Eq. (comp) makes a set top bit sort last (unsigned order)
    hi = (1 << 63) | 1
    lo = 3
    got = pp.distinct_sorted([(hi,), (lo,)])
    assert got == [(lo,), (hi,)]


def test_indexing_invariants_and_permutation_independence():
    wl = make_custom(4, 3, 70, 2, 30, 25, (1, 2, 3), 400, 2, seed=11)
    ix = pp.index_expansion(wl.det_up, wl.det_dn, wl.c)
    U, V = len(ix["uniq_up"]), len(ix["uniq_dn"])
    # FCI bound (Sec. 1): at most C(M, n) distinct spin determinants
    assert U <= math.comb(wl.n_mo, wl.n_up) and V <= math.comb(wl.n_mo, wl.n_dn)
    # column-major order: nondecreasing (j, i), strictly increasing key
    assert np.all(np.diff(ix["key"]) > 0)
    # every entry maps back to its input product
    for t in range(wl.n_det):
        k = ix["src_pos"][t]
        assert tuple(ix["uniq_up"][ix["row_i"][t]]) == tuple(wl.det_up[k])
        assert tuple(ix["uniq_dn"][ix["col_j"][t]]) == tuple(wl.det_dn[k])
        assert ix["val"][t] == wl.c[k]
    # shuffling the input products changes only src_pos
    perm = np.random.default_rng(5).permutation(wl.n_det)
    ix2 = pp.index_expansion(wl.det_up[perm], wl.det_dn[perm], wl.c[perm])
    for name in ("uniq_up", "uniq_dn", "row_i", "col_j", "val"):
        assert np.array_equal(ix[name], ix2[name]), name
    assert np.array_equal(perm[ix2["src_pos"]], ix["src_pos"])
    # the reference is the product with the largest |c| (c_0 = 0.95)
    assert ix["ref_up"] == ix["row_i"][np.where(ix["src_pos"] == 0)[0][0]]


def test_indexing_two_word_config():
    wl = make_config(3)
    ix = pp.index_expansion(wl.det_up[:3000], wl.det_dn[:3000], wl.c[:3000])
    keys = [pp.sort_key(tuple(int(x) for x in r)) for r in ix["uniq_up"]]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
