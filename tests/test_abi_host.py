"""CPU tests of the C-ABI library: it loads, exports every symbol that
include/mdet.h declares, and its host pre-processing (Sec. 2.1) matches the
oracle's independent one bit for bit.  No GPU is used (host-only context)."""
import os
import re

import numpy as np
import pytest

from gen.workloads import encode, make_config, make_custom
from oracle import preprocess as pp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdet.h")

mdet = pytest.importorskip("paper_1510_00730_amd")
from paper_1510_00730_amd import binding  # noqa: E402


def declared_symbols():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:mdet_status|void|const char \*)\s*(mdet_\w+)\s*\(",
                                 src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    syms = declared_symbols()
    assert len(syms) >= 9
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(binding.EXPORTED) == syms


def host_ctx(wl):
    ev = mdet.Evaluator(device=-1)
    ev.load_workload(wl)
    return ev


@pytest.mark.parametrize("cid", [1, 2, 3])
def test_indexing_bit_exact_vs_oracle(cid):
    wl = make_config(cid)
    ev = host_ctx(wl)
    got = ev.indexing()
    ref = pp.index_expansion(wl.det_up, wl.det_dn, wl.c)
    for k in ("uniq_up", "uniq_dn", "row_i", "col_j", "src_pos"):
        assert np.array_equal(got[k], ref[k]), k
    assert got["val"].tobytes() == ref["val"].tobytes()
    assert got["ref_up"] == ref["ref_up"] and got["ref_dn"] == ref["ref_dn"]
    st = ev.stats()
    assert st.n_det == wl.n_det and st.n_uniq_up == len(ref["uniq_up"])
    assert sum(st.n_by_degree_up) == st.n_uniq_up


@pytest.mark.parametrize("n_mo", [200, 300, 512])
def test_indexing_bit_exact_many_words(n_mo):
    """Encodings of 4, 5 and 8 words per determinant (orbitals beyond 128)."""
    from gen.workloads import make_custom
    wl = make_custom(9, 8, n_mo, 2, 400, 300, (1, 2, 3, 4), 4000, 4, seed=n_mo)
    assert wl.n_int == (n_mo + 63) // 64 >= 4
    ev = host_ctx(wl)
    got = ev.indexing()
    ref = pp.index_expansion(wl.det_up, wl.det_dn, wl.c)
    for k in ("uniq_up", "uniq_dn", "row_i", "col_j", "src_pos"):
        assert np.array_equal(got[k], ref[k]), k


@pytest.mark.slow
def test_indexing_bit_exact_largest_config():
    wl = make_config(4)
    ev = host_ctx(wl)
    got = ev.indexing()
    ref = pp.index_expansion(wl.det_up, wl.det_dn, wl.c)
    for k in ("uniq_up", "uniq_dn", "row_i", "col_j", "src_pos"):
        assert np.array_equal(got[k], ref[k]), k


def test_indexing_permutation_invariant_and_ties():
    wl = make_custom(5, 4, 130, 2, 40, 30, (1, 2, 3, 4), 600, 2, seed=3)   # 3 words
    # two dets with equal omega: words (a, b, 0) and (a^x, b^x, 0)
    ev = host_ctx(wl)
    a = ev.indexing()
    perm = np.random.default_rng(1).permutation(wl.n_det)
    ev.set_expansion(wl.n_up, wl.n_dn, wl.det_up[perm], wl.det_dn[perm], wl.c[perm])
    b = ev.indexing()
    for k in ("uniq_up", "uniq_dn", "row_i", "col_j", "val"):
        assert np.array_equal(a[k], b[k]), k
    ref = pp.index_expansion(wl.det_up[perm], wl.det_dn[perm], wl.c[perm])
    assert np.array_equal(b["src_pos"], ref["src_pos"])


def test_equal_omega_tie_break():
    # three 2-word up determinants with the same xor key {1, 2}: the order
    # must follow the words from the last to the first (unsigned)
    du = encode([[1, 64 + 2], [2, 64 + 1], [1, 2]], 2)
    assert len({pp.omega(tuple(int(x) for x in r)) for r in du}) == 1
    dd = encode([[0], [1], [2]], 2)
    wl = make_custom(2, 1, 100, 1, 3, 3, (1,), 3, 1, seed=0)
    c = np.array([0.9, 0.1, 0.2])
    ev = mdet.Evaluator(device=-1)
    ev.init_orbitals(wl.pow_abc, wl.alpha, wl.coef)
    ev.set_expansion(2, 1, du, dd, c)
    got = ev.indexing()
    ref = pp.index_expansion(du, dd, c)
    assert np.array_equal(got["uniq_up"], ref["uniq_up"])
    assert [int(r[1]) for r in got["uniq_up"]] == [0, 2, 4]


def _expect(code, fn):
    with pytest.raises(binding.MdetError) as ei:
        fn()
    assert ei.value.code == code, str(ei.value)


def test_error_codes():
    wl = make_config(1)
    ev = mdet.Evaluator(device=-1)
    _expect(-9, lambda: ev.set_expansion(5, 5, wl.det_up, wl.det_dn, wl.c))   # ESTATE
    ev.init_orbitals(wl.pow_abc, wl.alpha, wl.coef)
    _expect(-6, lambda: ev.set_expansion(4, 5, wl.det_up, wl.det_dn, wl.c))   # ESPIN
    bad = wl.det_up.copy(); bad[3, 0] |= np.uint64(1 << 19) | np.uint64(1 << 18)
    _expect(-3, lambda: ev.set_expansion(5, 5, bad, wl.det_dn, wl.c))         # EPOPCOUNT
    hi = wl.det_up.copy(); hi[2, 0] = np.uint64((1 << 25) | 0b1111)
    _expect(-4, lambda: ev.set_expansion(5, 5, hi, wl.det_dn, wl.c))          # EORBITAL
    _expect(-4, lambda: ev.set_expansion(5, 5, wl.det_up, wl.det_dn, wl.c, n_int=2))
    dup_u = np.concatenate([wl.det_up, wl.det_up[7:8]])
    dup_d = np.concatenate([wl.det_dn, wl.det_dn[7:8]])
    _expect(-5, lambda: ev.set_expansion(5, 5, dup_u, dup_d, np.append(wl.c, 0.01)))  # EDUPLICATE
    far = encode([[15, 16, 17, 18, 19]], 1)                                    # degree 5 from ref
    # a degree above 4 is a table-method degree (s x s minors up to 8 x 8)
    ev.set_expansion(5, 5, np.concatenate([wl.det_up, far]),
                     np.concatenate([wl.det_dn, wl.det_dn[:1]]), np.append(wl.c, 0.001))
    st = ev.stats()
    assert sum(st.n_by_degree_up) == st.n_uniq_up and st.n_by_degree_up[5] == 1
    # degree 9 (above MDET_MAX_DEGREE): accepted for the chain method, outside the counts
    ev10 = mdet.Evaluator(device=-1)
    ev10.init_orbitals(np.zeros((20, 1, 3), np.int32), np.full((20, 1), 0.5), np.ones((20, 1)))
    ref10 = list(range(10))
    up = encode([ref10, [0] + list(range(11, 20))], 1)
    dn = encode([list(range(9)), list(range(9))], 1)
    ev10.set_expansion(10, 9, up, dn, np.array([0.9, 0.1]))
    st = ev10.stats()
    assert sum(st.n_by_degree_up) == st.n_uniq_up - 1
    ev.set_expansion(5, 5, wl.det_up, wl.det_dn, wl.c)                         # still usable
    _expect(-9, lambda: ev.eval_raw(1, None, 0, None, None, None, None, None, None))
    _expect(-1, lambda: ev.set_fallback_threshold(-1.0))


def test_table_size_limit():
    """n_up * n_mo above 6144 is refused (the derivative kernel's per-walker
    tables must fit in LDS); 6144 itself is accepted."""
    for n_mo, n_up, code in ((512, 13, -2), (512, 12, 0)):
        rng = np.random.default_rng(5)
        ev = mdet.Evaluator(device=-1)
        ev.init_orbitals(np.zeros((n_mo, 1, 3), np.int32), np.ones((n_mo, 1)),
                         rng.normal(size=(n_mo, 1)))
        up = encode([list(range(n_up)), list(range(1, n_up + 1))], 8)
        dn = encode([list(range(n_up)), list(range(n_up))], 8)
        c = np.array([0.9, 0.1])
        if code:
            _expect(code, lambda: ev.set_expansion(n_up, n_up, up, dn, c, n_int=8))
        else:
            ev.set_expansion(n_up, n_up, up, dn, c, n_int=8)
