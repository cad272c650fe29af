"""FP64 CPU oracle for the multideterminant evaluator.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product library.  It
shares no code with the GPU path.

* ``oracle.c`` (built here with gcc into ``liboracle.so``): orbitals, one LU
  per distinct spin determinant, analytic derivative ratios, Eq. (1) and
  Eq. (main) sums.
* ``sm_chain.c`` (same library): the paper's own method, Sherman-Morrison
  substitutions along the sorted determinant list (Sec. 2.2), a CPU baseline
  checked against the direct LU of ``oracle.c``.
* ``preprocess.py``: the paper's determinant ordering and sparse indexing
  (Sec. 2.1), written independently of the library's C++ version.
* ``brute.py``: brute-force references for tiny inputs.
* ``extended.py``: the same sums in extended precision for a few walkers,
  to tell which of two disagreeing FP64 evaluations is the more accurate.
* ``mlp.py``, ``vmc.py``: FP64 references for the learned proposal and the
  Metropolis step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "sm_chain.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c and sm_chain.c with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", *_SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("MDET_ORACLE_LIB_OVERRIDE")   # mutation tests only
        if path is None:
            path = _LIB
            if not os.path.exists(path):
                build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.orc_eval.restype = ctypes.c_int
        lib.orc_eval.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P,
                                 P, P, P, ctypes.c_int, ctypes.c_int64, P, P, P, ctypes.c_int64,
                                 P, P, ctypes.c_int, P, P, P, P, P, ctypes.c_int]
        lib.orc_orbitals.restype = None
        lib.orc_orbitals.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P]
        lib.orc_slater.restype = ctypes.c_int
        lib.orc_slater.argtypes = [ctypes.c_int, P, P, P, P, P, P]
        I, L = ctypes.c_int, ctypes.c_int64
        lib.orc_sm_eval.restype = ctypes.c_int
        lib.orc_sm_eval.argtypes = [I, I, I, I, P, P, P, P, P, P, I, L, P, L, P, L, P, P, P, L, P,
                                    ctypes.c_double, I, P, P, P, P]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _orbital_set(wl, spin):
    """(pow_abc, alpha, coef) of the orbitals of `spin` (the down set if the
    workload has its own)."""
    if spin == 1 and getattr(wl, "alpha_dn", None) is not None:
        return wl.pow_abc_dn, wl.alpha_dn, wl.coef_dn
    return wl.pow_abc, wl.alpha, wl.coef


def _down_arrays(wl):
    if getattr(wl, "alpha_dn", None) is None:
        return None, None, None
    return (np.ascontiguousarray(wl.pow_abc_dn, dtype=np.int32),
            np.ascontiguousarray(wl.alpha_dn, dtype=np.float64),
            np.ascontiguousarray(wl.coef_dn, dtype=np.float64))


def orbitals(wl, r, spin=0):
    """[5][n_mo] values, grad x,y,z and Laplacian of every orbital of `spin` at point r."""
    lib = _load()
    pw0, al0, cf0 = _orbital_set(wl, spin)
    pw = np.ascontiguousarray(pw0, dtype=np.int32)
    al = np.ascontiguousarray(al0, dtype=np.float64)
    cf = np.ascontiguousarray(cf0, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.zeros((5, wl.n_mo))
    lib.orc_orbitals(wl.n_mo, wl.n_prim, _p(pw), _p(al), _p(cf), _p(r), _p(out))
    return out


def slater(S, G):
    """(sign, ln|det S|, ratio[n][4]) for S [n][n] and G [4][n][n]."""
    lib = _load()
    n = S.shape[0]
    S = np.ascontiguousarray(S, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    sg = np.zeros(1)
    la = np.zeros(1)
    rt = np.zeros((n, 4))
    work = np.zeros(2 * n * n + n)
    lib.orc_slater(n, _p(S), _p(G), _p(sg), _p(la), _p(rt), _p(work))
    return float(sg[0]), float(la[0]), rt


class Result:
    """sign [W], logabs [W], gl [W][N][4], rs_psi [W], rs_gl [W][N][4]."""

    def __init__(self, sign, logabs, gl, rs_psi, rs_gl):
        self.sign, self.logabs, self.gl, self.rs_psi, self.rs_gl = sign, logabs, gl, rs_psi, rs_gl


def evaluate(wl, R=None, max_degree="auto", mode=0, n_threads=0, c=None,
             det_up=None, det_dn=None):
    """Evaluate the wavefunction of workload ``wl`` at walkers ``R``.

    mode 0 = Eq. (1) compensated sum over products, 1 = Eq. (main) bilinear form.
    """
    lib = _load()
    R = wl.R if R is None else R
    R = np.ascontiguousarray(R, dtype=np.float64)
    W, N = R.shape[0], wl.n_up + wl.n_dn
    if isinstance(max_degree, str) and max_degree == "auto":
        max_degree = wl.max_degree
    md = None if max_degree is None else np.ascontiguousarray(max_degree, dtype=np.int8)
    c = np.ascontiguousarray(wl.c if c is None else c, dtype=np.float64)
    du = np.ascontiguousarray(wl.det_up if det_up is None else det_up, dtype=np.uint64)
    dd = np.ascontiguousarray(wl.det_dn if det_dn is None else det_dn, dtype=np.uint64)
    pw = np.ascontiguousarray(wl.pow_abc, dtype=np.int32)
    al = np.ascontiguousarray(wl.alpha, dtype=np.float64)
    cf = np.ascontiguousarray(wl.coef, dtype=np.float64)
    sign = np.zeros(W)
    logabs = np.zeros(W)
    gl = np.zeros((W, N, 4))
    rs_psi = np.zeros(W)
    rs_gl = np.zeros((W, N, 4))
    pwd, ald, cfd = _down_arrays(wl)
    rc = lib.orc_eval(wl.n_up, wl.n_dn, wl.n_mo, wl.n_prim, _p(pw), _p(al), _p(cf), _p(pwd),
                      _p(ald), _p(cfd), wl.n_int,
                      int(c.shape[0]), _p(du), _p(dd), _p(c), W, _p(R), _p(md), int(mode),
                      _p(sign), _p(logabs), _p(gl), _p(rs_psi), _p(rs_gl), int(n_threads))
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return Result(sign, logabs, gl, rs_psi, rs_gl)


class SMResult:
    """sign [W], logabs [W], gl [W][N][4] and the chain counters summed over
    walkers and both spins: n_subst (column substitutions done), n_inv
    (factorisations from scratch), n_fail (postponed substitution attempts)."""

    def __init__(self, sign, logabs, gl, stats, W):
        self.sign, self.logabs, self.gl = sign, logabs, gl
        self.n_subst, self.n_inv, self.n_fail = (int(x) for x in stats)
        self.n_walk = W


_INDEX_CACHE = {}


def _indexed(det_up, det_dn, c):
    """preprocess.index_expansion, remembered by the content of its inputs."""
    import hashlib
    from . import preprocess
    h = hashlib.sha256()
    for a in (det_up, det_dn, c):
        a = np.ascontiguousarray(a)
        h.update(str((a.dtype, a.shape)).encode())
        h.update(a.tobytes())
    key = h.hexdigest()
    if key not in _INDEX_CACHE:
        if len(_INDEX_CACHE) > 8:
            _INDEX_CACHE.clear()
        _INDEX_CACHE[key] = preprocess.index_expansion(det_up, det_dn, c)
    return _INDEX_CACHE[key]


def sm_evaluate(wl, R=None, threshold=1e-3, n_threads=0, det_up=None, det_dn=None, c=None):
    """Psi and grad~Psi/Psi by the paper's Sherman-Morrison chain (Sec. 2.2).

    The distinct spin determinants are visited in the order of Eq. (comp)
    (``preprocess.index_expansion``); every walker runs its own chain.  The
    whole expansion is used (no per-walker excitation limit).
    """
    lib = _load()
    R = wl.R if R is None else R
    R = np.ascontiguousarray(R, dtype=np.float64)
    W, N = R.shape[0], wl.n_up + wl.n_dn
    idx = _indexed(wl.det_up if det_up is None else det_up,
                   wl.det_dn if det_dn is None else det_dn, wl.c if c is None else c)
    uu = np.ascontiguousarray(idx["uniq_up"])
    ud = np.ascontiguousarray(idx["uniq_dn"])
    ri = np.ascontiguousarray(idx["row_i"], dtype=np.int32)
    cj = np.ascontiguousarray(idx["col_j"], dtype=np.int32)
    val = np.ascontiguousarray(idx["val"], dtype=np.float64)
    pw = np.ascontiguousarray(wl.pow_abc, dtype=np.int32)
    al = np.ascontiguousarray(wl.alpha, dtype=np.float64)
    cf = np.ascontiguousarray(wl.coef, dtype=np.float64)
    sign = np.zeros(W)
    logabs = np.zeros(W)
    gl = np.zeros((W, N, 4))
    stats = np.zeros(3, dtype=np.int64)
    pwd, ald, cfd = _down_arrays(wl)
    rc = lib.orc_sm_eval(wl.n_up, wl.n_dn, wl.n_mo, wl.n_prim, _p(pw), _p(al), _p(cf), _p(pwd),
                         _p(ald), _p(cfd), uu.shape[1], uu.shape[0], _p(uu), ud.shape[0], _p(ud), val.shape[0],
                         _p(ri), _p(cj), _p(val), W, _p(R), float(threshold), int(n_threads),
                         _p(sign), _p(logabs), _p(gl), _p(stats))
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return SMResult(sign, logabs, gl, stats, W)
