"""ctypes binding of libmdet (include/mdet.h).  Argument marshalling only:
every step of the evaluation runs in the HIP kernels of libmdet.so.

PyTorch supplies device memory and the current stream; nothing here falls
back to a CPU path.  If the library is missing the import of this module
raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdet.so")

MDET_FP64, MDET_MIXED = 0, 1
W_OK, W_FALLBACK, W_NODE = 0, 1, 2
MAX_DEGREE = 8

STATUS = {0: "MDET_OK", -1: "MDET_EINVAL", -2: "MDET_EDIM", -3: "MDET_EPOPCOUNT",
          -4: "MDET_EORBITAL", -5: "MDET_EDUPLICATE", -6: "MDET_ESPIN", -7: "MDET_ENOMEM",
          -8: "MDET_EHIP", -9: "MDET_ESTATE", -10: "MDET_EDEGREE"}

# every symbol include/mdet.h declares (checked by the CPU tests)
EXPORTED = ["mdet_create", "mdet_destroy", "mdet_last_error", "mdet_init_orbitals",
            "mdet_set_expansion", "mdet_get_indexing", "mdet_eval_walkers",
            "mdet_set_fallback_threshold", "mdet_get_stats", "mdet_set_profiling",
            "mdet_get_kernel_times", "mdet_rng_fill", "mdet_vmc_step", "mdet_mlp_forward",
            "mdet_mlp_backward", "mdet_mlp_adam", "mdet_mlp_train_step", "mdet_set_launch_config",
            "mdet_get_launch_config", "mdet_eval_graph", "mdet_autotune",
            "mdet_norm_truncation", "mdet_set_method", "mdet_get_sm_counters",
            "mdet_set_jastrow", "mdet_dmc_step", "mdet_init_orbitals_dn",
            "mdet_set_profiling_mask", "mdet_eval_walkers_noalloc"]
METHOD_TABLE, METHOD_SM_CHAIN = 0, 1
PROP_GAUSSIAN, PROP_DRIFT, PROP_MLP = 0, 1, 2
OBJ_JUMP, OBJ_POTENTIAL = 0, 1
RNG_UNIFORM, RNG_NORMAL = 0, 1


class MdetError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int64), ("n_uniq_up", ctypes.c_int64),
                ("n_uniq_dn", ctypes.c_int64), ("n_up", ctypes.c_int32),
                ("n_dn", ctypes.c_int32), ("n_mo", ctypes.c_int32), ("n_prim", ctypes.c_int32),
                ("n_int", ctypes.c_int32), ("ref_up", ctypes.c_int64), ("ref_dn", ctypes.c_int64),
                ("n_by_degree_up", ctypes.c_int64 * (MAX_DEGREE + 1)),
                ("n_by_degree_dn", ctypes.c_int64 * (MAX_DEGREE + 1)),
                ("workspace_bytes", ctypes.c_int64), ("expansion_bytes", ctypes.c_int64),
                ("preprocess_seconds", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("spmm_row_splits", ctypes.c_int32), ("direct_split", ctypes.c_int32),
                ("sort_walkers", ctypes.c_int32), ("overlap_fallback", ctypes.c_int32),
                ("n_candidates", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmdet.  When PyTorch is installed it is imported first: its HIP
    runtime carries the same soname (libamdhip64.so.7), so the dynamic loader
    binds libmdet to it and the process holds one HIP runtime -- PyTorch's
    device pointers and streams are then valid in libmdet's calls.  Loading
    libmdet first would bring in a second runtime."""
    if not os.path.exists(path):
        raise ImportError(f"libmdet.so not built at {path}; run __graft_entry__.build()")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "mdet_create": (I32, [ctypes.POINTER(P), I32]),
        "mdet_destroy": (None, [P]),
        "mdet_last_error": (ctypes.c_char_p, [P]),
        "mdet_init_orbitals": (I32, [P, I32, I32, P, P, P]),
        "mdet_set_expansion": (I32, [P, I32, I32, I32, I64, P, P, P]),
        "mdet_get_indexing": (I32, [P, P, P, P, P, P, P, P, P, P, P]),
        "mdet_eval_walkers": (I32, [P, I64, P, I32, P, P, P, P, P, P]),
        "mdet_eval_walkers_noalloc": (I32, [P, I64, P, I32, P, P, P, P, P, P]),
        "mdet_set_fallback_threshold": (I32, [P, I32, D]),
        "mdet_get_stats": (I32, [P, P]),
        "mdet_set_profiling": (I32, [P, I32]),
        "mdet_get_kernel_times": (I32, [P, I32, P, P, P, P]),
        "mdet_rng_fill": (I32, [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, I64, I32, P, P]),
        "mdet_vmc_step": (I32, [P, I64, I32, D, P, I32, P, P, P, P, P, P, D, I32, P, P, P]),
        "mdet_mlp_forward": (I32, [P, I32, I32, I32, P, I64, P, P, P]),
        "mdet_mlp_backward": (I32, [P, I32, I32, I32, P, I64, P, P, P, P, P]),
        "mdet_mlp_adam": (I32, [P, I64, P, P, P, P, I32, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float, P]),
        "mdet_mlp_train_step": (I32, [P, I64, I32, P, P, P, I32, ctypes.c_float, P, P, I32, D, I32,
                                      D, P, P, P]),
        "mdet_set_launch_config": (I32, [P, I32, I32, I32, I32]),
        "mdet_get_launch_config": (I32, [P, P, P, P, P]),
        "mdet_eval_graph": (I32, [P, I64, P, I32, P, P, P, P, P, P]),
        "mdet_autotune": (I32, [P, I64, P, I32, P, I32, P]),
        "mdet_norm_truncation": (I32, [I32, I64, P, P, P, D, D, P, P, P, P]),
        "mdet_set_method": (I32, [P, I32, D, I32]),
        "mdet_get_sm_counters": (I32, [P, P]),
        "mdet_set_jastrow": (I32, [P, I32, D, D, D]),
        "mdet_init_orbitals_dn": (I32, [P, P, P, P]),
        "mdet_set_profiling_mask": (I32, [P, ctypes.c_uint32]),
        "mdet_dmc_step": (I32, [P, I64, D, D, D, I32, P, P, P, P, P, P, P, P, D, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB = load_library()


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Evaluator:
    """One libmdet context on one HIP device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        rc = _LIB.mdet_create(ctypes.byref(h), int(device))
        if rc != 0:
            raise MdetError(rc, f"mdet_create(device={device}) failed")
        self._h = h
        self.device = device
        self.n_up = self.n_dn = self.n_mo = 0

    def close(self):
        if getattr(self, "_h", None):
            _LIB.mdet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise MdetError(rc, _LIB.mdet_last_error(self._h).decode())

    # -------------------------------------------------------------- setup
    def init_orbitals(self, pow_abc, alpha, coef):
        pw = np.ascontiguousarray(pow_abc, dtype=np.int32)
        al = np.ascontiguousarray(alpha, dtype=np.float64)
        cf = np.ascontiguousarray(coef, dtype=np.float64)
        n_mo, n_prim = al.shape
        self._check(_LIB.mdet_init_orbitals(self._h, n_mo, n_prim, _ptr(pw), _ptr(al), _ptr(cf)))
        self.n_mo = n_mo

    def init_orbitals_dn(self, pow_abc, alpha, coef):
        """Separate orbitals for the down electrons (same shapes as init_orbitals)."""
        pw = np.ascontiguousarray(pow_abc, dtype=np.int32)
        al = np.ascontiguousarray(alpha, dtype=np.float64)
        cf = np.ascontiguousarray(coef, dtype=np.float64)
        self._check(_LIB.mdet_init_orbitals_dn(self._h, _ptr(pw), _ptr(al), _ptr(cf)))

    def set_expansion(self, n_up, n_dn, det_up, det_dn, c, n_int=None):
        du = np.ascontiguousarray(det_up, dtype=np.uint64)
        dd = np.ascontiguousarray(det_dn, dtype=np.uint64)
        cc = np.ascontiguousarray(c, dtype=np.float64)
        if du.ndim == 1:
            du = du.reshape(-1, 1)
            dd = dd.reshape(-1, 1)
        n_int = du.shape[1] if n_int is None else n_int
        self._check(_LIB.mdet_set_expansion(self._h, int(n_up), int(n_dn), int(n_int),
                                            int(cc.shape[0]), _ptr(du), _ptr(dd), _ptr(cc)))
        self.n_up, self.n_dn = int(n_up), int(n_dn)

    def load_workload(self, wl):
        self.init_orbitals(wl.pow_abc, wl.alpha, wl.coef)
        if getattr(wl, "alpha_dn", None) is not None:
            self.init_orbitals_dn(wl.pow_abc_dn, wl.alpha_dn, wl.coef_dn)
        self.set_expansion(wl.n_up, wl.n_dn, wl.det_up, wl.det_dn, wl.c, wl.n_int)

    def set_fallback_threshold(self, kappa_max: float, precision: int = -1):
        """Conditioning threshold of the table method for `precision`
        (MDET_FP64, MDET_MIXED, or -1 = both)."""
        self._check(_LIB.mdet_set_fallback_threshold(self._h, int(precision), float(kappa_max)))

    def set_method(self, method: int, sm_threshold: float = 1e-3, sm_chunk: int = 64):
        """METHOD_TABLE (default) or METHOD_SM_CHAIN (Sec. 2.2 update chain)."""
        self._check(_LIB.mdet_set_method(self._h, int(method), float(sm_threshold),
                                         int(sm_chunk)))

    def sm_counters(self):
        """Chain counters of the last chain evaluation (synchronises):
        dict(n_subst, n_inv, n_fail, n_start)."""
        out = np.zeros(4, dtype=np.int64)
        self._check(_LIB.mdet_get_sm_counters(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return dict(n_subst=int(out[0]), n_inv=int(out[1]), n_fail=int(out[2]),
                    n_start=int(out[3]))

    def indexing(self):
        nu = ctypes.c_int64()
        nd = ctypes.c_int64()
        self._check(_LIB.mdet_get_indexing(self._h, ctypes.byref(nu), ctypes.byref(nd),
                                           None, None, None, None, None, None, None, None))
        st = self.stats()
        n_int, Z = st.n_int, st.n_det
        out = dict(uniq_up=np.zeros((nu.value, n_int), np.uint64),
                   uniq_dn=np.zeros((nd.value, n_int), np.uint64),
                   row_i=np.zeros(Z, np.int32), col_j=np.zeros(Z, np.int32),
                   val=np.zeros(Z, np.float64), src_pos=np.zeros(Z, np.int64))
        ru, rd = ctypes.c_int64(), ctypes.c_int64()
        self._check(_LIB.mdet_get_indexing(self._h, None, None, _ptr(out["uniq_up"]),
                                           _ptr(out["uniq_dn"]), _ptr(out["row_i"]),
                                           _ptr(out["col_j"]), _ptr(out["val"]),
                                           _ptr(out["src_pos"]), ctypes.byref(ru),
                                           ctypes.byref(rd)))
        out["ref_up"], out["ref_dn"] = ru.value, rd.value
        return out

    def set_profiling(self, enable: bool, kernels=None):
        """Per-kernel HIP-event timing of later evaluations: every kernel, or
        only those named in `kernels` (names as kernel_times reports them)."""
        if not enable or kernels is None:
            self._check(_LIB.mdet_set_profiling(self._h, 1 if enable else 0))
            return
        order = list(self.kernel_times()[0])
        mask = 0
        for name in kernels:
            mask |= 1 << order.index(name)
        self._check(_LIB.mdet_set_profiling_mask(self._h, ctypes.c_uint32(mask)))

    def kernel_times(self):
        """{kernel name: total ms} over the profiled calls, and the call count."""
        cap = 32
        ms = np.zeros(cap)
        names = (ctypes.c_char_p * cap)()
        nk = ctypes.c_int32()
        nc = ctypes.c_int64()
        self._check(_LIB.mdet_get_kernel_times(self._h, cap, _ptr(ms), ctypes.cast(names, ctypes.c_void_p),
                                               ctypes.byref(nk), ctypes.byref(nc)))
        return {names[k].decode(): float(ms[k]) for k in range(nk.value)}, nc.value

    def stats(self) -> Stats:
        s = Stats()
        self._check(_LIB.mdet_get_stats(self._h, ctypes.byref(s)))
        return s

    # -------------------------------------------------------------- hot path
    def eval_raw(self, n_walk, R_ptr, precision, maxdeg_ptr, sign_ptr, logabs_ptr, gl_ptr,
                 wstatus_ptr, stream_ptr):
        """Direct call with raw device pointers (ints or c_void_p)."""
        self._check(_LIB.mdet_eval_walkers(self._h, int(n_walk), R_ptr, int(precision),
                                           maxdeg_ptr, sign_ptr, logabs_ptr, gl_ptr,
                                           wstatus_ptr, stream_ptr))

    def eval_walkers(self, R, precision=MDET_FP64, max_degree=None, out=None, stream=None):
        """R: torch float64 [W][N][3] on this device.  Returns (sign, logabs, gl, wstatus)
        torch tensors on the device; the call is asynchronous on ``stream``
        (default: torch's current stream)."""
        import torch
        if not (R.is_cuda and R.dtype == torch.float64 and R.is_contiguous()):
            raise ValueError("R must be a contiguous float64 tensor on the GPU")
        W, N = R.shape[0], R.shape[1]
        if N != self.n_up + self.n_dn or R.shape[2] != 3:
            raise ValueError("R must have shape [W][n_up+n_dn][3]")
        if max_degree is not None and not (max_degree.is_cuda and max_degree.dtype == torch.int8
                                           and max_degree.shape == (W,)):
            raise ValueError("max_degree must be an int8 [W] tensor on the GPU")
        if out is None:
            out = (torch.empty(W, dtype=torch.float64, device=R.device),
                   torch.empty(W, dtype=torch.float64, device=R.device),
                   torch.empty((W, N, 4), dtype=torch.float64, device=R.device),
                   torch.empty(W, dtype=torch.int32, device=R.device))
        sign, logabs, gl, ws = out
        if stream is None:
            stream = torch.cuda.current_stream(R.device)
        self.eval_raw(W, _dptr(R), precision, _dptr(max_degree), _dptr(sign), _dptr(logabs),
                      _dptr(gl), _dptr(ws), ctypes.c_void_p(stream.cuda_stream))
        return out

    def eval_walkers_noalloc(self, R, sign, logabs, gl, wstatus=None, precision=MDET_FP64,
                             max_degree=None, stream=None):
        """The allocation-free evaluation (mdet_eval_walkers_noalloc) into the
        caller's output tensors; the library's work buffers come from its
        static device scratch."""
        import torch
        W = R.shape[0]
        if stream is None:
            stream = torch.cuda.current_stream(R.device)
        self._check(_LIB.mdet_eval_walkers_noalloc(
            self._h, int(W), _dptr(R), int(precision), _dptr(max_degree), _dptr(sign),
            _dptr(logabs), _dptr(gl), _dptr(wstatus), ctypes.c_void_p(stream.cuda_stream)))
        return sign, logabs, gl, wstatus

    # -------------------------------------------------------------- VMC / MLP
    @staticmethod
    def _stream(stream):
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        return ctypes.c_void_p(s.cuda_stream)

    def rng_fill(self, out, seed, stream_id, step, kind=RNG_NORMAL, stream=None):
        """Fill the float64 device tensor `out` with Philox uniforms or normals."""
        self._check(_LIB.mdet_rng_fill(self._h, int(seed), int(stream_id), int(step), out.numel(),
                                       int(kind), _dptr(out), self._stream(stream)))
        return out

    def vmc_step(self, R, sign, logabs, gl, noise, uniform, elocal, accepted, proposal=PROP_GAUSSIAN,
                 step=0.3, mlp_params=None, n_hidden=0, nuclear_charge=None, precision=MDET_FP64,
                 stream=None):
        """One VMC step on device tensors, in place (see mdet_vmc_step)."""
        Z = float(self.n_up + self.n_dn) if nuclear_charge is None else float(nuclear_charge)
        self._check(_LIB.mdet_vmc_step(self._h, R.shape[0], int(proposal), float(step),
                                       _dptr(mlp_params), int(n_hidden), _dptr(R), _dptr(sign),
                                       _dptr(logabs), _dptr(gl), _dptr(noise), _dptr(uniform), Z,
                                       int(precision), _dptr(elocal), _dptr(accepted),
                                       self._stream(stream)))

    def set_jastrow(self, enable=True, b_ee=1.0, a_en=0.0, b_en=1.0):
        """Slater-Jastrow trial function exp(J) Psi (see mdet_set_jastrow)."""
        self._check(_LIB.mdet_set_jastrow(self._h, 1 if enable else 0, float(b_ee), float(a_en),
                                          float(b_en)))

    def dmc_step(self, R, sign, logabs, gl, elocal, weight, noise, uniform, comb_u, sums, accepted,
                 tau=0.01, e_trial=0.0, nuclear_charge=None, precision=MDET_FP64, stream=None):
        """One fixed-node DMC step on device tensors, in place (see mdet_dmc_step)."""
        Z = float(self.n_up + self.n_dn) if nuclear_charge is None else float(nuclear_charge)
        self._check(_LIB.mdet_dmc_step(self._h, R.shape[0], float(tau), float(e_trial), Z,
                                       int(precision), _dptr(R), _dptr(sign), _dptr(logabs),
                                       _dptr(gl), _dptr(elocal), _dptr(weight), _dptr(noise),
                                       _dptr(uniform), float(comb_u), _dptr(sums), _dptr(accepted),
                                       self._stream(stream)))

    def mlp_forward(self, params, X, n_hidden, n_out, Y=None, stream=None):
        import torch
        Y = torch.empty((X.shape[0], n_out), dtype=torch.float32, device=X.device) if Y is None else Y
        self._check(_LIB.mdet_mlp_forward(self._h, X.shape[1], int(n_hidden), int(n_out),
                                          _dptr(params), X.shape[0], _dptr(X), _dptr(Y),
                                          self._stream(stream)))
        return Y

    def mlp_backward(self, params, X, dY, n_hidden, want_dX=True, stream=None):
        import torch
        dp = torch.empty_like(params)
        dX = torch.empty_like(X) if want_dX else None
        self._check(_LIB.mdet_mlp_backward(self._h, X.shape[1], int(n_hidden), dY.shape[1],
                                           _dptr(params), X.shape[0], _dptr(X), _dptr(dY), _dptr(dp),
                                           _dptr(dX), self._stream(stream)))
        return dp, dX

    def mlp_adam(self, params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self._check(_LIB.mdet_mlp_adam(self._h, params.numel(), _dptr(params), _dptr(grads), _dptr(m),
                                       _dptr(v), int(t), float(lr), float(b1), float(b2), float(eps),
                                       self._stream(stream)))

    def mlp_train_step(self, params, m, v, t, lr, R, noise, n_hidden, loss, grad=None,
                       precision=MDET_FP64, jump_ref=0.0, objective=OBJ_JUMP,
                       nuclear_charge=None, stream=None):
        """One training step (see mdet_mlp_train_step); jump_ref > 0 weighs each
        electron's squared jump by 1 / (|r_e|^2 + jump_ref^2); objective
        OBJ_POTENTIAL maximises the expected squared change of the Coulomb
        potential energy (nucleus of charge nuclear_charge, default N)."""
        Z = float(self.n_up + self.n_dn) if nuclear_charge is None else float(nuclear_charge)
        self._check(_LIB.mdet_mlp_train_step(self._h, R.shape[0], int(n_hidden), _dptr(params),
                                             _dptr(m), _dptr(v), int(t), float(lr), _dptr(R),
                                             _dptr(noise), int(precision), float(jump_ref),
                                             int(objective), Z, _dptr(loss), _dptr(grad),
                                             self._stream(stream)))

    # -------------------------------------------------------------- tuning / graphs
    def set_launch_config(self, spmm_row_splits=0, direct_split=0, sort_walkers=True,
                          overlap_fallback=False):
        self._check(_LIB.mdet_set_launch_config(self._h, int(spmm_row_splits), int(direct_split),
                                                1 if sort_walkers else 0,
                                                1 if overlap_fallback else 0))

    def launch_config(self):
        a, b, c, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(_LIB.mdet_get_launch_config(self._h, ctypes.byref(a), ctypes.byref(b),
                                                ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, bool(c.value), bool(d.value)

    def eval_graph(self, R, precision=MDET_FP64, max_degree=None, out=None, stream=None):
        """Like eval_walkers, replaying a captured HIP graph of the whole step."""
        import torch
        W, N = R.shape[0], R.shape[1]
        if out is None:
            out = (torch.empty(W, dtype=torch.float64, device=R.device),
                   torch.empty(W, dtype=torch.float64, device=R.device),
                   torch.empty((W, N, 4), dtype=torch.float64, device=R.device),
                   torch.empty(W, dtype=torch.int32, device=R.device))
        sign, logabs, gl, ws = out
        st = ctypes.c_void_p(None) if stream is None else ctypes.c_void_p(stream.cuda_stream)
        self._check(_LIB.mdet_eval_graph(self._h, W, _dptr(R), int(precision), _dptr(max_degree),
                                         _dptr(sign), _dptr(logabs), _dptr(gl), _dptr(ws), st))
        return out

    def autotune(self, R, precision=MDET_FP64, max_degree=None, n_rep=10) -> TuneResult:
        r = TuneResult()
        self._check(_LIB.mdet_autotune(self._h, R.shape[0], _dptr(R), int(precision),
                                       _dptr(max_degree), int(n_rep), ctypes.byref(r)))
        return r


def norm_truncation(det_up, det_dn, c, eps_up, eps_dn=None):
    """Norm-based truncation (Sec. 3): keep mask [n_det] (bool) of the products
    whose up and down determinants both contribute more than eps to the norm,
    and the numbers of kept products and distinct up / down determinants."""
    import numpy as np
    du = np.ascontiguousarray(det_up, dtype=np.uint64)
    dd = np.ascontiguousarray(det_dn, dtype=np.uint64)
    cc = np.ascontiguousarray(c, dtype=np.float64)
    if du.ndim == 1:
        du = du[:, None]
        dd = dd[:, None]
    n_det, n_int = du.shape
    keep = np.zeros(n_det, dtype=np.uint8)
    nk, nu, nd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = _LIB.mdet_norm_truncation(int(n_int), int(n_det), _ptr(du), _ptr(dd), _ptr(cc),
                                   float(eps_up), float(eps_up if eps_dn is None else eps_dn),
                                   _ptr(keep), ctypes.byref(nk), ctypes.byref(nu), ctypes.byref(nd))
    if rc != 0:
        raise MdetError(rc, "mdet_norm_truncation failed")
    return keep.astype(bool), nk.value, nu.value, nd.value
