"""Helpers of the GPU parity tests: run the library through the C ABI and
compare with the FP64 oracle using the scaled error metric (each output's
error divided by the oracle's sum of absolute terms)."""
import math
import sys

import numpy as np

import oracle

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_eval(ev, R, precision=0, max_degree=None):
    import torch
    Rt = torch.as_tensor(np.ascontiguousarray(R), dtype=torch.float64, device="cuda")
    md = None
    if max_degree is not None:
        md = torch.as_tensor(np.asarray(max_degree, dtype=np.int8), device="cuda")
    sign, logabs, gl, ws = ev.eval_walkers(Rt, precision=precision, max_degree=md)
    torch.cuda.synchronize()
    return sign.cpu().numpy(), logabs.cpu().numpy(), gl.cpu().numpy(), ws.cpu().numpy()


def scaled_errors(ref, sign, logabs, gl, idx=None):
    """Per-walker scaled errors of the GPU outputs against the oracle.

    Psi:   |sigma sigma* exp(l - l*) - 1| * |Psi*| / S_Psi      (log domain)
    grad~: |x Psi - x* Psi*| / S_grad = |x sigma sigma* exp(l - l*) - x*| / (S_grad/|Psi*|)
    i.e. the error of grad~Psi itself (not of the quotient grad~Psi/Psi) over the
    oracle's sum of the absolute values of its terms, max over electrons and
    components.  idx maps oracle rows to GPU rows (default identity)."""
    W = ref.sign.shape[0]
    idx = np.arange(W) if idx is None else np.asarray(idx)
    ep = np.zeros(W)
    eg = np.zeros(W)
    for r in range(W):
        w = idx[r]
        if ref.sign[r] == 0.0:
            ep[r] = 0.0 if sign[w] == 0.0 else np.inf
            eg[r] = 0.0
            continue
        f = sign[w] * ref.sign[r] * math.exp(min(700.0, logabs[w] - ref.logabs[r]))
        ep[r] = abs(f - 1.0) / ref.rs_psi[r]
        eg[r] = np.max(np.abs(gl[w] * f - ref.gl[r]) / ref.rs_gl[r])
    return ep, eg


def ratio_errors(ref, gl, idx=None):
    """max |x - x*| / (S_grad/|Psi*|) for the quotient x = grad~Psi/Psi."""
    W = ref.sign.shape[0]
    idx = np.arange(W) if idx is None else np.asarray(idx)
    out = np.zeros(W)
    for r in range(W):
        if ref.sign[r] != 0.0:
            out[r] = np.max(np.abs(gl[idx[r]] - ref.gl[r]) / ref.rs_gl[r])
    return out


def rel_errors(ref, gl, idx=None):
    W = ref.sign.shape[0]
    idx = np.arange(W) if idx is None else np.asarray(idx)
    out = np.zeros(W)
    for r in range(W):
        d = np.linalg.norm(ref.gl[r])
        out[r] = np.linalg.norm(gl[idx[r]] - ref.gl[r]) / d if d > 0 else 0.0
    return out


def summary(name, ep, eg, ws=None):
    s = (f"{name}: psi scaled err p50 {np.median(ep):.2e} max {ep.max():.2e} | "
         f"grad/lap scaled err p50 {np.median(eg):.2e} p99 {np.percentile(eg, 99):.2e} "
         f"max {eg.max():.2e}")
    if ws is not None:
        s += f" | fallback {np.mean(ws == 1):.3f} node {np.mean(ws == 2):.3f}"
    log(s)
    return s
