"""Benchmark: walker-steps/s of the multideterminant evaluation (Psi, grad,
Laplacian of every electron) on the 1e5-determinant workload
(9+8 electrons, 100 orbitals, 1000 distinct determinants per spin, 1024
walkers), mixed precision and FP64, on one GPU.

A step is one call of the whole hot path (orbitals, reference LU, table,
ratios, sparse combination, derivatives) on a batch of 1024 walkers whose
coordinates already sit in HBM; a pool of 8 walker batches is rotated so
consecutive steps see different walkers.  The launch configuration is chosen
by the library's autotuner during the warm-up.  `value` is the eager rate
(kernels launched one by one); during the timed steps HIP events on the
library's stream bracket the dominant kernel only (found by an untimed
profiled pass, which also gives the other kernels' per-launch times);
`graph_value` is the same steps replayed as captured HIP graphs.  Prints one
JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64 = 78.6e12      # FP64 vector (and matrix) flop/s
PEAK_FP32 = 157.3e12     # FP32 vector flop/s
PEAK_HBM = 8.0e12        # bytes/s

# algorithmic flops of the small dense steps (an FMA counts 2)
DET_FLOPS = {0: 0, 1: 0, 2: 3, 3: 2 * 27 // 3, 4: 2 * 64 // 3}   # determinant of an s x s minor
ADJ_FLOPS = {0: 0, 1: 0, 2: 0, 3: 2 * 27, 4: 2 * 64}             # its cofactors (det M times M^-1)
EXP_FLOPS = 1                                                     # an exp counts as one flop


class Shape:
    """Per-walker algorithmic sizes of a workload: the electron counts, the
    distinct determinants of each spin by excitation degree, the products,
    and, for a batch with per-walker degree limits, the averages over the
    walkers of what each walker's limit keeps."""

    def __init__(self, wl):
        from oracle.preprocess import occupied
        self.n = (wl.n_up, wl.n_dn)
        self.N, self.M, self.P = wl.n_up + wl.n_dn, wl.n_mo, wl.n_prim
        k0 = int(np.argmax(np.abs(wl.c)))
        degs = []
        for dets in (wl.det_up, wl.det_dn):
            uniq, inv = np.unique(dets, axis=0, return_inverse=True)
            ref = set(occupied(dets[k0]))
            d = np.array([len(ref - set(occupied(u))) for u in uniq])
            degs.append((d, d[inv.ravel()]))
        md = wl.max_degree
        if md is None:
            lims, cnts = [1 << 30], [1]
        else:
            lims, cnts = np.unique(np.asarray(md, dtype=int), return_counts=True)
        self.U, self.V, self.Z = 0.0, 0.0, 0.0
        self.by_deg = [np.zeros(9), np.zeros(9)]
        for big, cnt in zip(lims, cnts):
            for sp in range(2):
                du = degs[sp][0]
                self.by_deg[sp] += cnt * np.bincount(du[du <= big], minlength=9)[:9]
            self.U += cnt * np.sum(degs[0][0] <= big)
            self.V += cnt * np.sum(degs[1][0] <= big)
            self.Z += cnt * np.sum((degs[0][1] <= big) & (degs[1][1] <= big))
        nl = float(np.sum(cnts))
        self.U, self.V, self.Z = self.U / nl, self.V / nl, self.Z / nl
        self.by_deg = [b / nl for b in self.by_deg]
        self.Z_total = wl.n_det


def kernel_model(name, sh, W, precision, n_fallback=0):
    """Algorithmic flops and HBM bytes of one launch of kernel `name` on W
    walkers, from the method's own operation counts (not this design's
    re-reads): an FMA is 2 flops, an exp 1; bytes are what the step must read
    or write at least once.  Returns (flops, bytes, dtype of the arithmetic).

    k_reference  orbitals with derivatives (N M P primitives, ~30 flops and one
                 exp each) and the reference LU, inverse and one residual
                 step per spin (6 n^3); reads the positions.
    k_ratios     the table T = A^-1 Phi on the virtual orbitals (2 n^2 (M-n)
                 per spin) and the s x s minor of every distinct determinant;
                 writes the ratio vectors.
    k_spmm       u = C R_dn, v = C^T R_up, psi = R_up.u: 4 Z + 2 U flops per
                 walker; reads C once per launch and the ratio vectors, writes
                 u and v.
    k_deriv      the derivative table B (8 n^2 (M-n) per spin), the cofactors
                 and weights of every distinct determinant (s x s inverse plus
                 2 s^2), the contraction; reads u and v, writes the outputs.
    k_finalize   writes sign, ln|Psi| and the outputs.
    k_direct_*   the direct-LU fallback's own algorithm on the flagged
                 (walker, spin) pairs: an LU per determinant (2 n^3 / 3), and
                 for the derivatives the n columns of its inverse (2 n^3) and
                 8 n^2 row-replacement sums.
    """
    n, M, P, N = sh.n, sh.M, sh.P, sh.N
    b = 4 if precision == 1 else 8
    uv = (sh.U + sh.V) * b
    if name == "k_reference":
        flops = N * M * P * (30 + EXP_FLOPS) + sum(6 * nn ** 3 for nn in n)
        return W * flops, W * N * 3 * 8, "fp64"
    if name == "k_ratios":
        flops = sum(2 * nn * nn * (M - nn) for nn in n)
        flops += sum(sum(c * DET_FLOPS.get(s, 2 * s ** 3 // 3) for s, c in enumerate(bd))
                     for bd in sh.by_deg)
        return W * flops, W * uv, "fp64"
    if name == "k_spmm":
        flops = 4 * sh.Z + 2 * sh.U
        byts = sh.Z_total * (8 + 4) * 2 + W * 2 * uv
        return W * flops, byts, ("fp32" if b == 4 else "fp64")
    if name == "k_deriv":
        flops = sum(8 * nn * nn * (M - nn) for nn in n)
        flops += sum(sum(c * (ADJ_FLOPS.get(s, 2 * s ** 3) + 2 * s * s) for s, c in enumerate(bd))
                     for bd in sh.by_deg)
        return W * flops, W * (uv + N * 4 * 8), "fp64"
    if name == "k_finalize":
        return W * 4 * N, W * (N * 4 * 8 + 3 * 8), "fp64"
    if name in ("k_direct_ratios", "k_direct_deriv"):
        nn = max(n)
        per = 2 * nn ** 3 // 3
        if name == "k_direct_deriv":
            per = 2 * nn ** 3 + 8 * nn * nn
        ndet = max(sh.U, sh.V)
        return n_fallback * ndet * per, n_fallback * 5 * nn * M * 8, "fp64"
    return 0, 0, "fp64"


def roofline(name, sh, W, precision, ms, n_fallback=0, traffic=None):
    """Roofline entry of one kernel: the binding roof is the larger of the
    minimum ALU time and the minimum HBM time of its algorithmic work."""
    flops, byts, kdt = kernel_model(name, sh, W, precision, n_fallback)
    t = ms * 1e-3
    if t <= 0 or (flops == 0 and byts == 0):
        return None
    peak_f = PEAK_FP32 if kdt == "fp32" else PEAK_FP64
    if byts / PEAK_HBM >= flops / peak_f:
        r = {"bound": "hbm", "achieved": byts / t / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    else:
        r = {"bound": "alu", "achieved": flops / t / 1e12, "peak": peak_f / 1e12,
             "unit": "TFLOP/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = traffic
    r["kernel"] = name
    r["avg_launch_ms"] = ms
    r["algorithmic_flops"] = float(flops)
    r["algorithmic_bytes"] = float(byts)
    r["arith"] = kdt
    return r


def run_gpu(wl, precision, steps, warmup, pool, tune=True):
    """Eager timed region (HIP events on the stream around the dominant
    kernel), then the same steps replayed as captured HIP graphs (launch
    overhead removed).  A workload with per-walker degree limits passes them
    with every batch.  Returns timings, the last batch's outputs and the
    index of the pool batch they belong to."""
    import torch
    import paper_1510_00730_amd as mdet
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    W, N = wl.R.shape[0], wl.n_elec
    Rpool = [torch.as_tensor(r, dtype=torch.float64, device="cuda") for r in pool]
    md = None
    if wl.max_degree is not None:
        md = torch.as_tensor(np.asarray(wl.max_degree, dtype=np.int8), device="cuda")
    out = (torch.empty(W, dtype=torch.float64, device="cuda"),
           torch.empty(W, dtype=torch.float64, device="cuda"),
           torch.empty((W, N, 4), dtype=torch.float64, device="cuda"),
           torch.empty(W, dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream()

    def step(k):
        ev.eval_walkers(Rpool[k % len(Rpool)], precision=precision, max_degree=md, out=out,
                        stream=stream)

    tuned = None
    if tune:  # the library's launch-configuration search (part of the warm-up)
        tuned = ev.autotune(Rpool[0], precision=precision, max_degree=md, n_rep=5)
    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    # per-kernel times over an untimed pass; the timed steps then carry HIP
    # events around the dominant kernel only (two records per step)
    ev.set_profiling(True)
    for k in range(min(steps, 20)):
        step(k)
    torch.cuda.synchronize()
    all_times, all_calls = ev.kernel_times()
    dom = max(all_times, key=lambda k: all_times[k])
    ev.set_profiling(True, kernels=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_times, calls = ev.kernel_times()
    ev.set_profiling(False)
    # every kernel's figure from the untimed pass, the dominant one's from the timed steps
    times = {k: v / max(all_calls, 1) * calls for k, v in all_times.items()}
    times[dom] = dom_times[dom]
    last = (steps - 1) % len(Rpool)
    outs = tuple(t.cpu().numpy() for t in out)
    # graph replay of the same steps (one capture per walker buffer, untimed)
    for k in range(len(Rpool)):
        ev.eval_graph(Rpool[k], precision=precision, max_degree=md, out=out, stream=stream)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for k in range(steps):
        ev.eval_graph(Rpool[k % len(Rpool)], precision=precision, max_degree=md, out=out,
                      stream=stream)
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    st = ev.stats()
    cfg = ev.launch_config() if tuned is None else (
        tuned.spmm_row_splits, tuned.direct_split, bool(tuned.sort_walkers),
        bool(tuned.overlap_fallback))
    ev.close()
    return dict(dt=t1 - t0, dt_graph=g1 - g0, times=times, calls=calls, st=st, ws=outs[3],
                cfg=cfg, outs=outs, last=last, dom=dom)


def timed_walker_errors(wl, R, outs, n_sample=64):
    """Errors of the outputs of a timed step against the FP64 oracle on a
    sample of its walkers: the scaled errors (each output's error over the
    oracle's sum of the absolute values of its terms; the parity gate) and
    the plain normwise relative error of grad~Psi/Psi (p50 / p99 / max)."""
    import math
    import oracle
    W = R.shape[0]
    rows = np.unique(np.linspace(0, W - 1, min(n_sample, W)).astype(int))
    md = None if wl.max_degree is None else np.asarray(wl.max_degree)[rows]
    ref = oracle.evaluate(wl, R[rows], max_degree=md, n_threads=0)
    sign, logabs, gl, _ = outs
    ep, eg, rel = [], [], []
    for r, w in enumerate(rows):
        if ref.sign[r] == 0.0:
            continue
        f = sign[w] * ref.sign[r] * math.exp(min(700.0, logabs[w] - ref.logabs[r]))
        ep.append(abs(f - 1.0) / ref.rs_psi[r])
        eg.append(float(np.max(np.abs(gl[w] * f - ref.gl[r]) / ref.rs_gl[r])))
        d = np.linalg.norm(ref.gl[r])
        rel.append(float(np.linalg.norm(gl[w] - ref.gl[r]) / d) if d > 0 else 0.0)
    rel = np.array(rel)
    return {"walkers": int(len(rows)), "max_scaled_psi": float(max(ep)),
            "max_scaled_grad_lap": float(max(eg)),
            "plain_rel_grad_lap": {"p50": float(np.median(rel)), "p99": float(np.percentile(rel, 99)),
                                   "max": float(rel.max())}}


def run_chain(wl, precision, steps, warmup, pool, chunks=(16, 32, 64, 128)):
    """The paper's Sherman-Morrison chain (Sec. 2.2) on the same walkers: the
    piece length is picked by a short sweep during the warm-up, then `steps`
    eager steps are timed like the table method's."""
    import torch
    import paper_1510_00730_amd as mdet
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    W, N = wl.R.shape[0], wl.n_elec
    Rpool = [torch.as_tensor(r, dtype=torch.float64, device="cuda") for r in pool]
    out = (torch.empty(W, dtype=torch.float64, device="cuda"),
           torch.empty(W, dtype=torch.float64, device="cuda"),
           torch.empty((W, N, 4), dtype=torch.float64, device="cuda"),
           torch.empty(W, dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream()
    best, sweep = None, {}
    for L in chunks:
        ev.set_method(mdet.METHOD_SM_CHAIN, 1e-3, L)
        for k in range(2):
            ev.eval_walkers(Rpool[k], precision=precision, out=out, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(5):
            ev.eval_walkers(Rpool[k % len(Rpool)], precision=precision, out=out, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sweep[str(L)] = 1e3 * dt / 5
        if best is None or dt < best[1]:
            best = (L, dt)
    L = best[0]
    ev.set_method(mdet.METHOD_SM_CHAIN, 1e-3, L)
    for k in range(warmup):
        ev.eval_walkers(Rpool[k % len(Rpool)], precision=precision, out=out, stream=stream)
    torch.cuda.synchronize()
    ev.set_profiling(True)
    counts = {"n_subst": 0, "n_inv": 0, "n_fail": 0, "n_start": 0}
    t0 = time.perf_counter()
    for k in range(steps):
        ev.eval_walkers(Rpool[k % len(Rpool)], precision=precision, out=out, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    times, calls = ev.kernel_times()
    ev.set_profiling(False)
    for k in range(len(Rpool)):  # counters of one pass over the walker pool (untimed)
        ev.eval_walkers(Rpool[k], precision=precision, out=out, stream=stream)
        c = ev.sm_counters()
        for key in counts:
            counts[key] += c[key]
    st = ev.stats()
    ev.close()
    nws = len(Rpool) * W
    ndet = st.n_uniq_up + st.n_uniq_dn
    # algorithmic FP64 work of k_sm_chain per walker-step from the measured
    # counts: a substitution is a mat-vec and a rank-1 update (4 n^2 flops), a
    # factorisation 2 n^3, the derivative ratios of a determinant 8 n^2 (n^2
    # weighted over the two spin lists)
    n2 = (wl.n_up ** 2 * st.n_uniq_up + wl.n_dn ** 2 * st.n_uniq_dn) / ndet
    n3 = (wl.n_up ** 3 * st.n_uniq_up + wl.n_dn ** 3 * st.n_uniq_dn) / ndet
    per = {k: v / nws for k, v in counts.items()}
    flops = W * (4 * n2 * per["n_subst"] + 2 * n3 * (per["n_inv"] + per["n_start"]) + 8 * n2 * ndet)
    t_k = times.get("k_sm_chain", 0.0) / max(calls, 1) * 1e-3
    roof = None
    if t_k > 0:
        roof = {"bound": "alu", "kernel": "k_sm_chain", "achieved": flops / t_k / 1e12,
                "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "avg_launch_ms": t_k * 1e3,
                "algorithmic_flops": flops}
        roof["frac"] = roof["achieved"] / roof["peak"]
    return {"value": steps * W / (t1 - t0), "unit": "walker-steps/s",
            "ms_per_step": 1e3 * (t1 - t0) / steps, "precision": "mixed" if precision else "fp64",
            "threshold": 1e-3, "piece_length": L,
            "piece_sweep_ms_per_step": sweep,
            "per_walker_step": {k: v / nws for k, v in counts.items()},
            "per_determinant": {"substitutions": counts["n_subst"] / (nws * ndet),
                                "factorisations": (counts["n_inv"] + counts["n_start"]) / (nws * ndet),
                                "retry_factorisations": counts["n_inv"] / (nws * ndet)},
            "kernel_ms_per_launch": {k: v / max(calls, 1) for k, v in times.items() if v > 0},
            "roofline": roof}


def cpu_chain_baseline(wl, seconds):
    """The paper's chain on the host cores (the oracle's CPU version), timed
    on batches of the same walkers for about `seconds`."""
    import oracle
    cores = host_cores()
    batch = 64
    oracle.sm_evaluate(wl, wl.R[:cores], n_threads=cores)
    done, k = 0, 0
    t0 = time.perf_counter()
    while True:
        b0 = (k * batch) % wl.n_walk
        oracle.sm_evaluate(wl, wl.R[b0:b0 + batch], n_threads=cores)
        done += min(batch, wl.n_walk - b0)
        k += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "walker-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} walker evaluations by the CPU Sherman-Morrison chain "
                      f"(threshold 1e-3, one chain per walker and spin), {dt:.1f} s wall"}


def host_cores():
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    return max(1, min(cores, os.cpu_count() or 1))


def cpu_baseline(wl, seconds, threads=None):
    """The FP64 oracle on `threads` host cores (default: all), on batches of
    the same walkers until `seconds` of wall time have passed (at least one
    batch)."""
    import oracle
    cores = host_cores() if threads is None else threads
    batch = max(8, min(128, 8 * cores))
    md = None if wl.max_degree is None else np.asarray(wl.max_degree)
    oracle.evaluate(wl, wl.R[:cores], max_degree=None if md is None else md[:cores],
                    n_threads=cores)   # warm-up (page-in, thread pool)
    done, k = 0, 0
    t0 = time.perf_counter()
    while True:
        b0 = (k * batch) % wl.n_walk
        b1 = min(wl.n_walk, b0 + batch)
        oracle.evaluate(wl, wl.R[b0:b1], max_degree=None if md is None else md[b0:b1],
                        n_threads=cores)
        done += b1 - b0
        k += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "walker-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} walker evaluations ({k} batches of up to {batch} of the same "
                      f"{wl.n_walk} walkers), FP64 oracle (one LU per distinct determinant, "
                      f"Eq. (1) compensated sum), {dt:.1f} s wall on {cores} thread(s)"}


def copy_probe(mib, reps):
    """A plain device copy of known size (for scaling HBM traffic counters)."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                      "reps": reps}), flush=True)


def kernel_source_sha():
    """sha256 over the sources of the table-method kernels (the kernel file and
    the device helpers it includes), as recorded in the counter summaries."""
    import hashlib
    h = hashlib.sha256()
    for f in ("mdet_kernels.hip", "mdet_device.h"):
        h.update(open(os.path.join(ROOT, "paper_1510_00730_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def read_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.md")
    try:
        text = open(path).read()
        sha = kernel_source_sha()
    except OSError:
        return None
    vals = {}
    for ln in text.splitlines():
        if ":" in ln and ln.startswith("- "):
            k, v = ln[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel source sha256") != sha:
        return None
    try:
        return float(vals["HBM bytes per launch (scaled)"])
    except (KeyError, ValueError):
        return None


WORKLOAD_LABEL = {
    1: "tiny: 5+5 electrons, 20 orbitals x 3 primitives, 50+50 distinct dets, 500 products, "
       "8 walkers",
    2: "c2_1e4: 9+8 electrons, 60 orbitals x 4 primitives, 300+300 distinct dets, 1e4 products, "
       "256 walkers",
    3: "c3_1e5: 9+8 electrons, 100 orbitals x 4 primitives, 1000+1000 distinct dets, "
       "1e5 products, 1024 walkers",
    4: "c4_uneven_7.5e5: 9+8 electrons, 120 orbitals x 4 primitives, 2500+2500 distinct dets, "
       "7.5e5 products, 4096 walkers with per-walker degree limits U{1..4}",
}


def measure_config(cid, steps, warmup, tune, n_sample, precisions=(1, 0), raw_order=False):
    """Both precisions of one workload: rates (eager and graph replay), every
    kernel's time and roofline entry, and the errors of a timed step's walkers
    against the oracle."""
    from gen.workloads import make_config, walker_pool
    wl = make_config(cid, raw_orbital_order=raw_order)
    pool = walker_pool(wl, 8)
    sh = Shape(wl)
    W = wl.n_walk
    res = {}
    for p in precisions:
        r = run_gpu(wl, p, steps, warmup, pool, tune=tune)
        n_fb = int(np.sum(r["ws"] == 1))
        kr = {}
        for k, v in r["times"].items():
            ms = v / max(r["calls"], 1)
            e = roofline(k, sh, W, p, ms, n_fallback=n_fb,
                         traffic=read_traffic(k) if k == r["dom"] else None)
            if e is not None:
                kr[k] = e
        err = timed_walker_errors(wl, pool[r["last"]], r["outs"], n_sample)
        name = "mixed" if p else "fp64"
        res[name] = {"value": steps * W / r["dt"], "graph_value": steps * W / r["dt_graph"],
                     "ms_per_step": 1e3 * r["dt"] / steps, "launch_config": list(r["cfg"]),
                     "fallback_fraction": float(np.mean(r["ws"] == 1)),
                     "dominant_kernel": r["dom"], "kernels": kr, "errors": err}
        print(f"[bench] config {cid} {name}: {res[name]['value']:.4g} walker-steps/s eager, "
              f"{res[name]['graph_value']:.4g} graph, {res[name]['ms_per_step']:.3f} ms/step, "
              f"config {r['cfg']}, errors {err['max_scaled_psi']:.1e}/{err['max_scaled_grad_lap']:.1e}"
              f" scaled, kernels: " + ", ".join(
                  f"{k} {e['avg_launch_ms']:.4f} ms ({e['bound']} {e['frac']:.3f})"
                  for k, e in kr.items()), file=sys.stderr, flush=True)
    return wl, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4],
                    help="workload of the headline line (3: 1e5 products; 4: the uneven "
                         "7.5e5-product batch)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-chain", action="store_true",
                    help="skip the Sherman-Morrison chain comparison run")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the other workloads' rows")
    ap.add_argument("--sample", type=int, default=64,
                    help="walkers of a timed step checked against the oracle")
    ap.add_argument("--raw-orbital-order", action="store_true",
                    help="keep the orbitals in the order drawn (near-singular reference at "
                         "most walkers: the conditioning fallback's stress case); headline only")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB buffer (traffic-counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); walkers are independent, "
              "so more GPUs would each run this same per-GPU workload.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe, 5)
        return
    prec = 1 if args.precision == "mixed" else 0
    pname = "mixed" if prec else "fp64"
    if args.raw_orbital_order:
        args.headline_only, args.no_chain = True, True
    wl, res = measure_config(args.config, args.steps, args.warmup, not args.no_tune, args.sample,
                             precisions=(prec, 1 - prec), raw_order=args.raw_orbital_order)
    r = res[pname]
    W = wl.n_walk
    roof = dict(r["kernels"][r["dominant_kernel"]])
    line = {
        "metric": "walker-steps/s (Psi,∇,∇²) at 1e5 dets: FP64 vs mixed prec at rel err 1e-5",
        "value": r["value"],
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if prec == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_LABEL[args.config] +
                   (" (orbitals in drawn order)" if args.raw_orbital_order else ""),
                   "precision": pname,
                   "walker_batch": W, "launch_config": r["launch_config"],
                   "fallback_fraction": r["fallback_fraction"]},
        "fp64_value": res["fp64"]["value"],
        "mixed_value": res["mixed"]["value"],
        "graph_value": r["graph_value"],
        "errors": {k: v["errors"] for k, v in res.items()},
        "kernel_ms_per_launch": {k: e["avg_launch_ms"] for k, e in r["kernels"].items()},
        "roofline": roof,
        "kernel_roofline": {k: {kk: e[kk] for kk in ("bound", "frac", "achieved", "unit",
                                                     "avg_launch_ms")}
                            for k, e in r["kernels"].items()},
    }
    cpu_main = None
    if not args.no_cpu:
        cpu_main = cpu_baseline(wl, args.cpu_seconds)
        cpu_1 = cpu_baseline(wl, min(args.cpu_seconds, 8.0), threads=1)
        line["cpu_baseline_1thread"] = cpu_1
    if not args.headline_only:
        rows = {}
        for cid in (1, 2, 3, 4):
            if cid == args.config:
                rr = res
            else:
                _, rr = measure_config(cid, min(args.steps, 50), min(args.warmup, 5),
                                       not args.no_tune, min(args.sample, 32))
            row = {k: {"value": v["value"], "graph_value": v["graph_value"],
                       "ms_per_step": v["ms_per_step"], "fallback_fraction": v["fallback_fraction"],
                       "errors": v["errors"],
                       "kernel_roofline": {kk: {"bound": e["bound"], "frac": e["frac"],
                                                "avg_launch_ms": e["avg_launch_ms"]}
                                           for kk, e in v["kernels"].items()}}
                   for k, v in rr.items()}
            if not args.no_cpu and cid != args.config:
                from gen.workloads import make_config
                wc = make_config(cid)
                row["cpu_oracle"] = {"all_cores": cpu_baseline(wc, 2.0)["value"],
                                     "one_thread": cpu_baseline(wc, 2.0, threads=1)["value"],
                                     "cores": host_cores()}
            rows[WORKLOAD_LABEL[cid].split(":")[0]] = row
        line["all_configs"] = rows
    if not args.no_chain and args.config == 3:
        from gen.workloads import walker_pool
        ch = run_chain(wl, prec, min(args.steps, 50), min(args.warmup, 5), walker_pool(wl, 8))
        print(f"[bench] sm chain ({ch['precision']}, pieces of {ch['piece_length']}): "
              f"{ch['value']:.4g} walker-steps/s, {ch['ms_per_step']:.3f} ms/step, "
              f"{ch['per_walker_step']}", file=sys.stderr, flush=True)
        if not args.no_cpu:
            ch["cpu_baseline"] = cpu_chain_baseline(wl, min(args.cpu_seconds, 6.0))
        line["sm_chain"] = ch
    if cpu_main is not None:
        line["cpu_baseline"] = cpu_main
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
