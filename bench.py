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


def kernel_model(name, wl, st, W, precision, n_fallback=0):
    """Algorithmic flops and HBM bytes of one launch of kernel `name` on W walkers.

    Counts follow the algorithm, not the implementation: an FMA is 2 flops,
    an exp is counted as 1 flop; bytes are what the kernel must read or write
    at least once (C once per launch, per-walker vectors once).
    Returns (flops, bytes, arithmetic type of the dominant operations).
    """
    n = (wl.n_up, wl.n_dn)
    M, P, N = wl.n_mo, wl.n_prim, wl.n_up + wl.n_dn
    U, V, Z = st.n_uniq_up, st.n_uniq_dn, st.n_det
    degs = (list(st.n_by_degree_up), list(st.n_by_degree_dn))
    b = 4 if precision == 1 else 8
    det_flops = {0: 0, 1: 0, 2: 3, 3: 2 * 27 // 3, 4: 2 * 64 // 3}     # LU of s x s
    adj_flops = {1: 0, 2: 0, 3: 2 * 27, 4: 2 * 64}                     # Gauss-Jordan
    if name == "k_spmm":
        flops = W * (4 * Z + 2 * U)
        byts = 2 * Z * (b + 4) + 4 * (U + V + 2) + W * (U + V) * 2 * b + W * 8
        return flops, byts, ("fp32" if b == 4 else "fp64")
    if name == "k_ratios":
        flops = W * sum(sum(c * det_flops[s] for s, c in enumerate(d)) for d in degs)
        byts = W * sum(nn * M * 8 for nn in n) + W * (U + V) * b
        return flops, byts, "fp64"
    if name == "k_deriv":
        f = 0
        for d, nn in zip(degs, n):
            f += sum(c * (adj_flops[s] + 2 * s * s) for s, c in enumerate(d) if s > 0)
            f += 2 * M * nn * nn + 2 * nn * nn * M + 4 * nn * 2 * (M + nn)
        byts = W * (sum(nn * M * 8 + nn * nn * 8 for nn in n) + (U + V) * b + 4 * N * M * 8
                    + N * 4 * 8 * 2)
        return W * f, byts, "fp64"
    if name == "k_reference":
        f = N * M * P * 36
        for nn in n:
            f += 2 * nn ** 3 + 4 * nn ** 3 + 2 * nn * nn * M + 8 * nn * nn
        byts = W * (N * 3 * 8 + 5 * N * M * 8 + sum(2 * nn * M * 8 for nn in n))
        return W * f, byts, "fp64"
    if name in ("k_direct_ratios", "k_direct_deriv"):
        # n_fallback (walker, spin) pairs, one LU per distinct determinant
        nn = max(n)
        per = 2 * nn ** 3 // 3 + (2 * nn ** 3 + 8 * nn * nn if name == "k_direct_deriv" else 0)
        return n_fallback * max(U, V) * per, n_fallback * 5 * nn * M * 8, "fp64"
    return 0, 0, "fp64"


def run_gpu(wl, precision, steps, warmup, pool, tune=True):
    """Eager timed region (per-kernel HIP events on the stream), then the same
    steps replayed as captured HIP graphs (launch overhead removed)."""
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
    if tune:  # the library's launch-configuration search (part of the warm-up)
        ev.autotune(Rpool[0], precision=precision, n_rep=5)
    for k in range(warmup):
        ev.eval_walkers(Rpool[k % len(Rpool)], precision=precision, out=out, stream=stream)
    torch.cuda.synchronize()
    # per-kernel times over an untimed pass; the timed steps then carry HIP
    # events around the dominant kernel only (two records per step)
    ev.set_profiling(True)
    for k in range(min(steps, 20)):
        ev.eval_walkers(Rpool[k % len(Rpool)], precision=precision, out=out, stream=stream)
    torch.cuda.synchronize()
    all_times, all_calls = ev.kernel_times()
    dom = max(all_times, key=lambda k: all_times[k])
    ev.set_profiling(True, kernels=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev.eval_walkers(Rpool[k % len(Rpool)], precision=precision, out=out, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_times, calls = ev.kernel_times()
    ev.set_profiling(False)
    # every kernel's figure from the untimed pass, the dominant one's from the timed steps
    times = {k: v / max(all_calls, 1) * calls for k, v in all_times.items()}
    times[dom] = dom_times[dom]
    ws = out[3].cpu().numpy()
    # graph replay of the same steps (one capture per walker buffer, untimed)
    for k in range(len(Rpool)):
        ev.eval_graph(Rpool[k], precision=precision, out=out, stream=stream)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for k in range(steps):
        ev.eval_graph(Rpool[k % len(Rpool)], precision=precision, out=out, stream=stream)
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    st = ev.stats()
    cfg = ev.launch_config()
    ev.close()
    return dict(dt=t1 - t0, dt_graph=g1 - g0, times=times, calls=calls, st=st, ws=ws, cfg=cfg)


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
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    cores = max(1, min(cores, os.cpu_count() or 1))
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


def cpu_baseline(wl, seconds):
    """The FP64 oracle on the host cores, on batches of the same walkers until
    `seconds` of wall time have passed (at least one batch)."""
    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    cores = max(1, min(cores, os.cpu_count() or 1))
    batch = 128
    oracle.evaluate(wl, wl.R[:cores], n_threads=cores)   # warm-up (page-in, thread pool)
    done, k = 0, 0
    t0 = time.perf_counter()
    while True:
        b0 = (k * batch) % wl.n_walk
        oracle.evaluate(wl, wl.R[b0:b0 + batch], n_threads=cores)
        done += min(batch, wl.n_walk - b0)
        k += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "walker-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} walker evaluations ({k} batches of up to {batch} of the same "
                      f"{wl.n_walk} walkers), FP64 oracle (one LU per distinct determinant, "
                      f"Eq. (1) compensated sum), {dt:.1f} s wall"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-chain", action="store_true",
                    help="skip the Sherman-Morrison chain comparison run")
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
    from gen.workloads import make_config, walker_pool
    wl = make_config(args.config)
    pool = walker_pool(wl, 8)
    prec = 1 if args.precision == "mixed" else 0
    res = {}
    for p in (prec, 1 - prec):
        r = run_gpu(wl, p, args.steps, args.warmup, pool, tune=not args.no_tune)
        res[p] = r
        print(f"[bench] precision {'mixed' if p else 'fp64'}: {args.steps * wl.n_walk / r['dt']:.4g} "
              f"walker-steps/s eager, {args.steps * wl.n_walk / r['dt_graph']:.4g} graph, "
              f"{1e3 * r['dt'] / args.steps:.3f} ms/step, config {r['cfg']}, kernels (ms/launch): "
              + ", ".join(f"{k} {v / max(r['calls'], 1):.4f}" for k, v in r["times"].items()),
              file=sys.stderr, flush=True)
    r = res[prec]
    W = wl.n_walk
    value = args.steps * W / r["dt"]
    dom = max(r["times"], key=lambda k: r["times"][k])
    avg_ms = r["times"][dom] / max(r["calls"], 1)
    n_fb = int(np.sum(r["ws"] == 1))
    flops, byts, kdt = kernel_model(dom, wl, r["st"], W, prec, n_fallback=n_fb)
    t = avg_ms * 1e-3
    peak_f = PEAK_FP32 if kdt == "fp32" else PEAK_FP64
    if byts / PEAK_HBM >= flops / peak_f:
        roof = {"bound": "hbm", "achieved": byts / t / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": flops / t / 1e12, "peak": peak_f / 1e12,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = read_traffic(dom)
    roof["kernel"] = dom
    roof["avg_launch_ms"] = avg_ms
    roof["algorithmic_flops"] = flops
    roof["algorithmic_bytes"] = byts
    line = {
        "metric": "walker-steps/s (Psi,∇,∇²) at 1e5 dets: FP64 vs mixed prec at rel err 1e-5",
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["dt"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if prec == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: 9+8 electrons, 100 orbitals x 4 primitives, "
                               f"1000+1000 distinct dets, 1e5 products, {W} walkers",
                   "precision": args.precision, "walker_batch": W,
                   "launch_config": list(r["cfg"]),
                   "fallback_fraction": float(np.mean(r["ws"] == 1))},
        "fp64_value": args.steps * W / res[0]["dt"],
        "mixed_value": args.steps * W / res[1]["dt"],
        "graph_value": args.steps * W / r["dt_graph"],
        "kernel_ms_per_launch": {k: v / max(r["calls"], 1) for k, v in r["times"].items()},
        "roofline": roof,
    }
    if not args.no_chain:
        ch = run_chain(wl, prec, min(args.steps, 50), min(args.warmup, 5), pool)
        print(f"[bench] sm chain ({ch['precision']}, pieces of {ch['piece_length']}): "
              f"{ch['value']:.4g} walker-steps/s, {ch['ms_per_step']:.3f} ms/step, "
              f"{ch['per_walker_step']}", file=sys.stderr, flush=True)
        if not args.no_cpu:
            ch["cpu_baseline"] = cpu_chain_baseline(wl, min(args.cpu_seconds, 6.0))
        line["sm_chain"] = ch
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
