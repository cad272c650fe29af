"""Learned Metropolis proposal vs the plain Gaussian proposal on the
1e5-determinant wavefunction (9+8 electrons, 100 orbitals), 2048 walkers.

1. Plain VMC with the Gaussian proposal; its step is tuned over a small grid
   by the expected squared jump distance (ESJD).
2. About 1e6 walker configurations are sampled from that chain (thinned).
3. The MLP proposal (51 -> 128 -> 128 -> 68, tanh, FP32) is trained on them
   with the library's training step (ESJD with the exact acceptance).
4. Both proposals run from the same equilibrated walkers; reported per
   proposal: acceptance, ESJD, integrated autocorrelation time of the
   walker-averaged local energy and of sum r^2, wall time per step, and
   effective samples per second = walkers * steps / time / tau_int.

Run: python -m paper_1510_00730_amd.learned_proposal [--quick]
Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def esjd_of(walkers, run_fn, n_steps, proposal, step, mlp=None):
    import torch
    R_prev = walkers.R.clone()
    jump = []
    for _ in range(n_steps):
        walkers.step(proposal, step, mlp)
        jump.append(torch.mean(torch.sum((walkers.R - R_prev) ** 2, dim=(1, 2))))
        R_prev.copy_(walkers.R)
    return float(torch.stack(jump).mean())


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="small sizes (test)")
    ap.add_argument("--walkers", type=int, default=2048)
    ap.add_argument("--samples", type=int, default=1_000_000)
    ap.add_argument("--train-iters", type=int, default=1500)
    ap.add_argument("--compare-steps", type=int, default=2000)
    ap.add_argument("--config", type=int, default=5)
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    from gen.workloads import make_config, mlp_init
    from . import Evaluator
    from .binding import PROP_GAUSSIAN, PROP_MLP
    from .vmc import Walkers, run, tau_int, train_proposal

    if args.quick:
        args.walkers, args.samples, args.train_iters, args.compare_steps = 512, 60_000, 200, 300
    wl = make_config(args.config, n_walk=args.walkers)
    ev = Evaluator(0)
    ev.load_workload(wl)
    N, H = wl.n_elec, 128
    W = args.walkers
    out = {"workload": f"{wl.name}: {wl.n_up}+{wl.n_dn} electrons, {wl.n_mo} orbitals, "
                       f"{wl.n_det} products, {W} walkers", "nuclear_charge": N}
    t_start = time.perf_counter()
    # 1. equilibrate and tune the Gaussian step by ESJD
    w = Walkers(ev, wl.R, seed=101)
    run(w, 150 if not args.quick else 60, PROP_GAUSSIAN, 0.2, record=False)
    best = None
    for s in (0.1, 0.15, 0.2, 0.3, 0.45):
        e = esjd_of(w, run, 40 if not args.quick else 15, PROP_GAUSSIAN, s)
        if best is None or e > best[1]:
            best = (s, e)
    step = best[0]
    out["gaussian_step"] = step
    # 2. samples from plain VMC (thinned by 5 steps)
    snaps = []
    n_snap = max(1, args.samples // W)
    for _ in range(n_snap):
        run(w, 5, PROP_GAUSSIAN, step, record=False)
        snaps.append(w.R.float().cpu().numpy())
    samples = np.concatenate(snaps).astype(np.float64)
    out["training_samples"] = int(samples.shape[0])
    # 3. training
    p0 = mlp_init(3 * N, H, 4 * N, seed=7)
    t0 = time.perf_counter()
    params, losses = train_proposal(ev, samples, p0, H, args.train_iters, min(2048, W), lr=1e-3)
    out["train_seconds"] = time.perf_counter() - t0
    out["train_loss_first_last"] = [float(np.mean(losses[:20])), float(np.mean(losses[-20:]))]
    # 4. comparison from the same equilibrated walkers
    R_eq = w.R.cpu().numpy()
    res = {}
    for name, prop, stp, mlp in (("gaussian", PROP_GAUSSIAN, step, None),
                                 ("mlp", PROP_MLP, 0.0, (params, H))):
        wk = Walkers(ev, R_eq, seed=202)
        run(wk, 50, prop, stp, mlp, record=False)
        jd = esjd_of(wk, run, 50, prop, stp, mlp)
        el, r2, acc, dt = run(wk, args.compare_steps, prop, stp, mlp)
        t_el, t_r2 = tau_int(el), tau_int(r2)
        rate = W * args.compare_steps / dt
        res[name] = {"acceptance": float(acc.mean()), "esjd": jd, "ms_per_step": 1e3 * dt / args.compare_steps,
                     "tau_int_E_L": t_el, "tau_int_sum_r2": t_r2, "mean_E_L": float(np.mean(el)),
                     "mean_sum_r2": float(np.mean(r2)),
                     "effective_samples_per_s_E_L": rate / t_el,
                     "effective_samples_per_s_sum_r2": rate / t_r2}
    out["proposals"] = res
    g, m = res["gaussian"], res["mlp"]
    out["gain_E_L"] = m["effective_samples_per_s_E_L"] / g["effective_samples_per_s_E_L"]
    out["gain_sum_r2"] = m["effective_samples_per_s_sum_r2"] / g["effective_samples_per_s_sum_r2"]
    out["total_seconds"] = time.perf_counter() - t_start
    print(json.dumps(out), flush=True)
    ev.close()
    return out


if __name__ == "__main__":
    main()
