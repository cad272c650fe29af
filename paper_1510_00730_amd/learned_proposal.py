"""Learned Metropolis proposal vs the plain Gaussian proposal on the
1e5-determinant wavefunction (9+8 electrons, 100 orbitals), 2048 walkers.

1. Plain VMC with the Gaussian proposal; its step is tuned over a small grid
   by the expected squared jump distance (ESJD).
2. About 1e6 walker configurations are sampled from that chain (thinned).
3. The MLP proposal (51 -> 128 -> 128 -> 68, tanh, FP32) is trained on them
   with the library's training step (jump objective with the exact
   acceptance), once per jump weighting: the plain squared jump, and the
   jump of each electron relative to its distance from the nucleus
   (weights 1 / (r^2 + ref^2)), which counts the moves of the inner
   electrons that dominate the local energy.
4. Every proposal runs from the same equilibrated walkers -- the Gaussian at
   every step of the grid, so that the best Gaussian for the local energy is
   the baseline -- reporting acceptance, ESJD, integrated autocorrelation
   time of the walker-averaged local energy and of sum r^2, wall time per
   step, and effective samples per second = walkers * steps / time / tau_int.

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
    ap.add_argument("--compare-steps", type=int, default=6000)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--jump-refs", type=float, nargs="+", default=[0.0, 4.0],
                    help="jump weightings to train (0: plain squared jump)")
    ap.add_argument("--checkpoints", type=int, nargs="+", default=[100, 400, 1500],
                    help="training iterations at which the network is compared")
    ap.add_argument("--potential", action="store_true",
                    help="also train on the jump of the potential energy")
    ap.add_argument("--lr", type=float, default=1e-3)
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    from gen.workloads import make_config, mlp_init
    from . import Evaluator
    from .binding import OBJ_JUMP, OBJ_POTENTIAL, PROP_GAUSSIAN, PROP_MLP
    from .vmc import Walkers, run, tau_int, tau_int_walkers, train_proposal

    if args.quick:
        args.walkers, args.samples, args.compare_steps = 512, 60_000, 300
        args.checkpoints = [50, 200]
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
    grid = (0.1, 0.15, 0.2, 0.3, 0.45)
    for s in grid:
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
    # 3. training, one network per jump weighting, kept at a few points of
    #    its training (checkpoints)
    p0 = mlp_init(3 * N, H, 4 * N, seed=7)
    nets = {}
    objectives = [(f"jump_ref={ref:g}", OBJ_JUMP, ref) for ref in args.jump_refs]
    if args.potential:
        objectives.append(("potential", OBJ_POTENTIAL, 0.0))
    for oname, obj, ref in objectives:
        t0 = time.perf_counter()
        params, done, losses, state = p0, 0, [], {}
        for ck in sorted(args.checkpoints):
            params, ls = train_proposal(ev, samples, params, H, ck - done, min(2048, W),
                                        lr=args.lr, jump_ref=ref, seed=5, state=state,
                                        objective=obj, nuclear_charge=N)
            params = params.cpu().numpy()
            losses.extend(ls.tolist())
            done = ck
            nets[(oname, ck)] = params
        out.setdefault("training", {})[oname] = {
            "seconds": time.perf_counter() - t0,
            "loss_first_last": [float(np.mean(losses[:20])), float(np.mean(losses[-20:]))]}
    # 4. comparison from the same equilibrated walkers
    R_eq = w.R.cpu().numpy()
    res = {}
    runs = [(f"gaussian_step={s:g}", PROP_GAUSSIAN, s, None) for s in grid]
    runs += [(f"mlp_{oname}_iters={ck}", PROP_MLP, 0.0,
              (torch.as_tensor(p, dtype=torch.float32, device="cuda"), H))
             for (oname, ck), p in nets.items()]
    for name, prop, stp, mlp in runs:
        wk = Walkers(ev, R_eq, seed=202)
        run(wk, 50, prop, stp, mlp, record=False)
        jd = esjd_of(wk, run, 50, prop, stp, mlp)
        el, r2, acc, dt, (elw, r2w) = run(wk, args.compare_steps, prop, stp, mlp,
                                          per_walker=True)
        t_el, t_r2 = tau_int_walkers(elw), tau_int_walkers(r2w)
        t_el_avg = tau_int(el)
        del elw, r2w
        rate = W * args.compare_steps / dt
        res[name] = {"acceptance": float(acc.mean()), "esjd": jd,
                     "ms_per_step": 1e3 * dt / args.compare_steps,
                     "tau_int_E_L": t_el, "tau_int_sum_r2": t_r2,
                     "tau_int_E_L_from_averaged_series": t_el_avg, "mean_E_L": float(np.mean(el)),
                     "err_E_L": float(np.std(el) * np.sqrt(t_el / el.size)),
                     "mean_sum_r2": float(np.mean(r2)),
                     "effective_samples_per_s_E_L": rate / t_el,
                     "effective_samples_per_s_sum_r2": rate / t_r2}
        print(f"[proposal] {name}: {res[name]}", file=sys.stderr, flush=True)
    out["proposals"] = res
    gauss = {k: v for k, v in res.items() if k.startswith("gaussian")}
    best_g = max(gauss, key=lambda k: gauss[k]["effective_samples_per_s_E_L"])
    esjd_g = f"gaussian_step={step:g}"
    out["baseline_best_gaussian_E_L"] = best_g
    out["gain_E_L_vs_best_gaussian"] = {
        k: v["effective_samples_per_s_E_L"] / gauss[best_g]["effective_samples_per_s_E_L"]
        for k, v in res.items() if k.startswith("mlp")}
    out["gain_E_L_vs_esjd_tuned_gaussian"] = {
        k: v["effective_samples_per_s_E_L"] / gauss[esjd_g]["effective_samples_per_s_E_L"]
        for k, v in res.items() if k.startswith("mlp")}
    out["gain_sum_r2_vs_esjd_tuned_gaussian"] = {
        k: v["effective_samples_per_s_sum_r2"] / gauss[esjd_g]["effective_samples_per_s_sum_r2"]
        for k, v in res.items() if k.startswith("mlp")}
    out["total_seconds"] = time.perf_counter() - t_start
    print(json.dumps(out), flush=True)
    ev.close()
    return out


if __name__ == "__main__":
    main()
