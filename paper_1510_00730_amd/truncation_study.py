"""Truncation study on a synthetic expansion (analogue of the paper's Table 5,
Sec. 4): for the standard scheme (remove products with |c_k| <= eps) and the
norm-based scheme of Sec. 3 (remove spin determinants whose contribution to
the norm is <= eps), the numbers of products and distinct spin determinants
kept, and, with a GPU, the time of one evaluation of the truncated
expansion for the workload's walkers.

Run: python -m paper_1510_00730_amd.truncation_study [--config 4] [--no-gpu]
Prints a markdown table.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np


def _rows(d):
    return [tuple(int(x) for x in r) for r in np.asarray(d, dtype=np.uint64).reshape(len(d), -1)]


def counts(det_up, det_dn, keep):
    up, dn = _rows(det_up), _rows(det_dn)
    return (int(keep.sum()), len({up[k] for k in np.flatnonzero(keep)}),
            len({dn[k] for k in np.flatnonzero(keep)}))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--no-gpu", action="store_true")
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from gen.workloads import make_config
    from . import binding
    wl = make_config(args.config)
    c = wl.c / np.sqrt(np.sum(wl.c ** 2))
    gpu = None
    if not args.no_gpu:
        import torch
        if torch.cuda.is_available():
            ev = binding.Evaluator(0)
            ev.init_orbitals(wl.pow_abc, wl.alpha, wl.coef)
            R = torch.as_tensor(wl.R, dtype=torch.float64, device="cuda")
            gpu = (ev, R, torch)

    def timed(keep):
        if gpu is None or keep.sum() == 0:
            return None
        ev, R, torch = gpu
        ev.set_expansion(wl.n_up, wl.n_dn, wl.det_up[keep], wl.det_dn[keep], c[keep], wl.n_int)
        for _ in range(3):
            ev.eval_walkers(R, precision=binding.MDET_FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.reps):
            ev.eval_walkers(R, precision=binding.MDET_FP64)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / args.reps

    print(f"Workload {wl.name}: {wl.n_det} products, {wl.n_walk} walkers, c normalised; "
          f"GPU time = one FP64 evaluation of all walkers (ms)\n")
    print("| scheme | eps | products | up dets | down dets | GPU ms |")
    print("|---|---|---|---|---|---|")
    for eps in (0.5, 1e-2, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 0.0):
        keep = np.abs(c) > eps
        nk, nu, nd = counts(wl.det_up, wl.det_dn, keep)
        t = timed(keep)
        print(f"| abs(c_k) > eps | {eps:g} | {nk} | {nu} | {nd} | "
              f"{'-' if t is None else f'{t:.3f}'} |", flush=True)
    for eps in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 0.0):
        keep, nk, nu, nd = binding.norm_truncation(wl.det_up, wl.det_dn, c, eps)
        t = timed(keep)
        print(f"| N_i > eps | {eps:g} | {nk} | {nu} | {nd} | "
              f"{'-' if t is None else f'{t:.3f}'} |", flush=True)
    if gpu is not None:
        gpu[0].close()


if __name__ == "__main__":
    main()
