"""Variational Monte Carlo driver on top of libmdet (all arithmetic in the
library's HIP kernels; this module only sequences calls and keeps
statistics).

* `Walkers`: the walker state on the device (positions, sign, ln|Psi|,
  grad~Psi/Psi) and the Philox stream counters for move noise and
  acceptance uniforms.
* `run`: VMC steps with the Gaussian, drift-diffusion or MLP proposal,
  returning the walker-averaged local energy per step and the acceptance.
* `train_proposal`: the MLP proposal trained on walker configurations
  sampled by plain VMC, one library training step per batch.
* `tau_int`: integrated autocorrelation time with Sokal's automatic
  window (c = 5); `tau_int_walkers` the same for a walker average from the
  per-walker autocovariances.
"""
from __future__ import annotations

import time

import numpy as np

from .binding import (MDET_FP64, PROP_DRIFT, PROP_GAUSSIAN, PROP_MLP, RNG_NORMAL, RNG_UNIFORM,
                      Evaluator)

NOISE_STREAM, UNIFORM_STREAM, TRAIN_STREAM = 1, 2, 3


class Walkers:
    def __init__(self, ev: Evaluator, R0, seed=1, precision=MDET_FP64):
        import torch
        self.ev, self.seed, self.precision = ev, int(seed), precision
        self.R = torch.as_tensor(np.ascontiguousarray(R0), dtype=torch.float64, device="cuda").clone()
        W, N = self.R.shape[0], self.R.shape[1]
        self.N, self.W = N, W
        self.sign, self.logabs, self.gl, _ = ev.eval_walkers(self.R, precision=precision)
        self.noise = torch.empty((W, N, 3), dtype=torch.float64, device="cuda")
        self.uniform = torch.empty(W, dtype=torch.float64, device="cuda")
        self.elocal = torch.empty(W, dtype=torch.float64, device="cuda")
        self.accepted = torch.empty(W, dtype=torch.int32, device="cuda")
        self.step_count = 0

    def step(self, proposal=PROP_GAUSSIAN, step=0.3, mlp=None):
        ev = self.ev
        ev.rng_fill(self.noise, self.seed, NOISE_STREAM, self.step_count, RNG_NORMAL)
        ev.rng_fill(self.uniform, self.seed, UNIFORM_STREAM, self.step_count, RNG_UNIFORM)
        params, n_hidden = (None, 0) if mlp is None else mlp
        ev.vmc_step(self.R, self.sign, self.logabs, self.gl, self.noise, self.uniform, self.elocal,
                    self.accepted, proposal=proposal, step=step, mlp_params=params,
                    n_hidden=n_hidden, precision=self.precision)
        self.step_count += 1


def run(walkers: Walkers, n_steps, proposal=PROP_GAUSSIAN, step=0.3, mlp=None, record=True,
        per_walker=False):
    """n_steps VMC steps; returns (mean E_L per step, mean sum r^2 per step,
    acceptance per step, wall seconds), and with per_walker also the series
    of every walker, (E_L [steps][W], sum r^2 [steps][W]) as device tensors."""
    import torch
    el, r2, acc, elw, r2w = [], [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        walkers.step(proposal, step, mlp)
        if record:
            rr = torch.sum(walkers.R * walkers.R, dim=(1, 2))
            el.append(torch.nanmean(walkers.elocal))
            r2.append(torch.mean(rr))
            acc.append(walkers.accepted.double().mean())
            if per_walker:
                elw.append(walkers.elocal.clone())
                r2w.append(rr)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if not record:
        return None, None, None, dt
    out = (torch.stack(el).cpu().numpy(), torch.stack(r2).cpu().numpy(),
           torch.stack(acc).cpu().numpy(), dt)
    if per_walker:
        return out + ((torch.stack(elw), torch.stack(r2w)),)
    return out


def tau_int(x, c=5.0):
    """Integrated autocorrelation time (Sokal's automatic windowing)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    x = x - x.mean()
    f = np.fft.rfft(x, 2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n]
    if acf[0] <= 0:
        return 1.0
    rho = acf / acf[0]
    tau = 1.0
    for m in range(1, n):
        tau = 1.0 + 2.0 * np.sum(rho[1:m + 1])
        if m >= c * tau:
            break
    return max(tau, 1.0)


def tau_int_walkers(x, c=5.0):
    """Integrated autocorrelation time of the walker average of x [steps][W]
    (a device or host array), from the autocovariance averaged over the
    walkers: the chains are independent, so the autocorrelation of the
    average is that of the summed per-walker autocovariances -- the same
    quantity as tau_int of the averaged series, with far less noise.  Sokal's
    automatic window (c = 5).  Non-finite entries are replaced by the walker's
    mean."""
    import torch
    x = torch.as_tensor(x, dtype=torch.float64)
    n = x.shape[0]
    m = torch.nanmean(x, dim=0, keepdim=True)
    x = torch.where(torch.isfinite(x), x, m) - m
    f = torch.fft.rfft(x, 2 * n, dim=0)
    acf = torch.fft.irfft(f * torch.conj(f), dim=0)[:n].sum(dim=1).cpu().numpy()
    if acf[0] <= 0:
        return 1.0
    rho = acf / acf[0]
    tau = 1.0
    for k in range(1, n):
        tau = 1.0 + 2.0 * np.sum(rho[1:k + 1])
        if k >= c * tau:
            break
    return max(float(tau), 1.0)


def train_proposal(ev: Evaluator, samples, params0, n_hidden, n_iter, batch, lr=1e-3, seed=5,
                   precision=MDET_FP64, log_every=0, jump_ref=0.0, state=None, objective=0,
                   nuclear_charge=None):
    """Train the MLP proposal on `samples` [S][N][3] (host), `n_iter` library
    training steps on random batches (jump_ref, objective: the jump weighting
    and objective of mdet_mlp_train_step).  `state` (a dict, nullable) carries the Adam moments
    and step count from one call to the next.  Returns (params tensor, losses)."""
    import torch
    p = torch.as_tensor(params0, dtype=torch.float32, device="cuda").clone()
    if state is not None and "m" in state:
        m, v, t_done = state["m"], state["v"], state["t"]
    else:
        m, v, t_done = torch.zeros_like(p), torch.zeros_like(p), 0
    S = samples.shape[0]
    rng = np.random.default_rng(seed)
    Rb = torch.empty((batch,) + samples.shape[1:], dtype=torch.float64, device="cuda")
    noise = torch.empty_like(Rb)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    dev_samples = torch.as_tensor(samples, dtype=torch.float64, device="cuda")
    losses = []
    for t in range(t_done + 1, t_done + n_iter + 1):
        idx = torch.as_tensor(rng.integers(0, S, batch), device="cuda")
        Rb.copy_(dev_samples.index_select(0, idx))
        ev.rng_fill(noise, seed, TRAIN_STREAM, t, RNG_NORMAL)
        ev.mlp_train_step(p, m, v, t, lr, Rb, noise, n_hidden, loss, precision=precision,
                          jump_ref=jump_ref, objective=objective, nuclear_charge=nuclear_charge)
        losses.append(loss.clone())
        if log_every and t % log_every == 0:
            print(f"[train] iter {t} loss {float(loss):.5f}", flush=True)
    if state is not None:
        state.update(m=m, v=v, t=t_done + n_iter)
    return p, torch.cat(losses).cpu().numpy()
