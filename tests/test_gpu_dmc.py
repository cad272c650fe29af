"""GPU Slater-Jastrow outputs and fixed-node DMC steps through the C ABI,
against the CPU oracle with the same random numbers, and the helium
ground-state energy from a GPU DMC run."""
import math

import numpy as np
import pytest

from gen.workloads import make_config, make_helium
from oracle import dmc, vmc
from parity_util import gpu_eval, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_1510_00730_amd as mdet  # noqa: E402

PARAMS = (1.0, -2.0, 1.0)


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


@pytest.mark.parametrize("cid", [1, 2])
def test_jastrow_applied_to_the_evaluators_outputs(cid):
    log(f"[dmc] Jastrow on config {cid}")
    wl = make_config(cid)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    s0, l0, g0, _ = gpu_eval(ev, wl.R)
    ev.set_jastrow(True, *PARAMS)
    s1, l1, g1, _ = gpu_eval(ev, wl.R)
    la, gl = dmc.apply_jastrow(wl.R, wl.n_up, PARAMS, l0, g0)
    assert np.array_equal(s0, s1)
    live = np.isfinite(l0)
    np.testing.assert_allclose(l1[live], la[live], rtol=0, atol=1e-12 * (1 + np.abs(la[live]).max()))
    scale = 1.0 + np.abs(gl[live]).max(axis=(1, 2), keepdims=True)
    assert np.max(np.abs(g1[live] - gl[live]) / scale) < 1e-12
    ev.set_jastrow(False)
    s2, l2, g2, _ = gpu_eval(ev, wl.R)
    assert np.array_equal(l2, l0) and np.array_equal(g2, g0)


def _run_gpu_and_oracle(wl, Z, steps, tau, seed):
    W, N = wl.R.shape[0], wl.n_elec
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    ev.set_jastrow(True, *PARAMS)
    s, la, gl = dmc.trial(wl, wl.R, PARAMS)
    el = vmc.local_energy(wl.R, gl, Z)
    st = dict(R=wl.R.copy(), sign=s, logabs=la, gl=gl, elocal=el, weight=np.ones(W))
    g = dict(R=dev(wl.R), sign=dev(s), logabs=dev(la), gl=dev(gl), elocal=dev(el),
             weight=dev(np.ones(W)))
    sums = torch.zeros(4, dtype=torch.float64, device="cuda")
    acc = torch.zeros(W, dtype=torch.int32, device="cuda")
    rng = np.random.default_rng(seed)
    for k in range(steps):
        xi, u, cu = rng.standard_normal((W, N, 3)), rng.random(W), float(rng.random())
        et = -2.9 if Z == 2.0 else float(np.nanmean(st["elocal"]))
        st, osums, oacc = dmc.dmc_step(wl, st, tau, et, Z, xi, u, cu, PARAMS)
        ev.dmc_step(g["R"], g["sign"], g["logabs"], g["gl"], g["elocal"], g["weight"], dev(xi),
                    dev(u), cu, sums, acc, tau=tau, e_trial=et, nuclear_charge=Z)
        torch.cuda.synchronize()
        assert np.array_equal(acc.cpu().numpy().astype(bool), oacc), k
        np.testing.assert_allclose(sums.cpu().numpy(), osums, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(g["R"].cpu().numpy(), st["R"], rtol=0, atol=1e-10)
        np.testing.assert_allclose(g["elocal"].cpu().numpy(), st["elocal"], rtol=1e-8, atol=1e-8)
        assert np.array_equal(g["sign"].cpu().numpy(), st["sign"])
        assert np.all(g["weight"].cpu().numpy() == 1.0)


def test_dmc_steps_match_oracle_helium():
    log("[dmc] helium, 256 walkers, 6 steps against the oracle")
    _run_gpu_and_oracle(make_helium(256, seed=3), 2.0, 6, 0.02, seed=11)


def test_dmc_steps_match_oracle_multideterminant():
    log("[dmc] config 1 (5+5 electrons, 500 products), 3 steps against the oracle")
    wl = make_config(1)
    _run_gpu_and_oracle(wl, 10.0, 3, 0.005, seed=12)


def test_helium_fixed_node_dmc_energy_on_gpu():
    """He ground state -2.903724 hartree (nodeless: fixed-node DMC is exact)."""
    log("[dmc] helium GPU run, 4096 walkers x 3000 steps")
    W, steps, tau = 4096, 3000, 0.02
    wl = make_helium(W, seed=4)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    ev.set_jastrow(True, *PARAMS)
    s, la, gl = dmc.trial(wl, wl.R, PARAMS)
    g = dict(R=dev(wl.R), sign=dev(s), logabs=dev(la), gl=dev(gl),
             elocal=dev(vmc.local_energy(wl.R, gl, 2.0)), weight=dev(np.ones(W)))
    sums = torch.zeros(4, dtype=torch.float64, device="cuda")
    acc = torch.zeros(W, dtype=torch.int32, device="cuda")
    noise = torch.empty((W, 2, 3), dtype=torch.float64, device="cuda")
    uni = torch.empty(W, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(9)
    es, et = [], -2.9
    hist = torch.zeros((steps, 4), dtype=torch.float64, device="cuda")
    for k in range(steps):
        ev.rng_fill(noise, seed=77, stream_id=0, step=k, kind=mdet.binding.RNG_NORMAL)
        ev.rng_fill(uni, seed=77, stream_id=1, step=k, kind=mdet.binding.RNG_UNIFORM)
        ev.dmc_step(g["R"], g["sign"], g["logabs"], g["gl"], g["elocal"], g["weight"], noise, uni,
                    float(rng.random()), sums, acc, tau=tau, e_trial=et, nuclear_charge=2.0)
        hist[k] = sums
        if k % 100 == 99:  # update the trial energy from the running estimate
            h = hist[: k + 1].cpu().numpy()
            es = h[:, 1] / h[:, 0]
            et = float(np.mean(es[50:]))
    h = hist.cpu().numpy()
    es = (h[:, 1] / h[:, 0])[steps // 4:]
    nb = 30
    b = es[: len(es) // nb * nb].reshape(nb, -1).mean(axis=1)
    e, err = es.mean(), b.std(ddof=1) / math.sqrt(nb)
    log(f"[dmc] helium E = {e:.5f} +- {err:.5f} (exact -2.903724), acceptance "
        f"{h[-1, 3] / W:.3f}")
    assert abs(e - (-2.903724)) < 4 * err + 0.004


def test_jastrow_inside_captured_graph_replays_bitwise():
    log("[dmc] Jastrow under graph capture, config 2")
    wl = make_config(2)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    ev.set_jastrow(True, *PARAMS)
    s0, l0, g0, _ = gpu_eval(ev, wl.R)
    R = dev(wl.R)
    out = (torch.empty(R.shape[0], dtype=torch.float64, device="cuda"),
           torch.empty(R.shape[0], dtype=torch.float64, device="cuda"),
           torch.empty((R.shape[0], wl.n_elec, 4), dtype=torch.float64, device="cuda"),
           torch.empty(R.shape[0], dtype=torch.int32, device="cuda"))
    for rep in range(3):
        ev.eval_graph(R, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out[1].cpu().numpy(), l0) and np.array_equal(out[2].cpu().numpy(), g0)
        gpu_eval(ev, wl.R)  # eager work between the replays


def test_vmc_with_jastrow_is_variational_for_helium():
    """VMC energy of the Slater-Jastrow helium trial function lies above the
    exact ground state and below the determinant-only trial function's."""
    log("[dmc] helium VMC with and without the Jastrow factor")
    W, steps = 2048, 400
    energies = {}
    for jas in (False, True):
        wl = make_helium(W, seed=6)
        ev = mdet.Evaluator(0)
        ev.load_workload(wl)
        if jas:
            ev.set_jastrow(True, *PARAMS)
        R = dev(wl.R)
        sign, logabs, gl, _ = ev.eval_walkers(R)
        el = torch.empty(W, dtype=torch.float64, device="cuda")
        acc = torch.empty(W, dtype=torch.int32, device="cuda")
        noise = torch.empty((W, 2, 3), dtype=torch.float64, device="cuda")
        uni = torch.empty(W, dtype=torch.float64, device="cuda")
        es = []
        for k in range(steps):
            ev.rng_fill(noise, seed=5, stream_id=0, step=k, kind=mdet.binding.RNG_NORMAL)
            ev.rng_fill(uni, seed=5, stream_id=1, step=k, kind=mdet.binding.RNG_UNIFORM)
            ev.vmc_step(R, sign, logabs, gl, noise, uni, el, acc, proposal=mdet.binding.PROP_DRIFT,
                        step=0.05, nuclear_charge=2.0)
            if k >= steps // 2:
                es.append(el.mean().item())
        energies[jas] = float(np.mean(es))
    log(f"[dmc] helium VMC: determinant only {energies[False]:.4f}, with Jastrow {energies[True]:.4f}")
    assert -2.9037 < energies[True] < energies[False]
