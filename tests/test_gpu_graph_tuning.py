"""Captured steps, launch configurations, walker sorting and the autotuner."""
import numpy as np
import pytest

import oracle
from gen.workloads import make_config
from parity_util import FP64_TOL, MIXED_TOL, gpu_eval, log, scaled_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_1510_00730_amd as mdet  # noqa: E402


def dev(x, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_equal_eager(precision):
    """Every replay of the captured step equals the eager evaluation bit for
    bit, with eager work (input updates, other evaluations) between replays."""
    log(f"[graph] replays precision {precision}")
    wl = make_config(2)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    R = dev(wl.R)
    outs = tuple(t.clone() for t in ev.eval_walkers(R, precision=precision))
    rng = np.random.default_rng(3)
    for rep in range(4):
        R.add_(dev(rng.normal(0, 0.05, wl.R.shape)))          # new inputs, same buffer
        ref = [t.clone() for t in ev.eval_walkers(R, precision=precision)]
        torch.cuda.synchronize()
        got = ev.eval_graph(R, precision=precision, out=outs)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), f"replay {rep} differs"
        ev.eval_walkers(dev(wl.R[:17]), precision=precision)  # unrelated eager call in between


def test_walker_sorting_is_bitwise_neutral_and_configs_pass_parity():
    log("[graph] uneven batch, sorting on/off, launch configurations")
    wl = make_config(4, n_walk=512)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    R = dev(wl.R)
    md = dev(wl.max_degree, torch.int8)
    res = {}
    for prec in (0, 1):
        for sort in (True, False):
            for ovl in (True, False):
                ev.set_launch_config(0, 4, sort, ovl)
                res[(prec, sort, ovl)] = [t.cpu() for t in
                                          ev.eval_walkers(R, precision=prec, max_degree=md)]
        for key in ((prec, True, False), (prec, False, True), (prec, False, False)):
            for a, b in zip(res[(prec, True, True)], res[key]):
                assert torch.equal(a, b), key
    rows = list(range(0, 512, 16))
    ref = oracle.evaluate(wl, wl.R[rows], max_degree=wl.max_degree[rows], n_threads=16)
    for rs, ds in ((1, 1), (4, 8), (16, 2)):
        ev.set_launch_config(rs, ds, True)
        for prec, tol in ((0, FP64_TOL), (1, MIXED_TOL)):
            s, l, g, w = gpu_eval(ev, wl.R, precision=prec, max_degree=wl.max_degree)
            ep, eg = scaled_errors(ref, s, l, g, idx=rows)
            assert ep.max() <= tol and eg.max() <= tol, (rs, ds, prec, ep.max(), eg.max())


def test_autotune_picks_a_valid_config():
    log("[graph] autotune")
    wl = make_config(3)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    R = dev(wl.R)
    r = ev.autotune(R, precision=1, n_rep=3)
    log(f"autotune: splits {r.spmm_row_splits} direct {r.direct_split} sort {r.sort_walkers} "
        f"overlap {r.overlap_fallback} "
        f"best {r.best_ms:.4f} ms default {r.default_ms:.4f} ms over {r.n_candidates} candidates")
    assert r.n_candidates == 24 and r.best_ms <= r.default_ms
    rows = list(range(0, 1024, 64))
    ref = oracle.evaluate(wl, wl.R[rows], n_threads=16)
    s, l, g, w = gpu_eval(ev, wl.R, precision=1)
    ep, eg = scaled_errors(ref, s, l, g, idx=rows)
    assert ep.max() <= MIXED_TOL and eg.max() <= MIXED_TOL


def _graph_eval(ev, R, precision, max_degree=None):
    Rt = dev(R)
    md = None if max_degree is None else dev(max_degree, torch.int8)
    out = ev.eval_graph(Rt, precision=precision, max_degree=md)
    torch.cuda.synchronize()
    out = ev.eval_graph(Rt, precision=precision, max_degree=md, out=out)  # a replay
    torch.cuda.synchronize()
    return tuple(t.cpu().numpy() for t in out)


def test_graph_replay_parity_c3_mixed():
    """The captured step that the benchmark replays, against the oracle on the
    full 1e5-product batch in mixed precision (and FP64)."""
    log("[graph] config 3 replay vs oracle")
    wl = make_config(3)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    ref = oracle.evaluate(wl, wl.R, n_threads=16)
    for prec, tol in ((1, MIXED_TOL), (0, FP64_TOL)):
        s, l, g, w = _graph_eval(ev, wl.R, prec)
        ep, eg = scaled_errors(ref, s, l, g)
        log(f"c3 graph precision {prec}: psi {ep.max():.2e} grad {eg.max():.2e} "
            f"fallback {np.mean(w == 1):.3f}")
        assert ep.max() <= tol and eg.max() <= tol, (prec, ep.max(), eg.max())


@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_graph_replay_parity_c4_uneven(precision, tol):
    """Uneven batch (per-walker degree limits, walkers sorted by degree inside
    the captured step) against the oracle on sampled walkers."""
    log(f"[graph] config 4 replay vs oracle, precision {precision}")
    wl = make_config(4)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    s, l, g, w = _graph_eval(ev, wl.R, precision, wl.max_degree)
    rows = list(range(0, wl.n_walk, wl.n_walk // 48))
    ref = oracle.evaluate(wl, wl.R[rows], max_degree=wl.max_degree[rows], n_threads=16)
    ep, eg = scaled_errors(ref, s, l, g, idx=rows)
    log(f"c4 graph precision {precision}: psi {ep.max():.2e} grad {eg.max():.2e}")
    assert ep.max() <= tol and eg.max() <= tol


def test_threshold_change_reaches_captured_steps():
    """A new conditioning threshold takes effect on the next replay (the
    captured step is dropped and captured again)."""
    log("[graph] threshold change after capture")
    wl = make_config(2)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    R = wl.R[:64]
    s, l, g, w = _graph_eval(ev, R, 0)
    assert np.mean(w == mdet.W_FALLBACK) < 0.5
    ev.set_fallback_threshold(1e-300)
    s, l, g, w = _graph_eval(ev, R, 0)
    assert np.all(w == mdet.W_FALLBACK)
    ref = oracle.evaluate(wl, R, n_threads=16)
    ep, eg = scaled_errors(ref, s, l, g)
    assert ep.max() <= FP64_TOL and eg.max() <= FP64_TOL
    # per precision: only the mixed threshold lowered
    ev.set_fallback_threshold(3e4, precision=0)
    s, l, g, w = _graph_eval(ev, R, 0)
    assert np.mean(w == mdet.W_FALLBACK) < 0.5
    s, l, g, w = _graph_eval(ev, R, 1)
    assert np.all(w == mdet.W_FALLBACK)
