"""The allocation-free evaluation (mdet_eval_walkers_noalloc) through the C
ABI: the same outputs as mdet_eval_walkers, bit for bit, on two calls in a
row with a smaller batch the second time (the static scratch keeps the first
call's contents), in both precisions and with per-walker degree limits; and
the size limit reported before any work is queued."""
import numpy as np
import pytest

import oracle
from gen.workloads import make_config
from parity_util import FP64_TOL, MIXED_TOL, log, scaled_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_1510_00730_amd as mdet  # noqa: E402


def dev(x, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def _outputs(W, N):
    return (torch.full((W,), 7.0, dtype=torch.float64, device="cuda"),
            torch.full((W,), 7.0, dtype=torch.float64, device="cuda"),
            torch.full((W, N, 4), 7.0, dtype=torch.float64, device="cuda"),
            torch.full((W,), 7, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("cid,sizes", [(2, (256, 100)), (4, (160, 37))])
def test_noalloc_equals_eval_walkers(cid, sizes):
    wl = make_config(cid, n_walk=max(sizes))
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    N = wl.n_elec
    for W in sizes:
        R = dev(wl.R[:W])
        md = None if wl.max_degree is None else dev(wl.max_degree[:W], torch.int8)
        ref = oracle.evaluate(wl, wl.R[:W], max_degree=None if md is None else wl.max_degree[:W],
                              n_threads=16)
        for prec, tol in ((mdet.MDET_FP64, FP64_TOL), (mdet.MDET_MIXED, MIXED_TOL)):
            log(f"[noalloc] config {cid} W={W} precision {prec}")
            a = ev.eval_walkers(R, precision=prec, max_degree=md)
            b = ev.eval_walkers_noalloc(R, *_outputs(W, N), precision=prec, max_degree=md)
            torch.cuda.synchronize()
            for x, y in zip(a, b):
                assert torch.equal(x, y)
            s, l, g, w = (t.cpu().numpy() for t in b)
            ep, eg = scaled_errors(ref, s, l, g)
            assert ep.max() <= tol and eg.max() <= tol, (W, prec, ep.max(), eg.max())


def test_noalloc_rejects_batches_beyond_its_scratch():
    log("[noalloc] size limit")
    wl = make_config(3)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    W, N = wl.n_walk, wl.n_elec
    out = _outputs(W, N)
    with pytest.raises(mdet.MdetError) as ei:
        ev.eval_walkers_noalloc(dev(wl.R), *out)
    assert ei.value.code == -2
    torch.cuda.synchronize()
    assert torch.all(out[0] == 7.0)          # nothing was queued
    # a batch that fits runs and matches the allocating entry point
    R = dev(wl.R[:128])
    a = ev.eval_walkers(R, precision=mdet.MDET_MIXED)
    b = ev.eval_walkers_noalloc(R, *_outputs(128, N), precision=mdet.MDET_MIXED)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
