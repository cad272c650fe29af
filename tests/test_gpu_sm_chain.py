"""GPU Sherman-Morrison chain (Sec. 2.2) through the C ABI: against the
paper-method chain on the CPU (same decisions, counters compared) and the
direct-LU oracle.  The chain's own rounding growth is part of the method, so
its accuracy bar is the CPU chain's error against the direct LU, measured on
the same walkers; the degenerate settings that remove the updates (pieces of
one determinant, a threshold no ratio reaches) are held to the FP64 bar."""
import numpy as np
import pytest

import oracle
from gen.workloads import make_config
from parity_util import FP64_TOL, MIXED_TOL, gpu_eval, log, scaled_errors, summary

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_1510_00730_amd as mdet  # noqa: E402

_CACHE = {}


def case(cid, W):
    key = (cid, W)
    if key not in _CACHE:
        wl = make_config(cid, n_walk=W)
        wl.max_degree = None
        direct = oracle.evaluate(wl, max_degree=None, n_threads=16)
        chain = oracle.sm_evaluate(wl, n_threads=16)
        _CACHE[key] = (wl, direct, chain)
    return _CACHE[key]


def chain_eval(wl, precision=0, threshold=1e-3, chunk=1 << 20, R=None, max_degree=None):
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    ev.set_method(mdet.METHOD_SM_CHAIN, threshold, chunk)
    out = gpu_eval(ev, wl.R if R is None else R, precision=precision, max_degree=max_degree)
    return out, ev.sm_counters()


@pytest.mark.parametrize("cid,W", [(1, 8), (2, 128), (3, 64)])
def test_chain_matches_cpu_chain(cid, W):
    log(f"[sm] config {cid} W={W} one piece per chain, threshold 1e-3")
    wl, direct, chain = case(cid, W)
    (sign, logabs, gl, ws), cnt = chain_eval(wl)
    ep, eg = scaled_errors(direct, sign, logabs, gl)
    cp, cg = scaled_errors(direct, chain.sign, chain.logabs, chain.gl)
    summary(f"c{cid} gpu chain vs direct", ep, eg, ws)
    summary(f"c{cid} cpu chain vs direct", cp, cg)
    log(f"counters gpu {cnt} cpu subst {chain.n_subst} inv {chain.n_inv} fail {chain.n_fail}")
    assert np.all(ws == mdet.W_OK)
    assert cnt["n_start"] == 2 * W
    # same decisions as the CPU chain (a flip needs |r| within rounding of the threshold)
    for a, b in ((cnt["n_subst"], chain.n_subst), (cnt["n_fail"], chain.n_fail),
                 (cnt["n_inv"] + cnt["n_start"], chain.n_inv)):
        assert abs(a - b) <= 1e-3 * max(b, 1000), (a, b)
    # walker by walker against the CPU chain (same decisions, its rounding
    # differs): within the FP64 bar, or within ten times that walker's own
    # chain error against the direct LU where the chain amplifies rounding
    cpu = oracle.Result(chain.sign, chain.logabs, chain.gl, direct.rs_psi, direct.rs_gl)
    dp, dg = scaled_errors(cpu, sign, logabs, gl)
    summary(f"c{cid} gpu chain vs cpu chain", dp, dg)
    assert np.array_equal(np.sign(sign), np.sign(chain.sign))
    assert np.all(dp <= np.maximum(FP64_TOL, 10 * cp)), np.max(dp / np.maximum(FP64_TOL, 10 * cp))
    assert np.all(dg <= np.maximum(FP64_TOL, 10 * cg)), np.max(dg / np.maximum(FP64_TOL, 10 * cg))
    well = (cp <= 1e-12) & (cg <= 1e-12)
    log(f"walkers where the CPU chain is within 1e-12 of the direct LU: {well.sum()} of {W}; "
        f"gpu-cpu chain max there: psi {dp[well].max() if well.any() else 0:.2e} "
        f"grad {dg[well].max() if well.any() else 0:.2e}")
    assert np.all(dp[well] <= FP64_TOL) and np.all(dg[well] <= FP64_TOL)


@pytest.mark.parametrize("cid,W", [(2, 128), (3, 64)])
def test_single_determinant_pieces_are_direct(cid, W):
    """Pieces of one determinant: every determinant factorised from scratch."""
    log(f"[sm] config {cid} W={W} pieces of 1")
    wl, direct, _ = case(cid, W)
    (sign, logabs, gl, ws), cnt = chain_eval(wl, chunk=1)
    U = len(np.unique(wl.det_up, axis=0))
    V = len(np.unique(wl.det_dn, axis=0))
    ep, eg = scaled_errors(direct, sign, logabs, gl)
    summary(f"c{cid} pieces of 1", ep, eg, ws)
    assert cnt["n_subst"] == 0 and cnt["n_fail"] == 0 and cnt["n_start"] == W * (U + V)
    assert ep.max() <= FP64_TOL and eg.max() <= FP64_TOL


def test_unreachable_threshold_recomputes_every_determinant():
    log("[sm] config 2 W=64 threshold 1e300")
    wl, direct, _ = case(2, 128)
    R = wl.R[:64]
    (sign, logabs, gl, ws), cnt = chain_eval(wl, threshold=1e300, R=R)
    ref = oracle.sm_evaluate(wl, R=R, threshold=np.inf, n_threads=16)
    assert cnt["n_subst"] == 0 and cnt["n_inv"] + cnt["n_start"] == ref.n_inv
    assert cnt["n_fail"] == ref.n_fail
    ep, eg = scaled_errors(oracle.evaluate(wl, R, max_degree=None, n_threads=16), sign, logabs, gl)
    assert ep.max() <= FP64_TOL and eg.max() <= FP64_TOL


@pytest.mark.parametrize("chunk", [7, 64, 250])
def test_piece_length_changes_counts_not_results(chunk):
    log(f"[sm] config 2 pieces of {chunk}")
    wl, direct, chain = case(2, 128)
    (sign, logabs, gl, ws), cnt = chain_eval(wl, chunk=chunk)
    U = len(np.unique(wl.det_up, axis=0))
    V = len(np.unique(wl.det_dn, axis=0))
    assert cnt["n_start"] == 128 * ((U + chunk - 1) // chunk + (V + chunk - 1) // chunk)
    ep, eg = scaled_errors(direct, sign, logabs, gl)
    cp, cg = scaled_errors(direct, chain.sign, chain.logabs, chain.gl)
    summary(f"c2 pieces of {chunk}", ep, eg, ws)
    assert ep.max() <= max(FP64_TOL, 10 * cp.max()) and eg.max() <= max(FP64_TOL, 10 * cg.max())


def test_mixed_precision_chain():
    log("[sm] config 2 mixed precision chain")
    wl, direct, chain = case(2, 128)
    (sign, logabs, gl, ws), cnt = chain_eval(wl, precision=mdet.MDET_MIXED, chunk=64)
    ep, eg = scaled_errors(direct, sign, logabs, gl)
    summary("c2 mixed chain", ep, eg, ws)
    assert ep.max() <= MIXED_TOL and eg.max() <= MIXED_TOL


def test_chain_honours_max_degree_and_graphs():
    """Uneven batch through the chain, eager and graph replay bit for bit."""
    log("[sm] config 2 uneven degrees, eager and graph")
    wl, _, _ = case(2, 128)
    md = np.random.default_rng(3).integers(1, 5, size=128).astype(np.int8)
    ref = oracle.evaluate(wl, wl.R, max_degree=md, n_threads=16)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    ev.set_method(mdet.METHOD_SM_CHAIN, 1e-3, 1)  # pieces of one: FP64 bar applies
    sign, logabs, gl, ws = gpu_eval(ev, wl.R, max_degree=md)
    ep, eg = scaled_errors(ref, sign, logabs, gl)
    summary("c2 uneven chain", ep, eg, ws)
    assert ep.max() <= FP64_TOL and eg.max() <= FP64_TOL
    Rt = torch.as_tensor(wl.R, device="cuda")
    mdt = torch.as_tensor(md, device="cuda")
    for rep in range(3):
        s2, l2, g2, w2 = ev.eval_graph(Rt, max_degree=mdt)
        torch.cuda.synchronize()
        assert np.array_equal(s2.cpu().numpy(), sign) and np.array_equal(l2.cpu().numpy(), logabs)
        assert np.array_equal(g2.cpu().numpy(), gl)
    # switching back to the table method gives the table results
    ev.set_method(mdet.METHOD_TABLE)
    s3, l3, g3, w3 = gpu_eval(ev, wl.R, max_degree=md)
    ep, eg = scaled_errors(ref, s3, l3, g3)
    assert ep.max() <= FP64_TOL and eg.max() <= FP64_TOL


def test_excitation_degrees_up_to_eight_table_and_chain():
    """Degrees 1-8 from the reference: the table method (s x s minors up to
    8 x 8) and the chain (no degree limit along the sorted list) both match
    the direct-LU oracle."""
    from gen.workloads import make_custom
    log("[sm] degrees up to 8, 9+8 electrons, 60 orbitals")
    wl = make_custom(9, 8, 60, 3, 200, 150, (1, 2, 4, 6, 8), 3000, 64, seed=21)
    direct = oracle.evaluate(wl, max_degree=None, n_threads=16)
    chain = oracle.sm_evaluate(wl, n_threads=16)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    for prec, tol in ((0, FP64_TOL), (1, MIXED_TOL)):
        sign, logabs, gl, ws = gpu_eval(ev, wl.R, precision=prec)
        ep, eg = scaled_errors(direct, sign, logabs, gl)
        summary(f"degree 8, table method, precision {prec}", ep, eg, ws)
        assert ep.max() <= tol and eg.max() <= tol
    ev.set_method(mdet.METHOD_SM_CHAIN, 1e-3, 1)
    sign, logabs, gl, ws = gpu_eval(ev, wl.R)
    ep, eg = scaled_errors(direct, sign, logabs, gl)
    summary("degree 8, pieces of 1", ep, eg, ws)
    assert ep.max() <= FP64_TOL and eg.max() <= FP64_TOL
    ev.set_method(mdet.METHOD_SM_CHAIN, 1e-3, 1 << 20)
    sign, logabs, gl, ws = gpu_eval(ev, wl.R)
    cnt = ev.sm_counters()
    ep, eg = scaled_errors(direct, sign, logabs, gl)
    cp, cg = scaled_errors(direct, chain.sign, chain.logabs, chain.gl)
    summary("degree 8, one piece", ep, eg, ws)
    assert abs(cnt["n_subst"] - chain.n_subst) <= 1e-3 * max(chain.n_subst, 1000)
    assert ep.max() <= max(FP64_TOL, 10 * cp.max()) and eg.max() <= max(FP64_TOL, 10 * cg.max())


def test_degrees_above_eight_by_the_chain_only():
    """Degree 9 (10+9 electrons): the table method refuses the
    expansion with MDET_EDEGREE, the chain evaluates it."""
    from gen.workloads import make_custom
    log("[sm] degree 9, 10+9 electrons, 40 orbitals")
    wl = make_custom(10, 9, 40, 3, 80, 60, (1, 2, 9), 1200, 16, seed=23)
    direct = oracle.evaluate(wl, max_degree=None, n_threads=16)
    ev = mdet.Evaluator(0)
    ev.load_workload(wl)
    with pytest.raises(mdet.MdetError) as ei:
        gpu_eval(ev, wl.R)
    assert ei.value.code == -10
    ev.set_method(mdet.METHOD_SM_CHAIN, 1e-3, 1)
    sign, logabs, gl, ws = gpu_eval(ev, wl.R)
    ep, eg = scaled_errors(direct, sign, logabs, gl)
    summary("degree 9, pieces of 1", ep, eg, ws)
    assert ep.max() <= FP64_TOL and eg.max() <= FP64_TOL
