"""Launch choices and graph replay against the FP64 oracle.

Every forward gather a plan can be switched to, the configuration gt_plan_tune picks, and the
plan's own graph replays compute the transform to the same bars as the default launches
(relative l2 and max|err|/||input||_1, as in test_gpu_transform.py).  A second plan of the
same signature takes the cached choice without timing."""
import numpy as np
import pytest

import workloads as W
from oracle import index_set as oidx
from oracle import transform as otr
from paper_2010_10199_amd import lib
from tests.gpu_util import TOL, check, dtype_code, max_tol, say, to_dev

pytestmark = pytest.mark.gpu

# (name, d, ds, N, M, R): enough nodes per grid cell that every order can take the cell
# gather (and order 2 the polynomial gather in FP32)
CASES = [
    ("cells-3d-R2", 3, 3, (4, 4, 4), 30000, 2),
    ("order2-d5", 5, 2, (16, 8), 20000, 1),
]
NAMES = {lib.GT_GATHER_SORTED: "sorted", lib.GT_GATHER_CELL: "cell", lib.GT_GATHER_POLY: "poly"}


def _setup(case, prec):
    import torch
    name, d, ds, N, M, R = case
    cid = 40 + CASES.index(case)
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(cid, W.P_NODES), M, d, prec)
    fhat = W.complex_normal(W.rng(cid, W.P_COEFFS), (R, iset.n_coeffs), prec)
    y = W.complex_normal(W.rng(cid, W.P_SAMPLES), (R, M), prec)
    p, keep = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    ct = torch.complex64 if prec == "f32" else torch.complex128
    bufs = dict(fhat=to_dev(fhat.reshape(-1)), y=to_dev(y.reshape(-1)),
                f=torch.empty(R * M, dtype=ct, device="cuda"), a=torch.empty(R * iset.n_coeffs, dtype=ct, device="cuda"))
    torch.cuda.synchronize()
    ref_f = otr.forward(iset, x, fhat)
    ref_a = otr.adjoint(iset, x, y)
    return iset, x, fhat, y, plan, bufs, ref_f, ref_a


def _run(plan, bufs, stream, R, M, n):
    import torch
    plan.trafo(bufs["fhat"], bufs["f"], stream)
    plan.adjoint(bufs["y"], bufs["a"], stream)
    torch.cuda.synchronize()
    return (bufs["f"].cpu().numpy().astype(np.complex128).reshape(R, M),
            bufs["a"].cpu().numpy().astype(np.complex128).reshape(R, n))


def _check_both(label, got_f, got_a, fhat, y, ref_f, ref_a, prec, ds):
    check(f"{label} forward", got_f, ref_f, fhat, TOL[prec], max_tol(prec, ds))
    check(f"{label} adjoint", got_a, ref_a, y, TOL[prec], max_tol(prec, ds))


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_every_gather_form(case, prec):
    import torch
    name, d, ds, N, M, R = case
    say(f"[forms] {name} {prec}")
    iset, x, fhat, y, plan, bufs, ref_f, ref_a = _setup(case, prec)
    s = torch.cuda.Stream()
    for t in range(1, ds + 1):
        for path in (lib.GT_GATHER_SORTED, lib.GT_GATHER_CELL, lib.GT_GATHER_POLY):
            if path == lib.GT_GATHER_POLY and (t != 2 or prec == "f64"):
                with pytest.raises(lib.GroupedError) as e:
                    plan.set_gather_path(t, path)
                assert e.value.code == lib.GT_EUNSUPPORTED
                continue
            plan.set_gather_path(t, path)
            assert plan.gather_path(t) == path
            f, a = _run(plan, bufs, s.cuda_stream, R, M, iset.n_coeffs)
            _check_both(f"order {t} {NAMES[path]}", f, a, fhat, y, ref_f, ref_a, prec, ds)
    plan.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_tuned_plan_and_cached_choice(case, prec):
    import torch
    name, d, ds, N, M, R = case
    say(f"[tune] {name} {prec}")
    lib.release_all()   # no cached choice from earlier tests
    iset, x, fhat, y, plan, bufs, ref_f, ref_a = _setup(case, prec)
    assert plan.tuning() == {}
    s = torch.cuda.Stream()
    rep = plan.tune(s.cuda_stream)
    say(f"  report: {rep}")
    assert rep["cached"] is False and rep["forward_ms"] > 0 and rep["adjoint_ms"] > 0
    for t in range(1, ds + 1):
        chosen = rep["gather"][str(t)]["chosen"]
        assert NAMES[plan.gather_path(t)] == chosen
        assert rep["gather"][str(t)][chosen] == min(v for k, v in rep["gather"][str(t)].items() if k != "chosen")
    if ds >= 2:
        assert str(rep["tile_waves_cu"]["chosen"]) in rep["tile_waves_cu"]
    f, a = _run(plan, bufs, s.cuda_stream, R, M, iset.n_coeffs)
    _check_both("tuned", f, a, fhat, y, ref_f, ref_a, prec, ds)
    # a second plan of the same signature (other nodes) takes the cached choice
    x2 = W.uniform_nodes(W.rng(77, W.P_NODES), M, d, prec)
    p2, keep2 = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    plan2 = lib.Plan(p2, to_dev(x2), keepalive=keep2)
    rep2 = plan2.tuning()
    assert rep2["cached"] is True
    for t in range(1, ds + 1):
        assert plan2.gather_path(t) == plan.gather_path(t)
    f2, a2 = _run(plan2, bufs, s.cuda_stream, R, M, iset.n_coeffs)
    _check_both("cached", f2, a2, fhat, y, otr.forward(iset, x2, fhat), otr.adjoint(iset, x2, y), prec, ds)
    plan2.close()
    plan.close()
    lib.release_all()
    p3, keep3 = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    plan3 = lib.Plan(p3, to_dev(x2), keepalive=keep3)
    assert plan3.tuning() == {}   # the release cleared the cache
    plan3.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_graph_replays(case, prec):
    """Replays of the plan's captured graphs, with the program's own eager work and
    synchronisations between them and new input values in the same buffers, each checked
    against the oracle; a new output buffer gets a graph of its own."""
    import torch
    name, d, ds, N, M, R = case
    say(f"[graph] {name} {prec}")
    iset, x, fhat, y, plan, bufs, ref_f, ref_a = _setup(case, prec)
    s = torch.cuda.Stream()
    plan.set_graph(True)
    for rep in range(4):
        fh = W.complex_normal(W.rng(500 + rep, W.P_COEFFS), (R, iset.n_coeffs), prec)
        yy = W.complex_normal(W.rng(500 + rep, W.P_SAMPLES), (R, M), prec)
        bufs["fhat"].copy_(to_dev(fh.reshape(-1)))
        bufs["y"].copy_(to_dev(yy.reshape(-1)))
        junk = torch.randn(1 << 16, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        f, a = _run(plan, bufs, s.cuda_stream, R, M, iset.n_coeffs)
        assert torch.isfinite(junk)
        _check_both(f"replay {rep}", f, a, fh, yy, otr.forward(iset, x, fh), otr.adjoint(iset, x, yy), prec, ds)
    ct = bufs["f"].dtype
    other = dict(bufs, f=torch.empty(R * M, dtype=ct, device="cuda"),
                 a=torch.empty(R * iset.n_coeffs, dtype=ct, device="cuda"))
    fh = W.complex_normal(W.rng(500 + 3, W.P_COEFFS), (R, iset.n_coeffs), prec)
    yy = W.complex_normal(W.rng(500 + 3, W.P_SAMPLES), (R, M), prec)
    f, a = _run(plan, other, s.cuda_stream, R, M, iset.n_coeffs)
    _check_both("new buffers", f, a, fh, yy, otr.forward(iset, x, fh), otr.adjoint(iset, x, yy), prec, ds)
    plan.set_graph(False)
    f, a = _run(plan, other, s.cuda_stream, R, M, iset.n_coeffs)
    _check_both("eager again", f, a, fh, yy, otr.forward(iset, x, fh), otr.adjoint(iset, x, yy), prec, ds)
    plan.close()
