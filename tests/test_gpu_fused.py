"""Shared launches of orders 1 and 2 (gt_plan_set_fused) against the separate launches and
the FP64 oracle.

Each part of a shared launch runs the body, work items and summation order of its own
kernel, so forward and adjoint must equal the separate launches' results bit for bit, for
every gather form, ragged datasets, several right-hand sides, both precisions, graph replay
and the weighted solvers; and they meet the oracle bars of test_gpu_transform.py."""
import numpy as np
import pytest

import workloads as W
from oracle import index_set as oidx
from oracle import transform as otr
from paper_2010_10199_amd import lib
from tests.gpu_util import TOL, check, dtype_code, max_tol, nfft_model_error, say, to_dev

pytestmark = pytest.mark.gpu

# (name, d, ds, N, M, R, m): the d = 10 workload's shape at fewer nodes; several right-hand
# sides; a narrow window; ragged datasets (sizes below)
CASES = [
    ("d10-N64-16", 10, 2, (64, 16), 20000, 1, 0),
    ("d5-R3", 5, 2, (16, 8), 12000, 3, 0),
    ("d4-m3", 4, 2, (24, 12), 6000, 2, 3),
    ("ragged-3", 6, 2, (20, 10), 0, 3, 0),
]
RAGGED = (3000, 17, 5200)
NAMES = {lib.GT_GATHER_SORTED: "sorted", lib.GT_GATHER_CELL: "cell", lib.GT_GATHER_POLY: "poly"}


def _setup(case, prec):
    import torch
    name, d, ds, N, M, R, m = case
    cid = 90 + CASES.index(case)
    iset = oidx.grouped_index_set(d, ds, N)
    ragged = M == 0
    sizes = RAGGED if ragged else (M,)
    Mtot = int(sum(sizes))
    x = W.uniform_nodes(W.rng(cid, W.P_NODES), Mtot, d, prec)
    fhat = W.complex_normal(W.rng(cid, W.P_COEFFS), (R, iset.n_coeffs), prec)
    V = Mtot if ragged else R * M
    y = W.complex_normal(W.rng(cid, W.P_SAMPLES), (V,), prec)
    offsets = np.concatenate([[0], np.cumsum(sizes)]) if ragged else None
    p, keep = lib.make_problem(d, ds, N, M=0 if ragged else M, R=R, dtype=dtype_code(prec), m=m, offsets=offsets)
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    ct = torch.complex64 if prec == "f32" else torch.complex128
    bufs = dict(fhat=to_dev(fhat.reshape(-1)), y=to_dev(y),
                f=torch.empty(V, dtype=ct, device="cuda"), a=torch.empty(R * iset.n_coeffs, dtype=ct, device="cuda"))
    torch.cuda.synchronize()
    return iset, x, fhat, y, plan, bufs, offsets


def _refs(iset, x, fhat, y, offsets, R):
    if offsets is None:
        M = x.shape[0]
        return otr.forward(iset, x, fhat).reshape(-1), otr.adjoint(iset, x, y.reshape(R, M))
    f = [otr.forward(iset, x[offsets[r]:offsets[r + 1]], fhat[r:r + 1]).reshape(-1) for r in range(R)]
    a = [otr.adjoint(iset, x[offsets[r]:offsets[r + 1]], y[None, offsets[r]:offsets[r + 1]]).reshape(-1)
         for r in range(R)]
    return np.concatenate(f), np.stack(a)


def _check_all(label, f, a, fhat, y, ref_f, ref_a, offsets, prec, ds, m, R):
    """Oracle bars: relative l2 (widened to the window's error model for a narrow window) and
    max|err| / ||input||_1, per right-hand side or dataset."""
    l2 = max(TOL[prec], 20 * ds * nfft_model_error(m, 2.0)) if m else TOL[prec]
    mt = max_tol(prec, ds, m)
    f = f.astype(np.complex128)
    a = a.astype(np.complex128).reshape(R, -1)
    if offsets is None:
        check(f"{label} forward", f.reshape(R, -1), ref_f.reshape(R, -1), fhat, l2, mt)
        check(f"{label} adjoint", a, ref_a, y.reshape(R, -1), l2, mt)
        return
    for r in range(R):
        sl = slice(int(offsets[r]), int(offsets[r + 1]))
        check(f"{label} forward dataset {r}", f[sl], ref_f[sl], fhat[r], l2, mt)
        check(f"{label} adjoint dataset {r}", a[r], ref_a[r], y[sl], l2, mt)


def _run(plan, bufs, stream):
    import torch
    plan.trafo(bufs["fhat"], bufs["f"], stream)
    plan.adjoint(bufs["y"], bufs["a"], stream)
    torch.cuda.synchronize()
    return bufs["f"].cpu().numpy().copy(), bufs["a"].cpu().numpy().copy()


def _forms(prec):
    o2 = [lib.GT_GATHER_SORTED, lib.GT_GATHER_CELL] + ([lib.GT_GATHER_POLY] if prec == "f32" else [])
    return [(p1, p2) for p1 in (lib.GT_GATHER_SORTED, lib.GT_GATHER_CELL) for p2 in o2]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused_equals_separate_and_oracle(case, prec):
    import torch
    name, d, ds, N, M, R, m = case
    iset, x, fhat, y, plan, bufs, offsets = _setup(case, prec)
    ref_f, ref_a = _refs(iset, x, fhat, y, offsets, R)
    s = torch.cuda.Stream()
    for p1, p2 in _forms(prec):
        try:
            plan.set_gather_path(1, p1)
            plan.set_gather_path(2, p2)
        except lib.GroupedError as e:   # a form these nodes cannot take (too few per cell)
            assert e.code == lib.GT_EUNSUPPORTED
            continue
        label = f"{name} {prec} {NAMES[p1]}/{NAMES[p2]}"
        say(f"[fused] {label}")
        plan.set_fused(False)
        f0, a0 = _run(plan, bufs, s.cuda_stream)
        plan.set_fused(True)
        f1, a1 = _run(plan, bufs, s.cuda_stream)
        f2, a2 = _run(plan, bufs, s.cuda_stream)   # again: scratch from the last call must not leak in
        assert np.array_equal(f1, f0) and np.array_equal(a1, a0), label
        assert np.array_equal(f2, f0) and np.array_equal(a2, a0), label
        _check_all(label, f1, a1, fhat, y, ref_f, ref_a, offsets, prec, ds, m, R)
    plan.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_graph_replay_and_tuning(prec):
    """Graph replay of the shared launches (replays between eager work, every replay checked)
    and the tuner's report of its shared-launch trial."""
    import torch
    case = CASES[0]
    iset, x, fhat, y, plan, bufs, offsets = _setup(case, prec)
    s = torch.cuda.Stream()
    f0, a0 = _run(plan, bufs, s.cuda_stream)
    plan.set_fused(True)
    plan.set_graph(True)
    for rep in range(4):
        f1, a1 = _run(plan, bufs, s.cuda_stream)
        assert np.array_equal(f1, f0) and np.array_equal(a1, a0), f"replay {rep}"
        bufs["f"].zero_()
        bufs["a"].zero_()
        torch.cuda.synchronize()
    plan.set_graph(False)
    rep = plan.tune(s.cuda_stream)
    say(f"  tuning: {rep.get('fused')}")
    assert "fused" in rep and set(rep["fused"]) == {"on", "off", "chosen"}
    f2, a2 = _run(plan, bufs, s.cuda_stream)
    ref_f, ref_a = _refs(iset, x, fhat, y, offsets, 1)
    _check_all("tuned", f2, a2, fhat, y, ref_f, ref_a, offsets, prec, 2, 0, 1)
    plan.close()


def test_fused_availability():
    """Only plans of orders 1 and 2 with window forms and one window width take them; a form
    change that breaks this returns the plan to the separate launches."""
    import torch
    x = W.uniform_nodes(W.rng(97, W.P_NODES), 4000, 4, "f64")
    p3, k3 = lib.make_problem(4, 3, (8, 6, 4), M=4000, dtype=lib.GT_C128)
    plan3 = lib.Plan(p3, to_dev(x), keepalive=k3)
    with pytest.raises(lib.GroupedError) as e:
        plan3.set_fused(True)
    assert e.value.code == lib.GT_EUNSUPPORTED
    plan3.set_fused(False)
    plan3.close()
    case = CASES[2]
    iset, x2, fhat, y, plan, bufs, offsets = _setup(case, "f64")
    s = torch.cuda.Stream()
    plan.set_gather_path(2, lib.GT_GATHER_DIRECT)
    with pytest.raises(lib.GroupedError) as e:
        plan.set_fused(True)
    assert e.value.code == lib.GT_EUNSUPPORTED
    plan.set_gather_path(2, lib.GT_GATHER_SORTED)
    plan.set_fused(True)
    plan.set_gather_path(2, lib.GT_GATHER_DIRECT)   # now separate launches again
    f, a = _run(plan, bufs, s.cuda_stream)
    ref_f, ref_a = _refs(iset, x2, fhat, y, offsets, case[5])
    _check_all("direct after fused", f, a, fhat, y, ref_f, ref_a, offsets, "f64", 2, case[6], case[5])
    plan.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_weighted_lsqr_equals_separate(prec):
    """LSQR with Sobolev weights (the column scale enters the packs and the adjoint DFTs):
    the shared launches give the separate launches' iterate bit for bit."""
    import torch
    d, ds, N, M, R = 6, 2, (24, 10), 5000, 2
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(98, W.P_NODES), M, d, prec)
    y1 = W.complex_normal(W.rng(98, W.P_SAMPLES), (M,), prec)
    K = iset.full_frequencies()
    omega = np.prod((1.0 + np.abs(K)) ** 0.5, axis=1)
    p, keep = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    ct = torch.complex64 if prec == "f32" else torch.complex128
    outs = []
    for fused in (False, True):
        plan.set_fused(fused)
        out = torch.empty(R * iset.n_coeffs, dtype=ct, device="cuda")
        plan.lsqr(to_dev(np.tile(y1, R)), [0.5, 20.0], to_dev(omega), 12, 0.0, out)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
    say(f"  weighted lsqr {prec}: max |diff| {np.max(np.abs(outs[0] - outs[1])):.3e}")
    assert np.array_equal(outs[0], outs[1])
    plan.close()


def test_adjoint_repeats_bit_for_bit():
    """FP64 adjoint of orders 1 and 2, separate and shared launches, three times each: the
    order-1 spread sums its cells in a fixed order (grid copies per cell residue), the order-2
    spread and all folds in fixed orders, so every repeat gives the same bits."""
    import torch
    case = CASES[1]
    iset, x, fhat, y, plan, bufs, offsets = _setup(case, "f64")
    s = torch.cuda.Stream()
    for fused in (False, True):
        plan.set_fused(fused)
        outs = []
        for _ in range(3):
            plan.adjoint(bufs["y"], bufs["a"], s.cuda_stream)
            torch.cuda.synchronize()
            outs.append(bufs["a"].cpu().numpy().copy())
        assert all(np.array_equal(o, outs[0]) for o in outs[1:]), f"fused={fused}"
    plan.close()
