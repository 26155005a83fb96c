"""Autograd over the grouped transform: gradients with respect to the coefficients (adjoint)
and to the node positions (node-gradient kernel), against the oracle's analytic gradient,
finite differences (step 1e-3, FP64) and torch.autograd.gradcheck."""
import numpy as np
import pytest

import workloads as W
from oracle import index_set as oidx
from oracle import transform as otr
from tests.gpu_util import rel, say, to_dev

pytestmark = pytest.mark.gpu


def _ragged(seed, B, lo, hi, d, ds, N, prec):
    sizes = W.ragged_sizes(seed, B, lo, hi)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(seed, W.P_NODES), int(offs[-1]), d, prec)
    fh = W.complex_normal(W.rng(seed, W.P_COEFFS), (B, iset.n_coeffs), prec)
    v = W.complex_normal(W.rng(seed, W.P_GRAD), (int(offs[-1]),), prec)
    return iset, offs, x, fh, v


def _grads(iset, offs, x, fh, v, d, ds, N, prec):
    import torch
    from paper_2010_10199_amd.autograd import grouped_trafo
    xt = to_dev(x).requires_grad_(True)
    ft = to_dev(fh).requires_grad_(True)
    f = grouped_trafo(ft, xt, d, ds, N, offsets=offs)
    loss = (torch.conj(to_dev(v)) * f).real.sum()          # Re <v, f>
    loss.backward()
    torch.cuda.synchronize()
    return ft.grad.cpu().numpy().astype(complex), xt.grad.cpu().numpy().astype(float), f.detach().cpu().numpy()


def _oracle_grads(iset, offs, x, fh, v):
    B = len(offs) - 1
    gfh = np.zeros((B, iset.n_coeffs), complex)
    gx = np.zeros(x.shape)
    for b in range(B):
        a, e = int(offs[b]), int(offs[b + 1])
        if e == a:
            continue
        gfh[b] = otr.adjoint(iset, x[a:e], v[a:e])          # d Re<v, F f>/d conj(f) = F^H v
        D = otr.node_gradient(iset, x[a:e], fh[b])
        gx[a:e] = (np.conj(D) * v[a:e, None]).real
    return gfh, gx


def test_gradients_vs_oracle_fp32_config5_shape():
    """Config-5 shape (d=8, d_s=2, N=(32,10)), 12 ragged datasets of 300..3000 nodes."""
    d, ds, N = 8, 2, (32, 10)
    iset, offs, x, fh, v = _ragged(51, 12, 300, 3000, d, ds, N, "f32")
    say(f"[autograd] fp32 datasets=12 nodes={offs[-1]}")
    gfh, gx, _ = _grads(iset, offs, x, fh, v, d, ds, N, "f32")
    rfh, rgx = _oracle_grads(iset, offs, x, fh, v)
    e1, e2 = rel(gfh, rfh), rel(gx, rgx)
    say(f"  grad fhat {e1:.3e} grad x {e2:.3e}")
    assert e1 <= 1e-5 and e2 <= 1e-5


def test_config5_full_sampled():
    """64 datasets, M_b uniform in [1000, 20000], FP32: gradients on sampled datasets."""
    d, ds, N = 8, 2, (32, 10)
    iset, offs, x, fh, v = _ragged(5, 64, 1000, 20000, d, ds, N, "f32")
    say(f"[autograd config5] nodes={offs[-1]}")
    gfh, gx, _ = _grads(iset, offs, x, fh, v, d, ds, N, "f32")
    for b in (0, 17, 63):
        a, e = int(offs[b]), int(offs[b + 1])
        ref = otr.adjoint(iset, x[a:e], v[a:e])
        S = np.arange(a, min(e, a + 400))
        D = otr.node_gradient(iset, x[S], fh[b])
        rgx = (np.conj(D) * v[S, None]).real
        e1, e2 = rel(gfh[b], ref), rel(gx[S], rgx)
        say(f"  dataset {b} (M_b={e - a}) grad fhat {e1:.3e} grad x {e2:.3e}")
        assert e1 <= 1e-5 and e2 <= 1e-5


def test_finite_differences_fp64():
    """Central differences with step 1e-3 of L = Re<v, f(x)> on the FP64 GPU path; the
    truncation error (2 pi K h)^2/6 ~ 1.7e-3 relative for K = 16 sets the 1e-2 bar."""
    import torch
    from paper_2010_10199_amd.autograd import grouped_trafo
    d, ds, N = 4, 2, (32, 10)
    iset, offs, x, fh, v = _ragged(52, 3, 50, 200, d, ds, N, "f64")
    _, gx, _ = _grads(iset, offs, x, fh, v, d, ds, N, "f64")
    h = 1e-3
    g = np.random.default_rng(1)
    picks = [(int(i), int(j)) for i, j in zip(g.integers(0, x.shape[0], 12), g.integers(0, d, 12))]
    fd = []
    for i, j in picks:
        vals = []
        for s in (+1, -1):
            xp = x.copy()
            xp[i, j] += s * h
            f = grouped_trafo(to_dev(fh), to_dev(xp), d, ds, N, offsets=offs)
            vals.append(float((torch.conj(to_dev(v)) * f).real.sum()))
        fd.append((vals[0] - vals[1]) / (2 * h))
    an = np.array([gx[i, j] for i, j in picks])
    e = rel(an, np.array(fd))
    say(f"[fd] rel {e:.3e}")
    assert e <= 1e-2


def test_gradcheck_fp64():
    import torch
    from paper_2010_10199_amd.autograd import grouped_trafo
    d, ds, N = 3, 2, (6, 4)
    iset, offs, x, fh, v = _ragged(53, 2, 5, 9, d, ds, N, "f64")
    xt = to_dev(x).requires_grad_(True)
    ft = to_dev(fh).requires_grad_(True)
    ok = torch.autograd.gradcheck(lambda a, b: grouped_trafo(a, b, d, ds, N, offsets=offs), (ft, xt), eps=1e-6,
                                  atol=1e-6, rtol=1e-5)
    assert ok


def test_shared_nodes_batch_gradient_sums_over_rhs():
    """R right-hand sides on shared nodes: grad_x sums the contributions of every r."""
    d, ds, N, M, R = 3, 2, (10, 6), 500, 3
    iset = oidx.grouped_index_set(d, ds, N)
    x, fh, yv = W.trafo_inputs(54, d, ds, M, iset.n_coeffs, R, "f64")
    v = yv.reshape(R, M)
    import torch
    from paper_2010_10199_amd.autograd import grouped_trafo
    xt = to_dev(x).requires_grad_(True)
    ft = to_dev(fh).requires_grad_(True)
    f = grouped_trafo(ft, xt, d, ds, N)
    (torch.conj(to_dev(v)) * f).real.sum().backward()
    gx = xt.grad.cpu().numpy()
    ref = np.zeros_like(x)
    for r in range(R):
        ref += (np.conj(otr.node_gradient(iset, x, fh[r])) * v[r][:, None]).real
    e = rel(gx, ref)
    say(f"[shared grad] rel {e:.3e}")
    assert e <= 1e-11


def test_fixed_nodes_reuses_its_plan_and_matches():
    """GroupedTrafoFixedNodes: forward and coefficient gradient equal grouped_trafo's on the
    same ragged inputs (same kernels and plan contents: bit for bit) over three calls on the
    one plan, and the gradient matches the oracle's adjoint."""
    import torch
    from paper_2010_10199_amd.autograd import GroupedTrafoFixedNodes, grouped_trafo
    d, ds, N = 8, 2, (32, 10)
    iset, offs, x, fh, v = _ragged(52, 6, 300, 2000, d, ds, N, "f32")
    xt = to_dev(x)
    mod = GroupedTrafoFixedNodes(xt, d, ds, N, offsets=offs)
    vt = to_dev(v)
    for it in range(3):
        ft = to_dev(fh * (1.0 + it)).requires_grad_(True)
        f = mod(ft)
        (torch.conj(vt) * f).real.sum().backward()
        ft2 = to_dev(fh * (1.0 + it)).requires_grad_(True)
        f2 = grouped_trafo(ft2, xt, d, ds, N, offsets=offs)
        (torch.conj(vt) * f2).real.sum().backward()
        torch.cuda.synchronize()
        assert torch.equal(f, f2) and torch.equal(ft.grad, ft2.grad)
    gfh = ft.grad.cpu().numpy().astype(complex)
    rfh, _ = _oracle_grads(iset, offs, x, fh * 3.0, v)
    e = rel(gfh, rfh)
    say(f"[fixed nodes] grad fhat vs oracle {e:.3e}")
    assert e <= 1e-5
    mod.close()


def test_moving_nodes_match_fresh_plans_and_oracle():
    """GroupedTrafoMovingNodes over three node sets on one plan (device re-binning): forward
    and both gradients equal those of grouped_trafo's fresh plan for the same nodes, except
    for the gather forms (the moved plan takes the sorted gather; the fresh plan may take
    the cell or polynomial gather), so compared at the FP32 bar; the last step against the
    oracle."""
    import torch
    from paper_2010_10199_amd.autograd import GroupedTrafoMovingNodes
    d, ds, N = 8, 2, (32, 10)
    iset, offs, x, fh, v = _ragged(53, 6, 300, 2500, d, ds, N, "f32")
    mod = GroupedTrafoMovingNodes(to_dev(x), d, ds, N, offsets=offs)
    vt = to_dev(v)
    for it in range(3):
        xi = W.uniform_nodes(W.rng(530 + it, W.P_NODES), x.shape[0], d, "f32")
        xt = to_dev(xi).requires_grad_(True)
        ft = to_dev(fh).requires_grad_(True)
        f = mod(ft, xt)
        (torch.conj(vt) * f).real.sum().backward()
        gfh2, gx2, f2 = _grads(iset, offs, xi, fh, v, d, ds, N, "f32")
        torch.cuda.synchronize()
        e0 = rel(f.detach().cpu().numpy(), f2)
        e1 = rel(ft.grad.cpu().numpy(), gfh2)
        e2 = rel(xt.grad.cpu().numpy(), gx2)
        say(f"[moving nodes] step {it}: f {e0:.2e} grad fhat {e1:.2e} grad x {e2:.2e} (vs a fresh plan)")
        assert e0 <= 1e-5 and e1 <= 1e-5 and e2 <= 1e-5
    rfh, rgx = _oracle_grads(iset, offs, xi, fh, v)
    e1, e2 = rel(ft.grad.cpu().numpy(), rfh), rel(xt.grad.cpu().numpy(), rgx)
    say(f"[moving nodes] vs oracle: grad fhat {e1:.2e} grad x {e2:.2e}")
    assert e1 <= 1e-5 and e2 <= 1e-5
    # a second call before the first call's backward: the backward refuses
    ft = to_dev(fh).requires_grad_(True)
    fa = mod(ft, to_dev(x))
    mod(to_dev(fh), to_dev(xi))
    with pytest.raises(RuntimeError):
        (torch.conj(vt) * fa).real.sum().backward()
    mod.close()


def test_tuned_fixed_and_moving_nodes_vs_oracle():
    """tune=True: the objects' plans take measured launch forms (the shared launches of orders
    1 and 2 among them); the gradients still meet the FP32 bar against the oracle, for fixed
    nodes and for nodes moved twice on the tuned plan."""
    import torch
    from paper_2010_10199_amd.autograd import GroupedTrafoFixedNodes, GroupedTrafoMovingNodes
    d, ds, N = 8, 2, (32, 10)
    iset, offs, x, fh, v = _ragged(54, 6, 300, 2500, d, ds, N, "f32")
    vt = to_dev(v)
    fixed = GroupedTrafoFixedNodes(to_dev(x), d, ds, N, offsets=offs, tune=True)
    say(f"[tuned fixed] {fixed.tuning.get('fused')}")
    ft = to_dev(fh).requires_grad_(True)
    (torch.conj(vt) * fixed(ft)).real.sum().backward()
    rfh, _ = _oracle_grads(iset, offs, x, fh, v)
    e = rel(ft.grad.cpu().numpy(), rfh)
    say(f"[tuned fixed] grad fhat vs oracle {e:.3e}")
    assert e <= 1e-5
    fixed.close()
    moving = GroupedTrafoMovingNodes(to_dev(x), d, ds, N, offsets=offs, tune=True)
    for it in range(2):
        xi = W.uniform_nodes(W.rng(540 + it, W.P_NODES), x.shape[0], d, "f32")
        xt = to_dev(xi).requires_grad_(True)
        ft = to_dev(fh).requires_grad_(True)
        (torch.conj(vt) * moving(ft, xt)).real.sum().backward()
        torch.cuda.synchronize()
        rfh, rgx = _oracle_grads(iset, offs, xi, fh, v)
        e1, e2 = rel(ft.grad.cpu().numpy(), rfh), rel(xt.grad.cpu().numpy(), rgx)
        say(f"[tuned moving] step {it}: grad fhat {e1:.2e} grad x {e2:.2e}")
        assert e1 <= 1e-5 and e2 <= 1e-5
    moving.close()
