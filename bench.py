"""Benchmark of the grouped Fourier transform hot path on one MI355X.

Workload: d = 10, d_s = 2, bandwidths N = 64 (1-D terms) / 16 (2-D terms), 56 ANOVA terms,
10,756 coefficients, M = 50,000 nodes uniform on [-1/2, 1/2)^10, complex coefficients and
samples CN(0, 1), Kaiser-Bessel window m = 6, oversampling 2.  One step = one forward and
one adjoint transform on a plan built once for the node set (inputs resident in HBM).

metric: node-terms/s = 2 * M * |U| / (time of forward + adjoint), FP32 bulk arithmetic.
Prints one JSON line.  The timed steps run on a dedicated stream (the library forks its
order-1 kernels onto a second stream and joins them back).  A second timed pass of the same
steps runs on one stream with a HIP event pair around every kernel launch; the per-kernel
durations and the roofline of the dominant kernel come from that pass.
"""
from __future__ import annotations

import argparse
import hashlib
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

D, DS, NB, M, M_WIN, SIGMA = 10, 2, (64, 16), 50000, 6, 2.0
PEAK_FP32_VECTOR_TFLOPS = 157.3      # 256 CU x 2.4 GHz x 64 lanes x 2 (FMA) x 2 (packed)
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def flops_per_node_term(order: int, m: int) -> int:
    """Algorithmic FLOPs of one node-term gather or spread: w^t real x complex MACs plus the
    lower-dimensional partial sums (w = 2m), 4 flops per real x complex MAC."""
    w = 2 * m
    return 4 * sum(w ** k for k in range(1, order + 1))


def direct_flops_per_node_term(order: int, N: int, R: int) -> int:
    """Algorithmic FLOPs of one node-term of the direct sums: (N - 1)^order complex MACs per
    right-hand side, 8 flops each (the phases, computed on the vector units, not counted)."""
    return 8 * (N - 1) ** order * R


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels_impl.h", "gt_internal.h", "gather.h", "spread.h", "direct.h", "fused.h"):
        with open(os.path.join(ROOT, "paper_2010_10199_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted_bytes(tj: dict, record: str, tuning: dict, khash: str):
    """HBM bytes per launch of a timing record from the counter table, for the kernel form the tuner chose.

    A gather record may have been counted in several forms (a sorted, cell or polynomial sweep, and its
    packing kernel with it); the entry used is the one of the chosen form.  The kernels of any other record
    all run in each of its launches and are summed.  None when the table was taken with other kernel
    sources or lacks the form.
    """
    ent = tj.get("kernels", {}).get(record)
    if not ent or ent.get("kernel_hash") != khash:
        return None
    forms = ent.get("forms", {})
    if len(forms) <= 1:
        return ent.get("bytes_per_launch")
    if record in ("gather_12", "pack_fwd_12"):
        # shared launches of orders 1 and 2: the forms are template arguments, the gather's
        # <T, m, order-1 form, order-2 form>, the pack's <T, m> with m = 0 unless order 2 is polynomial
        code = {"sorted": 0, "cell": 1, "poly": 2}
        ch = {o: (tuning or {}).get("gather", {}).get(o, {}).get("chosen") for o in ("1", "2")}
        if record == "gather_12":
            if ch["1"] not in code or ch["2"] not in code:
                return None
            tail = f", {code[ch['1']]}, {code[ch['2']]}>"
            hit = [e for k, e in forms.items() if k.endswith(tail)]
        else:
            hit = [e for k, e in forms.items() if k.endswith(", 0>") == (ch["2"] != "poly")]
        return hit[0]["bytes_per_launch"] if len(hit) == 1 else None
    order = record.rsplit("_", 1)[-1][:-1]
    chosen = (tuning or {}).get("gather", {}).get(order, {}).get("chosen")
    want = {("gather", "cell"): "k_gather_cell<", ("gather", "sorted"): "k_gather_sorted<",
            ("gather", "poly"): "k_gather_poly2<", ("pack", "poly"): "k_pack_poly2<"}
    kind = "pack" if record.startswith("pack") else "gather" if record.startswith("gather") else None
    if kind is None:
        return sum(e["bytes_per_launch"] for e in forms.values())
    sub = want.get((kind, chosen), "k_pack_fwd<" if kind == "pack" else None)
    for k, e in forms.items():
        if sub and sub in k:
            return e["bytes_per_launch"]
    return None


def run_gpu(precision: str, steps: int, warmup: int, profile: bool, launch: str = "tuned",
            count_forms: bool = False):
    import torch
    import workloads as W
    from paper_2010_10199_amd import lib
    code = lib.GT_C64 if precision == "f32" else lib.GT_C128
    ncoef = lib.gt_num_coeffs(D, DS, NB)
    nterms = lib.gt_num_terms(D, DS)
    x, fhat, y = W.trafo_inputs(2, D, DS, M, ncoef, 1, precision)
    cdt = torch.complex64 if precision == "f32" else torch.complex128
    xd = torch.from_numpy(x).cuda()
    fd = torch.from_numpy(fhat.reshape(-1)).cuda()
    yd = torch.from_numpy(y).cuda()
    f_out = torch.empty(M, dtype=cdt, device="cuda")
    a_out = torch.empty(ncoef, dtype=cdt, device="cuda")
    stream = torch.cuda.Stream()          # a dedicated stream, default priority
    prob, keep = lib.make_problem(D, DS, NB, M=M, R=1, dtype=code, m=M_WIN, sigma=SIGMA)

    def timed(n, fwd=True, adj=True):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(n):
            if fwd:
                plan.trafo(fd, f_out)
            if adj:
                plan.adjoint(yd, a_out)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = lib.Plan(prob, xd, keepalive=keep)
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()    # a second plan for the same nodes: process-wide tables warm
        plan2 = lib.Plan(prob, xd, keepalive=keep)
        torch.cuda.synchronize()
        plan_ms_warm = (time.perf_counter() - t0) * 1e3
        plan2.close()
        t0 = time.perf_counter()
        tuning = plan.tune(stream.cuda_stream)   # launch forms measured on these nodes (off the clock)
        tune_ms = (time.perf_counter() - t0) * 1e3
        if launch != "tuned":                    # pin the orders' launch mode (profiling runs)
            plan.set_fused(launch == "shared")
            tuning = dict(tuning, launch=launch)
        for _ in range(max(warmup, 1)):          # (a graph, if chosen, is captured here)
            plan.trafo(fd, f_out)
            plan.adjoint(yd, a_out)
        ms = timed(steps)
        ms_fwd = timed(steps, adj=False)
        ms_adj = timed(steps, fwd=False)
        kern, ms_eager = {}, None
        if profile:                       # same steps, eager launches with a HIP event pair per launch
            lib.prof_enable(True)
            ms_eager = timed(steps)
            kern = lib.prof_report()
            lib.prof_enable(False)
        if count_forms:                   # one forward in every window-gather form (counter runs)
            keep_paths = (plan.gather_path(1), plan.gather_path(2))
            o2 = [lib.GT_GATHER_SORTED, lib.GT_GATHER_CELL] + ([lib.GT_GATHER_POLY] if precision == "f32" else [])
            for p1 in (lib.GT_GATHER_SORTED, lib.GT_GATHER_CELL):
                for p2 in o2:
                    plan.set_gather_path(1, p1)
                    plan.set_gather_path(2, p2)
                    plan.trafo(fd, f_out)
                    torch.cuda.synchronize()
            plan.set_gather_path(1, keep_paths[0])
            plan.set_gather_path(2, keep_paths[1])
    plan.close()
    return dict(ms=ms, ms_fwd=ms_fwd, ms_adj=ms_adj, ms_eager=ms_eager, plan_ms=plan_ms, plan_ms_warm=plan_ms_warm,
                nterms=nterms, tuning=tuning, tune_ms=tune_ms,
                ncoef=ncoef, kernels=kern)


# solver workload: the group-lasso configuration's shape (d = 12, d_s = 2, N = 48 / 16,
# 79 terms, 15,415 coefficients, M = 200,000) with 8 lambda values
SD, SDS, SN, SM, SR = 12, 2, (48, 16), 200000, 8
TAU = 1e-5                           # accuracy both forms must reach, relative l2 per lambda
REF_ITERS, REF_TOL = 4000, 1e-13     # FP64 reference runs: iteration cap and stopping tolerance
KMAX = 2048                          # largest iteration count tried in the search


def run_solvers():
    """Time to accuracy TAU of the two solvers, FP32 batched (all lambda values in one call)
    against FP64 plain (one call per lambda), on the same FP32-rounded nodes and samples.

    1. Reference: FP64, all lambda values in one call, run until the solver's own stopping
       test reaches REF_TOL (LSQR: normal-equation residual relative to its start; FISTA:
       relative step).
    2. Off the clock, for each form the smallest iteration count K whose solution is within
       TAU of the reference for every lambda it covers (relative l2 error; a reference that
       is zero, lambda at lambda_max, is compared by the error relative to the largest
       reference solution), by doubling from 8 and then bisection (the error is taken to
       stay below TAU once it is).  FP32 batched has one K for the batch; FP64 plain one K
       per lambda.
    3. On the clock: each form's solver calls at its K on plans built off the clock (one plan
       per precision and batch size: FP32 with all lambda values, FP64 with one right-hand
       side, reused by the per-lambda calls); each call synchronises.  Plan creation is
       reported beside it, and the totals with plans as second figures.
    FISTA runs take one step constant for all, L = 1.05 x a 50-step FP64 power-iteration
    estimate of ||F||^2 computed once off the clock, with constant steps."""
    import torch
    import workloads as W
    from paper_2010_10199_amd import lib
    x32 = W.uniform_nodes(W.rng(4, W.P_NODES), SM, SD, "f32")
    target = W.bspline_target(x32)
    y = W.add_noise(W.rng(4, W.P_NOISE), target.astype(np.complex128), 0.01).astype(np.complex64)
    ncoef = lib.gt_num_coeffs(SD, SDS, SN)
    _, offs = lib.gt_term_table(SD, SDS, SN)
    p64, k64 = lib.make_problem(SD, SDS, SN, M=SM, R=1, dtype=lib.GT_C128)
    xd = {"f32": torch.from_numpy(x32).cuda(), "f64": torch.from_numpy(x32.astype(np.float64)).cuda()}
    yd = {"f32": torch.from_numpy(y).cuda(), "f64": torch.from_numpy(y.astype(np.complex128)).cuda()}
    # lambda grids: group lasso from lambda_max = max_u ||(F^H y)_u|| (zero solution above it)
    g = torch.empty(ncoef, dtype=torch.complex128, device="cuda")
    lib.grouped_adjoint(p64, xd["f64"], yd["f64"], g)
    gh = g.cpu().numpy()
    lam_max = max(float(np.linalg.norm(gh[offs[i]:offs[i + 1]])) for i in range(len(offs) - 1))
    lams = {"fista": lam_max * 10.0 ** (-3.0 * np.arange(SR) / (SR - 1)), "lsqr": np.logspace(-4, 1, SR)}
    plan = lib.Plan(p64, xd["f64"], keepalive=k64)
    L = 1.05 * plan.norm_estimate(50)
    plan.close()
    out = {"workload": f"group-lasso shape: d={SD}, d_s={SDS}, N={SN[0]}/{SN[1]}, 79 terms, {ncoef} coefficients, "
                       f"M={SM} uniform nodes, target: 3 one- and 2 two-dimensional B-spline terms + 1% noise, "
                       f"{SR} lambda values", "tau": TAU, "fista_L": L,
           "timing": "wall time of the solver calls on plans built off the clock, at the smallest iteration "
                     "count whose solution is within tau of the converged FP64 reference (counts found off "
                     "the clock); plan creation reported beside it"}
    plans, tunings = {}, {}
    out["tunings"] = tunings

    def get_plan(prec, R):
        if (prec, R) not in plans:
            code = lib.GT_C64 if prec == "f32" else lib.GT_C128
            prob, keep = lib.make_problem(SD, SDS, SN, M=SM, R=R, dtype=code)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pl = lib.Plan(prob, xd[prec], keepalive=keep)
            torch.cuda.synchronize()
            plans[(prec, R)] = (pl, time.perf_counter() - t0)
            tunings[f"{prec}_R{R}"] = pl.tune(torch.cuda.current_stream().cuda_stream)   # off the clock
        return plans[(prec, R)][0]

    def solve(kind, prec, lam, iters, tol=0.0):
        R = len(lam)
        pl = get_plan(prec, R)
        cdt = torch.complex64 if prec == "f32" else torch.complex128
        yy = yd[prec].repeat(R)
        fh = torch.zeros(R * ncoef, dtype=cdt, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if kind == "fista":
            info = pl.fista(yy, lam, None, iters, L, 1.0, tol, fh)
        else:
            info = pl.lsqr(yy, lam, None, iters, tol, fh)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"[bench]   {kind} {prec} R={R} iters={iters} {dt:.3f} s", file=sys.stderr, flush=True)
        return dt, fh.cpu().numpy().reshape(R, ncoef).astype(np.complex128), info

    def smallest(ok):
        """Smallest K in [1, KMAX] with ok(K), assuming ok stays true past the first K."""
        hi = 8
        while not ok(hi):
            if hi >= KMAX:
                return None
            hi = min(2 * hi, KMAX)
        lo = hi // 2 if hi > 8 else 0     # ok(lo) is false (or lo = 0)
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if ok(mid):
                hi = mid
            else:
                lo = mid
        return hi

    for kind in ("fista", "lsqr"):
        lam = lams[kind]
        solve(kind, "f32", lam[:1], 2)           # warm-up (code objects, allocator)
        solve(kind, "f64", lam[:1], 2)
        _, ref, rinfo = solve(kind, "f64", lam, REF_ITERS, REF_TOL)
        nrm = np.linalg.norm(ref, axis=1)
        scale = np.where(nrm > 1e-10 * nrm.max(), nrm, nrm.max())

        def err(sol, idx):
            return float(max(np.linalg.norm(sol[k] - ref[j]) / scale[j] for k, j in enumerate(idx)))

        every = list(range(SR))
        k32 = smallest(lambda K: err(solve(kind, "f32", lam, K)[1], every) <= TAU)
        k64 = [smallest(lambda K, j=j: err(solve(kind, "f64", lam[j:j + 1], K)[1], [j]) <= TAU)
               for j in range(SR)]
        res = {"lambdas": [float(v) for v in lam],
               "reference": {"form": "FP64, all lambda values in one call", "iters": max(i.iters for i in rinfo),
                             "tol": REF_TOL, "final_test_value": max(i.resid for i in rinfo),
                             "converged": all(i.flags & 1 for i in rinfo)}}
        if k32 is None or None in k64:
            res["error"] = f"tau not reached within {KMAX} iterations"
            out[kind] = res
            continue
        t32, s32, _ = solve(kind, "f32", lam, k32)
        t64, e64 = 0.0, 0.0
        for j in range(SR):
            dt, sj, _ = solve(kind, "f64", lam[j:j + 1], k64[j])
            t64 += dt
            e64 = max(e64, err(sj, [j]))
        p32, p64 = plans[("f32", SR)][1], plans[("f64", 1)][1]
        res.update({"fp32_batched": {"iters": k32, "s": t32, "max_rel_err": err(s32, every), "plan_s": p32,
                                     "s_with_plan": t32 + p32},
                    "fp64_plain": {"iters_per_lambda": k64, "s": t64, "max_rel_err": e64, "plan_s": p64,
                                   "s_with_plan": t64 + p64, "s_with_plan_per_call": t64 + SR * p64},
                    "speedup": t64 / t32, "speedup_with_plans": (t64 + p64) / (t32 + p32)})
        out[kind] = res
    for pl, _ in plans.values():
        pl.close()
    return out


# batched-LSQR workload: d = 20, d_s = 3, N = 32 / 12 / 6 (1,351 terms, 166,111 coefficients),
# M = 500,000 uniform nodes, 16 lambda values
CD, CDS, CN, CM, CR = 20, 3, (32, 12, 6), 500000, 16
C3_FP64_TIMED = (0, 5, 10, 15)       # lambda indices whose FP64-plain solves are timed by default


def run_c3(steps: int, all_lambdas: bool, transform_only: bool = False, forms: str = "tune"):
    """The batched-LSQR workload (Sec. 4.1, eq. new_min_prob): d = 20, d_s = 3, N = 32/12/6,
    M = 500,000 uniform nodes, FP32 bulk arithmetic.

    1. Transform throughput with 16 right-hand sides in one launch (the batch the solver's
       lambda values make when each carries its own samples): forward + adjoint on a plan
       built once, node-terms/s = 2 M |U| R / t, per-kernel times from a pass with an event
       pair per launch, and the roofline of the dominant kernel.
    2. Time to accuracy TAU of LSQR for y = 8 random low-order trigonometric monomials + 1 %
       noise and lambda = logspace(-4, 1, 16):
       * reference: FP64, all 16 lambda in one lsqr_solve_path call (shared bidiagonalisation),
         run to a normal-equation residual of 1e-12 relative to its start;
       * FP32 batched: all 16 lambda in one FP32 lsqr_solve_path call at the smallest K with
         every lambda within TAU (relative l2) of the reference;
       * FP64 plain: one FP64 gt_plan_lsqr call per lambda at that lambda's smallest K (found
         off the clock with FP64 path runs, whose iterates are the plain runs' iterates);
         by default the lambda values C3_FP64_TIMED are timed (all 16 with all_lambdas).
       Plans are built off the clock (their creation time is reported separately); each timed
       call is the library call's wall time (launches + one synchronisation)."""
    import torch
    import workloads as W
    from paper_2010_10199_amd import lib
    ncoef = lib.gt_num_coeffs(CD, CDS, CN)
    nterms = lib.gt_num_terms(CD, CDS)
    x32 = W.uniform_nodes(W.rng(3, W.P_NODES), CM, CD, "f32")
    out = {"workload": f"batched-lsqr-d20: d={CD}, d_s={CDS}, N={'/'.join(map(str, CN))}, {nterms} terms, "
                       f"{ncoef} coefficients, M={CM} uniform nodes"}
    # ---- 1. transform, R = 16
    x_d = torch.from_numpy(x32).cuda()
    fh, y0 = W.complex_normal(W.rng(3, W.P_COEFFS), (CR, ncoef), "f32"), W.complex_normal(W.rng(3, W.P_SAMPLES),
                                                                                          (CR, CM), "f32")
    fd, yd = torch.from_numpy(fh.reshape(-1)).cuda(), torch.from_numpy(y0.reshape(-1)).cuda()
    f_out = torch.empty(CR * CM, dtype=torch.complex64, device="cuda")
    a_out = torch.empty(CR * ncoef, dtype=torch.complex64, device="cuda")
    p, keep = lib.make_problem(CD, CDS, CN, M=CM, R=CR, dtype=lib.GT_C64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = lib.Plan(p, x_d, keepalive=keep)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    if forms == "direct":                      # every order on the direct sums (for profiling)
        for t in range(1, CDS + 1):
            plan.set_gather_path(t, lib.GT_GATHER_DIRECT)
            plan.set_adjoint_form(t, lib.GT_ADJ_DIRECT)
        tuning = {"forms": "direct sums for every order, set by hand"}
    else:
        tuning = plan.tune(stream.cuda_stream)     # launch forms measured on these nodes (off the clock)
    tune_s = time.perf_counter() - t0
    print(f"[bench]   c3 tuning R={CR}: {tune_s:.1f} s {json.dumps(tuning)}", file=sys.stderr, flush=True)
    plan.trafo(fd, f_out)
    plan.adjoint(yd, a_out)

    def timed(fwd, adj):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(steps):
            if fwd:
                plan.trafo(fd, f_out)
            if adj:
                plan.adjoint(yd, a_out)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    ms, ms_f, ms_a = timed(True, True), timed(True, False), timed(False, True)
    lib.prof_enable(True)
    plan.trafo(fd, f_out)
    plan.adjoint(yd, a_out)
    kern = lib.prof_report()
    lib.prof_enable(False)
    m3 = plan.order_info(3)[0]
    plan.close()
    del f_out, a_out, fd, yd
    nt = CM * nterms * CR          # node-terms per transform
    name, (cnt, tot) = max(kern.items(), key=lambda kv: kv[1][1])
    order = 2 if "2d" in name else (1 if "1d" in name else 3)
    from math import comb
    if name.startswith("direct"):   # MFMA contraction: useful flops per node-term and right-hand side
        fl = CM * comb(CD, order) * direct_flops_per_node_term(order, CN[order - 1], CR)
    else:
        fl = CM * comb(CD, order) * CR * flops_per_node_term(order, m3)
    out["transform"] = {
        "R": CR, "m": m3, "plan_s": plan_s, "steps": steps, "tune_s": tune_s, "tuning": tuning,
        "fwd_adj": {"value": 2 * nt / (ms * 1e-3), "unit": "node-terms/s", "ms": ms},
        "forward": {"value": nt / (ms_f * 1e-3), "unit": "node-terms/s", "ms": ms_f},
        "adjoint": {"value": nt / (ms_a * 1e-3), "unit": "node-terms/s", "ms": ms_a},
        "kernels_ms": {k: {"launches": v[0], "avg_ms": v[1] / v[0]} for k, v in sorted(kern.items())},
        "roofline": {"bound": "mfma" if name.startswith("direct") else "alu", "kernel": name, "achieved": fl / (tot / cnt * 1e-3) / 1e12,
                     "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": fl / (tot / cnt * 1e-3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, "flops_per_launch": fl,
                     "avg_launch_ms": tot / cnt}}
    print(f"[bench]   c3 transform R={CR}: {ms:.1f} ms per fwd+adj ({2 * nt / (ms * 1e-3):.3e} node-terms/s)",
          file=sys.stderr, flush=True)
    if transform_only:
        return out
    # ---- 2. LSQR time to accuracy
    target, _ = W.sparse_trig_target(3, x32, CN)
    y = W.add_noise(W.rng(3, W.P_NOISE), target, 0.01).astype(np.complex64)
    lams = np.logspace(-4, 1, CR)
    y32, y64 = torch.from_numpy(y).cuda(), torch.from_numpy(y.astype(np.complex128)).cuda()
    x64 = torch.from_numpy(x32.astype(np.float64)).cuda()
    plans = {}
    for prec, xd_ in (("f32", x_d), ("f64", x64)):
        pp, kk = lib.make_problem(CD, CDS, CN, M=CM, R=1, dtype=lib.GT_C64 if prec == "f32" else lib.GT_C128)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plans[prec] = (lib.Plan(pp, xd_, keepalive=kk), time.perf_counter() - t0)
    tunings = {}
    for prec in plans:                         # off the clock, as the plans
        tunings[prec] = plans[prec][0].tune(torch.cuda.current_stream().cuda_stream)
        print(f"[bench]   c3 tuning lsqr plan {prec}: {json.dumps(tunings[prec])}", file=sys.stderr, flush=True)
    cdt = {"f32": torch.complex64, "f64": torch.complex128}

    def path_run(prec, K, tol=0.0):
        buf = torch.empty(CR * ncoef, dtype=cdt[prec], device="cuda")
        info = plans[prec][0].lsqr_path(y32 if prec == "f32" else y64, lams, None, K, tol, buf)
        return buf.cpu().numpy().astype(np.complex128).reshape(CR, ncoef), info

    t0 = time.perf_counter()
    ref, rinfo = path_run("f64", 400, 1e-12)
    ref_s = time.perf_counter() - t0
    ref_norm = np.linalg.norm(ref, axis=1)

    def errs(sol):
        return np.linalg.norm(sol - ref, axis=1) / ref_norm

    cache = {}

    def errs_at(prec, K):
        if (prec, K) not in cache:
            cache[(prec, K)] = errs(path_run(prec, K)[0])
            print(f"[bench]   c3 lsqr {prec} K={K}: max err {cache[(prec, K)].max():.2e}", file=sys.stderr,
                  flush=True)
        return cache[(prec, K)]

    def smallest_k(prec, j=None, guess=None):
        """Smallest K whose error is within TAU (for lambda j, or for all).  Without a guess:
        doubling from 8, then bisection; with one: steps of one from the guess (the error
        falls monotonically in K here)."""
        sel = (lambda e: e.max()) if j is None else (lambda e: e[j])
        if guess is not None:
            K = guess
            if sel(errs_at(prec, K)) <= TAU:
                while K > 1 and sel(errs_at(prec, K - 1)) <= TAU:
                    K -= 1
                return K
            while sel(errs_at(prec, K)) > TAU:
                K += 1
                if K > 256:
                    return None
            return K
        lo, hi = 0, 8
        while sel(errs_at(prec, hi)) > TAU:
            lo, hi = hi, 2 * hi
            if hi > 256:
                return None
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if sel(errs_at(prec, mid)) <= TAU:
                hi = mid
            else:
                lo = mid
        return hi

    k32 = smallest_k("f32")
    timed_idx = list(range(CR)) if all_lambdas else list(C3_FP64_TIMED)
    # FP64 plain: one search per lambda, started from the FP32 count (path runs give every
    # lambda's error at once, so the searches share their runs)
    k64 = {j: smallest_k("f64", j, guess=k32) for j in timed_idx}
    # on the clock
    buf32 = torch.empty(CR * ncoef, dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans["f32"][0].lsqr_path(y32, lams, None, k32, 0.0, buf32)
    t32 = time.perf_counter() - t0
    e32 = errs(buf32.cpu().numpy().astype(np.complex128).reshape(CR, ncoef))
    buf64 = torch.empty(ncoef, dtype=torch.complex128, device="cuda")
    t64, e64 = 0.0, []
    for j in timed_idx:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plans["f64"][0].lsqr(y64, [float(lams[j])], None, k64[j], 0.0, buf64)
        t64 += time.perf_counter() - t0
        sol = buf64.cpu().numpy().astype(np.complex128)
        e64.append(float(np.linalg.norm(sol - ref[j]) / ref_norm[j]))
    for pl_, _ in plans.values():
        pl_.close()
    out["lsqr"] = {
        "lambdas": [float(v) for v in lams], "tau": TAU,
        "reference": {"form": "FP64, all 16 lambda in one lsqr_solve_path call (m = 8)",
                      "iters": int(max(i[0].iters for i in rinfo)), "tol": 1e-12, "s": ref_s,
                      "converged": all(bool(i[0].flags & lib.GT_SOLVE_CONVERGED) for i in rinfo)},
        "fp32_batched": {"form": "FP32, 16 lambda in one call, one shared bidiagonalisation", "iters": k32,
                         "s": t32, "max_rel_err": float(e32.max()), "plan_s": plans["f32"][1],
                         "tuning": tunings["f32"]},
        "fp64_plain": {"form": "FP64, one gt_plan_lsqr call per lambda", "lambdas_timed": timed_idx,
                       "iters_per_lambda": [k64[j] for j in timed_idx], "s": t64, "max_rel_err": max(e64),
                       "plan_s": plans["f64"][1], "tuning": tunings["f64"]},
        "speedup": (t64 / len(timed_idx) * CR) / t32,
        "speedup_measured_only": t64 / t32,
        "note": ("speedup: FP64-plain time per lambda (timed lambda values) x 16 over the FP32 batched call; "
                 "speedup_measured_only: the timed FP64-plain calls (a subset unless all lambda are timed) "
                 "over the FP32 call for all 16, a lower bound without extrapolation")}
    print(f"[bench]   c3 lsqr: fp32 batched K={k32} {t32:.2f} s; fp64 plain {t64:.2f} s over {len(timed_idx)} lambda",
          file=sys.stderr, flush=True)
    return out


def run_cosine(steps: int):
    """The non-periodic variant (Sec. 5, half-period cosine basis on [0, 1]^d) on the shape of
    the paper's adult-data model: d = 12, d_s = 2, N = 82 / 10 (79 terms, 6,319
    coefficients), M = 36,160 synthetic nodes uniform on [0, 1]^12 (the paper's training size;
    the census data itself is not used), FP32.  Forward + adjoint throughput on a plan, and an
    LSQR fit over 8 lambda values in one lsqr_solve_path call (40 iterations) for samples of a
    smooth target with five active ANOVA terms + 1 % noise."""
    import torch
    import workloads as W
    from paper_2010_10199_amd import lib
    d, ds, N, M = 12, 2, (82, 10), 36160
    ncoef, nterms = lib.gt_num_coeffs(d, ds, N), lib.gt_num_terms(d, ds)
    x = W.unit_cube_nodes(W.rng(8, W.P_NODES), M, d, "f32")
    fh = W.complex_normal(W.rng(8, W.P_COEFFS), (ncoef,), "f32")
    yv = W.complex_normal(W.rng(8, W.P_SAMPLES), (M,), "f32")
    xd, fd, yd = (torch.from_numpy(a).cuda() for a in (x, fh, yv))
    f_out = torch.empty(M, dtype=torch.complex64, device="cuda")
    a_out = torch.empty(ncoef, dtype=torch.complex64, device="cuda")
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C64, basis=lib.GT_BASIS_COS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = lib.Plan(p, xd, keepalive=keep)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    plan.trafo(fd, f_out)
    plan.adjoint(yd, a_out)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        plan.trafo(fd, f_out)
        plan.adjoint(yd, a_out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    # smooth target: 3 one- and 2 two-dimensional terms built from cos(pi x) pieces, + 1 % noise
    xs = x.astype(np.float64)
    tgt = (np.cos(np.pi * xs[:, 0]) + 0.5 * np.cos(2 * np.pi * xs[:, 1]) + xs[:, 2] ** 2 - 1.0 / 3.0
           + np.cos(np.pi * xs[:, 3]) * np.cos(np.pi * xs[:, 4]) + (xs[:, 5] - 0.5) * (xs[:, 6] - 0.5))
    y = W.add_noise(W.rng(8, W.P_NOISE), tgt, 0.01).astype(np.complex64)
    lams = np.logspace(-2, 2, 8)
    path = torch.empty(len(lams) * ncoef, dtype=torch.complex64, device="cuda")
    yt = torch.from_numpy(y).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = plan.lsqr_path(yt, lams, None, 40, 0.0, path)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    sols = path.reshape(len(lams), ncoef)
    resid = []
    for j in range(len(lams)):
        plan.trafo(sols[j].contiguous(), f_out)
        torch.cuda.synchronize()
        resid.append(float(np.linalg.norm(f_out.cpu().numpy() - y) / np.linalg.norm(y)))
    rho = torch.empty(nterms, dtype=torch.float64, device="cuda")
    best = int(np.argmin(resid))
    lib.sensitivity(p, sols[best].contiguous(), rho)
    r = rho.cpu().numpy()
    coords, _ = lib.gt_term_table(d, ds, N)
    top = [tuple(int(c) for c in coords[i] if c >= 0) for i in np.argsort(-r)[:5]]
    plan.close()
    print(f"[bench]   cosine: {ms:.3f} ms per fwd+adj; lsqr path {fit_s:.3f} s", file=sys.stderr, flush=True)
    return {"workload": f"cosine basis, adult-data shape: d={d}, d_s={ds}, N={N[0]}/{N[1]}, {nterms} terms, "
                        f"{ncoef} coefficients, M={M} uniform nodes on [0,1]^12, FP32",
            "plan_s": plan_s, "fwd_adj": {"value": 2 * M * nterms / (ms * 1e-3), "unit": "node-terms/s", "ms": ms},
            "lsqr_path": {"lambdas": [float(v) for v in lams], "iters": 40, "s": fit_s,
                          "rel_residual": resid, "best_lambda": float(lams[best]),
                          "top5_terms_by_sensitivity": top,
                          "true_terms": [(0,), (1,), (2,), (3, 4), (5, 6)]}}


def run_active_set():
    """The pipeline of Sec. 4.1 on the solver workload (B-spline target with 3 one- and 2
    two-dimensional terms, 1 % noise), FP32: LSQR fit on U_2, global sensitivity indices
    (eq. gsi) on the GPU, active set U* (eq. activeset) with thresholds 0.01, and the LSQR
    refit on I_N(U*) with larger bandwidths.  Each stage is the one-shot library call (plan
    included) timed by wall clock with the stream synchronised; the indices' kernels read
    the coefficients once (|I| complex values)."""
    import torch
    import workloads as W
    from paper_2010_10199_amd import lib
    x32 = W.uniform_nodes(W.rng(4, W.P_NODES), SM, SD, "f32")
    y = W.add_noise(W.rng(4, W.P_NOISE), W.bspline_target(x32).astype(np.complex128), 0.01).astype(np.complex64)
    xd, yd = torch.from_numpy(x32).cuda(), torch.from_numpy(y).cuda()
    K, lam, eps, N2 = 10, 1e-3, (0.01, 0.01), (64, 24)
    stages = {}

    def timed(name, fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        stages[name] = time.perf_counter() - t0
        return res

    p, keep = lib.make_problem(SD, SDS, SN, M=SM, R=1, dtype=lib.GT_C64)
    nt, nc = lib.problem_size(p)
    fh = torch.zeros(nc, dtype=torch.complex64, device="cuda")
    timed("fit_s", lambda: lib.lsqr_solve(p, xd, yd, [lam], None, K, 0.0, fh))
    rho = torch.empty(nt, dtype=torch.float64, device="cuda")
    timed("sensitivity_s", lambda: lib.sensitivity(p, fh, rho))
    reps = 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lib.sensitivity(p, fh, rho)
    gsi_us = (time.perf_counter() - t0) / reps * 1e6
    rh = rho.cpu().numpy()
    mask, na = timed("active_set_s", lambda: lib.active_set(p, rh, eps))
    terms = [u for u, k in zip(itertools.chain.from_iterable(
        itertools.combinations(range(SD), t) for t in range(SDS + 1)), mask) if k]
    true = {(0,), (1,), (2,), (3, 4), (5, 6)}
    p2, keep2 = lib.make_problem(SD, SDS, N2, M=SM, R=1, dtype=lib.GT_C64, term_mask=mask)
    nt2, nc2 = lib.problem_size(p2)
    f2 = torch.zeros(nc2, dtype=torch.complex64, device="cuda")
    timed("refit_s", lambda: lib.lsqr_solve(p2, xd, yd, [0.0], None, K, 0.0, f2))

    def resid(prob, f):
        r = torch.empty(SM, dtype=torch.complex64, device="cuda")
        lib.grouped_trafo(prob, xd, f, r)
        return float(torch.linalg.norm(r - yd) / torch.linalg.norm(yd))

    out = {"workload": f"solver workload (d={SD}, d_s={SDS}, N={SN[0]}/{SN[1]}, M={SM}), FP32, LSQR {K} "
                       f"iterations for the fit (lambda {lam}) and the refit (lambda 0, N={N2[0]}/{N2[1]})",
           "thresholds": list(eps), "terms": nt, "active": [list(u) for u in terms if u],
           "true_terms_found": all(u in terms for u in true), "false_terms": sum(1 for u in terms if u and u not in true),
           "refit_coeffs": nc2, "rel_residual_fit": resid(p, fh), "rel_residual_refit": resid(p2, f2),
           "sensitivity_call_us": gsi_us, "sensitivity_bytes": nc * 8,
           **{k: v for k, v in stages.items()}}
    out["pipeline_s"] = sum(stages.values())
    del keep, keep2
    return out


def run_testfun(draw: int = 0):
    """The paper's LSQR experiments on its test function (Sec. 4, eq. testfun; Sec. 4.1 (i) to
    (iv)): d = 9, d_s = 3, M = 10,000 uniform nodes; (i) N = 26/6/4 (3,394 coefficients),
    exact samples, no weights; (ii) (i) with 10 % noise (standard deviation 0.1 x RMS of the
    samples); (iii) N = 352/20/8 (44,968 coefficients, more than nodes), Sobolev weights
    omega(k) = prod (1 + |k_j|)^1.5 (eq. sobolevweights), exact samples; (iv) (iii) with 10 %
    noise.  Each: one batched FP32 LSQR call for lambda = e^0 .. e^10, the relative L2 error
    of eq. L2error per lambda (Parseval with the exact coefficients), the sensitivity indices
    of the best solution, the active set with thresholds 0.001 and the refit on it (same
    bandwidths, weights and lambda).  One node draw (the paper averages 100)."""
    import torch
    import workloads as W
    from paper_2010_10199_amd import lib
    d, ds, M = 9, 3, 10000
    lams = np.exp(np.arange(11.0))
    R = len(lams)
    x = W.uniform_nodes(W.rng(7, W.P_NODES, draw), M, d, "f32")
    y0 = W.testfun(x)
    xd = torch.from_numpy(x).cuda()
    n2 = W.testfun_norm2()
    want = set()
    for g in W.TESTFUN_GROUPS:
        for t in (1, 2, 3):
            want.update(itertools.combinations(g, t))

    def experiment(N, noise, s_w, iters, printed):
        y = (W.add_noise(W.rng(7, W.P_NOISE, draw), y0, noise) if noise else y0).astype(np.complex64)
        yd = torch.from_numpy(y).cuda()

        def band(n):
            return [k for k in range(-n // 2, n // 2) if k != 0]

        def freqs(ts):
            return [np.array(list(itertools.product(band(N[len(u) - 1]), repeat=len(u)))) if u
                    else np.zeros((1, 0), dtype=np.int64) for u in ts]

        def weights(ts):   # eq. sobolevweights, one per coefficient in coefficient order
            return np.concatenate([np.prod((1.0 + np.abs(f)) ** s_w, axis=1) if u else np.ones(1)
                                   for u, f in zip(ts, freqs(ts))])

        def l2(fh, ex):    # eq. L2error by Parseval
            return float(np.sqrt(max(n2 + np.sum(np.abs(fh - ex) ** 2) - np.sum(np.abs(ex) ** 2), 0.0) / n2))

        coords, offs = lib.gt_term_table(d, ds, N)
        terms = [tuple(int(c) for c in row if c >= 0) for row in coords]
        nc = int(offs[-1])
        exact = W.testfun_coeffs(terms, freqs(terms))
        om = torch.from_numpy(weights(terms)).cuda() if s_w else None
        p, keep = lib.make_problem(d, ds, N, M=M, R=R, dtype=lib.GT_C64)
        fh = torch.zeros(R * nc, dtype=torch.complex64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lib.lsqr_solve(p, xd, yd.repeat(R), lams, om, iters, 0.0, fh)
        torch.cuda.synchronize()
        t_fit = time.perf_counter() - t0
        fhs = fh.cpu().numpy().reshape(R, nc).astype(np.complex128)
        errs = [l2(fhs[r], exact) for r in range(R)]
        best = int(np.argmin(errs))
        p1, keep1 = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C64)
        rho = torch.empty(len(terms), dtype=torch.float64, device="cuda")
        lib.sensitivity(p1, fh[best * nc:(best + 1) * nc], rho)
        mask, na = lib.active_set(p1, rho.cpu().numpy(), (1e-3, 1e-3, 1e-3))
        act = [u for u, k in zip(terms, mask) if k]
        p2, keep2 = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C64, term_mask=mask)
        nt2, nc2 = lib.problem_size(p2)
        f2 = torch.zeros(nc2, dtype=torch.complex64, device="cuda")
        om2 = torch.from_numpy(weights(act)).cuda() if s_w else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lib.lsqr_solve(p2, xd, yd, [float(lams[best])], om2, iters, 0.0, f2)
        torch.cuda.synchronize()
        t_refit = time.perf_counter() - t0
        err_refit = l2(f2.cpu().numpy().astype(np.complex128), W.testfun_coeffs(act, freqs(act)))
        del keep, keep1, keep2
        print(f"[bench]   test function N={N} noise={noise} s={s_w}: best {min(errs):.4f}, refit {err_refit:.4f}",
              file=sys.stderr, flush=True)
        return {"N": list(N), "coefficients": nc, "noise": noise, "s": s_w, "lsqr_iterations": iters,
                "l2_error": {f"e^{r}": errs[r] for r in range(R)}, "best_lambda": f"e^{best}",
                "active_terms": len(act) - 1, "active_set_is_printed_U*": set(act) - {()} == want,
                "refit_coeffs": nc2, "l2_error_refit": err_refit, "fit_s": t_fit, "refit_s": t_refit,
                "paper": printed}

    return {"workload": f"test function, d={d}, d_s={ds}, M={M} uniform nodes, FP32, lambda = e^0..e^10 in one "
                        "LSQR call, one node draw (the paper averages 100)",
            "i": experiment((26, 6, 4), 0.0, 0.0, 50, "about 9.1e-2 after the refit on U*"),
            "ii": experiment((26, 6, 4), 0.1, 0.0, 50, "about 0.165 after the refit on U*"),
            "iii": experiment((352, 20, 8), 0.0, 1.5, 100, "about 1.8e-2 after the refit on U*"),
            "iv": experiment((352, 20, 8), 0.1, 1.5, 100, "about 0.189 after the refit on U*")}


def run_testfun_fista(draw: int = 0):
    """The paper's FISTA experiments on its test function (Sec. 4.2 (i) to (iv), Algorithm
    algo:fista as printed): the settings of run_testfun, group lasso over lambda = e^10, e^9,
    .., e^0 in one library call (fista_group_lasso_path: one plan, the first lambda from zero
    and each next one started from the previous solution), KF iterations per lambda with
    backtracking from L_0 = M (every column of F has squared norm M, so ||F||^2 >= M) and
    eta = 2; the relative L2 error on U_3 (no refit) per lambda and the active set of the best
    solution (indices > 0.001).  FP32, one node draw."""
    import torch
    import workloads as W
    from paper_2010_10199_amd import lib
    d, ds, M, KF, ETA = 9, 3, 10000, 200, 2.0
    lams = np.exp(np.arange(10.0, -1.0, -1.0))
    x = W.uniform_nodes(W.rng(7, W.P_NODES, draw), M, d, "f32")
    y0 = W.testfun(x)
    xd = torch.from_numpy(x).cuda()
    n2 = W.testfun_norm2()
    want = set()
    for g in W.TESTFUN_GROUPS:
        for t in (1, 2, 3):
            want.update(itertools.combinations(g, t))

    def experiment(N, noise, s_w, printed):
        y = (W.add_noise(W.rng(7, W.P_NOISE, draw), y0, noise) if noise else y0).astype(np.complex64)
        yd = torch.from_numpy(y).cuda()

        def band(n):
            return [k for k in range(-n // 2, n // 2) if k != 0]

        coords, offs = lib.gt_term_table(d, ds, N)
        terms = [tuple(int(c) for c in row if c >= 0) for row in coords]
        fr = [np.array(list(itertools.product(band(N[len(u) - 1]), repeat=len(u)))) if u
              else np.zeros((1, 0), dtype=np.int64) for u in terms]
        nc = int(offs[-1])
        exact = W.testfun_coeffs(terms, fr)
        om = None
        if s_w:
            w = np.concatenate([np.prod((1.0 + np.abs(f)) ** s_w, axis=1) if u else np.ones(1)
                                for u, f in zip(terms, fr)])
            om = torch.from_numpy(w).cuda()
        p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C64)
        path = torch.zeros(len(lams) * nc, dtype=torch.complex64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = lib.fista_group_lasso_path(p, xd, yd, lams, om, KF, float(M), ETA, 0.0, None, path)
        torch.cuda.synchronize()
        t_path = time.perf_counter() - t0
        sols = path.reshape(len(lams), nc)
        errs = []
        for j in range(len(lams)):
            fv = sols[j].cpu().numpy().astype(np.complex128)
            errs.append(float(np.sqrt(max(n2 + np.sum(np.abs(fv - exact) ** 2) - np.sum(np.abs(exact) ** 2), 0.0)
                                      / n2)))
        best = int(np.argmin(errs))
        rho = torch.empty(len(terms), dtype=torch.float64, device="cuda")
        lib.sensitivity(p, sols[best].contiguous(), rho)
        mask, na = lib.active_set(p, rho.cpu().numpy(), (1e-3, 1e-3, 1e-3))
        act = {u for u, k in zip(terms, mask) if k and u}
        print(f"[bench]   fista test function N={N} noise={noise} s={s_w}: best {min(errs):.4f}",
              file=sys.stderr, flush=True)
        return {"N": list(N), "coefficients": nc, "noise": noise, "s": s_w, "iterations_per_lambda": KF,
                "L0": float(M), "eta": ETA, "L_final": [inf[0].L for inf in infos],
                "capped": any(inf[0].flags & lib.GT_SOLVE_BACKTRACK_CAP for inf in infos),
                "l2_error": {f"e^{int(round(np.log(l)))}": e for l, e in zip(lams, errs)},
                "best_lambda": f"e^{int(round(np.log(lams[best])))}", "best_l2_error": errs[best],
                "active_terms": len(act), "active_set_is_printed_U*": act == want, "path_s": t_path,
                "paper": printed}

    return {"workload": f"test function, d={d}, d_s={ds}, M={M} uniform nodes, FP32, group lasso (FISTA with "
                        "backtracking) on the warm-started path lambda = e^10 .. e^0 in one call, one node draw "
                        "(the paper averages 100)",
            "i": experiment((26, 6, 4), 0.0, 0.0, "about 9.2e-2 on U_3"),
            "ii": experiment((26, 6, 4), 0.1, 0.0, "about 0.202 on U_3"),
            "iii": experiment((352, 20, 8), 0.0, 1.5, "about 1.7e-2 on U_3"),
            "iv": experiment((352, 20, 8), 0.1, 1.5, "about 0.203 on U_3")}


def run_autograd(steps: int = 10):
    """The differentiable transform on the ragged workload (64 datasets of 1,000 .. 20,000
    nodes, d = 8, d_s = 2, N = 32/10, 37 terms, FP32): forward + backward of Re<v, f> with
    respect to the coefficients and the nodes.  (a) Whole steps through the
    torch.autograd.Function (a plan per forward: node sort included); (b) the three passes
    (forward, adjoint, node gradient) on one plan; (c) forward + coefficient gradient with
    GroupedTrafoFixedNodes (one plan for all steps); (d) whole steps with
    GroupedTrafoMovingNodes, the nodes moved by a small descent step each time (one plan,
    its nodes re-binned on the device per step).  Rates in node-terms/s of the passes."""
    import torch
    import workloads as W
    from paper_2010_10199_amd import lib
    from paper_2010_10199_amd.autograd import grouped_trafo
    d, ds, N, B = 8, 2, (32, 10), 64
    sizes = W.ragged_sizes(5, B, 1000, 20000)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    Mt = int(offs[-1])
    nterms, nc = lib.gt_num_terms(d, ds), lib.gt_num_coeffs(d, ds, N)
    x = torch.from_numpy(W.uniform_nodes(W.rng(5, W.P_NODES), Mt, d, "f32")).cuda()
    fh = torch.from_numpy(W.complex_normal(W.rng(5, W.P_COEFFS), (B, nc), "f32")).cuda()
    v = torch.from_numpy(W.complex_normal(W.rng(5, W.P_GRAD), (Mt,), "f32")).cuda()
    xt, ft = x.clone().requires_grad_(True), fh.clone().requires_grad_(True)

    def step():
        f = grouped_trafo(ft, xt, d, ds, N, offsets=offs)
        (torch.conj(v) * f).real.sum().backward()

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps
    from paper_2010_10199_amd.autograd import GroupedTrafoFixedNodes
    fixed = GroupedTrafoFixedNodes(x, d, ds, N, offsets=offs, tune=True)   # tuned off the clock
    fc = fh.clone().requires_grad_(True)

    def step_fixed():
        f = fixed(fc)
        (torch.conj(v) * f).real.sum().backward()

    for _ in range(2):
        step_fixed()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_fixed()
    torch.cuda.synchronize()
    t_fixed = (time.perf_counter() - t0) / steps
    fixed.close()
    # (d) nodes moving every step on one plan: GroupedTrafoMovingNodes (device re-binning)
    from paper_2010_10199_amd.autograd import GroupedTrafoMovingNodes
    moving = GroupedTrafoMovingNodes(x, d, ds, N, offsets=offs, tune=True)   # tuned off the clock
    xm, fm = x.clone().requires_grad_(True), fh.clone().requires_grad_(True)

    def step_moving():
        f = moving(fm, xm)
        (torch.conj(v) * f).real.sum().backward()
        with torch.no_grad():                     # a descent step on the nodes: they move
            xm.add_(xm.grad, alpha=-1e-9)
            xm.grad = None

    for _ in range(2):
        step_moving()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_moving()
    torch.cuda.synchronize()
    t_moving = (time.perf_counter() - t0) / steps
    tunings = {"fixed_nodes": fixed.tuning, "moving_nodes": moving.tuning}
    moving.close()
    p, keep = lib.make_problem(d, ds, N, M=0, R=B, dtype=lib.GT_C64, offsets=offs)
    plan = lib.Plan(p, x, keepalive=keep)
    plan.tune(torch.cuda.current_stream().cuda_stream)   # (the same signature: the cached choice)
    f = torch.empty(Mt, dtype=torch.complex64, device="cuda")
    g = torch.empty(B * nc, dtype=torch.complex64, device="cuda")
    gx = torch.empty((Mt, d), dtype=torch.float32, device="cuda")
    times = {}
    for name, fn in (("forward", lambda: plan.trafo(fh, f)), ("adjoint", lambda: plan.adjoint(v, g)),
                     ("node_grad", lambda: plan.node_grad(fh, v, gx))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / steps
    plan.close()
    nt = Mt * nterms
    passes = sum(times.values())
    return {"workload": f"ragged: {B} datasets, {Mt} nodes, d={d}, d_s={ds}, N={N[0]}/{N[1]}, {nterms} terms, "
                        f"{nc} coefficients per dataset, FP32",
            "autograd_step_ms": t_step * 1e3,
            "autograd_node_terms_per_s": 3 * nt / t_step,
            "moving_nodes_step_ms": t_moving * 1e3,
            "moving_nodes_node_terms_per_s": 3 * nt / t_moving,
            "moving_over_fixed_plan_passes": t_moving / passes,
            "fixed_nodes_step_ms": t_fixed * 1e3,
            "fixed_nodes_node_terms_per_s": 2 * nt / t_fixed,
            "plan_passes_ms": {k: t * 1e3 for k, t in times.items()},
            "plan_passes_node_terms_per_s": {k: nt / t for k, t in times.items()},
            "tunings": tunings,
            "note": "the fixed-nodes and moving-nodes objects and the passes' plan are tuned off the clock; "
                    "autograd steps build a plan (node sort) per forward and count three passes (forward, "
                    "adjoint, node gradient); moving-nodes steps move one plan's nodes (device re-binning) "
                    "before the same three passes, and moving_over_fixed_plan_passes compares them with the "
                    "three passes on a plan whose nodes stay; fixed-nodes steps reuse one plan and count two "
                    "(forward, adjoint)"}


def cpu_baseline(sample_nodes: int):
    """The FP64 oracle (direct sums) on the first `sample_nodes` nodes, forward + adjoint."""
    import workloads as W
    from oracle import index_set as oidx
    from oracle import transform as otr
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    iset = oidx.grouped_index_set(D, DS, NB)
    x, fhat, y = W.trafo_inputs(2, D, DS, M, iset.n_coeffs, 1, "f32")
    xs, ys = x[:sample_nodes], y[:sample_nodes]
    t0 = time.perf_counter()
    otr.forward(iset, xs, fhat[0])
    otr.adjoint(iset, xs, ys)
    dt = time.perf_counter() - t0
    return dict(value=2 * sample_nodes * iset.n_terms / dt, unit="node-terms/s", cores=int(threads), kind="oracle",
                sample=f"forward + adjoint of the FP64 direct-sum oracle on the first {sample_nodes} of the "
                       f"{M} nodes (all {iset.n_terms} terms), {dt:.1f} s on {os.cpu_count()} visible host cores; "
                       "BLAS threads as counted, exponentials single-threaded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=20000, help="nodes for the oracle baseline (0 = skip)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-solvers", action="store_true", help="skip the FP32-batched vs FP64 solver timing")
    ap.add_argument("--draws", type=int, default=1,
                    help="node draws of the test-function experiments (the paper averages 100); means are reported")
    ap.add_argument("--no-c3", action="store_true", help="skip the batched-LSQR workload (d=20, M=500,000)")
    ap.add_argument("--autograd-only", action="store_true",
                    help="of the legs after the transform, run only the autograd one (profiles of the node updates)")
    ap.add_argument("--c3-steps", type=int, default=3, help="timed forward + adjoint steps of the d=20 workload")
    ap.add_argument("--c3-all-lambdas", action="store_true",
                    help="time the FP64-plain solve of all 16 lambda values (default: 4 of them)")
    ap.add_argument("--c3-transform-only", action="store_true",
                    help="d=20 workload: the transform leg only (no LSQR time to accuracy)")
    ap.add_argument("--launch", choices=["tuned", "separate", "shared"], default="tuned",
                    help="d=10 workload: the tuner's launch mode, or orders 1 and 2 pinned to separate launches "
                         "(second stream as tuned) or to shared launches; profilers change the timings the tuner "
                         "sees, so profiling runs pin the mode the unprofiled run takes")
    ap.add_argument("--c3-forms", choices=["tune", "direct"], default="tune",
                    help="d=20 transform leg: tuned launch forms, or the direct sums for every order")
    ap.add_argument("--count-forms", action="store_true",
                    help="after the timed steps, one forward in every window-gather form (counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy 4 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no multi-GPU "
              "path to time", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)          # reads and writes 256 MiB each
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] fp32 steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    r32 = run_gpu("f32", args.steps, args.warmup, profile=True, launch=args.launch, count_forms=args.count_forms)
    node_terms = 2 * M * r32["nterms"]
    value = node_terms * args.steps / (r32["ms"] * 1e-3)
    out = {
        "metric": "grouped NFFT fwd+adj node-terms/s",
        "value": value,
        "unit": "node-terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "trafo-d10: grouped transform forward + adjoint, d=10, d_s=2, N=64/16, "
                               "56 terms, 10,756 coefficients, M=50,000 uniform nodes, Kaiser-Bessel m=6, sigma=2",
                   "d": D, "ds": DS, "N": list(NB), "M": M, "m": M_WIN, "sigma": SIGMA,
                   "plan_ms": round(r32["plan_ms"], 3), "plan_ms_warm": round(r32["plan_ms_warm"], 3),
                   "tune_ms": round(r32["tune_ms"], 1), "tuning": r32["tuning"]},
        "forward": {"value": M * r32["nterms"] * args.steps / (r32["ms_fwd"] * 1e-3), "unit": "node-terms/s",
                    "ms": r32["ms_fwd"] / args.steps},
        "adjoint": {"value": M * r32["nterms"] * args.steps / (r32["ms_adj"] * 1e-3), "unit": "node-terms/s",
                    "ms": r32["ms_adj"] / args.steps},
    }
    # dominant kernel and its roofline
    kern = r32["kernels"]
    if kern:
        name, (count, total) = max(kern.items(), key=lambda kv: kv[1][1])
        avg_s = total / count * 1e-3
        # a shared launch of orders 1 and 2 ("..._12") counts both orders' work
        orders = [1, 2] if name.endswith("_12") else [2 if "2d" in name else (1 if "1d" in name else 3)]
        nterms_of = {1: D, 2: D * (D - 1) // 2, 3: D * (D - 1) * (D - 2) // 6}
        fl = M * sum(nterms_of[o] * flops_per_node_term(o, M_WIN) for o in orders)
        achieved = fl / avg_s / 1e12
        traffic = None
        tf = os.path.join(ROOT, "profiles", "traffic.json")
        hbm = {}
        if os.path.exists(tf):
            with open(tf) as fh:
                tj = json.load(fh)
            khash = kernel_hash()
            traffic = counted_bytes(tj, name, r32["tuning"], khash)
            # every kernel's HBM rate from the counted bytes (when taken with these sources)
            for k, (cnt, tot) in kern.items():
                b = counted_bytes(tj, k, r32["tuning"], khash)
                if b is not None and cnt > 0 and tot > 0:
                    gbs = b / (tot / cnt * 1e-3) / 1e9
                    hbm[k] = {"bytes_per_launch": b, "GB/s": gbs, "frac": gbs / PEAK_HBM_GBS}
        out["roofline"] = {"bound": "alu", "kernel": name, "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
                           "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
                           "avg_launch_us": avg_s * 1e6, "flops_per_launch": fl}
        out["kernels_ms"] = {k: {"launches": v[0], "avg_us": v[1] / v[0] * 1e3} for k, v in sorted(kern.items())}
        if traffic is not None:
            out["roofline"]["traffic_GB/s"] = traffic / avg_s / 1e9
            out["roofline"]["traffic_frac_of_hbm_peak"] = traffic / avg_s / 1e9 / PEAK_HBM_GBS
        out["kernels_hbm"] = hbm or None   # counted HBM bytes per launch / launch time, per kernel
        out["roofline"]["timing"] = ("per-launch HIP events over a second pass of the same steps, launched eagerly on one "
                                     "stream (the timed pass uses the tuned launch forms: graph replay and the "
                                     "order-1 kernels on a second stream where the tuning chose them)")
        out["eager_ms_per_step"] = r32["ms_eager"] / args.steps
    if not args.no_fp64:
        print("[bench] fp64", file=sys.stderr, flush=True)
        r64 = run_gpu("f64", args.steps, args.warmup, profile=False)
        out["fp64"] = {"value": node_terms * args.steps / (r64["ms"] * 1e-3), "unit": "node-terms/s",
                       "ms_per_step": r64["ms"] / args.steps, "forward_ms": r64["ms_fwd"] / args.steps,
                       "adjoint_ms": r64["ms_adj"] / args.steps, "tuning": r64["tuning"]}
    if not args.no_solvers and not args.autograd_only:
        print("[bench] solvers", file=sys.stderr, flush=True)
        out["solvers"] = run_solvers()
        print("[bench] active set", file=sys.stderr, flush=True)
        out["active_set"] = run_active_set()
        print("[bench] test function", file=sys.stderr, flush=True)
        runs = [run_testfun(k) for k in range(max(1, args.draws))]
        fruns = [run_testfun_fista(k) for k in range(max(1, args.draws))]
        out["testfun"], out["testfun_fista"] = runs[0], fruns[0]
        if args.draws > 1:
            exps = ("i", "ii", "iii", "iv")
            out["testfun"]["mean_over_draws"] = {
                e: {"draws": len(runs), "best_l2_error": float(np.mean([min(r[e]["l2_error"].values()) for r in runs])),
                    "l2_error_refit": float(np.mean([r[e]["l2_error_refit"] for r in runs])),
                    "active_set_is_printed_U*": sum(r[e]["active_set_is_printed_U*"] for r in runs)} for e in exps}
            out["testfun_fista"]["mean_over_draws"] = {
                e: {"draws": len(fruns), "best_l2_error": float(np.mean([r[e]["best_l2_error"] for r in fruns])),
                    "active_set_is_printed_U*": sum(r[e]["active_set_is_printed_U*"] for r in fruns)} for e in exps}
    if not args.no_solvers or args.autograd_only:
        print("[bench] autograd", file=sys.stderr, flush=True)
        out["autograd"] = run_autograd()
    if not args.no_solvers and not args.autograd_only:
        print("[bench] cosine basis", file=sys.stderr, flush=True)
        out["cosine"] = run_cosine(max(5, args.steps // 2))
    if not args.no_c3:
        print("[bench] batched-lsqr workload (d=20)", file=sys.stderr, flush=True)
        out["batched_lsqr_d20"] = run_c3(args.c3_steps, args.c3_all_lambdas, args.c3_transform_only, args.c3_forms)
    if args.cpu_sample > 0:
        print(f"[bench] cpu oracle sample {args.cpu_sample}", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
