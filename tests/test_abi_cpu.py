"""C-ABI library checks that need no GPU: it loads, exports every declared symbol, and its
host-side index-set functions agree with the oracle and the printed counts."""
import os
import re

import numpy as np
import pytest

from oracle import index_set as oidx
from paper_2010_10199_amd import lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "grouped.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)) - {"if", "sizeof"})


def test_library_loads_and_exports_every_declared_symbol():
    L = lib.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), f"missing export {name}"
    assert sorted(lib.EXPORTS) == names


def test_num_terms_and_coeffs_match_printed_counts():
    assert lib.gt_num_coeffs(9, 3, [26, 6, 4]) == 3394
    assert lib.gt_num_coeffs(9, 3, [352, 20, 8]) == 44968
    assert lib.gt_num_coeffs(12, 2, [82, 10]) == 6319
    assert lib.gt_num_terms(12, 2) == 79


@pytest.mark.parametrize("d,ds,N", [(1, 1, [4]), (4, 3, [6, 4, 4]), (6, 2, [16, 8]), (20, 3, [32, 12, 6]), (5, 0, [])])
def test_term_table_matches_oracle_ordering(d, ds, N):
    coords, offs = lib.gt_term_table(d, ds, N)
    iset = oidx.grouped_index_set(d, ds, N)
    assert np.array_equal(offs, iset.offsets)
    for row, u in zip(coords, iset.terms):
        assert tuple(int(v) for v in row if v >= 0) == u
    assert lib.gt_num_coeffs(d, ds, N) == iset.n_coeffs == oidx.count_coeffs(d, ds, N)


def test_invalid_index_arguments():
    assert lib.gt_num_terms(0, 0) == -1
    assert lib.gt_num_terms(3, 4) == -1
    assert lib.gt_num_coeffs(3, 2, [7, 4]) == -1
    with pytest.raises(lib.GroupedError) as e:
        lib.gt_term_table(6, 4, [8, 6, 4, 4])
    assert e.value.code == lib.GT_EUNSUPPORTED


@pytest.mark.parametrize("d,ds,N,seed", [(4, 3, [6, 4, 4], 1), (7, 2, [16, 8], 2), (20, 3, [32, 12, 6], 3)])
def test_masked_index_set_matches_oracle(d, ds, N, seed):
    """A term mask (the empty set's flag cleared: it stays anyway) gives the oracle's
    subset index set: sizes, coordinates and coefficient offsets."""
    nt = lib.gt_num_terms(d, ds)
    mask = (np.random.default_rng(seed).random(nt) < 0.5).astype(np.uint8)
    mask[0] = 0
    p, keep = lib.make_problem(d, ds, N, M=1, term_mask=mask)
    sub = oidx.grouped_index_set(d, ds, N, keep=mask)
    assert lib.problem_size(p) == (sub.n_terms, sub.n_coeffs)
    coords, offs = lib.gt_term_table(d, ds, N, term_mask=mask)
    want = np.array([list(u) + [-1] * (3 - len(u)) for u in sub.terms], dtype=np.int32)
    assert np.array_equal(coords, want)
    assert np.array_equal(offs, sub.offsets)


@pytest.mark.parametrize("masked", [False, True])
def test_active_set_matches_oracle(masked):
    """gt_active_set against the oracle's rule (eq. activeset) on random indices, with and
    without a term mask on the problem the indices belong to."""
    from oracle import sensitivity as osens
    d, ds, N = 6, 3, [8, 6, 4]
    g = np.random.default_rng(7)
    nt = lib.gt_num_terms(d, ds)
    mask = (g.random(nt) < 0.6).astype(np.uint8) if masked else None
    p, keep = lib.make_problem(d, ds, N, M=1, term_mask=mask)
    sub = oidx.grouped_index_set(d, ds, N, keep=mask)
    rho = g.random(sub.n_terms) * 0.2
    rho[0] = 0.0
    eps = [0.1, 0.05, 0.15]
    got, na = lib.active_set(p, rho, eps)
    want = osens.active_set(sub, rho, eps)
    assert np.array_equal(got, want)
    assert na == int(want.sum())


def test_allocation_failure_hook_and_plan_handles_on_cpu():
    """Error paths that need no GPU: an armed allocation-failure hook turns the first device
    allocation of a plan into GT_ENOMEM before anything reaches the device; a handle that is
    not a live plan is rejected without being dereferenced; releasing everything with no live
    plans is a no-op."""
    import ctypes as C
    import numpy as np
    L = lib.load()
    x = np.zeros((4, 3))
    p, keep = lib.make_problem(3, 2, [4, 4], M=4, dtype=lib.GT_C128)
    h = C.c_void_p()
    lib.debug_fail_alloc(1)
    try:
        rc = L.gt_plan_create(C.byref(p), x.ctypes.data, None, C.byref(h))
        assert rc == lib.GT_ENOMEM and h.value is None
        assert "allocation" in L.gt_last_error().decode()
        assert lib.debug_alloc_count() == 1
    finally:
        lib.debug_fail_alloc(0)
    with pytest.raises(lib.GroupedError) as e:
        lib.debug_fail_alloc(-1)
    assert e.value.code == lib.GT_EINVAL
    bogus = C.c_void_p(0x1000)       # never a plan; must not be dereferenced
    assert L.gt_plan_destroy(bogus) == lib.GT_EINVAL
    assert L.gt_plan_trafo(bogus, None, None, None) == lib.GT_EINVAL
    assert L.gt_plan_tune(bogus, None) == lib.GT_EINVAL
    assert L.gt_plan_tuning(bogus, None, 0) == lib.GT_EINVAL
    assert L.gt_plan_set_graph(bogus, 1) == lib.GT_EINVAL
    assert L.gt_plan_set_fused(bogus, 1) == lib.GT_EINVAL
    assert L.gt_plan_set_gather_path(bogus, 1, lib.GT_GATHER_SORTED) == lib.GT_EINVAL
    assert L.gt_plan_destroy(None) == lib.GT_OK
    assert L.gt_release_all() == lib.GT_OK
    pb, keepb = lib.make_problem(3, 2, [4, 4], M=4, dtype=lib.GT_C128, basis=7)
    assert L.gt_plan_create(C.byref(pb), x.ctypes.data, None, C.byref(h)) == lib.GT_EINVAL
    assert "basis" in L.gt_last_error().decode()
