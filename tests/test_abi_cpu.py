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
