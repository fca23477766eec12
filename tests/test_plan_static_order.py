"""The symbolic plan (nested-dissection order, supernodes, front maps, selected-block
owners) checked on the CPU: the selected-inversion recurrences (Sec. 3), run through the
plan's fronts with LAPACK per front, reproduce the selected blocks of the dense inverse."""
import numpy as np
import pytest

import oracle
from paper_1707_08874_amd.inputs import gen_links
from parity import block_errors
from static_pivoting_floor import static_order_selected


@pytest.mark.parametrize("dims,kw", [
    ((4, 4, 4, 4), {}),                                   # default plan
    ((4, 4, 4, 4), dict(max_pivot_rows=48)),              # separators split into chains
    ((4, 6, 4, 4), dict(leaf_sites=12)),                  # larger leaves, non-cubic
])
def test_plan_fronts_give_the_selected_inverse(dims, kw):
    U = gen_links(dims, 3, 0.1)
    sel, D = static_order_selected(U, dims, 0.05, 0.25, **kw)
    ref = oracle.selected_blocks(oracle.inverse_dense(D), dims)
    # rounding gives ~1e-11 here; a wrong order, front map or block owner gives O(1)
    assert block_errors(sel, ref).max() < 1e-10
