"""CPU checks of the leaf-set comparison the GPU parity tests use: a differing leaf is
excused only by a near-tie node that contains it, and the rest of the field is still
compared.  Runs the oracle twice on a small grid and edits one run's leaf set."""
import numpy as np
import pytest

import oracle
import workloads
from parity_util import compare_adaptive, excused_cells


def _run():
    W = workloads.field3d_trig(0, m=60, npts=17)
    W.min_leaf = 1
    M = oracle.fit(W)
    leaves, skipped, recs = oracle.adaptive(M, W)
    return W, M, leaves, skipped, recs


def _subtree(keys, node, dim):
    lk, ln = keys >> np.uint64(58), node >> 58
    shift = (lk.astype(np.int64) - ln) * dim
    return ((keys & np.uint64((1 << 58) - 1)) >> shift.astype(np.uint64)) == np.uint64(node & ((1 << 58) - 1))


def test_difference_below_a_tie_node_is_excused_and_only_its_cells():
    W, M, leaves, skipped, recs = _run()
    refined = recs[(recs["subdivide"] == 1) & (recs["level"] == 2)]
    assert len(refined) >= 2
    node = int(refined["key"][0])
    other = int(refined["key"][1])
    drop = _subtree(leaves, node, 3)
    assert drop.any()
    got = leaves[~drop]
    sym = set(map(int, got)) ^ set(map(int, leaves))
    mask = excused_cells(W, sym, {node})
    inside = oracle.level_field(W, np.array([node], np.uint64)).reshape(-1) != 255
    assert np.array_equal(mask, inside)
    # a near-tie elsewhere at the same level does not excuse the difference
    with pytest.raises(AssertionError):
        excused_cells(W, sym, {other})
    # the field outside the excused node is compared: an edit there is caught
    out = oracle.lcp_leaves(M, W, got).reshape(-1)
    lev = oracle.level_field(W, np.concatenate([got, skipped])).reshape(-1)
    compare_adaptive(W, M, out, got, lev, leaves, skipped, {node})
    bad = out.copy()
    j = int(np.flatnonzero(~inside & (out > 0))[0])
    bad[j] += 1.0 / W.n_samples
    with pytest.raises(AssertionError):
        compare_adaptive(W, M, bad, got, lev, leaves, skipped, {node})
