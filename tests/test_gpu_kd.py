"""Parity of the K-D tree variant of the adaptive query (lcp_adapt.split = LCP_SPLIT_KD,
Sec. 9) with the FP64 oracle: leaf sets (exact, except below nodes the oracle flags as
near-ties), Monte Carlo counts inside the leaves (exact in binary64) and the depth field.
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2512_12442_amd as lcp
from parity_util import compare_adaptive, counts, gpu_model, near_tie_keys, say, zbank

pytestmark = pytest.mark.gpu


def _cases():
    W1 = workloads.field3d_trig(0, m=120, npts=33)
    W2 = workloads.field3d_trig(3, m=150, npts=29)
    W2.npts[:] = [29, 23, 19]
    W2.min_leaf = 2
    W3 = workloads.make("cfg1_2d")
    W3.min_leaf = 2
    W4 = workloads.sgpr_field(154, m=64, npts=17, train_npts=10, ell=0.25)
    W4.min_leaf = 1
    return {"trig33": W1, "ragged": W2, "cfg1_2d": W3, "sgpr17_leaf1": W4}


@pytest.mark.parametrize("case,bound", [("trig33", 0), ("ragged", 0), ("cfg1_2d", 0), ("sgpr17_leaf1", 0),
                                        ("trig33", 1), ("ragged", 1)])
def test_adaptive_kd_matches_oracle(case, bound):
    W = _cases()[case]
    say(f"adaptive K-D {case} bound={bound} npts={W.npts} m={W.m} min_leaf={W.min_leaf}")
    M = oracle.fit(W)
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, bound_kind=bound, split=oracle.SPLIT_KD)
    G = gpu_model(W)
    A = lcp.adapt_of(W, bound_kind=bound, split=lcp.SPLIT_KD)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, A, zbank(W), "fp64")
    n = int(nl.item())
    got = leaves[:n].cpu().numpy().astype(np.uint64)
    ties = near_tie_keys(recs, W.alpha) if bound == 0 else {
        int(r["key"]) for r in recs if np.isfinite(r["ub"]) and abs(r["ub"] - W.alpha) <= 1e-6 * W.alpha}
    assert np.all(np.diff(got.astype(np.int64)) > 0)
    _, Lmax = oracle.octree_shape(W)
    sym, excused = compare_adaptive(W, M, out.cpu().numpy(), got, lf.cpu().numpy(), leaves_ref, skipped_ref, ties,
                                    split=1)
    say(f"  leaves gpu={n} oracle={len(leaves_ref)} skipped={len(skipped_ref)} differ={len(sym)} "
        f"near-ties={len(ties)} excused cells={int(excused.sum())}")
    assert lf.cpu().numpy().max() <= W.dim * Lmax


def test_kd_and_octree_agree_where_the_oracle_says_so():
    """On the trig field the two trees emit the same leaves (the oracle shows it); the GPU
    runs must then agree with each other and equal the dense field inside the leaves."""
    W = _cases()["trig33"]
    M = oracle.fit(W)
    lo, _, _ = oracle.adaptive(M, W)
    lk, _, _ = oracle.adaptive(M, W, split=oracle.SPLIT_KD)
    assert np.array_equal(lo, lk)
    G = gpu_model(W)
    grid = lcp.grid_of(W)
    a_oct = G.lcp_adaptive(grid, W.theta, lcp.adapt_of(W), zbank(W), "f16x3")
    a_kd = G.lcp_adaptive(grid, W.theta, lcp.adapt_of(W, split=lcp.SPLIT_KD), zbank(W), "f16x3")
    no, nk = int(a_oct[2].item()), int(a_kd[2].item())
    assert no == nk and np.array_equal(a_oct[1][:no].cpu().numpy(), a_kd[1][:nk].cpu().numpy())
    assert np.array_equal(a_oct[0].cpu().numpy(), a_kd[0].cpu().numpy())


def test_kd_level_outside_the_field_emits_nothing():
    """The K-D tree with a level far above every posterior value: the root's bound is far
    below alpha, so the tree stops at its root with no leaf and a zero field, as the
    oracle's K-D variant of Alg. 1 gives."""
    W = workloads.random_small(8, 3, 40, 24, signal_var=0.3, ell=0.3, min_leaf=2)
    W.theta = float(W.y.max() + 10.0)
    say(f"K-D tree, level outside the field: theta={W.theta:.3f}")
    M = oracle.fit(W)
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, split=oracle.SPLIT_KD)
    assert len(leaves_ref) == 0
    G = gpu_model(W)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, lcp.adapt_of(W, split=lcp.SPLIT_KD), zbank(W),
                                            "fp64")
    assert int(nl.item()) == 0
    assert float(out.abs().sum()) == 0.0
    sym, _ = compare_adaptive(W, M, out.cpu().numpy(), np.zeros(0, np.uint64), lf.cpu().numpy(), leaves_ref,
                              skipped_ref, near_tie_keys(recs, W.alpha), split=1)
    assert len(sym) == 0
