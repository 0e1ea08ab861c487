"""Pins of the oracle's K-D tree variant of Alg. 1 (Sec. 9: split the axes in turn instead
of all at once).  CPU only.

  * every D-th depth is an octree level: nodes at depth D l are the octree nodes of level l
    (same code, same box), so their region tests agree bit for bit with the octree run;
  * each child halves its parent along the axis of its depth (z, y, x in turn), and a node
    is refined exactly when Alg. 1's rules say so;
  * leaves and skipped nodes tile the cell grid once; the field inside the leaves equals
    the dense field; the level field reports each cell's depth;
  * with the certified bound, no skipped node holds a cell whose smooth LCP exceeds alpha.
"""
import numpy as np
import pytest

import oracle
import workloads
from test_oracle_pins import small

MASK = (1 << 58) - 1


def _decode(key, D):
    L, code = key >> 58, key & MASK
    c = [0, 0, 0]
    for j in range(L):
        a = D - 1 - j % D
        c[a] = 2 * c[a] + ((code >> (L - 1 - j)) & 1)
    return L, c


def _box(key, D, S0, nc):
    L, c = _decode(key, D)
    lo, hi = [0, 0, 0], [1, 1, 1]
    for d in range(D):
        s = S0 >> (L // D + (1 if d >= D - L % D else 0))
        lo[d], hi[d] = c[d] * s, min((c[d] + 1) * s, nc[d])
    return L, lo, hi


def _cases():
    W1 = workloads.field3d_trig(0, m=120, npts=33)
    W2 = small(170, 3, 15, 9, ell=0.3, signal_var=0.05, noise_var=1e-4, min_leaf=1)
    W2.npts[:] = [9, 7, 6]
    W3 = workloads.make("cfg1_2d")
    W3.min_leaf = 2
    return [W1, W2, W3]


@pytest.mark.parametrize("case", range(3))
def test_kd_depths_multiple_of_dim_are_octree_levels(case):
    W = _cases()[case]
    M = oracle.fit(W)
    _, _, ro = oracle.adaptive(M, W)
    _, _, rk = oracle.adaptive(M, W, split=oracle.SPLIT_KD)
    D = W.dim
    octree = {(int(r["level"]), int(r["key"]) & MASK): r for r in ro}
    n = 0
    for r in rk:
        L = int(r["level"])
        if L % D:
            continue
        o = octree.get((L // D, int(r["key"]) & MASK))
        if o is None:
            continue
        n += 1
        for f in ("n_obs", "path", "subdivide", "d"):
            assert o[f] == r[f], (f, hex(int(r["key"])))
        for f in ("p1", "p2", "gmin", "ub"):
            assert (np.isnan(o[f]) and np.isnan(r[f])) or o[f] == r[f], (f, hex(int(r["key"])))
    assert n > 10


@pytest.mark.parametrize("case", range(3))
def test_kd_children_halve_the_split_axis_and_follow_alg1(case):
    W = _cases()[case]
    M = oracle.fit(W)
    _, _, rk = oracle.adaptive(M, W, split=oracle.SPLIT_KD)
    D = W.dim
    S0, Lmax = oracle.octree_shape(W)
    nc = [int(W.npts[d]) - 1 for d in range(D)] + [1] * (3 - D)
    recs = {int(r["key"]): r for r in rk}
    for key, r in recs.items():
        L, lo, hi = _box(key, D, S0, nc)
        assert r["d"] == np.prod([hi[d] - lo[d] + 1 for d in range(D)])
        # Alg. 1: refined iff both sides are above alpha, or the bound exceeds alpha
        if r["path"] == 0:
            assert r["subdivide"] == 1
        elif r["path"] == 3:
            assert L == D * Lmax and r["subdivide"] == 1
        else:
            assert r["subdivide"] == (r["ub"] > W.alpha)
        if L == 0:
            continue
        pkey = ((L - 1) << 58) | ((key & MASK) >> 1)
        assert pkey in recs and recs[pkey]["subdivide"] == 1
        _, plo, phi = _box(pkey, D, S0, nc)
        a = D - 1 - (L - 1) % D
        for d in range(D):
            if d != a:
                assert (lo[d], hi[d]) == (plo[d], phi[d])
        half = (S0 >> (L // D + (1 if a >= D - L % D else 0)))
        assert lo[a] in (plo[a], plo[a] + half) and hi[a] <= phi[a]


@pytest.mark.parametrize("case", range(3))
def test_kd_tiles_the_grid_and_matches_dense_in_leaves(case):
    W = _cases()[case]
    M = oracle.fit(W)
    leaves, skipped, _ = oracle.adaptive(M, W, split=oracle.SPLIT_KD)
    D = W.dim
    S0, Lmax = oracle.octree_shape(W)
    nc = [int(W.npts[d]) - 1 for d in range(D)] + [1] * (3 - D)
    cover = np.zeros(nc[::-1], np.int32)
    for key in list(map(int, oracle.kd_leaf_keys(W, leaves))) + list(map(int, skipped)):
        _, lo, hi = _box(key, D, S0, nc)
        cover[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += 1
    assert np.all(cover == 1)
    assert np.all(leaves >> np.uint64(58) == Lmax)
    dense = oracle.lcp_dense(M, W).reshape(-1)
    got = oracle.lcp_leaves(M, W, leaves).reshape(-1)
    lev = oracle.level_field_kd(W, np.concatenate([oracle.kd_leaf_keys(W, leaves), skipped])).reshape(-1)
    inleaf = oracle.level_field_kd(W, oracle.kd_leaf_keys(W, leaves)).reshape(-1) != 255
    assert np.array_equal(got[inleaf], dense[inleaf]) and np.all(got[~inleaf] == 0)
    assert np.all(lev != 255) and np.all(lev[inleaf] == D * Lmax)


def test_kd_leaves_equal_octree_leaves_with_every_node_refined():
    """alpha below every bound: both trees refine everything down to the same finest nodes."""
    W = small(171, 3, 12, 9, ell=0.3, signal_var=0.5, noise_var=1e-3, min_leaf=2)
    M = oracle.fit(W)
    lo, _, _ = oracle.adaptive(M, W, alpha=1e-300)
    lk, sk, _ = oracle.adaptive(M, W, alpha=1e-300, split=oracle.SPLIT_KD)
    assert len(sk) == 0 and np.array_equal(lo, lk) and len(lo) == 64


def test_kd_certified_skips_only_safe_nodes():
    W = small(172, 3, 15, 17, kind=workloads.SE, ell=0.4, signal_var=0.05, noise_var=1e-3, min_leaf=2)
    W.zbank = np.random.default_rng(173).standard_normal((3000, 8))
    M = oracle.fit(W)
    W.theta = float(np.quantile(oracle.grid_posterior(M, W)[0], 0.95))
    leaves, skipped, _ = oracle.adaptive(M, W, bound_kind=oracle.BOUND_CERTIFIED, split=oracle.SPLIT_KD)
    S0, _ = oracle.octree_shape(W)
    lcp = oracle.lcp_sov_dense(M, W)
    n = 0
    for key in map(int, skipped):
        _, lo, hi = _box(key, 3, S0, [16, 16, 16])
        sl = lcp[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        n += sl.size
        if sl.size:
            assert sl.max() <= W.alpha + 5e-4
    assert n > 100
