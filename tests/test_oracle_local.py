"""Pins of the oracle's local model M' of Sec. 5.2, used by the region test of Alg. 1 when
lcp_adapt.bound_kind = BOUND_LOCAL.  CPU only.

  * selection: M' holds exactly the points inside the closed node box enlarged by beta
    lengthscales per axis (brute force, including points on the enlarged faces); the root
    keeps every point;
  * exact GP: the local posterior is the GP conditioned on the selected observations alone,
    written here with numpy's dense solve;
  * sparse model: eq. (sgp) with mu_M and A_M restricted to M' (numpy, dense solves);
  * with every point selected, the local model is the model itself bit for bit, and so is
    the whole octree run; with two clusters whose cross-covariances underflow to zero the
    local model of one cluster equals the full model there bit for bit;
  * an empty M' gives the prior.
"""
import numpy as np
import pytest

import oracle
import workloads
from test_oracle_pins import small


def _se(A, B, s2, ell):
    d = (A[:, None, :] - B[None, :, :]) / ell
    return s2 * np.exp(-0.5 * (d * d).sum(-1))


def _select(X, blo, bhi, beta, ell):
    r = beta * np.asarray(ell)[: X.shape[1]]
    return np.all((X >= np.asarray(blo) - r) & (X <= np.asarray(bhi) + r), axis=1)


def test_local_exact_gp_conditions_on_the_selected_observations():
    W = small(180, 3, 60, 5, ell=0.15, signal_var=0.4, noise_var=1e-3)
    M = oracle.fit(W)
    ell = W.lengthscale[:3]
    rng = np.random.default_rng(181)
    for beta in (0.5, 1.0, 2.0):
        blo = rng.random(3) * 0.6
        bhi = blo + 0.2
        P = blo + (bhi - blo) * rng.random((17, 3))
        mean, var, ml = oracle.local_posterior(M, blo, bhi, beta, P)
        sel = _select(W.X, blo, bhi, beta, ell)
        assert ml == sel.sum() and 0 < ml < W.m
        Xs, ys = W.X[sel], W.y[sel]
        K = _se(Xs, Xs, W.signal_var, ell) + W.noise_var * np.eye(ml)
        ks = _se(P, Xs, W.signal_var, ell)
        ref_mean = ks @ np.linalg.solve(K, ys)
        ref_var = W.signal_var - np.einsum("ij,ji->i", ks, np.linalg.solve(K, ks.T))
        assert np.allclose(mean, ref_mean, rtol=1e-9, atol=1e-12 * np.abs(ys).max())
        assert np.allclose(var, ref_var, rtol=1e-8, atol=1e-12 * W.signal_var)


def test_local_sparse_restricts_mu_and_A():
    W = workloads.sgpr_field(182, m=64, npts=9, train_npts=8, ell=0.25)
    M = oracle.fit(W)
    ell = W.lengthscale
    blo, bhi = np.array([0.3, 0.2, 0.4]), np.array([0.55, 0.45, 0.65])
    P = blo + (bhi - blo) * np.random.default_rng(183).random((11, 3))
    mean, var, ml = oracle.local_posterior(M, blo, bhi, 0.6, P)
    sel = _select(W.X, blo, bhi, 0.6, ell)
    assert ml == sel.sum() and 0 < ml < W.m
    Z, mu, A = W.X[sel], W.y[sel], W.A_M[np.ix_(sel, sel)]
    K = _se(Z, Z, W.signal_var, ell) + W.noise_var * np.eye(ml)
    ks = _se(P, Z, W.signal_var, ell)
    Wt = np.linalg.solve(K, ks.T)                       # K_M'M'^-1 K_M'I
    ref_mean = Wt.T @ mu
    ref_var = W.signal_var - np.einsum("ij,ji->i", ks, Wt) + np.einsum("ji,jk,ki->i", Wt, A, Wt)
    assert np.allclose(mean, ref_mean, rtol=1e-8, atol=1e-10 * np.abs(mu).max())
    assert np.allclose(var, ref_var, rtol=1e-6, atol=1e-9 * W.signal_var)


def test_local_selection_is_the_closed_enlarged_box():
    W = small(184, 3, 8, 5, ell=0.125, signal_var=0.3, noise_var=1e-3)
    # node box [0.25, 0.5]^3, beta 2 -> enlarged box [0, 0.75]^3 (exact in binary64)
    W.lengthscale[:] = 0.125
    X = np.array([[0.0, 0.3, 0.3], [0.75, 0.75, 0.75], [0.3, 0.3, 0.7500000000000001],
                  [-1e-17, 0.3, 0.3], [0.4, 0.4, 0.4], [0.9, 0.1, 0.1], [0.5, 0.0, 0.75], [0.2, 0.8, 0.3]])
    W.X = X
    M = oracle.fit(W)
    _, _, ml = oracle.local_posterior(M, [0.25] * 3, [0.5] * 3, 2.0, np.array([[0.3, 0.3, 0.3]]))
    assert ml == 4          # rows 0, 1 and 6 lie on enlarged faces, row 4 inside; 2, 3 are one ulp out
    inside = _select(X, [0.25] * 3, [0.5] * 3, 2.0, W.lengthscale)
    assert ml == inside.sum()
    _, _, mw = oracle.local_posterior(M, [0.25] * 3, [0.5] * 3, 2.0, np.array([[0.3, 0.3, 0.3]]), whole=True)
    assert mw == W.m


def test_local_with_every_point_is_the_model_bit_for_bit():
    W = small(185, 3, 40, 5, kind=workloads.MATERN52, ell=0.2, signal_var=0.5, noise_var=1e-3)
    M = oracle.fit(W)
    P = np.random.default_rng(186).random((23, 3))
    m0, v0 = oracle.posterior(M, P)
    m1, v1, ml = oracle.local_posterior(M, [0.4] * 3, [0.6] * 3, 1e3, P)
    assert ml == W.m and np.array_equal(m0, m1) and np.array_equal(v0, v1)
    Ws = workloads.sgpr_field(187, m=27, npts=9, train_npts=6, ell=0.3)
    Ms = oracle.fit(Ws)
    m0, v0 = oracle.posterior(Ms, P)
    m1, v1, ml = oracle.local_posterior(Ms, [0.4] * 3, [0.6] * 3, 0.0, P, whole=True)
    assert ml == Ws.m and np.array_equal(m0, m1) and np.array_equal(v0, v1)


def test_local_of_an_isolated_cluster_equals_the_model_there():
    """SE covariances at 40+ lengthscales underflow to zero: K is block diagonal and the
    full model near the first cluster only sums exact zeros from the second."""
    rng = np.random.default_rng(188)
    W = small(188, 3, 30, 5, ell=0.01, signal_var=0.2, noise_var=1e-3)
    W.lengthscale[:] = 0.01
    X = np.concatenate([0.1 + 0.05 * rng.random((15, 3)), 0.85 + 0.05 * rng.random((15, 3))])
    W.X = X
    W.y = rng.standard_normal(30) * 0.3
    M = oracle.fit(W)
    blo, bhi = np.array([0.1] * 3), np.array([0.15] * 3)
    P = blo + (bhi - blo) * rng.random((9, 3))
    m0, v0 = oracle.posterior(M, P)
    m1, v1, ml = oracle.local_posterior(M, blo, bhi, 6.0, P)
    assert ml == 15
    assert np.array_equal(m0, m1) and np.array_equal(v0, v1)


def test_local_empty_set_gives_the_prior():
    W = small(189, 2, 10, 5, ell=0.05, signal_var=0.7, noise_var=1e-3)
    W.X = 0.1 * np.random.default_rng(189).random((10, 2))
    M = oracle.fit(W)
    mean, var, ml = oracle.local_posterior(M, [0.8, 0.8], [0.9, 0.9], 2.0, np.array([[0.85, 0.85], [0.8, 0.9]]))
    assert ml == 0 and np.all(mean == 0.0) and np.all(var == W.signal_var)


@pytest.mark.parametrize("split", [oracle.SPLIT_OCTREE, oracle.SPLIT_KD])
def test_octree_local_with_huge_beta_is_the_search(split):
    W = workloads.field3d_trig(0, m=120, npts=33)
    M = oracle.fit(W)
    l0, s0, r0 = oracle.adaptive(M, W, split=split)
    l1, s1, r1 = oracle.adaptive(M, W, bound_kind=oracle.BOUND_LOCAL, beta=1e6, split=split)
    assert np.array_equal(l0, l1) and np.array_equal(s0, s1)
    for f in ("gmin", "ub", "lattice_gap"):
        assert np.array_equal(r0[f], r1[f], equal_nan=True), f
    tested = r1["n_local"] >= 0
    assert tested.any() and np.all(r1["n_local"][tested] == W.m)
    assert np.array_equal(tested, np.isfinite(r0["ub"]))


@pytest.mark.parametrize("beta", [1.0, 2.5])
def test_octree_local_records_count_the_enlarged_box(beta):
    W = workloads.field3d_trig(1, m=150, npts=29)
    W.npts[:] = [29, 23, 19]
    M = oracle.fit(W)
    _, _, recs = oracle.adaptive(M, W, bound_kind=oracle.BOUND_LOCAL, beta=beta)
    S0, _ = oracle.octree_shape(W)
    nc = W.npts - 1
    h = (W.hi - W.lo) / nc
    n = 0
    for r in recs:
        if r["n_local"] < 0:
            continue
        L, code = int(r["level"]), int(r["key"]) & ((1 << 58) - 1)
        c = [0, 0, 0]
        for j in range(L):
            for d in range(3):
                c[d] |= ((code >> (3 * j + d)) & 1) << j
        s = S0 >> L
        lo = np.array([c[d] * s for d in range(3)])
        hi = np.minimum(lo + s, nc)
        blo, bhi = W.lo + lo * h, W.lo + hi * h
        want = W.m if L == 0 else int(_select(W.X, blo, bhi, beta, W.lengthscale).sum())
        assert r["n_local"] == want, (hex(int(r["key"])), r["n_local"], want)
        n += 1
    assert n > 20


def test_local_factor_failure_refines_the_node():
    """R14 / Alg. 1: a node whose local model cannot be factored has no bound and must be
    refined (a skipped node would need a bound).  Two identical observations make every
    local K' that holds both singular once the local fit runs without noise; the stored
    full factor is the one with noise, so the preliminary test and the rest of the tree are
    unchanged.  Every record that reached the region test with a failed local fit (no
    |M'| recorded) must carry g_min = -inf, UB = 1 and be subdivided, and exactly those
    records are the ones whose enlarged box holds the duplicated point."""
    W = small(190, 3, 30, 9, signal_var=0.05, ell=0.2, noise_var=1e-4, min_leaf=1)
    W.X[1] = W.X[0]
    W.y[0] = W.y[1] = W.theta + 3.0
    M = oracle.fit(W)
    M.s.noise = 0.0                 # local fits only: K' + 0 I is singular with both copies
    beta = 0.5
    leaves, skipped, recs = oracle.adaptive(M, W, bound_kind=oracle.BOUND_LOCAL, beta=beta)
    S0, L = oracle.octree_shape(W)
    tested = recs[np.isin(recs["path"], [1, 2])]
    failed = tested[tested["n_local"] == -1]
    assert len(failed) >= 5
    assert (failed["subdivide"] == 1).all() and (failed["ub"] == 1.0).all()
    assert np.isneginf(failed["gmin"]).all()
    ell = W.lengthscale[:3]
    for r in tested:
        lvl = int(r["level"])
        mc = int(r["key"]) & ((1 << 58) - 1)
        c = [sum(((mc >> (b * 3 + d)) & 1) << b for b in range(lvl)) for d in range(3)]
        s = S0 >> lvl
        lo = np.array([c[d] * s for d in range(3)])
        hi = np.minimum(lo + s, W.npts[:3] - 1)
        h = 1.0 / (W.npts[0] - 1)
        dup = _select(W.X[:1], lo * h, hi * h, beta, ell)[0] or lvl == 0
        assert dup == (r["n_local"] == -1), (lvl, c)
