"""Pins of the FP64 oracle against values fixed by the paper, by mathematics or by
independent library routines (never by the oracle itself or by the GPU path).

Each test names the passage of the paper it checks.  CPU only.
"""
import os

import numpy as np
import pytest
from scipy import linalg as sla
from scipy import stats
from sklearn.gaussian_process import GaussianProcessRegressor
from sklearn.gaussian_process.kernels import RBF, ConstantKernel, Matern

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def sk_kernel(W):
    """The same covariance, built from scikit-learn's own kernel implementations."""
    ell = W.lengthscale[: W.dim]
    base = RBF(ell, "fixed") if W.kind == workloads.SE else Matern(ell, "fixed", nu=2.5)
    return ConstantKernel(W.signal_var, "fixed") * base


def sk_gpr(W):
    g = GaussianProcessRegressor(sk_kernel(W), alpha=W.noise_var, optimizer=None, normalize_y=False)
    return g.fit(W.X, W.y)


def small(seed=0, dim=3, m=12, npts=5, kind=workloads.SE, **kw):
    return workloads.random_small(seed, dim, m, npts, kind=kind, **kw)


# ---------------------------------------------------------------- kernels (Sec. 3)

@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_matches_sklearn(kind, dim):
    W = small(1, dim, 6, 4, kind=kind, signal_var=0.7)
    W.lengthscale[:dim] = [0.08, 0.12, 0.1][:dim]
    K = sk_kernel(W)(W.X)
    for i in range(W.m):
        for j in range(W.m):
            v = oracle.kernel(kind, dim, W.signal_var, W.lengthscale, W.X[i], W.X[j])
            assert abs(v - K[i, j]) <= 1e-14 * max(1.0, abs(K[i, j]))


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_kernel_gradient_finite_difference(kind):
    rng = np.random.default_rng(3)
    ell = np.array([0.1, 0.2, 0.15])
    for _ in range(20):
        x, z = rng.random(3), rng.random(3) * 0.3
        g = oracle.kernel_grad(kind, 3, 1.3, ell, x, z)
        h = 1e-6
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            fd = (oracle.kernel(kind, 3, 1.3, ell, x + e, z) - oracle.kernel(kind, 3, 1.3, ell, x - e, z)) / (2 * h)
            assert abs(g[d] - fd) <= 1e-6 * max(1.0, abs(fd))


# ------------------------------------------------------ factor and posterior (Sec. 3)

@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_cholesky_matches_numpy(kind):
    W = small(2, 3, 40, 4, kind=kind)
    M = oracle.fit(W)
    K = sk_kernel(W)(W.X) + W.noise_var * np.eye(W.m)
    Lr = np.linalg.cholesky(K)
    assert np.abs(M.L - Lr).max() <= 1e-12 * np.abs(Lr).max()
    assert np.allclose(np.triu(M.L, 1), 0.0)
    a_ref = sla.cho_solve((Lr, True), W.y)
    assert np.abs(M.a - a_ref).max() <= 1e-10 * np.abs(a_ref).max()


def test_fit_rejects_non_pd():
    W = small(0, 3, 6, 3, noise_var=0.0)
    W.X[3] = W.X[1]          # duplicate location, no noise: K is singular
    Mx = oracle.FitModel(W.kind, W.dim, W.signal_var, W.lengthscale, 0.0, W.X, W.y)
    assert Mx.rc == oracle.ORC_ENOTPD


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
@pytest.mark.parametrize("dim", [2, 3])
def test_posterior_matches_sklearn(kind, dim):
    W = small(4, dim, 30, 4, kind=kind, signal_var=0.5, ell=0.2)
    M = oracle.fit(W)
    P = np.random.default_rng(5).random((200, dim))
    mean, var = oracle.posterior(M, P)
    mu_ref, sd_ref = sk_gpr(W).predict(P, return_std=True)
    assert np.abs(mean - mu_ref).max() <= 1e-9
    assert np.abs(var - sd_ref ** 2).max() <= 1e-10


def test_posterior_equals_sgpr_formula_with_inducing_set_equal_to_data():
    """eq. (sgp) with M = X, mu_M = K (K + s_n^2 I)^-1 y, A_M = K - K (K + s_n^2 I)^-1 K."""
    W = small(6, 3, 15, 4, signal_var=0.8, ell=0.3, noise_var=1e-2)
    M = oracle.fit(W)
    P = np.random.default_rng(7).random((50, 3))
    kern = sk_kernel(W)
    K = kern(W.X)
    Kn = K + W.noise_var * np.eye(W.m)
    mu_M = K @ np.linalg.solve(Kn, W.y)
    A_M = K - K @ np.linalg.solve(Kn, K)
    K_IM = kern(P, W.X)
    Kinv_KMI = np.linalg.solve(K, K_IM.T)
    mu_sgp = K_IM @ np.linalg.solve(K, mu_M)
    var_sgp = (np.diag(kern(P)) - np.einsum("ij,ji->i", K_IM, Kinv_KMI)
               + np.einsum("ji,jk,ki->i", Kinv_KMI, A_M, Kinv_KMI))
    mean, var = oracle.posterior(M, P)
    assert np.abs(mean - mu_sgp).max() <= 1e-8
    assert np.abs(var - var_sgp).max() <= 1e-8


def test_posterior_single_observation_closed_form():
    W = small(8, 3, 1, 3, signal_var=1.7, noise_var=0.3)
    M = oracle.fit(W)
    P = np.random.default_rng(9).random((20, 3))
    k = np.array([oracle.kernel(W.kind, 3, W.signal_var, W.lengthscale, p, W.X[0]) for p in P])
    mean, var = oracle.posterior(M, P)
    den = W.signal_var + W.noise_var
    assert np.allclose(mean, k * W.y[0] / den, rtol=1e-13, atol=1e-15)
    assert np.allclose(var, W.signal_var - k * k / den, rtol=1e-13, atol=1e-15)


def test_posterior_interpolates_as_noise_vanishes_and_is_bounded():
    W = small(10, 3, 25, 3, ell=0.2, noise_var=1e-10)
    M = oracle.fit(W)
    mean, var = oracle.posterior(M, W.X)
    assert np.abs(mean - W.y).max() <= 1e-5
    assert var.max() <= 1e-8
    P = np.random.default_rng(11).random((500, 3))
    _, var = oracle.posterior(M, P)
    assert (var >= 0).all() and (var <= W.signal_var + 1e-12).all()


def test_posterior_far_field_reverts_to_prior():
    W = small(12, 3, 10, 3, ell=0.05)
    M = oracle.fit(W)
    far = np.array([[10.0, 10.0, 10.0], [-7.0, 3.0, 20.0]])
    mean, var = oracle.posterior(M, far)
    assert np.abs(mean).max() < 1e-12 and np.abs(var - W.signal_var).max() < 1e-12


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_posterior_gradient_finite_difference(kind):
    W = small(13, 3, 20, 3, kind=kind, ell=0.25, signal_var=0.6)
    M = oracle.fit(W)
    rng = np.random.default_rng(14)
    for _ in range(10):
        x = rng.random(3)
        mu, var, dmu, dvar = oracle.posterior_grad(M, x)
        for d in range(3):
            e = np.zeros(3)
            e[d] = 1e-6
            (mp, vp), (mm, vm) = [oracle.posterior(M, (x + s * e)[None]) for s in (1, -1)]
            assert abs(dmu[d] - (mp[0] - mm[0]) / 2e-6) <= 1e-5 * max(1, abs(dmu[d]))
            assert abs(dvar[d] - (vp[0] - vm[0]) / 2e-6) <= 1e-5 * max(1, abs(dvar[d]))


# ------------------------------------------------ cell covariance and MC LCP (Sec. 4)

def test_cell_moments_match_sklearn_joint_posterior():
    for dim in (2, 3):
        W = small(15, dim, 20, 6, ell=0.3, signal_var=0.9)
        M = oracle.fit(W)
        cell = [2, 1, 3][:dim]
        corners = np.array([[(cell[d] + ((q >> d) & 1)) / (W.npts[d] - 1) for d in range(dim)]
                            for q in range(1 << dim)])
        mu_ref, cov_ref = sk_gpr(W).predict(corners, return_cov=True)
        mu, S = oracle.cell_moments(M, W, cell)
        assert np.abs(mu - mu_ref).max() <= 1e-10
        assert np.abs(S - cov_ref).max() <= 1e-10


def test_chol_sd_full_rank_matches_numpy_and_semidefinite_reconstructs():
    rng = np.random.default_rng(16)
    A = rng.standard_normal((8, 8))
    S = A @ A.T + 0.1 * np.eye(8)
    Cm, r = oracle.chol_sd(S)
    assert r == 8 and np.abs(Cm - np.linalg.cholesky(S)).max() < 1e-12
    B = rng.standard_normal((8, 3))
    S = B @ B.T                                     # rank 3
    Cm, r = oracle.chol_sd(S)
    assert r == 3 and np.abs(Cm @ Cm.T - S).max() < 1e-10 and np.allclose(np.triu(Cm, 1), 0)


def _golden():
    rows = []
    with open(os.path.join(HERE, "golden", "orthant_exact.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, rho, p, lcp = line.split()
                rows.append((int(n), float(rho), float(p), float(lcp)))
    return rows


@pytest.mark.parametrize("n,rho,p_all,lcp", _golden())
def test_mc_lcp_matches_exact_orthant_values(n, rho, p_all, lcp):
    """Equicorrelated corners at theta = mean (closed forms in tests/golden)."""
    zb = np.random.default_rng(17).standard_normal((200000, n))
    S = np.full((n, n), rho) + (1 - rho) * np.eye(n)
    est = oracle.cell_lcp(np.zeros(n), S, 0.0, zb)
    se = np.sqrt(lcp * (1 - lcp) / zb.shape[0])
    assert abs(est - lcp) <= 4 * se + 1 / zb.shape[0]


def test_mc_lcp_duplicated_corners_reduce_to_sheppard():
    """A 2D cell whose corners 2,3 copy corners 0,1 (rank 2) has the bivariate LCP."""
    rho = 0.3
    S2 = np.array([[1.0, rho], [rho, 1.0]])
    T = np.array([[1, 0], [0, 1], [1, 0], [0, 1]], float)
    S = T @ S2 @ T.T
    zb = np.random.default_rng(18).standard_normal((200000, 4))
    est = oracle.cell_lcp(np.zeros(4), S, 0.0, zb)
    exact = 1 - 2 * (0.25 + np.arcsin(rho) / (2 * np.pi))
    assert abs(est - exact) <= 4 * np.sqrt(exact * (1 - exact) / 2e5) + 5e-6
    # three distinct variables copied onto eight corners: trivariate closed form
    r = np.array([[1, .2, .5], [.2, 1, .7], [.5, .7, 1]])
    T = np.eye(3)[[0, 1, 2, 0, 1, 2, 0, 1]]
    S = T @ r @ T.T
    zb = np.random.default_rng(19).standard_normal((200000, 8))
    est = oracle.cell_lcp(np.zeros(8), S, 0.0, zb)
    exact = 1 - 2 * (0.125 + (np.arcsin(.2) + np.arcsin(.5) + np.arcsin(.7)) / (4 * np.pi))
    assert abs(est - exact) <= 4 * np.sqrt(exact * (1 - exact) / 2e5) + 5e-6


def test_mc_lcp_independent_corners_product_formula_and_genz():
    rng = np.random.default_rng(20)
    zb = rng.standard_normal((200000, 8))
    mu = rng.normal(0.0, 0.5, 8)
    sd = rng.uniform(0.3, 1.0, 8)
    est = oracle.cell_lcp(mu, np.diag(sd ** 2), 0.1, zb)
    zc = (0.1 - mu) / sd
    exact = 1 - np.prod(stats.norm.cdf(zc)) - np.prod(stats.norm.sf(zc))
    assert abs(est - exact) <= 4 * np.sqrt(exact * (1 - exact) / 2e5) + 5e-6
    # a correlated 4-corner cell against scipy's Genz quasi-MC integration
    A = rng.standard_normal((4, 4))
    S = A @ A.T / 4 + 0.2 * np.eye(4)
    mu = rng.normal(0, 0.3, 4)
    theta = 0.05
    p_below = stats.multivariate_normal.cdf(np.full(4, theta), mu, S, abseps=1e-7, releps=1e-7)
    p_above = stats.multivariate_normal.cdf(np.full(4, -theta), -mu, S, abseps=1e-7, releps=1e-7)
    exact = 1 - p_below - p_above
    est = oracle.cell_lcp(mu, S, theta, zb[:, :4])
    assert abs(est - exact) <= 4 * np.sqrt(exact * (1 - exact) / 2e5) + 1e-5


def test_mc_lcp_rank_one_equal_means_is_zero_and_ties_count_as_crossed():
    S = np.full((8, 8), 0.4)
    zb = np.random.default_rng(21).standard_normal((1600, 8))
    assert oracle.cell_lcp(np.full(8, 0.2), S, 0.0, zb) == 0.0
    # zero covariance with the mean exactly at theta: every sample ties -> crossed
    assert oracle.cell_lcp(np.zeros(8), np.zeros((8, 8)), 0.0, zb) == 1.0


@pytest.mark.parametrize("dim", [2, 3])
def test_cell_lcp_matches_brute_force_joint_sampling(dim):
    """Sample the joint posterior of the whole tiny grid (scikit-learn covariance) and
    count crossings per cell; the per-cell oracle estimate must agree statistically."""
    W = small(22, dim, 6, 4 if dim == 3 else 6, ell=0.35, signal_var=0.5, noise_var=1e-3)
    M = oracle.fit(W)
    lcp = oracle.lcp_dense(M, W).reshape(-1)
    n = W.npts[:dim]
    axes = [np.linspace(W.lo[d], W.hi[d], n[d]) for d in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    # vertices in x-fastest order
    P = np.stack([g.transpose(*range(dim)[::-1]).reshape(-1) for g in grids], -1)
    mu, cov = sk_gpr(W).predict(P, return_cov=True)
    ns = 400000
    Y = np.random.default_rng(23).multivariate_normal(mu, cov, size=ns, method="eigh")
    Y = Y.reshape((ns,) + tuple(n[::-1]))
    if dim == 2:
        corners = [Y[:, j:j + n[1] - 1, i:i + n[0] - 1] for i in (0, 1) for j in (0, 1)]
    else:
        corners = [Y[:, k:k + n[2] - 1, j:j + n[1] - 1, i:i + n[0] - 1]
                   for i in (0, 1) for j in (0, 1) for k in (0, 1)]
    C = np.stack(corners, 0)
    below = (C < W.theta).all(0)
    above = (C > W.theta).all(0)
    freq = (~(below | above)).mean(0).reshape(-1)
    # oracle uses N_s = 1600 samples; add its own binomial spread to the tolerance
    tol = 4 * np.sqrt(freq * (1 - freq) / 1600) + 4 * np.sqrt(freq * (1 - freq) / ns) + 2 / 1600
    assert (np.abs(lcp - freq) <= tol).all()


# --------------------------------------------------------- region bound (Sec. 5.1)

def test_upper_bound_formula_and_stability():
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    for g, d in [(0.0, 1), (1.5, 10), (4.0, 125), (6.0, 2_000_000)]:
        t = Decimal(float(stats.norm.sf(g)))          # the tail, from scipy
        ref = float(1 - (1 - t) ** d)                   # exact power in 60-digit decimal
        assert abs(oracle.upper_bound(g, d) - ref) <= 1e-12 * ref + 1e-300
    # t = 1e-12 and d = 1e6: 1 - (1-t)^d = 1e-6 to relative 1e-6 (naive 1 - B^d loses it)
    g = -stats.norm.ppf(1e-12)
    assert abs(oracle.upper_bound(g, 10 ** 6) - 1e-6) <= 1e-11
    assert oracle.upper_bound(np.inf, 10) == 0.0 and oracle.upper_bound(-np.inf, 10) == 1.0


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_bound_search_not_worse_than_any_grid_vertex(kind):
    """The paper's failure mode (Sec. 9): a local search can miss the region's minimum,
    so UB_method may fall below UB_discrete = 1 - (min over grid vertices of P)^d.
    Count the failures that change a decision at alpha = 1e-3 over 800 random boxes."""
    bad = total = 0
    for seed in range(24, 34):
        W = small(seed, 3, 20, 9, kind=kind, ell=0.3, signal_var=0.3, noise_var=1e-4)
        M = oracle.fit(W)
        mean, var = oracle.grid_posterior(M, W)
        mean, var = mean.reshape(9, 9, 9), var.reshape(9, 9, 9)
        rng = np.random.default_rng(seed)
        for _ in range(40):
            lo = rng.integers(0, 6, 3)
            hi = np.minimum(lo + rng.integers(1, 4, 3), 8)
            sl = tuple(slice(lo[d], hi[d] + 1) for d in (2, 1, 0))
            d = int(np.prod(hi - lo + 1))
            for side in (1.0, -1.0):
                g_vert = (side * (W.theta - mean[sl]) / np.sqrt(var[sl])).min()
                gmin, _ = oracle.bound(M, W.theta, side, lo / 8.0, hi / 8.0)
                # the search's value is a value of g inside the box: never below the true minimum
                # over the box, and never above the best lattice point it started from
                total += 1
                bad += oracle.upper_bound(gmin, d) <= 1e-3 < oracle.upper_bound(g_vert, d)
    assert total == 800 and bad <= 1


def test_bound_dominates_cell_lcp_in_region():
    """UB(node) >= LCP of every cell in the node (Sec. 5.1: the region bound is an upper bound
    on the probability of a crossing anywhere in the region), up to MC slack."""
    W = small(26, 3, 15, 9, ell=0.3, signal_var=0.05, noise_var=1e-4)
    M = oracle.fit(W)
    lcp = oracle.lcp_dense(M, W)
    leaves, skipped, recs = oracle.adaptive(M, W, min_leaf=2)
    S0, _ = oracle.octree_shape(W, 2)
    bad = 0
    for r in recs:
        if r["path"] == 0 or np.isnan(r["ub"]):
            continue
        lvl = int(r["level"])
        c = _decode(int(r["key"]), 3)
        s = S0 >> lvl
        sl = tuple(slice(c[d] * s, min((c[d] + 1) * s, 8)) for d in (2, 1, 0))
        if lcp[sl].size:
            bad += lcp[sl].max() > r["ub"] + 3 / 1600
    assert bad == 0


# ---------------------------------------------------------- octree query (Alg. 1)

def _decode(key, dim):
    lvl = key >> 58
    mc = key & ((1 << 58) - 1)
    c = [0] * dim
    for b in range(lvl):
        for d in range(dim):
            c[d] |= ((mc >> (b * dim + d)) & 1) << b
    return c


def test_octree_shape():
    for n, leaf, S0, L in [(128, 4, 128, 5), (64, 4, 64, 4), (65, 4, 64, 4), (66, 4, 128, 5), (9, 1, 8, 3),
                           (256, 4, 256, 6)]:
        W = small(0, 3, 2, 3)
        W.npts[:] = n
        assert oracle.octree_shape(W, leaf) == (S0, L)


@pytest.mark.parametrize("dim,npts,leaf", [(3, 9, 1), (3, 12, 2), (2, 20, 1), (2, 33, 4)])
def test_adaptive_partitions_grid_and_matches_dense_in_leaves(dim, npts, leaf):
    W = small(27, dim, 12, npts, ell=0.25, signal_var=0.02, noise_var=1e-5, min_leaf=leaf)
    M = oracle.fit(W)
    leaves, skipped, recs = oracle.adaptive(M, W)
    lev = oracle.level_field(W, np.concatenate([leaves, skipped]))
    assert (lev != 255).all()
    # partition: each cell is covered exactly once
    S0, L = oracle.octree_shape(W)
    cover = np.zeros(W.n_cells, int)
    for key in np.concatenate([leaves, skipped]):
        lvl = int(key) >> 58
        c = _decode(int(key), dim)
        s = S0 >> lvl
        f = cover.reshape(W.cell_shape)
        sl = tuple(slice(c[d] * s, min((c[d] + 1) * s, W.npts[d] - 1)) for d in range(dim - 1, -1, -1))
        f[sl] += 1
    assert (cover == 1).all()
    assert all(int(k) >> 58 == L for k in leaves)
    dense = oracle.lcp_dense(M, W)
    adapt = oracle.lcp_leaves(M, W, leaves)
    inleaf = oracle.level_field(W, leaves) != 255
    assert np.array_equal(adapt[inleaf], dense[inleaf])
    assert (adapt[~inleaf] == 0).all()
    # skipped cells: their dense MC LCP must stay at the level alpha allows (binomial slack)
    assert dense[~inleaf].max(initial=0) <= W.alpha + 4 / 1600


def test_adaptive_decisions_follow_alg1():
    """Re-derive every node decision from the records with scikit-learn's posterior at
    the observations (p1, p2) and the printed rules of Alg. 1."""
    W = small(28, 3, 30, 17, ell=0.2, signal_var=0.01, noise_var=1e-5, min_leaf=2)
    M = oracle.fit(W)
    leaves, skipped, recs = oracle.adaptive(M, W)
    mu, sd = sk_gpr(W).predict(W.X, return_std=True)
    qlo = stats.norm.cdf((W.theta - mu) / sd)
    qhi = stats.norm.sf((W.theta - mu) / sd)
    S0, L = oracle.octree_shape(W)
    assert len(recs) > 20 and len(leaves) > 0 and len(skipped) > 0
    for r in recs:
        lvl = int(r["level"])
        c = _decode(int(r["key"]), 3)
        s = S0 >> lvl
        lo = np.array([c[d] * s for d in range(3)])
        hi = np.minimum(lo + s, W.npts[:3] - 1)
        inside = np.all((W.X >= lo / 16.0 - 1e-15) & (W.X <= hi / 16.0 + 1e-15), axis=1)
        assert int(r["n_obs"]) == inside.sum()
        assert int(r["d"]) == np.prod(hi - lo + 1)
        if inside.any():
            p1, p2 = qlo[inside].max(), qhi[inside].max()
            assert abs(r["p1"] - p1) < 1e-9 and abs(r["p2"] - p2) < 1e-9
            if p1 > W.alpha and p2 > W.alpha:
                assert r["path"] == 0 and r["subdivide"] == 1
                continue
            assert r["path"] == (1 if p2 <= W.alpha else 2)
        assert r["subdivide"] == int(r["ub"] > W.alpha)
        assert abs(r["ub"] - oracle.upper_bound(r["gmin"], int(r["d"]))) == 0.0
    # a subdivided node at the finest level is a leaf, a refused one is skipped
    sub = {int(r["key"]) for r in recs if r["subdivide"] and r["level"] == L}
    assert sub == {int(k) for k in leaves}
    assert {int(r["key"]) for r in recs if not r["subdivide"]} == {int(k) for k in skipped}


def _g_single_obs(r, y0, theta, side, s2, noise, ell):
    """Standardised margin of Sec. 5.1 for an SE model with one observation at scaled
    distance r/ell, from the m = 1 closed form of eq. (sgp) (no oracle code)."""
    k = s2 * np.exp(-0.5 * (np.asarray(r, float) / ell) ** 2)
    mu = k * y0 / (s2 + noise)
    var = s2 - k * k / (s2 + noise)
    return side * (theta - mu) / np.sqrt(var)


@pytest.mark.parametrize("side,y0,theta,lo,w", [(1.0, 1.0, 0.2, 0.0, 1.0), (-1.0, -1.0, -0.2, 0.0, 1.0),
                                                 (1.0, 1.0, 0.2, 0.1, 0.5)])
def test_bound_descent_follows_the_schedule_to_an_interior_minimum(side, y0, theta, lo, w):
    """The search of reading S12 on a box whose minimum of g is interior and off the
    {lo, mid, hi} lattice: one observation x0 (SE, isotropic) makes g radial around x0, so
    the normalised box-scaled step on a cube of width w moves straight towards x0 by
    eta_k w = 2^-(k+1) w.  The signed distance along the line then follows
    s_{k+1} = s_k - 2^-(k+1) w sign(s_k) from s_0 = |x0 - best lattice point|, and the search
    must return min(g(lattice), g(|s_1|), ..., g(|s_T|)) from the m = 1 closed form.  A
    wrong sign walks away from x0 and leaves the lattice value; a wrong step schedule or
    normalisation lands at other distances.  g(x0) is the box's minimum (checked on a
    41^3 brute-force grid), and the search never goes below it."""
    s2, noise, ell = 1.0, 1e-4, 0.15
    x0 = lo + w * np.array([0.314, 0.357, 0.628])
    M = oracle.FitModel(workloads.SE, 3, s2, [ell] * 3, noise, x0[None, :], np.array([y0]))
    blo, bhi = np.full(3, lo), np.full(3, lo + w)
    lat = np.array([[lo + 0.5 * w * ((i // 3 ** d) % 3) for d in range(3)] for i in range(27)])
    g_lat = _g_single_obs(np.linalg.norm(lat - x0, axis=1), y0, theta, side, s2, noise, ell)
    p0 = lat[int(np.argmin(g_lat))]
    assert np.allclose(p0, lo + 0.5 * w)           # the centre is the lattice point nearest x0
    s = np.linalg.norm(p0 - x0)
    visited = [g_lat.min()]
    for k in range(4):
        s = s - 0.5 ** (k + 1) * w * np.sign(s)
        visited.append(float(_g_single_obs(abs(s), y0, theta, side, s2, noise, ell)))
        gmin, _ = oracle.bound(M, theta, side, blo, bhi, steps=k + 1)
        want = min(visited)
        assert abs(gmin - want) <= 1e-9 * abs(want) + 1e-12, (k, gmin, want)
    g0, _ = oracle.bound(M, theta, side, blo, bhi, steps=0)
    assert abs(g0 - g_lat.min()) <= 1e-12 * max(1.0, abs(g0))
    assert gmin < g0 - 5.0                         # the descent found the interior basin
    # the true minimum is g(x0): every point of a 41^3 brute-force grid is above it
    t = np.linspace(lo, lo + w, 41)
    P = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    g_true = float(_g_single_obs(0.0, y0, theta, side, s2, noise, ell))
    g_grid = _g_single_obs(np.linalg.norm(P - x0, axis=1), y0, theta, side, s2, noise, ell).min()
    assert g_true <= g_grid and g_true <= gmin
