"""Pins of the oracle's general sparse model (eq. (sgp) with stored mu_M, A_M) against
independent library routines and the special cases the formula reduces to.  CPU only.
"""
import numpy as np
import pytest
from scipy import stats
from sklearn.gaussian_process import GaussianProcessRegressor

import oracle
import workloads
from test_oracle_pins import _decode, sk_kernel, small


def sparse_of(W, mu_M, A_M, jitter):
    return oracle.SparseModel(W.kind, W.dim, W.signal_var, W.lengthscale, jitter, W.X, mu_M, A_M)


def identity_model(W):
    """eq. (sgp) with M = X, mu_M = K (K + s_n^2 I)^-1 y, A_M = K - K (K + s_n^2 I)^-1 K."""
    K = sk_kernel(W)(W.X)
    Kn = K + W.noise_var * np.eye(W.m)
    mu_M = K @ np.linalg.solve(Kn, W.y)
    A_M = K - K @ np.linalg.solve(Kn, K)
    return sparse_of(W, mu_M, 0.5 * (A_M + A_M.T), 0.0)


def corners_of(W, cell):
    return np.array([[(cell[d] + ((q >> d) & 1)) / (W.npts[d] - 1) for d in range(W.dim)]
                     for q in range(1 << W.dim)])


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_sparse_with_inducing_set_equal_to_data_is_the_exact_posterior(kind):
    """Sec. 3: with M = X the sparse posterior is the exact GP posterior (scikit-learn)."""
    W = small(31, 3, 14, 6, kind=kind, signal_var=0.8, ell=0.3, noise_var=1e-2)
    S = identity_model(W)
    gpr = GaussianProcessRegressor(sk_kernel(W), alpha=W.noise_var, optimizer=None).fit(W.X, W.y)
    P = np.random.default_rng(32).random((60, 3))
    mean, var = oracle.posterior(S, P)
    mu_ref, sd_ref = gpr.predict(P, return_std=True)
    assert np.abs(mean - mu_ref).max() <= 1e-8
    assert np.abs(var - sd_ref ** 2).max() <= 1e-8
    for cell in ([0, 0, 0], [2, 3, 1], [4, 4, 4]):
        mu_c, cov_c = gpr.predict(corners_of(W, cell), return_cov=True)
        mu, Sc = oracle.cell_moments(S, W, cell)
        assert np.abs(mu - mu_c).max() <= 1e-8
        assert np.abs(Sc - cov_c).max() <= 1e-8
    E = oracle.fit(W)
    for x in P[:5]:
        a, b = oracle.posterior_grad(S, x), oracle.posterior_grad(E, x)
        for u, v in zip(a, b):
            assert np.allclose(u, v, rtol=1e-7, atol=1e-9)


def test_sparse_single_inducing_point_closed_form():
    """m = 1: mu = k mu_M / c, var = s2 - k^2 / c + A k^2 / c^2 with c = s2 + jitter, and
    the corner covariance k(p, q) - k_p k_q / c + A k_p k_q / c^2."""
    W = small(33, 3, 1, 4, signal_var=1.3)
    jit, mu_M, A = 0.05, np.array([0.7]), np.array([[0.4]])
    S = sparse_of(W, mu_M, A, jit)
    P = np.random.default_rng(34).random((30, 3))
    k = np.array([oracle.kernel(W.kind, 3, W.signal_var, W.lengthscale, p, W.X[0]) for p in P])
    c = W.signal_var + jit
    mean, var = oracle.posterior(S, P)
    assert np.allclose(mean, k * 0.7 / c, rtol=1e-13, atol=1e-15)
    assert np.allclose(var, W.signal_var - k * k / c + 0.4 * k * k / c ** 2, rtol=1e-13, atol=1e-15)
    X8 = corners_of(W, [1, 2, 0])
    kc = np.array([oracle.kernel(W.kind, 3, W.signal_var, W.lengthscale, p, W.X[0]) for p in X8])
    ref = sk_kernel(W)(X8) - np.outer(kc, kc) / c + 0.4 * np.outer(kc, kc) / c ** 2
    _, Sc = oracle.cell_moments(S, W, [1, 2, 0])
    assert np.abs(Sc - ref).max() <= 1e-13


def test_sparse_prior_covariance_of_inducing_values_gives_the_prior():
    """A_M = K_MM + jitter I: the inducing values carry no information, so the variance
    and the corner covariance are the prior's."""
    W = small(35, 3, 20, 5, signal_var=0.6, ell=0.3)
    jit = 1e-3
    K = sk_kernel(W)(W.X) + jit * np.eye(W.m)
    S = sparse_of(W, W.y, K, jit)
    P = np.random.default_rng(36).random((40, 3))
    _, var = oracle.posterior(S, P)
    assert np.abs(var - W.signal_var).max() <= 1e-9
    _, Sc = oracle.cell_moments(S, W, [1, 3, 2])
    assert np.abs(Sc - sk_kernel(W)(corners_of(W, [1, 3, 2]))).max() <= 1e-9


def test_sparse_deterministic_inducing_values_interpolate_them():
    """A_M = 0: the posterior is that of noise-free observations mu_M at M (scikit-learn
    with alpha = jitter)."""
    W = small(37, 3, 18, 5, signal_var=0.9, ell=0.25)
    jit = 1e-6
    S = sparse_of(W, W.y, np.zeros((W.m, W.m)), jit)
    gpr = GaussianProcessRegressor(sk_kernel(W), alpha=jit, optimizer=None).fit(W.X, W.y)
    P = np.random.default_rng(38).random((40, 3))
    mean, var = oracle.posterior(S, P)
    mu_ref, sd_ref = gpr.predict(P, return_std=True)
    assert np.abs(mean - mu_ref).max() <= 1e-7
    assert np.abs(var - sd_ref ** 2).max() <= 1e-8


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_sparse_gradient_finite_difference(kind):
    W = workloads.sgpr_field(39, m=27, npts=9, train_npts=10, signal_var=0.5, ell=0.3)
    W.kind = kind
    S = oracle.fit(W)
    rng = np.random.default_rng(40)
    for _ in range(10):
        x = rng.random(3)
        mu, var, dmu, dvar = oracle.posterior_grad(S, x)
        for d in range(3):
            e = np.zeros(3)
            e[d] = 1e-6
            (mp, vp), (mm, vm) = [oracle.posterior(S, (x + s * e)[None]) for s in (1, -1)]
            assert abs(dmu[d] - (mp[0] - mm[0]) / 2e-6) <= 1e-5 * max(1, abs(dmu[d]))
            assert abs(dvar[d] - (vp[0] - vm[0]) / 2e-6) <= 1e-5 * max(1, abs(dvar[d]))


def test_sgpr_generator_gives_a_valid_inducing_distribution():
    """The synthetic fit: A_M is symmetric, PSD and below K_MM + jitter I, and the inducing
    means follow the field."""
    W = workloads.sgpr_field(41, m=64, npts=17, train_npts=16)
    K = sk_kernel(W)(W.X) + W.noise_var * np.eye(W.m)
    assert np.array_equal(W.A_M, W.A_M.T)
    assert np.linalg.eigvalsh(W.A_M).min() > -1e-12
    assert np.linalg.eigvalsh(K - W.A_M).min() > -1e-12
    f = workloads._trig_field(W.X, 41)
    assert np.sqrt(np.mean((W.y - f) ** 2)) < 0.5 * f.std()


def test_sparse_adaptive_decisions_use_the_inducing_marginals():
    """Sec. 5.3 on the sparse model: p1, p2 are the largest marginal probabilities of the
    inducing values N(mu_M_i, A_M_ii) inside the node; leaves reproduce the dense field."""
    W = workloads.sgpr_field(42, m=27, npts=17, train_npts=12, signal_var=0.5, ell=0.3)
    W.min_leaf = 2
    S = oracle.fit(W)
    leaves, skipped, recs = oracle.adaptive(S, W)
    sd = np.sqrt(np.diag(W.A_M))
    qlo = stats.norm.cdf((W.theta - W.y) / sd)
    qhi = stats.norm.sf((W.theta - W.y) / sd)
    S0, L = oracle.octree_shape(W)
    n_with_obs = 0
    for r in recs:
        lvl = int(r["level"])
        c = _decode(int(r["key"]), 3)
        s = S0 >> lvl
        lo = np.array([c[d] * s for d in range(3)])
        hi = np.minimum(lo + s, W.npts[:3] - 1)
        inside = np.all((W.X >= lo / 16.0 - 1e-15) & (W.X <= hi / 16.0 + 1e-15), axis=1)
        assert int(r["n_obs"]) == inside.sum()
        if inside.any():
            n_with_obs += 1
            assert abs(r["p1"] - qlo[inside].max()) < 1e-12 and abs(r["p2"] - qhi[inside].max()) < 1e-12
    assert n_with_obs > 5 and len(leaves) > 0
    dense = oracle.lcp_dense(S, W)
    adapt = oracle.lcp_leaves(S, W, leaves)
    inleaf = oracle.level_field(W, leaves) != 255
    assert np.array_equal(adapt[inleaf], dense[inleaf])
    assert dense[~inleaf].max(initial=0) <= W.alpha + 4 / 1600
