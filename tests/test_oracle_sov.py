"""Pins of the oracle's smooth cell LCP (Genz's separation of variables) and of the LCP
adjoint built on it: closed-form orthant values, agreement with the paper's counting
estimator, and central finite differences of every smooth forward.  CPU only.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
import workloads
from test_oracle_pins import _golden, small


@pytest.mark.parametrize("n,rho,p_all,lcp", _golden())
def test_sov_lcp_matches_exact_orthant_values(n, rho, p_all, lcp):
    """Equicorrelated corners at theta = mean: 1 - 2 P(all > 0) (closed forms in tests/golden).
    The estimator is unbiased; 20000 samples bound its error well inside 5e-3."""
    zb = np.random.default_rng(80).standard_normal((20000, n))
    S = np.full((n, n), rho) + (1 - rho) * np.eye(n)
    Cm, _ = oracle.chol_sd(S)
    assert abs(oracle.sov_lcp(np.zeros(n), Cm, 0.0, zb) - lcp) <= 5e-3


def test_sov_lcp_agrees_with_counting_and_scipy():
    """Random 8-corner cells: the smooth estimate, the paper's counting estimate (same
    z-bank) and scipy's Genz integration of the two orthants agree statistically."""
    rng = np.random.default_rng(81)
    zb = rng.standard_normal((4000, 8))
    for _ in range(6):
        B = rng.standard_normal((8, 8)) * 0.3 + np.eye(8)
        S = B @ B.T
        mu = rng.standard_normal(8) * 0.5
        Cm, _ = oracle.chol_sd(S)
        sov = oracle.sov_lcp(mu, Cm, 0.2, zb)
        mc = oracle.mc_count(mu, Cm, 0.2, zb) / zb.shape[0]
        lo = stats.multivariate_normal(mu, S).cdf(np.full(8, 0.2))
        hi = stats.multivariate_normal(-mu, S).cdf(np.full(8, -0.2))
        ref = 1 - lo - hi
        se = np.sqrt(max(ref * (1 - ref), 1e-4) / zb.shape[0])
        assert abs(mc - ref) <= 5 * se + 2e-3
        assert abs(sov - ref) <= 5 * se + 2e-3


def test_sov_gradient_matches_finite_differences():
    rng = np.random.default_rng(82)
    zb = rng.standard_normal((300, 8))
    B = rng.standard_normal((8, 8)) * 0.4 + np.eye(8)
    S = B @ B.T
    Cm, _ = oracle.chol_sd(S)
    mu = rng.standard_normal(8) * 0.5
    v, gmu, gC = oracle.sov_lcp_grad(mu, Cm, 0.1, zb)
    assert abs(v - oracle.sov_lcp(mu, Cm, 0.1, zb)) < 1e-15
    h = 1e-6
    for i in range(8):
        e = np.zeros(8)
        e[i] = h
        fd = (oracle.sov_lcp(mu + e, Cm, 0.1, zb) - oracle.sov_lcp(mu - e, Cm, 0.1, zb)) / (2 * h)
        assert abs(gmu[i] - fd) <= 1e-6 * max(1.0, abs(fd))
    for i in range(8):
        for j in range(i + 1):
            E = np.zeros((8, 8))
            E[i, j] = h
            fd = (oracle.sov_lcp(mu, Cm + E, 0.1, zb) - oracle.sov_lcp(mu, Cm - E, 0.1, zb)) / (2 * h)
            assert abs(gC[i, j] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, j)


def test_cholesky_adjoint_matches_finite_differences():
    rng = np.random.default_rng(83)
    B = rng.standard_normal((8, 8)) * 0.5 + np.eye(8)
    S = B @ B.T
    G = np.tril(rng.standard_normal((8, 8)))
    Cm, _ = oracle.chol_sd(S)
    gS = oracle.chol_sd_rev(Cm, G)
    h = 1e-6
    for i in range(8):
        for j in range(i + 1):
            E = np.zeros((8, 8))
            E[i, j] = h            # the factor reads the lower triangle only
            fd = ((oracle.chol_sd(S + E)[0] * G).sum() - (oracle.chol_sd(S - E)[0] * G).sum()) / (2 * h)
            assert abs(gS[i, j] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, j)
    assert np.allclose(np.triu(gS, 1), 0.0)


@pytest.mark.parametrize("kind,dim", [(workloads.SE, 3), (workloads.MATERN52, 3), (workloads.SE, 2)])
def test_lcp_backward_matches_finite_differences(kind, dim):
    """L = sum_c u_c LCP_c of the smooth field; gradients with respect to y and log(ell)
    against central differences of the re-fitted oracle (h = 1e-6)."""
    W = small(84, dim, 10, 5 if dim == 3 else 9, kind=kind, ell=0.35, signal_var=0.05, noise_var=1e-3)
    W.zbank = W.zbank[:200]
    rng = np.random.default_rng(85)
    u = rng.random(W.n_cells)

    def loss(y, ell):
        M = oracle.FitModel(W.kind, W.dim, W.signal_var, ell, W.noise_var, W.X, y)
        return float(u @ oracle.lcp_sov_dense(M, W).reshape(-1))

    M = oracle.fit(W)
    dy, dl = oracle.lcp_backward(M, W, u)
    assert np.abs(dy).max() > 0 and np.abs(dl).max() > 0
    h = 1e-6
    for j in range(W.m):
        e = np.zeros(W.m)
        e[j] = h
        fd = (loss(W.y + e, W.lengthscale) - loss(W.y - e, W.lengthscale)) / (2 * h)
        assert abs(dy[j] - fd) <= 2e-6 * max(1.0, abs(fd)), (j, dy[j], fd)
    for d in range(dim):
        e = np.zeros(3)
        e[d] = h
        fd = (loss(W.y, W.lengthscale * np.exp(e)) - loss(W.y, W.lengthscale * np.exp(-e))) / (2 * h)
        assert abs(dl[d] - fd) <= 2e-6 * max(1.0, abs(fd)), (d, dl[d], fd)
