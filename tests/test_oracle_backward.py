"""Pins of the oracle's posterior adjoint (gradients of the eq. (sgp) posterior with respect
to the observation values and the log-lengthscales) against central finite differences of
the oracle's own forward pass (re-fitted at each perturbed input) and, for the values,
against scikit-learn's linear predictor.  CPU only.
"""
import numpy as np
import pytest
from sklearn.gaussian_process import GaussianProcessRegressor

import oracle
import workloads
from test_oracle_pins import sk_kernel, small


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_kernel_dlogell_finite_difference(kind):
    rng = np.random.default_rng(50)
    ell = np.array([0.1, 0.2, 0.15])
    for _ in range(20):
        x, z = rng.random(3), rng.random(3) * 0.3
        g = oracle.kernel_dlogell(kind, 3, 1.3, ell, x, z)
        for d in range(3):
            e = np.zeros(3)
            e[d] = 1e-6
            fp = oracle.kernel(kind, 3, 1.3, ell * np.exp(e), x, z)
            fm = oracle.kernel(kind, 3, 1.3, ell * np.exp(-e), x, z)
            assert abs(g[d] - (fp - fm) / 2e-6) <= 1e-7 * max(1.0, abs(g[d]))


def _loss(W, y, ell, P, gm, gv):
    M = oracle.FitModel(W.kind, W.dim, W.signal_var, ell, W.noise_var, W.X, y)
    mu, var = oracle.posterior(M, P)
    return float(gm @ mu + gv @ var)


@pytest.mark.parametrize("kind,dim", [(workloads.SE, 3), (workloads.MATERN52, 3), (workloads.SE, 2),
                                      (workloads.MATERN52, 2)])
def test_posterior_backward_matches_finite_differences(kind, dim):
    W = small(51, dim, 15, 4, kind=kind, signal_var=0.7, ell=0.3, noise_var=1e-3)
    W.lengthscale[:dim] = [0.25, 0.35, 0.3][:dim]
    rng = np.random.default_rng(52)
    P = rng.random((40, dim))
    gm, gv = rng.standard_normal(40), rng.standard_normal(40)
    M = oracle.fit(W)
    dy, dl = oracle.posterior_backward(M, P, gm, gv)
    h = 1e-6
    for j in range(W.m):
        e = np.zeros(W.m)
        e[j] = h
        fd = (_loss(W, W.y + e, W.lengthscale, P, gm, gv) - _loss(W, W.y - e, W.lengthscale, P, gm, gv)) / (2 * h)
        assert abs(dy[j] - fd) <= 1e-6 * max(1.0, abs(fd)), (j, dy[j], fd)
    for d in range(dim):
        e = np.zeros(3)
        e[d] = h
        lp = _loss(W, W.y, W.lengthscale * np.exp(e), P, gm, gv)
        lm = _loss(W, W.y, W.lengthscale * np.exp(-e), P, gm, gv)
        fd = (lp - lm) / (2 * h)
        assert abs(dl[d] - fd) <= 1e-6 * max(1.0, abs(fd)), (d, dl[d], fd)


def test_posterior_backward_values_match_the_linear_predictor():
    """The mean is linear in y: dL/dy_j = sum_i g_i mu_i(y = e_j) (scikit-learn, exact)."""
    W = small(53, 3, 12, 4, signal_var=0.9, ell=0.3, noise_var=1e-3)
    P = np.random.default_rng(54).random((30, 3))
    gm = np.random.default_rng(55).standard_normal(30)
    dy, _ = oracle.posterior_backward(oracle.fit(W), P, gm, None)
    for j in range(W.m):
        e = np.zeros(W.m)
        e[j] = 1.0
        g = GaussianProcessRegressor(sk_kernel(W), alpha=W.noise_var, optimizer=None).fit(W.X, e)
        assert abs(dy[j] - gm @ g.predict(P)) <= 1e-9


def test_posterior_backward_rejects_the_sparse_model():
    W = workloads.sgpr_field(56, m=8, npts=5, train_npts=6)
    with pytest.raises(AssertionError):
        oracle.posterior_backward(oracle.fit(W), np.zeros((1, 3)), np.ones(1), None)


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_posterior_backward_variance_gives_no_value_gradient(kind):
    """The variance of eq. (sgp) does not involve y, so an upstream on the variance alone gives
    dL/dy = 0 exactly, while its log-lengthscale gradient is the one of the variance term of
    the combined upstream (the two terms of the loss are additive)."""
    W = small(57, 3, 14, 4, kind=kind, signal_var=0.8, ell=0.3, noise_var=1e-3)
    P = np.random.default_rng(58).random((25, 3))
    rng = np.random.default_rng(59)
    gm, gv = rng.standard_normal(25), rng.standard_normal(25)
    M = oracle.fit(W)
    dy_v, dl_v = oracle.posterior_backward(M, P, None, gv)
    assert np.all(dy_v == 0.0)
    dy_m, dl_m = oracle.posterior_backward(M, P, gm, None)
    dy_b, dl_b = oracle.posterior_backward(M, P, gm, gv)
    assert np.allclose(dy_b, dy_m, rtol=1e-12, atol=1e-12)
    assert np.allclose(dl_b, dl_m + dl_v, rtol=1e-10, atol=1e-12)
    assert np.any(dl_v != 0.0)
