"""Pins of the oracle's certified region bound: box bounds of the posterior mean and
variance that hold at every point of the box (the guarantee the search of Sec. 5.1 lacks,
Sec. 9).  CPU only.

  * the kernel Hessian against central differences of the kernel gradient;
  * the third-derivative envelope is the supremum, beyond a distance, of the kernel's third
    directional derivative (numerical differences of the oracle kernel, itself pinned to
    scikit-learn);
  * soundness: the posterior (mean and variance) at lattices and random points of random
    boxes stays inside the certified bounds, for exact and sparse models;
  * tightness to first order: on tiny boxes the bounds approach the centre value plus the
    box's linear spread, |grad| . h, with the gradient from central differences;
  * second and third order: on a box centred on a lone observation (zero gradient) the
    bound's spread is the exact quadratic term plus s2 H^(3/2) |a| C3(0) / 6;
  * the octree: the leaves found with the certified bound contain those of the search, and
    no skipped node contains a cell whose smooth LCP exceeds alpha.
"""
import numpy as np
import pytest

import oracle
import workloads
from test_oracle_pins import small


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_kernel_hessian_matches_gradient_differences(kind):
    rng = np.random.default_rng(99)
    ell = np.array([0.2, 0.35, 0.3])
    e = 1e-6
    for _ in range(6):
        x, z = rng.random(3), rng.random(3)
        Hm = oracle.kernel_hess(kind, 3, 0.8, ell, x, z)
        fd = np.stack([(oracle.kernel_grad(kind, 3, 0.8, ell, x + e * np.eye(3)[d], z)
                        - oracle.kernel_grad(kind, 3, 0.8, ell, x - e * np.eye(3)[d], z)) / (2 * e)
                       for d in range(3)])
        assert np.abs(Hm - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())
        assert np.allclose(Hm, Hm.T, rtol=0, atol=1e-15)
    # at the observation itself: -s2 |g(0)| / ell^2 on the diagonal (1 for SE, 5/3 Matern)
    Hm = oracle.kernel_hess(kind, 3, 0.8, ell, z, z)
    assert np.allclose(Hm, -np.diag(0.8 * (1.0 if kind == workloads.SE else 5.0 / 3.0) / ell ** 2), rtol=1e-14)


def _third_radius(kind, rho, h=2e-3):
    """max over unit directions v of |d^3/dt^3 k(z + t v)| at |z| = rho (s2 = 1, unit ell),
    by fourth-order-accurate differences along 65 directions in a plane through z."""
    z = np.array([rho, 0.0, 0.0])
    f = lambda p: oracle.kernel(kind, 3, 1.0, [1.0, 1.0, 1.0], p, np.zeros(3))
    best = 0.0
    for th in np.linspace(0.0, np.pi, 65):
        v = np.array([np.cos(th), np.sin(th), 0.0])
        d3 = (-f(z + 3 * h * v) + 8 * f(z + 2 * h * v) - 13 * f(z + h * v)
              + 13 * f(z - h * v) - 8 * f(z - 2 * h * v) + f(z - 3 * h * v)) / (8 * h ** 3)
        best = max(best, abs(d3))
    return best


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_third_derivative_envelope_is_the_supremum(kind):
    rho = np.linspace(0.01, 7.0, 500)
    rad = np.array([_third_radius(kind, r) for r in rho])
    for r in (0.0, 0.2, 0.3, 0.5, 0.8, 1.0, 1.3, 1.8, 2.2, 2.6, 3.5, 5.0):
        env = oracle.curv3_env(kind, r * r)
        sup = max(rad[rho >= r].max(), _third_radius(kind, max(r, 1e-3)))
        assert sup <= env * (1 + 1e-4) + 1e-9, (r, sup, env)
        assert sup >= env * (1 - 2e-2), (r, sup, env)           # a supremum, not a loose bound
    env = np.array([oracle.curv3_env(kind, x * x) for x in rho])
    assert np.all(np.diff(env) <= 1e-15)                          # non-increasing


def _models():
    out = []
    for kind in (workloads.SE, workloads.MATERN52):
        W = small(110 + kind, 3, 30, 5, kind=kind, ell=0.3, signal_var=0.5, noise_var=1e-3)
        W.lengthscale[:3] = [0.25, 0.35, 0.3]
        out.append((W, oracle.fit(W)))
    S = workloads.sgpr_field(112, m=27, npts=5, train_npts=8, ell=0.3)
    out.append((S, oracle.fit(S)))
    return out


@pytest.mark.parametrize("case", range(3))
def test_certified_bounds_hold_over_the_box(case):
    W, M = _models()[case]
    rng = np.random.default_rng(120 + case)
    for t in range(40):
        lo = rng.random(3) * 0.8
        width = rng.choice([0.01, 0.05, 0.1, 0.2]) * rng.random(3)
        if t % 10 == 0:
            width[rng.integers(3)] = 0.0                    # a flat box
        hi = lo + width
        cb = oracle.bound_certified(M, lo, hi)
        g = [np.linspace(lo[d], hi[d], 7) for d in range(3)]
        P = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, 3)
        P = np.vstack([P, lo + rng.random((300, 3)) * width])
        mean, var = oracle.posterior(M, P)[:2]
        scale = np.abs(mean).max() + W.signal_var
        assert mean.min() >= cb[1] - 1e-12 * scale
        assert mean.max() <= cb[2] + 1e-12 * scale
        assert var.max() <= cb[3] + 1e-12 * W.signal_var
        c_mean, c_var = oracle.posterior(M, 0.5 * (lo + hi)[None])[:2]
        assert abs(cb[0] - c_mean[0]) <= 1e-12 * scale
        assert cb[3] >= c_var[0] - 1e-12 * W.signal_var and cb[3] <= W.signal_var


@pytest.mark.parametrize("case", range(3))
def test_certified_bounds_are_first_order_tight(case):
    W, M = _models()[case]
    rng = np.random.default_rng(130 + case)
    e = 1e-6
    for _ in range(5):
        c = 0.2 + 0.6 * rng.random(3)
        h = 1e-7 * np.asarray(W.lengthscale[:3]) * (0.5 + rng.random(3))
        cb = oracle.bound_certified(M, c - h, c + h)
        gm, gv = np.zeros(3), np.zeros(3)
        for d in range(3):
            P = np.stack([c + e * np.eye(3)[d], c - e * np.eye(3)[d]])
            mean, var = oracle.posterior(M, P)[:2]
            gm[d], gv[d] = (mean[0] - mean[1]) / (2 * e), (var[0] - var[1]) / (2 * e)
        lin_m, lin_v = np.abs(gm) @ h, np.abs(gv) @ h
        assert abs((cb[2] - cb[0]) - lin_m) <= 1e-3 * lin_m
        assert abs((cb[0] - cb[1]) - lin_m) <= 1e-3 * lin_m
        c_var = oracle.posterior(M, c[None])[1][0]
        assert abs((cb[3] - c_var) - lin_v) <= 1e-3 * lin_v + 1e-13


@pytest.mark.parametrize("kind,c0", [(workloads.SE, 1.0), (workloads.MATERN52, 5.0 / 3.0)])
def test_certified_bound_at_a_lone_observation(kind, c0):
    """m = 1, box centred on the observation: the gradient vanishes and the Hessian is
    -a s2 c0 / ell^2 on the diagonal, so the mean's spread is [-(a s2 c0 H / 2) - R, R] with
    R = s2 H^(3/2) |a| C3(0) / 6, and the true extreme sits at the corners (r^2 = H)."""
    s2, ell, noise, y = 0.7, np.array([0.2, 0.3, 0.25]), 1e-3, 1.3
    x1 = np.array([0.4, 0.5, 0.6])
    M = oracle.FitModel(kind, 3, s2, ell, noise, x1[None], np.array([y]))
    a = y / (s2 + noise)
    C3 = oracle.curv3_env(kind, 0.0)
    for scale in (1e-2, 3e-3, 1e-3):
        h = scale * ell
        H = float(np.sum((h / ell) ** 2))
        R = s2 * H ** 1.5 * abs(a) * C3 / 6
        cb = oracle.bound_certified(M, x1 - h, x1 + h)
        assert cb[2] - cb[0] == pytest.approx(R, rel=1e-9)
        assert cb[0] - cb[1] == pytest.approx(0.5 * a * s2 * c0 * H + R, rel=1e-9)
        corner = oracle.posterior(M, (x1 + h)[None])[0][0]
        true_dev = cb[0] - corner
        assert (cb[0] - cb[1]) >= true_dev
        assert (cb[0] - cb[1]) / true_dev - 1.0 <= 2.0 * np.sqrt(H)        # ratio -> 1 as H -> 0
        # variance: var(x) = s2 - w k(x), w = s2 / (s2 + noise); bound spread 2 (w s2 c0 H / 2 + R_w)
        w = s2 / (s2 + noise)
        var_c = s2 - s2 * s2 / (s2 + noise)
        Rw = s2 * H ** 1.5 * w * C3 / 6
        assert cb[3] - var_c == pytest.approx(2 * (0.5 * w * s2 * c0 * H + Rw), rel=1e-6)


def test_certified_margin_reads_the_worst_mean_and_the_largest_sigma():
    cb = np.array([0.0, -0.5, 0.2, 0.04])
    assert oracle.certified_margin(1.0, 0.6, cb) == pytest.approx((0.6 - 0.2) / 0.2)
    assert oracle.certified_margin(-1.0, -1.1, cb) == pytest.approx((-0.5 + 1.1) / 0.2)
    assert oracle.certified_margin(1.0, 0.1, cb) == -np.inf      # theta below the mean's upper bound
    assert oracle.certified_margin(-1.0, 0.1, cb) == -np.inf
    assert oracle.certified_margin(1.0, 0.6, [0.0, -0.5, 0.2, 0.0]) == np.inf


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_certified_octree_contains_search_leaves_and_skips_only_safe_nodes(kind):
    W = small(140 + kind, 3, 15, 17, kind=kind, ell=0.4, signal_var=0.05, noise_var=1e-3)
    W.zbank = np.random.default_rng(141).standard_normal((3000, 8))
    M = oracle.fit(W)
    W.theta = float(np.quantile(oracle.grid_posterior(M, W)[0], 0.95))
    ls, _, _ = oracle.adaptive(M, W, min_leaf=2)
    lc, skipped, recs = oracle.adaptive(M, W, min_leaf=2, bound_kind=oracle.BOUND_CERTIFIED)
    assert set(ls.tolist()) <= set(lc.tolist())
    assert len(lc) < 4096 // 8
    assert np.all(np.isnan(recs["lattice_gap"]))
    # every cell of a skipped node has smooth LCP <= alpha (up to the estimator's error)
    lcp = oracle.lcp_sov_dense(M, W)
    S0, _ = oracle.octree_shape(W, 2)
    from test_oracle_pins import _decode
    n_checked = 0
    for key in skipped.tolist():
        lvl = key >> 58
        c = _decode(key, 3)
        s = S0 >> lvl
        sl = tuple(slice(c[d] * s, min((c[d] + 1) * s, 16)) for d in (2, 1, 0))
        if lcp[sl].size:
            n_checked += lcp[sl].size
            assert lcp[sl].max() <= W.alpha + 5e-4
    assert n_checked > 100
