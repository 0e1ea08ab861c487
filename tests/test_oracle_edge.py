"""Pins of the oracle's edge-crossing region bound (Sec. 9's tighter bound from edge
crossings, built here as a union bound over a spanning tree of a node's grid vertices).

What fixes each part, independently of the oracle:
  * the edge term against Sheppard's orthant formula (means at theta), the independent
    product form (rho = 0), scipy's bivariate normal CDF, the rank-1 limits and bivariate
    Monte Carlo;
  * the spanning tree through a prior-only node, where every edge term is Sheppard's value
    and the bound is (vertices - 1) times it;
  * the bound against brute-force joint sampling of a node's vertices (P(node crossed)) and
    against the cell LCPs inside it;
  * the octree option: it only removes deepest-level nodes whose bound is <= alpha, and the
    cells of those nodes have dense LCP within that bound.  CPU only.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads


def _ref_cross(mua, mub, va, vb, c, th):
    both = stats.multivariate_normal(mean=[mua, mub], cov=[[va, c], [c, vb]]).cdf([th, th])
    return stats.norm.cdf((th - mua) / math.sqrt(va)) + stats.norm.cdf((th - mub) / math.sqrt(vb)) - 2 * both


@pytest.mark.parametrize("rho", [0.0, 0.3, -0.5, 0.9, 0.997, 0.999999, -0.999999])
def test_edge_term_sheppard(rho):
    # both means at theta: P(crossed) = 1 - 2 (1/4 + asin(rho) / (2 pi)) = 1/2 - asin(rho) / pi
    va, vb = 0.7, 1.9
    p = oracle.edge_cross(0.25, 0.25, va, vb, rho * math.sqrt(va * vb), 0.25)
    # rho itself is rounded (c / (sa sb)); d/drho of the value is 1 / (pi sqrt(1 - rho^2))
    assert abs(p - (0.5 - math.asin(rho) / math.pi)) <= 1e-15 / math.sqrt(1 - rho * rho) + 1e-15


def test_edge_term_independent_and_scipy():
    rng = np.random.default_rng(5)
    for _ in range(60):
        mua, mub, th = rng.normal(0, 1.5, 3)
        va, vb = rng.uniform(0.05, 2.0, 2)
        h, k = (th - mua) / math.sqrt(va), (th - mub) / math.sqrt(vb)
        ph, pk = stats.norm.cdf(h), stats.norm.cdf(k)
        assert abs(oracle.edge_cross(mua, mub, va, vb, 0.0, th) - (ph + pk - 2 * ph * pk)) <= 1e-14
        rho = rng.uniform(-0.995, 0.995)
        c = rho * math.sqrt(va * vb)
        assert abs(oracle.edge_cross(mua, mub, va, vb, c, th) - _ref_cross(mua, mub, va, vb, c, th)) <= 1e-8


def test_edge_term_high_correlation_and_rank_one_limits():
    # near rho = 1 the term tends to |Phi(h) - Phi(k)| (the values move together), continuously
    va, vb, th = 0.5, 0.8, 0.1
    for mua, mub in [(0.0, 0.3), (0.2, -0.4), (0.1, 0.1), (1.5, 1.7)]:
        h, k = (th - mua) / math.sqrt(va), (th - mub) / math.sqrt(vb)
        lim = abs(stats.norm.cdf(h) - stats.norm.cdf(k))
        assert abs(oracle.edge_cross(mua, mub, va, vb, math.sqrt(va * vb), th) - lim) <= 1e-15
        near = oracle.edge_cross(mua, mub, va, vb, (1 - 1e-10) * math.sqrt(va * vb), th)
        assert abs(near - lim) <= 1e-4
        limm = 1 - abs(stats.norm.cdf(h) - stats.norm.cdf(-k))
        assert abs(oracle.edge_cross(mua, mub, va, vb, -math.sqrt(va * vb), th) - limm) <= 1e-15
        nearm = oracle.edge_cross(mua, mub, va, vb, -(1 - 1e-10) * math.sqrt(va * vb), th)
        assert abs(nearm - limm) <= 1e-4


def test_edge_term_degenerate_ends():
    # a zero-variance end is a constant: crossed unless the random end falls on its side
    assert oracle.edge_cross(0.0, 1.0, 0.0, 0.0, 0.0, 0.5) == 1.0
    assert oracle.edge_cross(0.0, 0.2, 0.0, 0.0, 0.0, 0.5) == 0.0
    assert oracle.edge_cross(0.5, 0.0, 0.0, 0.0, 0.0, 0.5) == 1.0          # a tie counts as crossed
    p = oracle.edge_cross(0.0, 1.0, 0.0, 0.25, 0.0, 0.5)
    assert abs(p - stats.norm.sf((0.5 - 1.0) / 0.5)) <= 1e-15
    p = oracle.edge_cross(2.0, 1.0, 0.25, 0.0, 0.0, 0.5)
    assert abs(p - stats.norm.cdf((0.5 - 2.0) / 0.5)) <= 1e-15


def test_edge_term_bivariate_monte_carlo():
    rng = np.random.default_rng(7)
    for _ in range(5):
        mua, mub = rng.normal(0, 0.5, 2)
        va, vb = rng.uniform(0.3, 1.0, 2)
        c = rng.uniform(0.5, 0.98) * math.sqrt(va * vb)
        th = 0.0
        z = rng.multivariate_normal([mua, mub], [[va, c], [c, vb]], size=400000)
        emp = np.mean(~((z < th).all(1) | (z > th).all(1)))
        p = oracle.edge_cross(mua, mub, va, vb, c, th)
        assert abs(emp - p) <= 4 * math.sqrt(p * (1 - p) / len(z)) + 1e-6


def test_tree_through_a_prior_only_node():
    # observations far away: the node sees the prior (mean 0, variance s2); with theta = 0
    # every edge term is Sheppard's 1/2 - asin(rho_h) / pi with rho_h = k(h) / s2, so the
    # bound is (vertices - 1) times it: the tree has exactly vertices - 1 edges
    for dim, n in [(3, 7), (2, 9)]:
        W = workloads.random_small(1, dim, 5, n, signal_var=0.8, ell=0.4)
        W.X = W.X + 50.0
        W.theta = 0.0
        M = oracle.fit(W)
        h = 1.0 / (n - 1)
        rho = oracle.kernel(W.kind, dim, W.signal_var, W.lengthscale, np.zeros(dim),
                            np.array([h] + [0.0] * (dim - 1))) / W.signal_var
        for vlo, vhi in [([0] * dim, [2] * dim), ([1] * dim, [4] * dim), ([0] * dim, [n - 1] * dim)]:
            nv = int(np.prod(np.array(vhi) - np.array(vlo) + 1))
            eb = oracle.node_edge_bound(M, W, vlo, vhi)
            assert abs(eb - (nv - 1) * (0.5 - math.asin(rho) / math.pi)) <= 1e-12 * nv


def _node_joint(M, W, vlo, vhi):
    """Joint posterior mean and covariance of a node's vertices (x fastest), from the
    oracle's cell moments of its cells (each covariance entry between two vertices that
    share a cell; the node here is one cell or a line of cells in each direction)."""
    idx = [np.arange(vlo[d], vhi[d] + 1) for d in range(W.dim)]
    pts = np.stack(np.meshgrid(*idx, indexing="ij"), -1).reshape(-1, W.dim)
    pts = pts[np.lexsort(pts.T[::1])] if W.dim == 2 else pts[np.lexsort((pts[:, 0], pts[:, 1], pts[:, 2]))]
    h = [(W.hi[d] - W.lo[d]) / (W.npts[d] - 1) for d in range(W.dim)]
    P = np.array([[W.lo[d] + p[d] * h[d] for d in range(W.dim)] for p in pts])
    mu, var, V = oracle.posterior(M, P, want_v=True)
    K = np.array([[oracle.kernel(W.kind, W.dim, W.signal_var, W.lengthscale, a, b) for b in P] for a in P])
    return mu, K - V @ V.T


def test_node_bound_dominates_joint_sampling_and_cells():
    W = workloads.random_small(4, 3, 30, 9, ell=0.3, noise_var=1e-3)
    M = oracle.fit(W)
    rng = np.random.default_rng(11)
    mu_all, _ = oracle.posterior(M, np.array([[0.5, 0.5, 0.5]]))
    for vlo, vhi in [([1, 1, 1], [3, 3, 3]), ([4, 2, 5], [6, 4, 7]), ([0, 0, 0], [2, 2, 2])]:
        mu, S = _node_joint(M, W, vlo, vhi)
        for theta in [float(np.median(mu)), float(mu.max()) + 0.05, float(mu.min()) - 0.3]:
            W.theta = theta
            eb = oracle.node_edge_bound(M, W, vlo, vhi)
            evals, evecs = np.linalg.eigh(S)
            Z = rng.standard_normal((200000, len(mu))) @ (evecs * np.sqrt(np.maximum(evals, 0))).T + mu
            crossed = ~((Z < theta).all(1) | (Z > theta).all(1))
            p = crossed.mean()
            assert eb >= p - 4 * math.sqrt(max(p * (1 - p), 1e-12) / len(Z)) - 1e-6
            # and every cell of the node (a cell is crossed only if the node is)
            for cz in range(vlo[2], vhi[2]):
                for cy in range(vlo[1], vhi[1]):
                    for cx in range(vlo[0], vhi[0]):
                        mc, Sc = oracle.cell_moments(M, W, (cx, cy, cz))
                        l = oracle.cell_lcp(mc, Sc, theta, W.zbank)
                        assert l <= eb + 4 * math.sqrt(max(eb * (1 - eb), 1e-12) / W.n_samples) + 1.0 / W.n_samples


def test_octree_with_edge_bound():
    W = workloads.field3d_trig(0, m=200, npts=33)
    M = oracle.fit(W)
    leaves0, _, _ = oracle.adaptive(M, W)
    leaves1, _, recs = oracle.adaptive(M, W, edge_bound=1)
    assert set(leaves1.tolist()) <= set(leaves0.tolist())
    ev = recs[~np.isnan(recs["eb"])]
    assert len(ev) == len(leaves0)           # every node the region test emits gets the bound
    assert (ev["subdivide"] == (ev["eb"] > W.alpha)).all()
    assert (ev["ub"] > W.alpha).all() or (ev["path"] == 0).any()
    removed = set(leaves0.tolist()) - set(leaves1.tolist())
    print(f"edge bound: {len(leaves0)} -> {len(leaves1)} leaves")
    assert len(removed) > 0
    # the cells of every removed node: dense LCP within the node's bound (<= alpha) + MC slack
    dense = oracle.lcp_dense(M, W).reshape(-1)
    nc = [int(v) - 1 for v in W.npts[:3]]
    S0, Lmax = oracle.octree_shape(W)
    edge = S0 >> Lmax
    ebs = {int(r["key"]): r["eb"] for r in ev}
    for key in removed:
        mc = key & ((1 << 58) - 1)
        c = [0, 0, 0]
        for b in range(Lmax):
            for d in range(3):
                c[d] |= ((mc >> (3 * b + d)) & 1) << b
        for cz in range(c[2] * edge, min((c[2] + 1) * edge, nc[2])):
            for cy in range(c[1] * edge, min((c[1] + 1) * edge, nc[1])):
                for cx in range(c[0] * edge, min((c[0] + 1) * edge, nc[0])):
                    assert dense[cx + nc[0] * (cy + nc[1] * cz)] <= ebs[key] + 4 * math.sqrt(W.alpha / 1600) + 1 / 1600


def _uv_cross(mua, mub, va, vb, c, th):
    """The edge term by another decomposition: Za = a U + b V, Zb = a U - b V with U, V
    independent, so for fixed V = v the edge is crossed when U lies between (h - b v) / a and
    (k + b v) / a; integrated with scipy's adaptive quadrature on either side of the kink."""
    from scipy import integrate
    sa, sb = math.sqrt(va), math.sqrt(vb)
    h, k = (th - mua) / sa, (th - mub) / sb
    rho = c / (sa * sb)
    flip = rho < 0
    if flip:
        rho, k = -rho, -k
    a, b = math.sqrt((1 + rho) / 2), math.sqrt((1 - rho) / 2)
    f = lambda v: stats.norm.pdf(v) * abs(stats.norm.cdf((h - b * v) / a) - stats.norm.cdf((k + b * v) / a))
    vs = (h - k) / (2 * b)
    pts = [-12.0] + ([vs] if -12 < vs < 12 else []) + [12.0]
    p = sum(integrate.quad(f, lo, hi, epsabs=1e-14, epsrel=1e-12, limit=200)[0] for lo, hi in zip(pts[:-1], pts[1:]))
    return 1 - p if flip else p


def test_edge_term_matches_independent_decomposition():
    rng = np.random.default_rng(13)
    for _ in range(80):
        mua, mub = rng.normal(0, 2, 2)
        va, vb = rng.uniform(0.02, 2, 2)
        r = [rng.uniform(-0.99, 0.99), 1 - 10 ** rng.uniform(-9, -1)][rng.integers(0, 2)]
        c = r * math.sqrt(va * vb)
        th = rng.normal(0, 2)
        assert abs(oracle.edge_cross(mua, mub, va, vb, c, th) - _uv_cross(mua, mub, va, vb, c, th)) <= 1e-9
