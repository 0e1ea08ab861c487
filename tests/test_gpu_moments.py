"""Corner moments of listed cells (lcp_cell_moments) against the oracle's cell moments.

The call runs the same posterior and cross-covariance kernels as lcp_dense and
lcp_adaptive, so this checks rows a1-a5 cell by cell rather than through Monte Carlo
counts.  Tolerances: binary64 mean 1e-9 and covariance 1e-10 absolute (s2 <= 1, as the
posterior parity tests); the split 16-bit product carries about 22 bits of V, so the
covariances are held to 2e-5 s2 and the means to the binary32 kernel-value bound.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2512_12442_amd as lcp
from parity_util import DEV, gpu_model, mean_error_bound32, say

pytestmark = pytest.mark.gpu


def _cells(W, n, seed):
    nc = int(np.prod(W.npts[: W.dim] - 1))
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.integers(0, nc, n), [0, nc - 1]]))


def _oracle_moments(M, W, cells):
    shape = [int(v) - 1 for v in W.npts[: W.dim]]
    mus, covs = [], []
    for e in cells:
        c, r = [], int(e)
        for d in range(W.dim):
            c.append(r % shape[d])
            r //= shape[d]
        mu, S = oracle.cell_moments(M, W, tuple(c))
        mus.append(mu)
        covs.append(S)
    return np.array(mus), np.array(covs)


@pytest.mark.parametrize("name", ["trig17", "cfg1_2d", "ragged"])
def test_cell_moments_fp64_match_oracle(name):
    W = {"trig17": lambda: workloads.field3d_trig(0, m=120, npts=17),
         "cfg1_2d": lambda: workloads.make("cfg1_2d"),
         "ragged": lambda: _ragged()}[name]()
    say(f"cell moments fp64 {name}")
    M = oracle.fit(W)
    cells = _cells(W, 300, 1)
    mu_ref, cov_ref = _oracle_moments(M, W, cells)
    G = gpu_model(W)
    mu, cov = G.cell_moments(lcp.grid_of(W), torch.as_tensor(cells, device=DEV), "fp64")
    mu, cov = mu.cpu().numpy(), cov.cpu().numpy()
    say(f"  {len(cells)} cells: max|dmu|={np.abs(mu - mu_ref).max():.2e} max|dcov|={np.abs(cov - cov_ref).max():.2e}")
    assert np.abs(mu - mu_ref).max() <= 1e-9 * max(1.0, np.abs(mu_ref).max())
    assert np.abs(cov - cov_ref).max() <= 1e-10
    assert np.array_equal(cov, np.swapaxes(cov, 1, 2))


def test_cell_moments_fp64_top_layer_96cube():
    """Every cell of the top z-layer of a 96^3-vertex grid against the oracle.  The
    cross-covariance launch deals tiles of x-lines to the eight XCDs; at this size an XCD's
    run count is not a multiple of the work-group's four waves, and the runs that end each
    XCD's sequence own the vertices of the top planes (a launch that stopped at the last
    whole work-group once left some of them unwritten)."""
    W = workloads.field3d_trig(0, m=60, npts=96)
    say("cell moments fp64 96^3 top layer")
    M = oracle.fit(W)
    n = 95
    cells = np.arange(n * n) + (n - 1) * n * n
    mu_ref, cov_ref = _oracle_moments(M, W, cells)
    G = gpu_model(W)
    mu, cov = G.cell_moments(lcp.grid_of(W), torch.as_tensor(cells, device=DEV), "fp64")
    mu, cov = mu.cpu().numpy(), cov.cpu().numpy()
    say(f"  {len(cells)} cells: max|dmu|={np.abs(mu - mu_ref).max():.2e} max|dcov|={np.abs(cov - cov_ref).max():.2e}")
    assert np.abs(mu - mu_ref).max() <= 1e-9 * max(1.0, np.abs(mu_ref).max())
    assert np.abs(cov - cov_ref).max() <= 1e-10


def _ragged():
    W = workloads.field3d_trig(2, m=77, npts=13)
    W.npts[:] = [13, 9, 7]
    return W


@pytest.mark.parametrize("prec", ["f16x3", "fp32"])
def test_cell_moments_reduced_precision_error(prec):
    W = workloads.field3d_trig(0, m=500, npts=33)
    say(f"cell moments {prec} trig33 m=500")
    M = oracle.fit(W)
    cells = _cells(W, 250, 2)
    mu_ref, cov_ref = _oracle_moments(M, W, cells)
    G = gpu_model(W)
    mu, cov = G.cell_moments(lcp.grid_of(W), torch.as_tensor(cells, device=DEV), prec)
    mu, cov = mu.cpu().numpy(), cov.cpu().numpy()
    shape = [int(v) - 1 for v in W.npts[:3]]
    h = [(float(W.hi[d]) - float(W.lo[d])) / (int(W.npts[d]) - 1) for d in range(3)]
    P = []
    for e in cells:
        c = [int(e) % shape[0], (int(e) // shape[0]) % shape[1], int(e) // (shape[0] * shape[1])]
        for q in range(8):
            v = [c[0] + (q & 1), c[1] + ((q >> 1) & 1), c[2] + ((q >> 2) & 1)]
            P.append([float(W.lo[d]) + v[d] * h[d] for d in range(3)])
    bound = mean_error_bound32(W, M, np.array(P)).reshape(mu.shape)
    dmu, dcov = np.abs(mu - mu_ref), np.abs(cov - cov_ref)
    say(f"  max|dmu|={dmu.max():.2e} (bound {bound.max():.2e}) max|dcov|={dcov.max():.2e} (s2 {W.signal_var})")
    assert (dmu <= bound).all()
    assert dcov.max() <= 2e-5 * W.signal_var


def test_cell_moments_out_of_range_cells_are_nan():
    W = workloads.field3d_trig(0, m=60, npts=9)
    G = gpu_model(W)
    nc = 8 ** 3
    cells = torch.as_tensor([-1, 0, nc - 1, nc, 1 << 40], dtype=torch.int64, device=DEV)
    mu, cov = G.cell_moments(lcp.grid_of(W), cells, "fp64")
    mu, cov = mu.cpu().numpy(), cov.cpu().numpy()
    bad = [0, 3, 4]
    assert np.isnan(mu[bad]).all() and np.isnan(cov[bad]).all()
    assert np.isfinite(mu[[1, 2]]).all() and np.isfinite(cov[[1, 2]]).all()
