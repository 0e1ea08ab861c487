"""Monte Carlo counts of the reduced-precision 3D paths against an exact bracket.

The 3D reduced-precision paths evaluate each sample's corner values y = mu - theta + C z
on the matrix cores as split FP16 products with binary32 accumulation, so a sample can be
classified differently from binary64 only where some corner value lies within the
rounding of that evaluation: below about 2^-20 (|mu_q - theta| + sum_r |C_qr| |z_r|) for
corner q.  This test takes the cell moments exactly as the LCP kernels compute them
(lcp_cell_moments at the same precision, same posterior and cross-covariance kernels),
factors them in binary64 (lower Cholesky, the factor the kernel uses) and, with margin
m_q = 2^-18 (|mu_q - theta| + sum_r |C_qr| |z_r|), counts the samples that are crossed
under every perturbation within the margins (some corner below -m_q, another above +m_q)
and those crossed under some perturbation.  The kernel's count must lie between the two,
for sample counts that leave a ragged last block of 32.
"""
import numpy as np
import pytest
import torch

import workloads
import paper_2512_12442_amd as lcp
from parity_util import DEV, gpu_model, say

pytestmark = pytest.mark.gpu


def _chol_sd(S):
    """Semidefinite lower Cholesky of a batch of symmetric matrices: a pivot at or below
    1e-12 of the largest diagonal entry gives a zero column (binary64)."""
    n = S.shape[-1]
    C = np.zeros_like(S)
    tol = 1e-12 * np.max(np.diagonal(S, axis1=1, axis2=2), axis=1)
    for k in range(n):
        d = S[:, k, k] - np.sum(C[:, k, :k] ** 2, axis=1)
        keep = d > tol
        ckk = np.where(keep, np.sqrt(np.where(keep, d, 1.0)), 0.0)
        inv = np.where(keep, 1.0 / np.where(keep, ckk, 1.0), 0.0)
        C[:, k, k] = ckk
        for i in range(k + 1, n):
            C[:, i, k] = (S[:, i, k] - np.sum(C[:, i, :k] * C[:, k, :k], axis=1)) * inv
    return C


def _bracket(mu, C, z, theta, rel=2.0 ** -18, chunk=256):
    """Per cell: (samples surely crossed, samples possibly crossed)."""
    lo = np.zeros(mu.shape[0], np.int64)
    hi = np.zeros(mu.shape[0], np.int64)
    for a in range(0, mu.shape[0], chunk):
        m = mu[a:a + chunk] - theta                                   # (c, 8)
        Cc = C[a:a + chunk]                                           # (c, 8, 8)
        y = m[:, None, :] + np.einsum("cqr,sr->csq", Cc, z)           # (c, s, 8)
        mag = np.abs(m)[:, None, :] + np.einsum("cqr,sr->csq", np.abs(Cc), np.abs(z))
        marg = rel * mag
        surely_below = (y < -marg).any(axis=2)
        surely_above = (y > marg).any(axis=2)
        maybe_below = (y <= marg).any(axis=2)       # some corner may be <= 0 ... below theta
        maybe_above = (y >= -marg).any(axis=2)
        all_above_sure = (y > marg).all(axis=2)
        all_below_sure = (y < -marg).all(axis=2)
        lo[a:a + chunk] = (surely_below & surely_above).sum(axis=1)
        hi[a:a + chunk] = (~all_above_sure & ~all_below_sure & maybe_below & maybe_above).sum(axis=1)
    return lo, hi


@pytest.mark.parametrize("prec", ["f16x3", "fp32", "bf16x3"])
@pytest.mark.parametrize("ns", [1, 31, 33, 1601])
def test_mc_counts_within_exact_bracket(prec, ns):
    W = workloads.field3d_trig(0, m=120, npts=17, n_samples=ns)
    say(f"mc bracket {prec} ns={ns} npts={list(W.npts)}")
    G = gpu_model(W)
    grid = lcp.grid_of(W)
    zb = torch.as_tensor(W.zbank, device=DEV)
    out, _ = G.lcp_dense(grid, W.theta, zb, prec)
    cnt = np.rint(out.cpu().numpy().astype(np.float64) * ns).astype(np.int64)
    ncell = int(np.prod(W.npts - 1))
    mu, cov = G.cell_moments(grid, torch.arange(ncell, device=DEV), prec)
    mu, cov = mu.cpu().numpy(), cov.cpu().numpy()
    lo, hi = _bracket(mu, _chol_sd(cov), W.zbank, W.theta)
    undecided = int((hi - lo).sum())
    outside = int(((cnt < lo) | (cnt > hi)).sum())
    say(f"  cells={ncell} crossing samples={int(cnt.sum())} undecided samples={undecided} "
        f"cells outside the bracket={outside}")
    assert (lo <= hi).all()
    assert outside == 0
    assert int(cnt.sum()) > 0 if ns > 1 else True
