"""Parity of the posterior adjoint (gp_posterior_backward) with the FP64 oracle's adjoint.

The library forms W = K^-1 K*^T on MFMA and reduces dL/dlog(ell) through the rank-n
product G = sum_p h_p w_p w_p^T; the oracle takes the printed per-point derivatives.
Tolerances:
  * binary64: 1e-8 relative to the largest component (the two routes sum the same terms
    in different orders and forms; the terms carry cond(K) eps relative error);
  * binary32 W: 1e-3 relative.  W = K^-1 k* in binary32 carries up to cond(K) 2^-24
    relative error per entry; these models have cond(K) of about 1e6, and the sums of the
    adjoint reach 8e-4 (SE) and 1e-4 (Matern-5/2).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2512_12442_amd as lcp
from parity_util import DEV, say

pytestmark = pytest.mark.gpu


def _case(kind, dim, m, seed=60):
    W = workloads.random_small(seed, dim, m, 4, kind=kind, ell=0.2, signal_var=0.7, noise_var=1e-4)
    W.lengthscale[:dim] = [0.18, 0.25, 0.22][:dim]
    return W


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("kind,dim,m,n", [(workloads.SE, 3, 37, 1000), (workloads.MATERN52, 3, 200, 4097),
                                          (workloads.SE, 2, 50, 333), (workloads.MATERN52, 3, 1, 64),
                                          (workloads.SE, 3, 700, 300)])
def test_posterior_backward_fp64_matches_oracle(kind, dim, m, n):
    say(f"posterior backward fp64 kind={kind} dim={dim} m={m} n={n}")
    W = _case(kind, dim, m)
    rng = np.random.default_rng(61)
    P = rng.random((n, dim))
    gm, gv = rng.standard_normal(n), rng.standard_normal(n)
    dy_ref, dl_ref = oracle.posterior_backward(oracle.fit(W), P, gm, gv)
    G = lcp.GPModel.from_workload(W, DEV)
    t = lambda a: torch.as_tensor(a, device=DEV)
    dy, dl = G.posterior_backward(t(P), t(gm), t(gv), "fp64")
    dy, dl = dy.cpu().numpy(), dl.cpu().numpy()
    say(f"  rel dy={_rel(dy, dy_ref):.2e} rel dlogell={_rel(dl, dl_ref):.2e}  dlogell={dl}")
    assert _rel(dy, dy_ref) <= 1e-8
    assert _rel(dl, dl_ref) <= 1e-8


@pytest.mark.parametrize("kind", [workloads.SE, workloads.MATERN52])
def test_posterior_backward_fp32_error(kind):
    W = _case(kind, 3, 300, seed=62)
    rng = np.random.default_rng(63)
    P = rng.random((2000, 3))
    gm, gv = rng.standard_normal(2000), rng.standard_normal(2000)
    dy_ref, dl_ref = oracle.posterior_backward(oracle.fit(W), P, gm, gv)
    G = lcp.GPModel.from_workload(W, DEV)
    t = lambda a: torch.as_tensor(a, device=DEV)
    dy, dl = G.posterior_backward(t(P), t(gm), t(gv), "fp32")
    dy, dl = dy.cpu().numpy(), dl.cpu().numpy()
    say(f"posterior backward fp32 kind={kind}: rel dy={_rel(dy, dy_ref):.2e} rel dlogell={_rel(dl, dl_ref):.2e}")
    # measured 7.9e-4 / 3.7e-4 (SE) and 5.9e-5 / 1.1e-4 (Matern): binary32 W of an
    # ill-conditioned K; the binary64 path is held to 1e-8 above
    assert _rel(dy, dy_ref) <= 1e-3
    assert _rel(dl, dl_ref) <= 1e-3


def test_posterior_backward_partial_upstreams_and_empty():
    W = _case(workloads.SE, 3, 90)
    rng = np.random.default_rng(64)
    P = rng.random((500, 3))
    gm, gv = rng.standard_normal(500), rng.standard_normal(500)
    M = oracle.fit(W)
    G = lcp.GPModel.from_workload(W, DEV)
    t = lambda a: torch.as_tensor(a, device=DEV)
    for a, b in ((gm, None), (None, gv), (None, None)):
        dy_ref, dl_ref = oracle.posterior_backward(M, P, a, b)
        dy, dl = G.posterior_backward(t(P), None if a is None else t(a), None if b is None else t(b), "fp64")
        assert np.allclose(dy.cpu().numpy(), dy_ref, rtol=0, atol=1e-8 * max(1.0, np.abs(dy_ref).max()))
        assert np.allclose(dl.cpu().numpy(), dl_ref, rtol=0, atol=1e-8 * max(1.0, np.abs(dl_ref).max()))
        if a is None:   # the variance does not involve y: no value gradient at all
            assert float(dy.abs().max()) == 0.0
    dy, dl = G.posterior_backward(torch.zeros((0, 3), dtype=torch.float64, device=DEV), None, None, "fp64")
    assert float(dy.abs().max()) == 0.0 and float(dl.abs().max()) == 0.0


def test_posterior_backward_is_deterministic():
    W = _case(workloads.MATERN52, 3, 150)
    P = torch.as_tensor(np.random.default_rng(65).random((5000, 3)), device=DEV)
    g = torch.as_tensor(np.random.default_rng(66).standard_normal(5000), device=DEV)
    G = lcp.GPModel.from_workload(W, DEV)
    a = G.posterior_backward(P, g, g, "fp32")
    b = G.posterior_backward(P, g, g, "fp32")
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_autograd_function_matches_gpu_finite_differences():
    """torch.autograd through posterior_fn against central differences of the GPU forward
    (re-fitted at each perturbed input, binary64, h = 1e-6)."""
    W = _case(workloads.SE, 3, 25, seed=67)
    X = torch.as_tensor(W.X, device=DEV)
    P = torch.as_tensor(np.random.default_rng(68).random((200, 3)), device=DEV)
    w1 = torch.as_tensor(np.random.default_rng(69).standard_normal(200), device=DEV)
    w2 = torch.as_tensor(np.random.default_rng(70).standard_normal(200), device=DEV)

    def loss(y, log_ell):
        mean, var = lcp.posterior_fn(y, log_ell, X, P, W.kind, W.signal_var, W.noise_var, "fp64")
        return (w1 * mean).sum() + (w2 * var).sum()

    y = torch.as_tensor(W.y, device=DEV).requires_grad_(True)
    log_ell = torch.log(torch.as_tensor(W.lengthscale[:3], device=DEV)).requires_grad_(True)
    loss(y, log_ell).backward()
    h = 1e-6
    with torch.no_grad():
        for j in (0, 7, 24):
            e = torch.zeros_like(y)
            e[j] = h
            fd = (loss(y + e, log_ell) - loss(y - e, log_ell)).item() / (2 * h)
            assert abs(y.grad[j].item() - fd) <= 1e-6 * max(1.0, abs(fd))
        for d in range(3):
            e = torch.zeros_like(log_ell)
            e[d] = h
            fd = (loss(y, log_ell + e) - loss(y, log_ell - e)).item() / (2 * h)
            say(f"autograd d={d}: {log_ell.grad[d].item():.9e} fd {fd:.9e}")
            assert abs(log_ell.grad[d].item() - fd) <= 1e-6 * max(1.0, abs(fd))


def test_posterior_backward_rejects_sparse_models():
    W = workloads.sgpr_field(71, m=27, npts=9, train_npts=10, ell=0.3)
    G = lcp.GPModel.from_workload(W, DEV)
    with pytest.raises(lcp.LcpError) as e:
        G.posterior_backward(torch.zeros((4, 3), dtype=torch.float64, device=DEV), None, None, "fp64")
    assert "gp_fit_sgpr" in str(e.value)
