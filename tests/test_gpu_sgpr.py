"""Parity of the sparse model of eq. (sgp) (gp_fit_sgpr) with the FP64 CPU oracle.

The library folds the third term of eq. (sgp) into its stored factor (T = F L^-1 with
E = I - L^-1 A_M L^-T = F^T F); the oracle evaluates the three terms as printed.  The two
share no arithmetic, so agreement checks the fold.  Tolerances as in test_gpu_parity,
plus the documented shift: a variance may rise by shift * s2 when E had to be shifted.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2512_12442_amd as lcp
from parity_util import DEV, compare_adaptive, counts, near_tie_keys, say, zbank

pytestmark = pytest.mark.gpu


def _ragged():
    W = workloads.sgpr_field(5, m=64, npts=21, train_npts=14, ell=0.2)
    W.npts[:] = [21, 17, 13]
    return W


CASES = {
    "sgpr27_17": lambda: workloads.sgpr_field(3, m=27, npts=17, train_npts=12, ell=0.3),
    "sgpr64_ragged": _ragged,
    "sgpr125_33": lambda: workloads.sgpr_field(4, m=125, npts=33, train_npts=20, ell=0.15),
}


def gpu_sparse(W):
    return lcp.GPModel.from_workload(W, DEV)


def _se_gram(W, A, B):
    d = (A[:, None, :] - B[None, :, :]) / W.lengthscale[: W.dim]
    return W.signal_var * np.exp(-0.5 * (d * d).sum(-1))


@pytest.mark.parametrize("case", list(CASES) + ["sgpr500"])
def test_sgpr_posterior_fp64_matches_oracle(case):
    W = workloads.sgpr_field(0, m=500, npts=9) if case == "sgpr500" else CASES[case]()
    say(f"sgpr posterior fp64 {case} m={W.m}")
    M = oracle.fit(W)
    P = np.random.default_rng(6).random((1500, 3))
    mu_ref, var_ref = oracle.posterior(M, P)
    G = gpu_sparse(W)
    mu, var = G.posterior(torch.as_tensor(P, device=DEV), "fp64")
    mu, var = mu.cpu().numpy(), var.cpu().numpy()
    say(f"  shift={G.shift:.1e} max|dmu|={np.abs(mu - mu_ref).max():.2e} max|dvar|={np.abs(var - var_ref).max():.2e}")
    assert np.abs(mu - mu_ref).max() <= 1e-9 * max(1.0, np.abs(mu_ref).max())
    assert np.abs(var - var_ref).max() <= 1e-10 + G.shift * W.signal_var


@pytest.mark.parametrize("case", list(CASES))
def test_sgpr_dense_fp64_matches_oracle(case):
    W = CASES[case]()
    say(f"sgpr dense fp64 {case} npts={W.npts} m={W.m}")
    M = oracle.fit(W)
    ref = oracle.lcp_dense(M, W).reshape(-1)
    G = gpu_sparse(W)
    out, _ = G.lcp_dense(lcp.grid_of(W), W.theta, zbank(W), "fp64")
    got = out.cpu().numpy()
    dc = counts(got, W.n_samples) - counts(ref, W.n_samples)
    say(f"  cells={ref.size} nonzero={np.count_nonzero(ref)} mismatched={np.count_nonzero(dc)}")
    assert np.count_nonzero(ref) > 0
    assert np.count_nonzero(dc) == 0


@pytest.mark.parametrize("prec", ["fp32", "f16x3"])
@pytest.mark.parametrize("case", ["sgpr27_17", "sgpr125_33"])
def test_sgpr_dense_mixed_rmse(case, prec):
    W = CASES[case]()
    M = oracle.fit(W)
    ref = oracle.lcp_dense(M, W).reshape(-1)
    G = gpu_sparse(W)
    out, _ = G.lcp_dense(lcp.grid_of(W), W.theta, zbank(W), prec)
    d = out.cpu().numpy() - ref
    rmse = float(np.sqrt(np.mean(d * d)))
    say(f"sgpr dense {prec} {case}: rmse={rmse:.2e} max={np.abs(d).max():.2e}")
    assert rmse <= 1e-4


@pytest.mark.parametrize("case", list(CASES))
def test_sgpr_adaptive_fp64_matches_oracle(case):
    W = CASES[case]()
    W.min_leaf = 2 if case == "sgpr27_17" else 4
    say(f"sgpr adaptive fp64 {case} npts={W.npts} m={W.m} min_leaf={W.min_leaf}")
    M = oracle.fit(W)
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W)
    G = gpu_sparse(W)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, lcp.adapt_of(W), zbank(W), "fp64")
    n = int(nl.item())
    got = leaves[:n].cpu().numpy().astype(np.uint64)
    ties = near_tie_keys(recs, W.alpha)
    assert len(leaves_ref) > 0 and len(skipped_ref) > 0
    sym, excused = compare_adaptive(W, M, out.cpu().numpy(), got, lf.cpu().numpy(), leaves_ref, skipped_ref, ties)
    say(f"  leaves gpu={n} oracle={len(leaves_ref)} skipped={len(skipped_ref)} differ={len(sym)} "
        f"near-ties={len(ties)} excused cells={int(excused.sum())}")


def test_sgpr_with_inducing_set_equal_to_data_equals_exact_gp_path():
    """Sec. 3: M = X, mu_M = K (K + s_n^2 I)^-1 y, A_M = K - K (K + s_n^2 I)^-1 K gives the
    exact GP; the sparse and exact library paths must agree."""
    W = workloads.random_small(7, 3, 60, 4, ell=0.3, signal_var=0.8, noise_var=1e-2)
    K = _se_gram(W, W.X, W.X)
    Kn = K + W.noise_var * np.eye(W.m)
    mu_M = K @ np.linalg.solve(Kn, W.y)
    A_M = K - K @ np.linalg.solve(Kn, K)
    A_M = 0.5 * (A_M + A_M.T)
    X = torch.as_tensor(W.X, device=DEV)
    S = lcp.GPModel(W.kind, 3, W.signal_var, list(W.lengthscale), 0.0, X, torch.as_tensor(mu_M, device=DEV),
                    torch.as_tensor(A_M, device=DEV))
    E = lcp.GPModel.from_workload(W, DEV)
    P = torch.as_tensor(np.random.default_rng(8).random((700, 3)), device=DEV)
    (ms, vs), (me, ve) = S.posterior(P, "fp64"), E.posterior(P, "fp64")
    say(f"identity: shift={S.shift:.1e} max|dmu|={(ms - me).abs().max().item():.2e} "
        f"max|dvar|={(vs - ve).abs().max().item():.2e}")
    assert (ms - me).abs().max().item() <= 1e-8
    assert (vs - ve).abs().max().item() <= 1e-9 + S.shift * W.signal_var


def test_sgpr_prior_covariance_is_shifted_and_gives_the_prior():
    """A_M = K_MM + jitter I makes E = 0: the fit shifts it and the variance is s2."""
    W = workloads.random_small(9, 3, 40, 4, ell=0.3, signal_var=0.6)
    jit = 1e-4
    A = _se_gram(W, W.X, W.X) + jit * np.eye(W.m)
    S = lcp.GPModel(W.kind, 3, W.signal_var, list(W.lengthscale), jit, torch.as_tensor(W.X, device=DEV),
                    torch.as_tensor(W.y, device=DEV), torch.as_tensor(A, device=DEV))
    _, var = S.posterior(torch.as_tensor(np.random.default_rng(10).random((300, 3)), device=DEV), "fp64")
    say(f"prior: shift={S.shift:.1e} max|var - s2|={(var - W.signal_var).abs().max().item():.2e}")
    assert 0.0 < S.shift <= 1e-6
    assert (var - W.signal_var).abs().max().item() <= S.shift * W.signal_var + 1e-10


def test_sgpr_rejects_inducing_covariance_above_the_prior():
    W = workloads.random_small(11, 3, 30, 4, ell=0.3)
    A = 2.0 * _se_gram(W, W.X, W.X) + 1e-2 * np.eye(W.m)
    with pytest.raises(lcp.LcpError) as e:
        lcp.GPModel(W.kind, 3, W.signal_var, list(W.lengthscale), 1e-6, torch.as_tensor(W.X, device=DEV),
                    torch.as_tensor(W.y, device=DEV), torch.as_tensor(A, device=DEV))
    assert "A_M is not below" in str(e.value)
    X = W.X.copy()
    X[4] = X[2]
    with pytest.raises(lcp.LcpError) as e:
        lcp.GPModel(W.kind, 3, W.signal_var, list(W.lengthscale), 0.0, torch.as_tensor(X, device=DEV),
                    torch.as_tensor(W.y, device=DEV), torch.as_tensor(np.zeros((30, 30)), device=DEV))
    assert "K_MM + jitter I" in str(e.value)


def test_sgpr_single_inducing_point():
    W = workloads.random_small(12, 3, 1, 9, signal_var=1.3)
    jit, mu_M, A = 0.05, np.array([0.7]), np.array([[0.4]])
    S = lcp.GPModel(W.kind, 3, W.signal_var, list(W.lengthscale), jit, torch.as_tensor(W.X, device=DEV),
                    torch.as_tensor(mu_M, device=DEV), torch.as_tensor(A, device=DEV))
    M = oracle.SparseModel(W.kind, 3, W.signal_var, W.lengthscale, jit, W.X, mu_M, A)
    P = np.random.default_rng(13).random((100, 3))
    mu_ref, var_ref = oracle.posterior(M, P)
    mu, var = S.posterior(torch.as_tensor(P, device=DEV), "fp64")
    assert np.abs(mu.cpu().numpy() - mu_ref).max() <= 1e-12
    assert np.abs(var.cpu().numpy() - var_ref).max() <= 1e-12
    W.theta = 0.2
    ref = oracle.lcp_dense(M, W).reshape(-1)
    out, _ = S.lcp_dense(lcp.grid_of(W), W.theta, zbank(W), "fp64")
    assert np.count_nonzero(counts(out.cpu().numpy(), W.n_samples) - counts(ref, W.n_samples)) == 0
