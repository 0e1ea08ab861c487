"""Parity of the certified region bound (lcp_bound_certified and lcp_adaptive with
LCP_BOUND_CERTIFIED) with the FP64 oracle.

Tolerances: the library forms w = Q k(c) as one binary64 product with Q = L^-T L^-1 (T^T T
for a sparse model) formed explicitly, the oracle by two triangular solves; they agree to
about cond(K) m eps relative to |w|.  The box bounds are compared to 1e-9 of the mean's scale
(|mu(c)| + the bound's spread + s2) and to 1e-7 s2 for the variance.  Leaf sets are compared
exactly, except below nodes whose bound lies within 1e-6 of alpha.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2512_12442_amd as lcp
from parity_util import DEV, compare_adaptive, counts, gpu_model, say, zbank

pytestmark = pytest.mark.gpu


def _models():
    out = []
    for kind in (workloads.SE, workloads.MATERN52):
        W = workloads.random_small(150 + kind, 3, 60, 5, kind=kind, ell=0.3, signal_var=0.5, noise_var=1e-3)
        W.lengthscale[:3] = [0.25, 0.35, 0.3]
        out.append(W)
    out.append(workloads.sgpr_field(152, m=64, npts=5, train_npts=8, ell=0.3))
    out.append(workloads.random_small(153, 2, 45, 5, kind=workloads.SE, ell=0.3, signal_var=0.5, noise_var=1e-3))
    return out


def _boxes(rng, D, n):
    lo = rng.random((n, D)) * 0.8
    width = rng.choice([0.0, 0.01, 0.05, 0.1, 0.3], size=(n, 1)) * rng.random((n, D))
    width[::7, 0] = 0.0                                         # flat boxes
    return np.concatenate([lo, lo + width], axis=1)


@pytest.mark.parametrize("case", range(4))
def test_bound_certified_matches_oracle(case):
    W = _models()[case]
    say(f"certified bound case={case} dim={W.dim} m={W.m} sparse={getattr(W, 'A_M', None) is not None}")
    M = oracle.fit(W)
    rng = np.random.default_rng(160 + case)
    B = _boxes(rng, W.dim, 333)
    ref = np.stack([oracle.bound_certified(M, b[:W.dim], b[W.dim:]) for b in B])
    got = gpu_model(W).bound_certified(torch.as_tensor(B, device=DEV)).cpu().numpy()
    scale = np.abs(ref[:, 0]) + (ref[:, 2] - ref[:, 1]) + W.signal_var
    err_m = (np.abs(got[:, :3] - ref[:, :3]) / scale[:, None]).max()
    err_v = np.abs(got[:, 3] - ref[:, 3]).max() / W.signal_var
    say(f"  max rel err mean bounds {err_m:.2e}, var bound {err_v:.2e}")
    assert err_m <= 1e-9
    assert err_v <= 1e-7
    # the bounds contain the GPU posterior at the box corners and centres, up to the rounding
    # of the mean's sum (m eps sum_i |a_i| s2: the bounds hold in exact arithmetic)
    P = np.concatenate([B[:, :W.dim], B[:, W.dim:], 0.5 * (B[:, :W.dim] + B[:, W.dim:])])
    mean, var = gpu_model(W).posterior(torch.as_tensor(P, device=DEV), "fp64")
    mean, var = mean.cpu().numpy().reshape(3, -1), var.cpu().numpy().reshape(3, -1)
    tol = 1e-12 * scale + 4 * W.m * 2.0 ** -52 * np.abs(M.a).sum() * W.signal_var
    assert np.all(mean >= got[:, 1] - tol) and np.all(mean <= got[:, 2] + tol)
    assert np.all(var <= got[:, 3] + 1e-12 * W.signal_var)


def test_bound_certified_empty_and_single():
    W = _models()[0]
    G = gpu_model(W)
    assert G.bound_certified(torch.zeros((0, 6), dtype=torch.float64, device=DEV)).shape == (0, 4)
    b = np.array([[0.3, 0.3, 0.3, 0.3, 0.3, 0.3]])          # a point box: the bounds are the posterior
    got = G.bound_certified(torch.as_tensor(b, device=DEV)).cpu().numpy()[0]
    mean, var = oracle.posterior(oracle.fit(W), b[:, :3])[:2]
    assert got[1] == got[0] == got[2]
    assert abs(got[0] - mean[0]) <= 1e-12 * (abs(mean[0]) + W.signal_var)
    assert abs(got[3] - var[0]) <= 1e-9 * W.signal_var


def _near(recs, alpha):
    return {int(r["key"]) for r in recs if np.isfinite(r["ub"]) and abs(r["ub"] - alpha) <= 1e-6 * alpha}


def _cases():
    W1 = workloads.field3d_trig(0, m=120, npts=33)
    W2 = workloads.field3d_trig(3, m=150, npts=29)
    W2.npts[:] = [29, 23, 19]
    W2.min_leaf = 2
    W3 = workloads.sgpr_field(154, m=64, npts=17, train_npts=10, ell=0.25)
    W3.min_leaf = 2
    W4 = workloads.random_small(155, 3, 15, 17, kind=workloads.MATERN52, ell=0.4, signal_var=0.05, noise_var=1e-3,
                                min_leaf=2)
    W4.theta = float(np.quantile(oracle.grid_posterior(oracle.fit(W4), W4)[0], 0.95))
    W5 = workloads.make("cfg1_2d")
    W5.min_leaf = 2
    return {"trig33": W1, "ragged": W2, "sgpr17": W3, "matern_q95": W4, "cfg1_2d": W5}


@pytest.mark.parametrize("case", ["trig33", "ragged", "sgpr17", "matern_q95", "cfg1_2d"])
def test_adaptive_certified_matches_oracle(case):
    W = _cases()[case]
    say(f"adaptive certified {case} npts={W.npts} m={W.m} min_leaf={W.min_leaf}")
    M = oracle.fit(W)
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, bound_kind=oracle.BOUND_CERTIFIED)
    leaves_search, _, _ = oracle.adaptive(M, W)
    G = gpu_model(W)
    A = lcp.adapt_of(W, bound_kind=lcp.BOUND_CERTIFIED)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, A, zbank(W), "fp64")
    n = int(nl.item())
    got = leaves[:n].cpu().numpy().astype(np.uint64)
    ties = _near(recs, W.alpha)
    assert set(map(int, leaves_search)) <= set(map(int, leaves_ref))
    assert np.all(np.diff(got.astype(np.int64)) > 0)
    sym, excused = compare_adaptive(W, M, out.cpu().numpy(), got, lf.cpu().numpy(), leaves_ref, skipped_ref, ties)
    say(f"  leaves gpu={n} oracle={len(leaves_ref)} (search {len(leaves_search)}) differ={len(sym)} "
        f"near-ties={len(ties)} excused cells={int(excused.sum())}")


def test_adaptive_certified_contains_gpu_search_leaves_and_equals_dense_inside():
    W = _cases()["trig33"]
    G = gpu_model(W)
    grid = lcp.grid_of(W)
    dense, _ = G.lcp_dense(grid, W.theta, zbank(W), "f16x3")
    _, ls, ns, _, _ = G.lcp_adaptive(grid, W.theta, lcp.adapt_of(W), zbank(W), "f16x3")
    out, lc, nc, lf, _ = G.lcp_adaptive(grid, W.theta, lcp.adapt_of(W, bound_kind=lcp.BOUND_CERTIFIED), zbank(W),
                                       "f16x3")
    search = set(ls[: int(ns.item())].cpu().numpy().tolist())
    cert = set(lc[: int(nc.item())].cpu().numpy().tolist())
    say(f"certified leaves {len(cert)} vs search {len(search)}")
    assert search <= cert
    mask = torch.as_tensor(oracle.level_field(W, np.array(sorted(cert), np.uint64)).reshape(-1) != 255)
    d, a = dense.cpu(), out.cpu()
    assert torch.equal(a[mask], d[mask]) and (a[~mask] == 0).all()
