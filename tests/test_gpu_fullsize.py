"""Parity at the benchmarked size: the 128^3 trig field with m = 500 observations, run in
the launch configuration the benchmark times (lcp_adaptive in FP16x3 with the binary64
bound, lcp_dense in binary64).  The oracle checks the leaf set of Alg. 1 in full and the
posterior and cell LCP on sampled vertices and cells it computes one by one."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2512_12442_amd as lcp
from parity_util import DEV, compare_adaptive, counts, gpu_model, mean_error_bound32, near_tie_keys, say, zbank

pytestmark = pytest.mark.gpu

N_SAMPLED = 1500


@pytest.fixture(scope="module")
def full():
    W = workloads.field3d_trig(0, m=500, npts=128)
    return W, oracle.fit(W), gpu_model(W)


def _vertex_coords(W, idx):
    h = (W.hi - W.lo) / (W.npts - 1)
    return W.lo[None, :] + idx * h[None, :]      # lo + i h, as the grid convention states


def _oracle_cells(M, W, cells):
    out = np.empty(len(cells))
    for i, c in enumerate(cells):
        mu, S = oracle.cell_moments(M, W, c)
        out[i] = oracle.cell_lcp(mu, S, W.theta, W.zbank)
    return out


def test_full_size_posterior_on_sampled_vertices(full):
    W, M, G = full
    idx = np.random.default_rng(11).integers(0, W.npts, size=(4000, 3))
    P = _vertex_coords(W, idx)
    mu_ref, var_ref = oracle.posterior(M, P)
    mu, var = (t.cpu().numpy() for t in G.posterior(torch.as_tensor(P, device=DEV), "fp64"))
    say(f"128^3 fp64 vertices: max|dmu|={np.abs(mu - mu_ref).max():.2e} max|dvar|={np.abs(var - var_ref).max():.2e}")
    assert np.abs(mu - mu_ref).max() <= 1e-9
    assert np.abs(var - var_ref).max() <= 1e-10
    mu, var = (t.cpu().numpy() for t in G.posterior(torch.as_tensor(P, device=DEV), "f16x3"))
    rel = np.abs(var - var_ref).max() / W.signal_var
    say(f"128^3 f16x3 vertices: max|dmu|={np.abs(mu - mu_ref).max():.2e} max|dvar|/s2={rel:.2e}")
    assert np.all(np.abs(mu - mu_ref) <= mean_error_bound32(W, M, P))
    assert rel <= 2e-5


def test_full_size_dense_fp64_on_sampled_cells(full):
    W, M, G = full
    out, _ = G.lcp_dense(lcp.grid_of(W), W.theta, zbank(W), "fp64")
    got = out.cpu().numpy().reshape(W.cell_shape)
    rng = np.random.default_rng(12)
    cells = rng.integers(0, W.npts - 1, size=(N_SAMPLED, 3))
    ref = _oracle_cells(M, W, cells)
    g = got[cells[:, 2], cells[:, 1], cells[:, 0]]
    mism = np.count_nonzero(counts(g, W.n_samples) != counts(ref, W.n_samples))
    say(f"128^3 dense fp64: {N_SAMPLED} sampled cells, nonzero {np.count_nonzero(ref)}, mismatched counts {mism}")
    assert mism == 0


def test_full_size_adaptive_f16x3_leaf_set_and_sampled_cells(full):
    W, M, G = full
    adapt = lcp.adapt_of(W, min_leaf=4, bound_at_max_depth=1, steps=4)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, adapt, zbank(W), "f16x3")
    n = int(nl.item())
    got_keys = leaves[:n].cpu().numpy().astype(np.uint64)
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, min_leaf=4, bound_at_max_depth=1, steps=4)
    ties = near_tie_keys(recs, W.alpha)
    assert np.all(np.diff(got_keys.astype(np.int64)) > 0)
    sym, excused = compare_adaptive(W, M, None, got_keys, lf.cpu().numpy(), leaves_ref, skipped_ref, ties,
                                    counts_exact=False)
    say(f"128^3 adaptive: leaves gpu={n} oracle={len(leaves_ref)} differ={len(sym)} near-ties={len(ties)} "
        f"excused cells={int(excused.sum())}")

    # every cell outside the GPU's leaves is zero; sampled leaf cells match the oracle
    inleaf = oracle.level_field(W, got_keys) != 255
    field = out.cpu().numpy().reshape(W.cell_shape)
    assert np.all(field[~inleaf] == 0)
    cand = np.argwhere(inleaf)                       # (z, y, x)
    pick = cand[np.random.default_rng(13).choice(len(cand), size=N_SAMPLED, replace=False)]
    cells = pick[:, ::-1]
    ref = _oracle_cells(M, W, cells)
    g = field[pick[:, 0], pick[:, 1], pick[:, 2]]
    dc = np.abs(counts(g, W.n_samples) - counts(ref, W.n_samples))
    rmse = float(np.sqrt(np.mean((g - ref) ** 2)))
    say(f"128^3 adaptive f16x3: {N_SAMPLED} sampled leaf cells, rmse={rmse:.2e}, max flipped samples={dc.max()}")
    assert rmse <= 1e-4
    assert dc.max() <= 8


def test_full_size_adaptive_local_bound_leaf_set(full):
    """The region test on local models (Sec. 5.2, beta = 6) at the benchmarked size: the
    leaf set against the oracle's local-model run, and the level field."""
    W, M, G = full
    adapt = lcp.adapt_of(W, min_leaf=4, bound_at_max_depth=1, steps=4, bound_kind=lcp.BOUND_LOCAL, beta=6.0)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, adapt, zbank(W), "f16x3")
    n = int(nl.item())
    got_keys = leaves[:n].cpu().numpy().astype(np.uint64)
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, min_leaf=4, bound_at_max_depth=1, steps=4,
                                                    bound_kind=oracle.BOUND_LOCAL, beta=6.0)
    ties = near_tie_keys(recs, W.alpha)
    tested = recs["n_local"] >= 0
    assert np.all(np.diff(got_keys.astype(np.int64)) > 0)
    sym, excused = compare_adaptive(W, M, None, got_keys, lf.cpu().numpy(), leaves_ref, skipped_ref, ties,
                                    counts_exact=False)
    say(f"128^3 local bound: leaves gpu={n} oracle={len(leaves_ref)} differ={len(sym)} near-ties={len(ties)} "
        f"excused cells={int(excused.sum())} region tests={tested.sum()} "
        f"mean |M'|={recs['n_local'][tested].mean():.1f}")
    field = out.cpu().numpy().reshape(W.cell_shape)
    assert np.all(field[oracle.level_field(W, got_keys) == 255] == 0)


def test_full_size_unit_signal_variance_f16x3():
    """The 128^3, m = 500 field at s2 = 1, noise 1e-5 (K conditioned about 1e8 times worse
    than the headline's s2 = 1e-3): the bound refines every node, so every cell is in a
    leaf; the leaf set equals the oracle's and the f16x3 field stays within the 1e-4 RMSE
    target against the oracle's binary64 field on a band of 16 cell layers (measured 2.8e-5
    over the whole grid against the dense binary64 GPU field)."""
    W = workloads.field3d_trig(0, m=500, npts=128)
    W.signal_var, W.noise_var = 1.0, 1e-5
    M = oracle.fit(W)
    G = gpu_model(W)
    adapt = lcp.adapt_of(W, min_leaf=4, bound_at_max_depth=1, steps=4)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, adapt, zbank(W), "f16x3")
    n = int(nl.item())
    got_keys = leaves[:n].cpu().numpy().astype(np.uint64)
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, min_leaf=4, bound_at_max_depth=1, steps=4)
    ties = near_tie_keys(recs, W.alpha)
    sym, excused = compare_adaptive(W, M, None, got_keys, lf.cpu().numpy(), leaves_ref, skipped_ref, ties,
                                    counts_exact=False)
    c0, c1 = 56, 72
    ref = oracle.lcp_dense(M, W, c0, c1)
    field = out.cpu().numpy().reshape(W.cell_shape)[c0:c1]
    d = field - ref
    rmse = float(np.sqrt(np.mean(d * d)))
    say(f"128^3 s2=1 adaptive f16x3: leaves gpu={n} oracle={len(leaves_ref)} differ={len(sym)} "
        f"near-ties={len(ties)}; band [{c0},{c1}) rmse={rmse:.2e} max={np.abs(d).max():.2e} "
        f"cells>1e-4={int((np.abs(d) > 1e-4).sum())} of {d.size}")
    assert len(sym) == 0 or len(ties) > 0
    assert rmse <= 1e-4


def test_full_size_sparse_model_leaf_set():
    """The benchmarked sparse workload (eq. (sgp): 500 inducing points, 128^3 grid) in the
    benchmarked configuration.  Its finest level has 32 768 nodes, so the certified box bound
    settles nodes between the lattice passes with the sparse model's operand (Q = T^T T); the
    leaf set and the level field must still equal the oracle's (up to its near-ties)."""
    W = workloads.sgpr_field(0, m=500, npts=128)
    M = oracle.fit(W)
    G = gpu_model(W)
    adapt = lcp.adapt_of(W, min_leaf=4, bound_at_max_depth=1, steps=4)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, adapt, zbank(W), "f16x3")
    n = int(nl.item())
    got = leaves[:n].cpu().numpy().astype(np.uint64)
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, min_leaf=4, bound_at_max_depth=1, steps=4)
    ties = near_tie_keys(recs, W.alpha)
    sym, excused = compare_adaptive(W, M, None, got, lf.cpu().numpy(), leaves_ref, skipped_ref, ties,
                                    counts_exact=False)
    say(f"128^3 sparse adaptive: leaves gpu={n} oracle={len(leaves_ref)} differ={len(sym)} near-ties={len(ties)} "
        f"excused cells={int(excused.sum())}")
    assert n > 0 and len(skipped_ref) > 0
    assert len(sym) == 0 or len(ties) > 0


def test_full_size_kd_leaf_set(full):
    """The benchmarked field with the K-D tree (Sec. 9) at 128^3: the leaf set and the depth
    field equal the oracle's (up to its near-ties).  Its depths 12 and 13 have about 100
    descent tiles, so their binary64 probes share each tile between two work-groups."""
    W, M, G = full
    adapt = lcp.adapt_of(W, min_leaf=4, bound_at_max_depth=1, steps=4, split=lcp.SPLIT_KD)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, adapt, zbank(W), "f16x3")
    n = int(nl.item())
    got = leaves[:n].cpu().numpy().astype(np.uint64)
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, min_leaf=4, bound_at_max_depth=1, steps=4,
                                                    split=oracle.SPLIT_KD)
    ties = near_tie_keys(recs, W.alpha)
    sym, excused = compare_adaptive(W, M, None, got, lf.cpu().numpy(), leaves_ref, skipped_ref, ties, split=1,
                                    counts_exact=False)
    say(f"128^3 K-D adaptive: leaves gpu={n} oracle={len(leaves_ref)} differ={len(sym)} near-ties={len(ties)} "
        f"excused cells={int(excused.sum())}")
    assert n > 0 and len(skipped_ref) > 0
    assert len(sym) == 0 or len(ties) > 0


def test_full_size_256_adaptive_leaf_set_and_sampled_cells():
    """The largest configuration of the mixed-precision workload: 256^3, m = 500, adaptive
    f16x3 with the binary64 bound.  Leaf set against the oracle's Alg. 1 (about a minute of
    host time), sampled leaf cells against the oracle's cell LCP."""
    W = workloads.field3d_trig(0, m=500, npts=256)
    M = oracle.fit(W)
    G = gpu_model(W)
    adapt = lcp.adapt_of(W, min_leaf=4, bound_at_max_depth=1, steps=4)
    out, leaves, nl, _, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, adapt, zbank(W), "f16x3")
    n = int(nl.item())
    got_keys = leaves[:n].cpu().numpy().astype(np.uint64)
    field = out.cpu().numpy().reshape(W.cell_shape)
    del out
    say(f"256^3 adaptive: {n} leaves on the GPU; running the oracle's Alg. 1")
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, min_leaf=4, bound_at_max_depth=1, steps=4)
    ties = near_tie_keys(recs, W.alpha)
    assert np.all(np.diff(got_keys.astype(np.int64)) > 0)
    sym, excused = compare_adaptive(W, M, None, got_keys, None, leaves_ref, skipped_ref, ties, counts_exact=False)
    say(f"256^3 adaptive: leaves gpu={n} oracle={len(leaves_ref)} differ={len(sym)} near-ties={len(ties)} "
        f"excused cells={int(excused.sum())}")
    inleaf = oracle.level_field(W, got_keys) != 255
    assert np.all(field[~inleaf] == 0)
    cand = np.argwhere(inleaf)
    pick = cand[np.random.default_rng(14).choice(len(cand), size=N_SAMPLED, replace=False)]
    ref = _oracle_cells(M, W, pick[:, ::-1])
    g = field[pick[:, 0], pick[:, 1], pick[:, 2]]
    dc = np.abs(counts(g, W.n_samples) - counts(ref, W.n_samples))
    rmse = float(np.sqrt(np.mean((g - ref) ** 2)))
    say(f"256^3 adaptive f16x3: {N_SAMPLED} sampled leaf cells, rmse={rmse:.2e}, max flipped samples={dc.max()}")
    assert rmse <= 1e-4
    assert dc.max() <= 8
