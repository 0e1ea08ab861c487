"""Helpers shared by the GPU parity tests (not a test module)."""
import numpy as np
import torch

import paper_2512_12442_amd as lcp
import oracle
import workloads

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def gpu_model(W):
    return lcp.GPModel.from_workload(W, DEV)


def zbank(W):
    return torch.as_tensor(W.zbank, device=DEV)


def counts(x, ns):
    return np.rint(np.asarray(x, np.float64) * ns).astype(np.int64)


def mean_error_bound32(W, M, P):
    """First-order bound on the mean error when each k(x_j, p) is evaluated in binary32.

    A binary32 kernel value carries a relative error of a few units of 2^-24 from the
    coordinate differences, the square root and exp2, plus one growing with the magnitude u
    of the exponent argument (its absolute error is u times a few units); summed with the
    weights |a_j| of the binary64 mean accumulation this gives
    sum_j (8 + 4 u_j) 2^-24 |k_j a_j|.
    """
    d = (P[:, None, :] - W.X[None, :, :]) / np.asarray(W.lengthscale)[:W.dim]
    r2 = (d * d).sum(-1)
    if W.kind == workloads.SE:
        u = 0.5 * r2
        k = W.signal_var * np.exp(-u)
    else:
        u = np.sqrt(5.0 * r2)
        k = W.signal_var * (1 + u + u * u / 3) * np.exp(-u)
    return ((8 + 4 * u) * np.abs(k * M.a)).sum(1) * 2.0 ** -24 + 1e-15


def near_tie_keys(recs, alpha):
    """Nodes whose decision depends on rounding: UB (or the edge-crossing bound) within 1e-8
    relative of alpha, p1/p2 within 1e-12 of alpha, or two lattice minima within 1e-9 of each
    other."""
    bad = set()
    for r in recs:
        if r["path"] in (1, 2) or (r["path"] != 0 and not np.isnan(r["ub"])):
            if abs(r["ub"] - alpha) <= 1e-8 * alpha or abs(r["lattice_gap"]) <= 1e-9 * max(1, abs(r["gmin"])):
                bad.add(int(r["key"]))
        if r["n_obs"] > 0 and (abs(r["p1"] - alpha) <= 1e-12 or abs(r["p2"] - alpha) <= 1e-12):
            bad.add(int(r["key"]))
        # the edge-crossing bound: the GPU's quadrature agrees with the oracle's to ~1e-13
        if "eb" in r.dtype.names and not np.isnan(r["eb"]) and abs(r["eb"] - alpha) <= 1e-8 * alpha:
            bad.add(int(r["key"]))
    return bad


_CODE = (1 << 58) - 1


def excused_cells(W, sym, ties, split=0):
    """Cells a leaf-set difference may touch.  Every leaf in the symmetric difference must
    lie inside a near-tie node (its key's code, shortened to the node's depth, is the node's
    code; leaves carry the octree key of the finest level, whose code is also the K-D code at
    depth dim * level).  Returns the per-cell mask of the near-tie nodes that excuse some
    difference; everything outside it must still agree cell by cell."""
    D = W.dim
    used = set()
    for k in sym:
        kb = (k >> 58) * D
        owner = None
        for t in ties:
            tb = (t >> 58) * (1 if split else D)
            if tb <= kb and ((k & _CODE) >> (kb - tb)) == (t & _CODE):
                owner = t
                break
        assert owner is not None, f"leaf {hex(k)} differs outside every near-tie node"
        used.add(owner)
    if not used:
        return np.zeros(W.n_cells, bool)
    keys = np.array(sorted(used), np.uint64)
    lev = oracle.level_field_kd(W, keys) if split else oracle.level_field(W, keys)
    return lev.reshape(-1) != 255


def compare_adaptive(W, M, out, got, lf, leaves_ref, skipped_ref, ties, split=0, counts_exact=True):
    """Leaf set, Monte Carlo counts and level field of an adaptive GPU run against the oracle's
    run.  Differences are allowed only below near-tie nodes (excused_cells); outside them the
    counts (binary64 runs: exactly) and the level field must be identical.  Returns the
    symmetric difference and the excused mask."""
    sym = set(map(int, got)) ^ set(map(int, leaves_ref))
    keep = ~excused_cells(W, sym, ties, split)
    if counts_exact:
        ref = oracle.lcp_leaves(M, W, leaves_ref).reshape(-1)
        dc = counts(np.asarray(out).reshape(-1), W.n_samples) - counts(ref, W.n_samples)
        assert np.count_nonzero(dc[keep]) == 0
    if lf is not None:
        if split:
            lev_ref = oracle.level_field_kd(W, np.concatenate([oracle.kd_leaf_keys(W, leaves_ref), skipped_ref]))
        else:
            lev_ref = oracle.level_field(W, np.concatenate([leaves_ref, skipped_ref]))
        assert np.array_equal(np.asarray(lf).reshape(-1)[keep], lev_ref.reshape(-1)[keep])
    return sym, ~keep
