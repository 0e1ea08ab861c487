"""Helpers shared by the GPU parity tests (not a test module)."""
import numpy as np
import torch

import paper_2512_12442_amd as lcp
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
    """Nodes whose decision depends on rounding: UB within 1e-8 relative of alpha, p1/p2
    within 1e-12 of alpha, or two lattice minima within 1e-9 of each other."""
    bad = set()
    for r in recs:
        if r["path"] in (1, 2) or (r["path"] != 0 and not np.isnan(r["ub"])):
            if abs(r["ub"] - alpha) <= 1e-8 * alpha or abs(r["lattice_gap"]) <= 1e-9 * max(1, abs(r["gmin"])):
                bad.add(int(r["key"]))
        if r["n_obs"] > 0 and (abs(r["p1"] - alpha) <= 1e-12 or abs(r["p2"] - alpha) <= 1e-12):
            bad.add(int(r["key"]))
    return bad
