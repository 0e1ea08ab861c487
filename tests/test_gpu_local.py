"""Parity of the region test on local models (lcp_adapt.bound_kind = LCP_BOUND_LOCAL, the
local model M' of Sec. 5.2 used by Alg. 1) with the FP64 oracle, for exact-GP and sparse
models: leaf sets (exact, except below nodes the oracle flags as near-ties), Monte Carlo
counts inside the leaves (exact in binary64), the level field, and the identities that do
not need the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2512_12442_amd as lcp
from parity_util import compare_adaptive, counts, gpu_model, near_tie_keys, say, zbank

pytestmark = pytest.mark.gpu


def _cases():
    W1 = workloads.field3d_trig(0, m=120, npts=33)
    W2 = workloads.field3d_trig(3, m=150, npts=29)
    W2.npts[:] = [29, 23, 19]
    W2.min_leaf = 2
    W3 = workloads.make("cfg1_2d")
    W3.min_leaf = 2
    W4 = workloads.field3d_trig(5, m=300, npts=33)
    # few observations, short lengthscale: many nodes have an empty M' (the prior decides)
    W5 = workloads.random_small(190, 3, 40, 17, ell=0.06, signal_var=0.01, noise_var=1e-4, min_leaf=1)
    W5.theta = 0.45
    W6 = workloads.sgpr_field(154, m=64, npts=17, train_npts=10, ell=0.25)
    W6.min_leaf = 1
    W7 = workloads.sgpr_field(155, m=216, npts=25, train_npts=12, ell=0.12)
    W7.min_leaf = 2
    return {"trig33": W1, "ragged": W2, "cfg1_2d": W3, "trig33_m300": W4, "sparse_obs17": W5, "sgpr17": W6,
            "sgpr25": W7}


def _run(W, beta, split=oracle.SPLIT_OCTREE, prec="fp64"):
    G = gpu_model(W)
    A = lcp.adapt_of(W, bound_kind=lcp.BOUND_LOCAL, beta=beta, split=split)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, A, zbank(W), prec)
    n = int(nl.item())
    return out.cpu().numpy(), leaves[:n].cpu().numpy().astype(np.uint64), lf.cpu().numpy()


@pytest.mark.parametrize("case,beta,split", [("trig33", 6.0, 0), ("trig33", 2.0, 0), ("trig33", 1.0, 0),
                                             ("ragged", 1.5, 0), ("cfg1_2d", 2.0, 0), ("trig33_m300", 6.0, 0),
                                             ("sparse_obs17", 0.0, 0), ("sparse_obs17", 1.0, 0),
                                             ("trig33", 1.0, 1), ("cfg1_2d", 2.0, 1),
                                             ("sgpr17", 1.0, 0), ("sgpr17", 3.0, 0), ("sgpr25", 2.0, 0),
                                             ("sgpr25", 1.0, 1)])
def test_local_bound_matches_oracle(case, beta, split):
    W = _cases()[case]
    say(f"local bound {case} beta={beta} split={split} npts={list(W.npts)} m={W.m} min_leaf={W.min_leaf}")
    M = oracle.fit(W)
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, bound_kind=oracle.BOUND_LOCAL, beta=beta, split=split)
    out, got, lf = _run(W, beta, split)
    ties = near_tie_keys(recs, W.alpha)
    tested = recs["n_local"] >= 0
    assert np.all(np.diff(got.astype(np.int64)) > 0)
    sym, excused = compare_adaptive(W, M, out, got, lf, leaves_ref, skipped_ref, ties, split=split)
    say(f"  leaves gpu={len(got)} oracle={len(leaves_ref)} differ={len(sym)} near-ties={len(ties)} "
        f"excused cells={int(excused.sum())} region tests={tested.sum()} "
        f"mean |M'|={recs['n_local'][tested].mean():.1f} min |M'|={recs['n_local'][tested].min()}")


def test_local_with_huge_beta_is_the_full_model_search():
    """Every observation is local: the leaves are those of the search on the full model
    (the GPU's two search paths agree, and both agree with the oracle)."""
    W = _cases()["trig33"]
    G = gpu_model(W)
    grid = lcp.grid_of(W)
    a_s = G.lcp_adaptive(grid, W.theta, lcp.adapt_of(W), zbank(W), "fp64")
    a_l = G.lcp_adaptive(grid, W.theta, lcp.adapt_of(W, bound_kind=lcp.BOUND_LOCAL, beta=1e6), zbank(W), "fp64")
    ns, nl = int(a_s[2].item()), int(a_l[2].item())
    M = oracle.fit(W)
    ref, _, _ = oracle.adaptive(M, W)
    assert ns == nl == len(ref)
    assert np.array_equal(a_s[1][:ns].cpu().numpy(), a_l[1][:nl].cpu().numpy())
    assert np.array_equal(a_s[0].cpu().numpy(), a_l[0].cpu().numpy())


def test_local_mixed_precision_reconstruction_matches_fp64_leaves():
    """The region test runs in binary64 whatever the reconstruction precision."""
    W = _cases()["trig33"]
    _, l64, _ = _run(W, 2.0, prec="fp64")
    _, l16, _ = _run(W, 2.0, prec="f16x3")
    assert np.array_equal(l64, l16)


def test_local_bound_rejects_bad_beta():
    W = _cases()["cfg1_2d"]
    G = gpu_model(W)
    for beta in (-1.0, float("inf"), float("nan")):
        with pytest.raises(lcp.LcpError) as e:
            G.lcp_adaptive(lcp.grid_of(W), W.theta, lcp.adapt_of(W, bound_kind=lcp.BOUND_LOCAL, beta=beta),
                           zbank(W), "fp64")
        assert e.value.status == lcp.lcp.LCP_EINVAL
