"""The edge-crossing region bound (lcp_adapt.edge_bound, the tighter bound Sec. 9 proposes)
against the oracle: leaf sets identical except below oracle-flagged near-ties, binary64
Monte Carlo counts and the level field identical elsewhere, and the reduced-precision field
equal to the dense field inside the kept leaves.  The GPU evaluates each edge term by a
different quadrature than the oracle (Gauss-Legendre on the U/V decomposition against
adaptive Simpson on Plackett's identity); the two agree to ~1e-13."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2512_12442_amd as lcp
from parity_util import DEV, compare_adaptive, gpu_model, near_tie_keys, say, zbank

pytestmark = pytest.mark.gpu


def _ragged():
    W = workloads.field3d_trig(2, m=150, npts=29)
    W.npts[:] = [29, 23, 19]
    return W


CASES = {
    "trig33": (lambda: workloads.field3d_trig(0, m=200, npts=33), {}),
    "aniso33": (lambda: workloads.field3d_aniso(1, m=200, npts=33), {}),
    "ragged": (_ragged, {}),
    "kd": (lambda: workloads.field3d_trig(0, m=200, npts=33), {"split": 1}),
    "certified": (lambda: workloads.field3d_trig(0, m=200, npts=33), {"bound_kind": 1}),
    "leaf1": (lambda: workloads.field3d_trig(3, m=60, npts=17), {"min_leaf": 1}),
}


@pytest.mark.parametrize("case", list(CASES))
def test_edge_bound_fp64_matches_oracle(case):
    make, kw = CASES[case]
    W = make()
    ml = kw.get("min_leaf", W.min_leaf)
    say(f"edge bound {case} npts={tuple(W.npts)} m={W.m}")
    M = oracle.fit(W)
    ref0, _, _ = oracle.adaptive(M, W, min_leaf=ml, split=kw.get("split", 0), bound_kind=kw.get("bound_kind", 0))
    leaves_ref, skipped_ref, recs = oracle.adaptive(M, W, min_leaf=ml, split=kw.get("split", 0),
                                                    bound_kind=kw.get("bound_kind", 0), edge_bound=1)
    G = gpu_model(W)
    A = lcp.adapt_of(W, min_leaf=ml, split=kw.get("split", 0), bound_kind=kw.get("bound_kind", 0), edge_bound=1)
    out, leaves, nl, lf, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, A, zbank(W), "fp64")
    n = int(nl.item())
    got = leaves[:n].cpu().numpy().astype(np.uint64)
    assert np.all(np.diff(got.astype(np.int64)) > 0)
    ties = near_tie_keys(recs, W.alpha)
    W.min_leaf = ml
    sym, excused = compare_adaptive(W, M, out.cpu().numpy(), got, lf.cpu().numpy(), leaves_ref, skipped_ref, ties,
                                    split=kw.get("split", 0))
    say(f"  leaves without edge bound {len(ref0)}, with: gpu {n} oracle {len(leaves_ref)}, differ {len(sym)}, "
        f"near-ties {len(ties)}")
    assert set(map(int, leaves_ref)) <= set(map(int, ref0))
    if case == "trig33":
        assert len(leaves_ref) < len(ref0)         # the bound removes some nodes here


def test_edge_bound_field_equals_dense_inside_kept_leaves():
    W = workloads.field3d_trig(0, m=200, npts=33)
    G = gpu_model(W)
    dense, _ = G.lcp_dense(lcp.grid_of(W), W.theta, zbank(W), "f16x3")
    out, leaves, nl, _, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, lcp.adapt_of(W, edge_bound=1), zbank(W), "f16x3")
    keys = leaves[: int(nl.item())].cpu().numpy().astype(np.uint64)
    mask = torch.as_tensor(oracle.level_field(W, keys).reshape(-1) != 255)
    d, a = dense.cpu(), out.cpu()
    assert torch.equal(a[mask], d[mask])
    assert float(a[~mask].abs().max()) == 0.0
    # cells dropped by the bound: their dense LCP stays within alpha (+ one-sample MC slack)
    out0, leaves0, nl0, _, _ = G.lcp_adaptive(lcp.grid_of(W), W.theta, lcp.adapt_of(W), zbank(W), "f16x3")
    keys0 = leaves0[: int(nl0.item())].cpu().numpy().astype(np.uint64)
    mask0 = torch.as_tensor(oracle.level_field(W, keys0).reshape(-1) != 255)
    dropped = mask0 & ~mask
    say(f"edge bound f16x3: {int(dropped.sum())} cells dropped, max dense LCP there "
        f"{float(d[dropped].max()) if dropped.any() else 0.0:.2e}")
    assert float(d[dropped].max()) <= W.alpha + 2.0 / W.n_samples
