"""lcp_dense_noalloc (the allocation-free variant of lcp_dense for callers that cannot
allocate) against lcp_dense through the C ABI: two calls in a row on the library's fixed
scratch, the second on a smaller grid, each bitwise equal to lcp_dense on a caller
workspace (same kernels, same reduction order), plus the size limit."""
import numpy as np
import pytest
import torch

import workloads
import paper_2512_12442_amd as lcp
from parity_util import DEV, gpu_model, say, zbank

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "f16x3"])
def test_noalloc_dense_equals_dense_twice_second_smaller(prec):
    W1 = workloads.field3d_trig(0, m=120, npts=21)
    W2 = workloads.field3d_trig(1, m=90, npts=13)
    W2.npts[:] = [13, 11, 9]
    for W in (W1, W2):
        G = gpu_model(W)
        grid = lcp.grid_of(W)
        zb = zbank(W)
        need = G.dense_workspace(grid, prec, W.n_samples)
        assert need <= lcp.lcp.NOALLOC_SCRATCH_BYTES
        ref, _ = G.lcp_dense(grid, W.theta, zb, prec)
        out = torch.full_like(ref, -1.0)
        G.lcp_dense_noalloc(grid, W.theta, zb, out, prec)
        torch.cuda.synchronize()
        say(f"noalloc {prec} npts={list(W.npts)} m={W.m}: scratch {need} B, "
            f"max|diff|={float((out - ref).abs().max()):.1e}")
        assert torch.equal(out, ref)


def test_noalloc_rejects_grids_beyond_the_scratch():
    W = workloads.field3d_trig(0, m=500, npts=64)
    G = gpu_model(W)
    grid = lcp.grid_of(W)
    assert G.dense_workspace(grid, "fp32", W.n_samples) > lcp.lcp.NOALLOC_SCRATCH_BYTES
    out = torch.zeros(63 ** 3, dtype=torch.float32, device=DEV)
    with pytest.raises(lcp.LcpError) as e:
        G.lcp_dense_noalloc(grid, W.theta, zbank(W), out, "fp32")
    assert e.value.status == lcp.lcp.LCP_ENOMEM and "scratch" in str(e.value)
    assert float(out.abs().sum()) == 0.0
