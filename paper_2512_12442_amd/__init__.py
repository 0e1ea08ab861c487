"""MI355X (gfx950) level-crossing probability for GP-modelled fields.

The hot path of Li, Michaud, Biswas, Shen (arXiv 2512.12442): GP posterior at grid
vertices (Sec. 3), per-cell Monte Carlo level-crossing probability (Sec. 4), and the
regional upper bound driving the octree query of Alg. 1 (Sec. 5.1-5.3).  The compute
runs in the HIP library liblcp.so (C ABI in include/lcp.h); this package only marshals
arguments.
"""
from .lcp import (BOUND_CERTIFIED, BOUND_LOCAL, BOUND_SEARCH, EST_COUNT, EST_SOV, SPLIT_KD, SPLIT_OCTREE, FP32, FP64, MATERN52, MIXED_BF16X3, MIXED_F16X3, PRECISIONS, SE, Adapt, GPModel, GPModelBatch, batch_tiles,  # noqa: F401
                  GPLcp, GPLcpPosterior, GPPosterior, Grid, LcpError, lcp_fn, lcp_posterior_fn,
                  StageTimer, adapt_of, grid_of, lib, make_grid, posterior_fn)
