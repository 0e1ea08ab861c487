"""Python binding of the gfx950 LCP library (include/lcp.h).

Argument marshalling only: every step of the computation runs in the HIP kernels of
liblcp.so.  PyTorch provides device memory and the current stream.  If the shared
library is missing the import of this module fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblcp.so")

LCP_OK, LCP_EINVAL, LCP_ENOTPD, LCP_ECAPACITY, LCP_ENOMEM, LCP_EDEVICE, LCP_ENOTSUPPORTED = range(7)
FP64, FP32, MIXED_BF16X3, MIXED_F16X3 = 0, 1, 2, 3
NOALLOC_SCRATCH_BYTES = 64 << 20     # LCP_NOALLOC_SCRATCH_BYTES of lcp.h
SE, MATERN52 = 0, 1
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": MIXED_BF16X3, "f16x3": MIXED_F16X3}


class LcpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lcp status {status}: {msg}")
        self.status = status


class Kernel(C.Structure):
    _fields_ = [("kind", C.c_int), ("dim", C.c_int), ("signal_var", C.c_double),
                ("lengthscale", C.c_double * 3), ("noise_var", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("npts", C.c_int64 * 3)]


class Adapt(C.Structure):
    _fields_ = [("alpha", C.c_double), ("min_leaf_cells", C.c_int), ("bound_at_max_depth", C.c_int),
                ("descent_steps", C.c_int), ("bound_kind", C.c_int), ("split", C.c_int), ("beta", C.c_double),
                ("edge_bound", C.c_int)]


BOUND_SEARCH, BOUND_CERTIFIED, BOUND_LOCAL = 0, 1, 2
SPLIT_OCTREE, SPLIT_KD = 0, 1


class MC(C.Structure):
    _fields_ = [("n_samples", C.c_int), ("zbank", C.c_void_p), ("estimator", C.c_int)]


EST_COUNT, EST_SOV = 0, 1


EXPORTS = ["lcp_status_str", "lcp_last_error", "lcp_model_bytes", "gp_fit_factor", "gp_fit_sgpr", "gp_model_free",
           "lcp_posterior_workspace", "lcp_dense_workspace", "lcp_adaptive_workspace", "gp_posterior",
           "lcp_dense", "lcp_adaptive", "lcp_backward", "lcp_profile_begin", "lcp_profile_end",
           "lcp_batch_model_bytes", "gp_fit_factor_batch", "gp_model_batch_free", "lcp_dense_batch_workspace",
           "lcp_dense_batch", "gp_posterior_backward_workspace", "gp_posterior_backward",
           "lcp_backward_workspace", "lcp_bound_workspace", "lcp_bound_certified", "lcp_dense_noalloc",
           "lcp_cell_moments_workspace", "lcp_cell_moments", "lcp_batch_precision",
           "lcp_dense_batch_mixed_workspace", "lcp_dense_batch_mixed", "lcp_batch_tiles", "lcp_batch_tiles_get"]

STAGES = ["factor", "posterior", "bound", "cross", "cells", "octree", "misc"]

_lib = None


def lib():
    """Load liblcp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2512_12442_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P, I64, SZ = C.c_void_p, C.c_int64, C.c_size_t
    L.lcp_status_str.restype = C.c_char_p
    L.lcp_status_str.argtypes = [C.c_int]
    L.lcp_last_error.restype = C.c_char_p
    L.lcp_last_error.argtypes = []
    L.lcp_model_bytes.restype = SZ
    L.lcp_model_bytes.argtypes = [C.c_int, C.c_int]
    L.gp_fit_factor.argtypes = [P, C.c_int, P, P, P, SZ, P, C.POINTER(P)]
    L.gp_fit_sgpr.argtypes = [P, C.c_int, P, P, P, P, SZ, P, C.POINTER(C.c_double), C.POINTER(P)]
    L.gp_model_free.argtypes = [P]
    L.gp_model_free.restype = None
    L.lcp_posterior_workspace.argtypes = [P, I64, C.c_int, C.POINTER(SZ)]
    L.lcp_dense_workspace.argtypes = [P, P, C.c_int, C.c_int, C.POINTER(SZ)]
    L.lcp_adaptive_workspace.argtypes = [P, P, P, C.c_int, C.c_int, C.POINTER(SZ)]
    L.gp_posterior.argtypes = [P, I64, P, C.c_int, P, P, P, SZ, P]
    L.lcp_dense.argtypes = [P, P, C.c_double, P, C.c_int, P, P, SZ, P]
    L.lcp_dense_noalloc.argtypes = [P, P, C.c_double, P, C.c_int, P, P]
    L.lcp_adaptive.argtypes = [P, P, C.c_double, P, P, C.c_int, P, P, I64, P, P, P, SZ, P]
    L.lcp_backward.argtypes = [P, P, C.c_double, P, C.c_int, P, P, P, P, SZ, P]
    L.lcp_backward_workspace.argtypes = [P, P, C.c_int, C.c_int, C.POINTER(SZ)]
    L.gp_posterior_backward_workspace.argtypes = [P, I64, C.c_int, C.POINTER(SZ)]
    L.gp_posterior_backward.argtypes = [P, I64, P, C.c_int, P, P, P, P, P, SZ, P]
    L.lcp_bound_workspace.argtypes = [P, I64, C.POINTER(SZ)]
    L.lcp_bound_certified.argtypes = [P, I64, P, P, P, SZ, P]
    L.lcp_cell_moments_workspace.argtypes = [P, P, I64, C.c_int, C.POINTER(SZ)]
    L.lcp_cell_moments.argtypes = [P, P, I64, P, C.c_int, P, P, P, SZ, P]
    L.lcp_profile_begin.argtypes = [C.c_uint]
    L.lcp_profile_end.argtypes = [P, P, C.c_int]
    L.lcp_batch_model_bytes.restype = SZ
    L.lcp_batch_model_bytes.argtypes = [C.c_int, P, C.c_int]
    L.gp_fit_factor_batch.argtypes = [C.c_int, P, P, P, P, P, SZ, P, C.POINTER(P)]
    L.gp_model_batch_free.argtypes = [P]
    L.gp_model_batch_free.restype = None
    L.lcp_dense_batch_workspace.argtypes = [P, P, C.c_int, C.c_int, C.POINTER(SZ)]
    L.lcp_dense_batch.argtypes = [P, P, P, P, C.c_int, P, P, SZ, P]
    L.lcp_batch_precision.argtypes = [P, C.c_int, C.c_double, P, P, P]
    L.lcp_dense_batch_mixed_workspace.argtypes = [P, P, P, C.c_int, C.POINTER(SZ)]
    L.lcp_dense_batch_mixed.argtypes = [P, P, P, P, P, P, P, SZ, P]
    L.lcp_batch_tiles.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
    L.lcp_batch_tiles_get.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    for name in EXPORTS:
        if name not in ("lcp_status_str", "lcp_last_error", "lcp_model_bytes", "gp_model_free",
                        "lcp_batch_model_bytes", "gp_model_batch_free"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status):
    if status != LCP_OK:
        raise LcpError(status, lib().lcp_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _buffer(nbytes: int, device) -> torch.Tensor:
    """Device byte buffer whose data pointer is 256-byte aligned."""
    t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + max(int(nbytes), 1)]


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def make_grid(dim, lo, hi, npts) -> Grid:
    g = Grid()
    g.dim = dim
    for d in range(3):
        g.lo[d] = float(lo[d]) if d < dim else 0.0
        g.hi[d] = float(hi[d]) if d < dim else 0.0
        g.npts[d] = int(npts[d]) if d < dim else 1
    return g


class GPModel:
    """A factored GP model living in caller-owned device memory: gp_fit_factor for
    observations (X, y), or gp_fit_sgpr when A_M (the inducing covariance of eq. (sgp))
    is given, with X the inducing points, y = mu_M and noise_var the jitter of K_MM."""

    def __init__(self, kind, dim, signal_var, lengthscale, noise_var, X: torch.Tensor, y: torch.Tensor,
                 A_M: torch.Tensor = None):
        L = lib()
        X = X.to(torch.float64).contiguous()
        y = y.to(torch.float64).contiguous()
        assert X.is_cuda and y.is_cuda and X.shape == (y.shape[0], dim)
        self.k = Kernel(kind, dim, float(signal_var), (C.c_double * 3)(*[float(v) for v in lengthscale[:3]]),
                        float(noise_var))
        self.dim, self.m = dim, int(X.shape[0])
        nb = L.lcp_model_bytes(self.m, dim)
        if nb == 0:
            raise LcpError(LCP_EINVAL, f"unsupported number of observations m={self.m}")
        self.mem = _buffer(nb, X.device)
        self.device = X.device
        self._X, self._y = X, y
        h = C.c_void_p()
        self.shift = 0.0
        if A_M is None:
            _check(L.gp_fit_factor(C.byref(self.k), self.m, _ptr(X), _ptr(y), _ptr(self.mem), nb, _stream(),
                                   C.byref(h)))
        else:
            A_M = A_M.to(torch.float64).contiguous()
            assert A_M.is_cuda and A_M.shape == (self.m, self.m)
            sh = C.c_double()
            _check(L.gp_fit_sgpr(C.byref(self.k), self.m, _ptr(X), _ptr(y), _ptr(A_M), _ptr(self.mem), nb,
                                 _stream(), C.byref(sh), C.byref(h)))
            self.shift = sh.value
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gp_model_free(h)
            self.h = None

    @classmethod
    def from_workload(cls, W, device="cuda"):
        X = torch.as_tensor(W.X, dtype=torch.float64, device=device)
        y = torch.as_tensor(W.y, dtype=torch.float64, device=device)
        A = getattr(W, "A_M", None)
        A = None if A is None else torch.as_tensor(A, dtype=torch.float64, device=device)
        return cls(W.kind, W.dim, W.signal_var, list(W.lengthscale), W.noise_var, X, y, A)

    # -------------------------------------------------------------- operations
    def posterior(self, Xq: torch.Tensor, prec="fp64"):
        Xq = Xq.to(torch.float64).contiguous()
        n = int(Xq.shape[0])
        mean = torch.empty(n, dtype=torch.float64, device=self.device)
        var = torch.empty(n, dtype=torch.float64, device=self.device)
        _check(lib().gp_posterior(self.h, n, _ptr(Xq), _prec(prec), _ptr(mean), _ptr(var), None, 0, _stream()))
        return mean, var

    def posterior_backward(self, Xq: torch.Tensor, dmean=None, dvar=None, prec="fp64", ws=None):
        """Adjoint of posterior(Xq): (dL/dy, dL/dlog(lengthscale)) for upstream dL/dmean, dL/dvar."""
        Xq = Xq.to(torch.float64).contiguous()
        n = int(Xq.shape[0])
        b = C.c_size_t()
        _check(lib().gp_posterior_backward_workspace(self.h, n, _prec(prec), C.byref(b)))
        if ws is None or ws.numel() < b.value:
            ws = _buffer(b.value, self.device)
        gm = None if dmean is None else dmean.to(torch.float64).contiguous()
        gv = None if dvar is None else dvar.to(torch.float64).contiguous()
        dy = torch.empty(self.m, dtype=torch.float64, device=self.device)
        dl = torch.empty(self.dim, dtype=torch.float64, device=self.device)
        _check(lib().gp_posterior_backward(self.h, n, _ptr(Xq), _prec(prec), _ptr(gm), _ptr(gv), _ptr(dy), _ptr(dl),
                                           _ptr(ws), b.value, _stream()))
        return dy, dl

    def bound_certified(self, boxes: torch.Tensor, ws=None):
        """Certified box bounds (lcp_bound_certified): boxes n x (2 dim) as lo then hi per box;
        returns n x 4 (mu at the centre, mu lower and upper bound, var upper bound)."""
        boxes = boxes.to(torch.float64).contiguous()
        n = int(boxes.shape[0])
        b = C.c_size_t()
        _check(lib().lcp_bound_workspace(self.h, n, C.byref(b)))
        if ws is None or ws.numel() < b.value:
            ws = _buffer(b.value, self.device)
        out = torch.empty((n, 4), dtype=torch.float64, device=self.device)
        _check(lib().lcp_bound_certified(self.h, n, _ptr(boxes), _ptr(out), _ptr(ws), b.value, _stream()))
        return out

    def cell_moments(self, grid: Grid, cells: torch.Tensor, prec="fp64"):
        """Corner means (n x 2^dim) and covariances (n x 2^dim x 2^dim) of the listed cells
        (linear indices, x fastest) as the LCP kernels compute them (lcp_cell_moments)."""
        cells = cells.to(torch.int64).contiguous()
        n = int(cells.shape[0])
        nc = 1 << grid.dim
        b = C.c_size_t()
        _check(lib().lcp_cell_moments_workspace(self.h, C.byref(grid), n, _prec(prec), C.byref(b)))
        ws = _buffer(b.value, self.device)
        mean = torch.empty((n, nc), dtype=torch.float64, device=self.device)
        cov = torch.empty((n, nc, nc), dtype=torch.float64, device=self.device)
        _check(lib().lcp_cell_moments(self.h, C.byref(grid), n, _ptr(cells), _prec(prec), _ptr(mean), _ptr(cov),
                                      _ptr(ws), b.value, _stream()))
        return mean, cov

    def dense_workspace(self, grid: Grid, prec, n_samples):
        b = C.c_size_t()
        _check(lib().lcp_dense_workspace(self.h, C.byref(grid), _prec(prec), int(n_samples), C.byref(b)))
        return b.value

    def adaptive_workspace(self, grid: Grid, adapt: Adapt, prec, n_samples):
        b = C.c_size_t()
        _check(lib().lcp_adaptive_workspace(self.h, C.byref(grid), C.byref(adapt), _prec(prec), int(n_samples),
                                            C.byref(b)))
        return b.value

    def lcp_dense(self, grid: Grid, theta: float, zbank: torch.Tensor, prec="fp64", out=None, ws=None,
                  estimator=EST_COUNT):
        zbank = zbank.to(torch.float64).contiguous()
        mc = MC(int(zbank.shape[0]), zbank.data_ptr(), int(estimator))
        nb = self.dense_workspace(grid, prec, mc.n_samples)
        if ws is None or ws.numel() < nb:
            ws = _buffer(nb, self.device)
        ncell = 1
        for d in range(grid.dim):
            ncell *= grid.npts[d] - 1
        if out is None:
            out = torch.empty(ncell, dtype=torch.float32, device=self.device)
        _check(lib().lcp_dense(self.h, C.byref(grid), float(theta), C.byref(mc), _prec(prec), _ptr(out), _ptr(ws),
                               ws.numel(), _stream()))
        return out, ws

    def lcp_dense_noalloc(self, grid: Grid, theta: float, zbank: torch.Tensor, out: torch.Tensor, prec="fp64",
                          estimator=EST_COUNT):
        """lcp_dense on the library's fixed scratch: no workspace; `out` (one binary32 per
        cell) and a binary64 z-bank on the device are the caller's."""
        if zbank.dtype != torch.float64 or not zbank.is_contiguous():
            raise ValueError("zbank must be a contiguous float64 device tensor")
        mc = MC(int(zbank.shape[0]), zbank.data_ptr(), int(estimator))
        _check(lib().lcp_dense_noalloc(self.h, C.byref(grid), float(theta), C.byref(mc), _prec(prec), _ptr(out),
                                       _stream()))
        return out

    def lcp_adaptive(self, grid: Grid, theta: float, adapt: Adapt, zbank: torch.Tensor, prec="bf16x3", leaf_cap=None,
                     level_field=True, out=None, ws=None, leaves=None, n_leaves=None):
        zbank = zbank.to(torch.float64).contiguous()
        mc = MC(int(zbank.shape[0]), zbank.data_ptr())
        nb = self.adaptive_workspace(grid, adapt, prec, mc.n_samples)
        if ws is None or ws.numel() < nb:
            ws = _buffer(nb, self.device)
        ncell = 1
        for d in range(grid.dim):
            ncell *= grid.npts[d] - 1
        if out is None:
            out = torch.empty(ncell, dtype=torch.float32, device=self.device)
        if leaf_cap is None:
            leaf_cap = ncell
        if leaves is None:
            leaves = torch.zeros(max(int(leaf_cap), 1), dtype=torch.int64, device=self.device)
        if n_leaves is None:
            n_leaves = torch.zeros(1, dtype=torch.int64, device=self.device)
        lf = torch.empty(ncell, dtype=torch.uint8, device=self.device) if level_field else None
        _check(lib().lcp_adaptive(self.h, C.byref(grid), float(theta), C.byref(adapt), C.byref(mc), _prec(prec),
                                  _ptr(out), _ptr(leaves), int(leaf_cap), _ptr(n_leaves), _ptr(lf), _ptr(ws),
                                  ws.numel(), _stream()))
        return out, leaves, n_leaves, lf, ws

    def lcp_backward(self, grid: Grid, theta: float, zbank: torch.Tensor, dL_dlcp: torch.Tensor, prec="fp64",
                     ws=None):
        """Adjoint of the smooth LCP field (lcp_dense with EST_SOV): (dL/dy, dL/dlog(lengthscale))."""
        zbank = zbank.to(torch.float64).contiguous()
        mc = MC(int(zbank.shape[0]), zbank.data_ptr(), EST_SOV)
        b = C.c_size_t()
        _check(lib().lcp_backward_workspace(self.h, C.byref(grid), _prec(prec), mc.n_samples, C.byref(b)))
        if ws is None or ws.numel() < b.value:
            ws = _buffer(b.value, self.device)
        g = dL_dlcp.to(torch.float64).contiguous()
        dy = torch.empty(self.m, dtype=torch.float64, device=self.device)
        dl = torch.empty(self.dim, dtype=torch.float64, device=self.device)
        _check(lib().lcp_backward(self.h, C.byref(grid), float(theta), C.byref(mc), _prec(prec), _ptr(g), _ptr(dy),
                                  _ptr(dl), _ptr(ws), b.value, _stream()))
        return dy, dl


def _operand_prec(p):
    """gp_posterior_backward's one product has a full operand: binary64 or binary32 (a split
    16-bit precision of the forward maps to binary32)."""
    return p if _prec(p) in (FP64, FP32) else "fp32"


class GPPosterior(torch.autograd.Function):
    """Posterior mean and variance at Xq as a differentiable function of the observation
    values y and the log-lengthscales: forward fits the model (gp_fit_factor) and evaluates
    gp_posterior; backward runs gp_posterior_backward (K* regenerated, not stored)."""

    @staticmethod
    def forward(ctx, y, log_ell, X, Xq, kind, signal_var, noise_var, prec):
        ell = torch.exp(log_ell.detach()).cpu().tolist()
        ell = ell + [1.0] * (3 - len(ell))
        G = GPModel(kind, X.shape[1], signal_var, ell, noise_var, X, y.detach())
        mean, var = G.posterior(Xq, prec)
        ctx.G, ctx.prec = G, prec
        ctx.save_for_backward(Xq)
        return mean, var

    @staticmethod
    def backward(ctx, gmean, gvar):
        (Xq,) = ctx.saved_tensors
        dy, dl = ctx.G.posterior_backward(Xq, gmean, gvar, _operand_prec(ctx.prec))
        return dy, dl, None, None, None, None, None, None


class GPLcp(torch.autograd.Function):
    """Smooth LCP field (separation-of-variables estimate) of a dense grid as a
    differentiable function of y and the log-lengthscales: forward fits the model and runs
    lcp_dense with EST_SOV; backward runs lcp_backward."""

    @staticmethod
    def forward(ctx, y, log_ell, X, grid, theta, zbank, kind, signal_var, noise_var, prec):
        ell = torch.exp(log_ell.detach()).cpu().tolist()
        ell = ell + [1.0] * (3 - len(ell))
        G = GPModel(kind, X.shape[1], signal_var, ell, noise_var, X, y.detach())
        out, _ = G.lcp_dense(grid, theta, zbank, prec, estimator=EST_SOV)
        ctx.G, ctx.grid, ctx.theta, ctx.zbank, ctx.prec = G, grid, theta, zbank, prec
        return out.to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        dy, dl = ctx.G.lcp_backward(ctx.grid, ctx.theta, ctx.zbank, g, ctx.prec)
        return dy, dl, None, None, None, None, None, None, None, None


def lcp_fn(y, log_ell, X, grid, theta, zbank, kind=SE, signal_var=1.0, noise_var=1e-4, prec="fp64"):
    """Differentiable smooth LCP field; gradients flow to y and log_ell."""
    return GPLcp.apply(y, log_ell, X, grid, theta, zbank, kind, signal_var, noise_var, prec)


class GPLcpPosterior(torch.autograd.Function):
    """The smooth LCP field of a grid and the posterior at points Xq from one fit, as a
    differentiable function of y and the log-lengthscales (backward: lcp_backward plus
    gp_posterior_backward, summed)."""

    @staticmethod
    def forward(ctx, y, log_ell, X, grid, theta, zbank, Xq, kind, signal_var, noise_var, prec):
        ell = torch.exp(log_ell.detach()).cpu().tolist()
        ell = ell + [1.0] * (3 - len(ell))
        G = GPModel(kind, X.shape[1], signal_var, ell, noise_var, X, y.detach())
        field, _ = G.lcp_dense(grid, theta, zbank, prec, estimator=EST_SOV)
        mean, var = G.posterior(Xq, prec)
        ctx.G, ctx.grid, ctx.theta, ctx.zbank, ctx.prec = G, grid, theta, zbank, prec
        ctx.save_for_backward(Xq)
        return field.to(torch.float64), mean, var

    @staticmethod
    def backward(ctx, gfield, gmean, gvar):
        (Xq,) = ctx.saved_tensors
        dy, dl = ctx.G.lcp_backward(ctx.grid, ctx.theta, ctx.zbank, gfield, ctx.prec)
        dy2, dl2 = ctx.G.posterior_backward(Xq, gmean, gvar, _operand_prec(ctx.prec))
        return dy + dy2, dl + dl2, None, None, None, None, None, None, None, None, None


def lcp_posterior_fn(y, log_ell, X, grid, theta, zbank, Xq, kind=SE, signal_var=1.0, noise_var=1e-4, prec="fp64"):
    """Differentiable (smooth LCP field, mean at Xq, variance at Xq) from one model fit."""
    return GPLcpPosterior.apply(y, log_ell, X, grid, theta, zbank, Xq, kind, signal_var, noise_var, prec)


def posterior_fn(y, log_ell, X, Xq, kind=SE, signal_var=1.0, noise_var=1e-4, prec="fp64"):
    """Differentiable (mean, var) at Xq; gradients flow to y and log_ell."""
    return GPPosterior.apply(y, log_ell, X, Xq, kind, signal_var, noise_var, prec)


class StageTimer:
    """Per-stage kernel time from hipEvents the library records on its launch stream."""

    def __init__(self, stages=None):
        names = stages or STAGES
        self.mask = 0
        for n in names:
            self.mask |= 1 << STAGES.index(n)
        self.ms = {}
        self.launches = {}

    def __enter__(self):
        _check(lib().lcp_profile_begin(self.mask))
        return self

    def __exit__(self, *exc):
        import numpy as np
        ms = np.zeros(len(STAGES))
        cnt = np.zeros(len(STAGES), np.int64)
        _check(lib().lcp_profile_end(ms.ctypes.data_as(C.c_void_p), cnt.ctypes.data_as(C.c_void_p), len(STAGES)))
        self.ms = {n: float(ms[i]) for i, n in enumerate(STAGES) if self.mask >> i & 1}
        self.launches = {n: int(cnt[i]) for i, n in enumerate(STAGES) if self.mask >> i & 1}
        return False


def grid_of(W) -> Grid:
    return make_grid(W.dim, W.lo, W.hi, W.npts)


def adapt_of(W, min_leaf=None, bound_at_max_depth=1, steps=4, alpha=None, bound_kind=BOUND_SEARCH,
             split=SPLIT_OCTREE, beta=6.0, edge_bound=0) -> Adapt:
    return Adapt(float(alpha if alpha is not None else W.alpha), int(min_leaf or W.min_leaf), int(bound_at_max_depth),
                 int(steps), int(bound_kind), int(split), float(beta), int(edge_bound))


class GPModelBatch:
    """Independent GP models factored together (gp_fit_factor_batch), for lcp_dense_batch."""

    def __init__(self, kernels, Xs, ys, device="cuda"):
        L = lib()
        nb = len(kernels)
        assert nb == len(Xs) == len(ys) and nb > 0
        dim = kernels[0][1]
        K = (Kernel * nb)()
        for b, (kind, kd, s2, ell, noise) in enumerate(kernels):
            K[b] = Kernel(kind, kd, float(s2), (C.c_double * 3)(*[float(v) for v in list(ell)[:3]]), float(noise))
        ms = (C.c_int * nb)(*[int(len(y)) for y in ys])
        X = torch.cat([torch.as_tensor(x, dtype=torch.float64).reshape(-1, dim) for x in Xs]).to(device).contiguous()
        y = torch.cat([torch.as_tensor(v, dtype=torch.float64).reshape(-1) for v in ys]).to(device).contiguous()
        nbytes = L.lcp_batch_model_bytes(nb, ms, dim)
        if nbytes == 0:
            raise LcpError(LCP_EINVAL, "unsupported batch (each m must be 1..1024)")
        self.mem = _buffer(nbytes, device)
        self.device, self.nb, self.dim = torch.device(device), nb, dim
        self._X, self._y, self._K, self._m = X, y, K, ms
        h = C.c_void_p()
        _check(L.gp_fit_factor_batch(nb, C.byref(K), ms, _ptr(X), _ptr(y), _ptr(self.mem), nbytes, _stream(),
                                     C.byref(h)))
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gp_model_batch_free(h)
            self.h = None

    @classmethod
    def from_workloads(cls, Ws, device="cuda"):
        return cls([(W.kind, W.dim, W.signal_var, list(W.lengthscale), W.noise_var) for W in Ws],
                   [W.X for W in Ws], [W.y for W in Ws], device)

    def precision(self, reduced="fp32", kappa_max=0.0):
        """Per-model precision codes (lcp_batch_precision): `reduced` where sqrt(s2) max|L^-1|
        <= kappa_max (0: the library default), binary64 elsewhere; and the kappa values."""
        pr = (C.c_int * self.nb)()
        kap = (C.c_double * self.nb)()
        _check(lib().lcp_batch_precision(self.h, _prec(reduced), float(kappa_max), pr, kap, _stream()))
        return list(pr), list(kap)

    def dense_workspace(self, grids, prec, n_samples):
        G = (Grid * self.nb)(*grids)
        b = C.c_size_t()
        if isinstance(prec, str):
            _check(lib().lcp_dense_batch_workspace(self.h, G, _prec(prec), int(n_samples), C.byref(b)))
        else:
            pr = (C.c_int * self.nb)(*[_prec(p) if isinstance(p, str) else int(p) for p in prec])
            _check(lib().lcp_dense_batch_mixed_workspace(self.h, G, pr, int(n_samples), C.byref(b)))
        return b.value

    def lcp_dense(self, grids, thetas, zbank: torch.Tensor, prec="fp32", out=None, ws=None):
        """Cell fields of every model, concatenated in model order.  prec: one precision for
        all models, or a sequence with one per model (lcp_dense_batch_mixed)."""
        G = (Grid * self.nb)(*grids)
        th = (C.c_double * self.nb)(*[float(t) for t in thetas])
        zbank = zbank.to(torch.float64).contiguous()
        mc = MC(int(zbank.shape[0]), zbank.data_ptr())
        nbytes = self.dense_workspace(grids, prec, mc.n_samples)
        if ws is None or ws.numel() < nbytes:
            ws = _buffer(nbytes, self.device)
        ncell = 0
        for g in grids:
            c = 1
            for d in range(g.dim):
                c *= g.npts[d] - 1
            ncell += c
        if out is None:
            out = torch.empty(ncell, dtype=torch.float32, device=self.device)
        if isinstance(prec, str):
            _check(lib().lcp_dense_batch(self.h, G, th, C.byref(mc), _prec(prec), _ptr(out), _ptr(ws), ws.numel(),
                                         _stream()))
        else:
            pr = (C.c_int * self.nb)(*[_prec(p) if isinstance(p, str) else int(p) for p in prec])
            _check(lib().lcp_dense_batch_mixed(self.h, G, th, C.byref(mc), pr, _ptr(out), _ptr(ws), ws.numel(),
                                               _stream()))
        return out, ws


def batch_tiles(prec, size_class, nt=None, nw=None):
    """Read (and with nt, nw set) the batched posterior's tile configuration for a
    precision and size class (m_pad = 128 (size_class + 1)); nt = 0 restores the default."""
    L = lib()
    if nt is not None:
        _check(L.lcp_batch_tiles(_prec(prec), int(size_class), int(nt), int(nw or 0)))
    a, b = C.c_int(), C.c_int()
    _check(L.lcp_batch_tiles_get(_prec(prec), int(size_class), C.byref(a), C.byref(b)))
    return a.value, b.value
