"""Seeded synthetic inputs shared by the oracle-based tests, the GPU path and the bench.

This module only *draws* inputs: observation locations, observation values of a
synthetic field, kernel hyper-parameters, the grid, the iso-value and the bank of
standard-normal draws used by the Monte Carlo cell estimate.  It contains none of
the method's arithmetic (no covariance, posterior, probability or bound), so the
oracle and the HIP path can both consume its arrays without sharing any code.

One generator, sgpr_field, also stands in for the SGPR fitting step that the paper
delegates to an external library (Sec. 3): for fixed inducing points and kernel
parameters it forms the optimal Gaussian N(mu_M, A_M) of the inducing values from a
noisy synthetic training grid (Titsias' closed form).  That step is model training,
not part of the method; the method's own arithmetic (eq. (sgp), the cell
probability, the bound) stays out of this module.

The paper evaluates on two datasets (Tangle, Ethanediol, Sec. 6.3) that are not
available here; the workloads below stand in for them at the paper's scale
(m = 50 / 500 observations, 128^3 target grid, Sec. 6.3 and Sec. 7.1), with the
Monte Carlo sample count of Sec. 6.4 (1600) and the threshold alpha = 1e-3 of
Sec. 7.3.  Every random number the method consumes (the z-bank) is drawn here
and passed in as an input.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

SE = 0        # squared-exponential (RBF) covariance, Sec. 3
MATERN52 = 1  # Matern-5/2 covariance (textbook form; not used by the paper)


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    kind: int
    signal_var: float
    lengthscale: np.ndarray      # (3,) float64, unused trailing entries = 1
    noise_var: float
    X: np.ndarray                # (m, dim) float64 observation locations
    y: np.ndarray                # (m,) float64 observation values
    lo: np.ndarray               # (3,) grid lower corner
    hi: np.ndarray               # (3,) grid upper corner
    npts: np.ndarray             # (3,) int64 vertices per axis (trailing = 1)
    theta: float                 # iso-value
    alpha: float                 # skip threshold of the octree query
    min_leaf: int                # finest octree node edge, in cells
    zbank: np.ndarray            # (n_samples, 2**dim) float64 N(0,1) draws
    seed: int = 0
    A_M: Optional[np.ndarray] = None  # sparse model: (m, m) covariance of the inducing
                                      # values; X are then the inducing points, y = mu_M and
                                      # noise_var the jitter added to K_MM's diagonal

    @property
    def m(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_vertices(self) -> int:
        return int(np.prod(self.npts[: self.dim]))

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.npts[: self.dim] - 1))

    @property
    def cell_shape(self) -> tuple:
        """Cell-array shape, slowest axis first (x is the fastest axis)."""
        return tuple(int(v - 1) for v in self.npts[: self.dim][::-1])

    @property
    def n_samples(self) -> int:
        return int(self.zbank.shape[0])


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def _bumps(P, amp, ctr, wid):
    """Sum of Gaussian bumps; wid has shape (nb,) (isotropic) or (nb, dim)."""
    d = P[:, None, :] - ctr[None, :, :]
    if wid.ndim == 1:
        q = (d * d).sum(-1) / (wid[None, :] ** 2)
    else:
        q = ((d / wid[None, :, :]) ** 2).sum(-1)
    return (amp[None, :] * np.exp(-0.5 * q)).sum(-1)


def _zbank(seed, n_samples, dim):
    return _rng(seed, 4).standard_normal((n_samples, 2 ** dim))


def _pad3(v, fill):
    out = np.full(3, fill, dtype=np.float64)
    out[: len(v)] = v
    return out


def field2d_bumps(seed: int, m: int = 50, npts: int = 64, n_samples: int = 1600,
                  name: str = "cfg1_2d") -> Workload:
    """2D plain method: m uniform locations, 5 isotropic bumps, SE l=0.1, s2=1."""
    X = _rng(seed, 1).random((m, 2))
    r = _rng(seed, 2)
    amp = r.uniform(0.5, 1.0, 5)
    wid = r.uniform(0.05, 0.2, 5)
    ctr = r.random((5, 2))
    y = _bumps(X, amp, ctr, wid)
    return Workload(name, 2, SE, 1.0, _pad3([0.1, 0.1], 1.0), 1e-4, X, y,
                    _pad3([0, 0], 0.0), _pad3([1, 1], 0.0),
                    np.array([npts, npts, 1], np.int64), 0.5, 1e-3, 4,
                    _zbank(seed, n_samples, 2), seed)


def field3d_aniso(seed: int, m: int = 200, npts: int = 64, n_samples: int = 1600,
                  signal_var: float = 0.1, name: str = "cfg2_3d") -> Workload:
    """3D plain vs FP32: Sobol locations, 8 anisotropic bumps + 0.01 N(0,1) noise,
    ARD SE lengthscales (0.08, 0.12, 0.1), iso-value = median of y."""
    import warnings
    from scipy.stats import qmc
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")  # m need not be a power of two
        X = qmc.Sobol(3, scramble=True, seed=_rng(seed, 1)).random(m)
    r = _rng(seed, 2)
    amp = r.uniform(0.5, 1.0, 8)
    wid = r.uniform(0.05, 0.2, (8, 3))
    ctr = r.random((8, 3))
    y = _bumps(X, amp, ctr, wid) + 0.01 * _rng(seed, 3).standard_normal(m)
    return Workload(name, 3, SE, signal_var, np.array([0.08, 0.12, 0.1]), 1e-4, X, y,
                    np.zeros(3), np.ones(3), np.array([npts] * 3, np.int64),
                    float(np.median(y)), 1e-3, 4, _zbank(seed, n_samples, 3), seed)


def field3d_trig(seed: int, m: int = 500, npts: int = 128, n_samples: int = 1600,
                 signal_var: float = 1e-3, name: Optional[str] = None,
                 iso_quantile: float = 0.5) -> Workload:
    """3D at the paper's scale: m uniform locations, f = sin(6x)cos(5y)sin(4z)
    + 0.3 * (8 isotropic bumps), noise variance 1e-5, Matern-5/2 l=0.1."""
    X = _rng(seed, 1).random((m, 3))
    r = _rng(seed, 2)
    amp = r.uniform(0.5, 1.0, 8)
    wid = r.uniform(0.05, 0.2, 8)
    ctr = r.random((8, 3))
    f = np.sin(6 * X[:, 0]) * np.cos(5 * X[:, 1]) * np.sin(4 * X[:, 2])
    y = f + 0.3 * _bumps(X, amp, ctr, wid) + np.sqrt(1e-5) * _rng(seed, 3).standard_normal(m)
    return Workload(name or f"cfg3_{npts}", 3, MATERN52, signal_var, np.array([0.1, 0.1, 0.1]),
                    1e-5, X, y, np.zeros(3), np.ones(3), np.array([npts] * 3, np.int64),
                    float(np.quantile(y, iso_quantile)), 1e-3, 4,
                    _zbank(seed, n_samples, 3), seed)


def local_blocks(seed: int, nblocks: int = 256, m_range=(64, 1024), side_range=(16, 64), n_samples: int = 1600,
                 signal_var: float = 1.0, noise_var: float = 1e-4, ell_range=(0.05, 0.2), nbumps: int = 4):
    """Batch of independent local GP models: block b has m_b ~ U{m_range} uniform
    observations on [0,1]^3 of its own field (nbumps isotropic bumps), an SE kernel with
    lengthscale ~ U[ell_range], a cubic grid of side s_b ~ U{side_range} vertices and its
    iso-value at the median of its observations.  All blocks share one z-bank."""
    r = _rng(seed, 10)
    zb = _zbank(seed, n_samples, 3)
    out = []
    for b in range(nblocks):
        m = int(r.integers(m_range[0], m_range[1] + 1))
        side = int(r.integers(side_range[0], side_range[1] + 1))
        ell = float(r.uniform(*ell_range))
        X = r.random((m, 3))
        amp = r.uniform(0.5, 1.0, nbumps)
        wid = r.uniform(0.05, 0.2, nbumps)
        ctr = r.random((nbumps, 3))
        y = _bumps(X, amp, ctr, wid)
        out.append(Workload(f"block{b}", 3, SE, signal_var, np.array([ell] * 3), noise_var, X, y,
                            np.zeros(3), np.ones(3), np.array([side] * 3, np.int64),
                            float(np.median(y)), 1e-3, 4, zb, seed))
    return out


def _trig_field(P, seed):
    r = _rng(seed, 2)
    amp = r.uniform(0.5, 1.0, 8)
    wid = r.uniform(0.05, 0.2, 8)
    ctr = r.random((8, 3))
    f = np.sin(6 * P[:, 0]) * np.cos(5 * P[:, 1]) * np.sin(4 * P[:, 2])
    return f + 0.3 * _bumps(P, amp, ctr, wid)


def _se_gram(A, B, s2, ell):
    """s2 exp(-|a - b|^2 / (2 ell^2)), row blocks of A at a time (training only)."""
    out = np.empty((A.shape[0], B.shape[0]))
    for i0 in range(0, A.shape[0], 256):
        d = (A[i0:i0 + 256, None, :] - B[None, :, :]) / ell
        out[i0:i0 + 256] = s2 * np.exp(-0.5 * (d * d).sum(-1))
    return out


def sgpr_field(seed: int, m: int = 500, npts: int = 128, train_npts: int = 32, n_samples: int = 1600,
               signal_var: float = 1e-3, ell: float = 0.12, noise_var: float = 1e-4, jitter: float = 1e-6,
               name: Optional[str] = None) -> Workload:
    """Sparse GP model of eq. (sgp) standing in for the paper's fitted SGPR models
    (Sec. 6.3: 50 or 500 inducing points, RBF kernel, a training grid of the field).

    Inducing points: one in each of m cells drawn without replacement from a c^3
    lattice (c = ceil(m^(1/3))), uniform in the central half of its cell.  Training data:
    the trig field of field3d_trig on a train_npts^3 grid plus N(0, noise_var) noise.
    N(mu_M, A_M) is Titsias' optimal distribution of the inducing values for an SE kernel
    (signal_var, ell) and that noise, with K_MM + jitter I in place of K_MM; the
    reconstruction grid is npts^3 on [0, 1]^3 and the iso-value the median of the data."""
    from scipy.linalg import cho_solve, cholesky, solve_triangular
    c = int(np.ceil(m ** (1.0 / 3.0) - 1e-9))
    r = _rng(seed, 1)
    cells = r.choice(c ** 3, m, replace=False)
    ijk = np.stack([cells % c, (cells // c) % c, cells // (c * c)], 1).astype(np.float64)
    Z = (ijk + 0.25 + 0.5 * r.random((m, 3))) / c
    g = np.linspace(0.0, 1.0, train_npts)
    gz, gy, gx = np.meshgrid(g, g, g, indexing="ij")
    P = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], 1)
    y = _trig_field(P, seed) + np.sqrt(noise_var) * _rng(seed, 3).standard_normal(P.shape[0])
    Kmm = _se_gram(Z, Z, signal_var, ell) + jitter * np.eye(m)
    L = cholesky(Kmm, lower=True)
    Phi = solve_triangular(L, _se_gram(Z, P, signal_var, ell), lower=True)   # L^-1 K_MN
    B = np.eye(m) + (Phi @ Phi.T) / noise_var
    LB = cholesky(B, lower=True)
    R = solve_triangular(LB, L.T, lower=True)                                # LB^-1 L^T
    A_M = R.T @ R                                                            # L B^-1 L^T
    A_M = 0.5 * (A_M + A_M.T)
    mu_M = L @ cho_solve((LB, True), Phi @ y) / noise_var
    return Workload(name or f"sgpr{m}_{npts}", 3, SE, signal_var, np.array([ell] * 3), jitter, Z, mu_M,
                    np.zeros(3), np.ones(3), np.array([npts] * 3, np.int64), float(np.median(y)), 1e-3, 4,
                    _zbank(seed, n_samples, 3), seed, A_M)


def grad_field(seed: int, m: int = 1000, npts: int = 96, n_heldout: int = 2000, n_samples: int = 1600):
    """Differentiation workload: the trig field of field3d_trig observed at m uniform points
    (noise variance 1e-5), an SE kernel with lengthscale 0.1 (the initial value of a learnable
    log-lengthscale), s2 = 1e-3, an npts^3 grid, per-cell loss weights u ~ U[0, 1] and
    n_heldout uniform points with their noise-free field values (for a mean-squared error).
    Returns (workload, weights, held-out points, held-out values)."""
    X = _rng(seed, 1).random((m, 3))
    y = _trig_field(X, seed) + np.sqrt(1e-5) * _rng(seed, 3).standard_normal(m)
    W = Workload(f"grad{npts}", 3, SE, 1e-3, np.array([0.1, 0.1, 0.1]), 1e-5, X, y, np.zeros(3), np.ones(3),
                 np.array([npts] * 3, np.int64), float(np.median(y)), 1e-3, 4, _zbank(seed, n_samples, 3), seed)
    u = _rng(seed, 11).random(W.n_cells)
    P = _rng(seed, 12).random((n_heldout, 3))
    return W, u, P, _trig_field(P, seed)


def random_small(seed: int, dim: int, m: int, npts, kind: int = SE, n_samples: int = 1600,
                 signal_var: float = 1.0, ell: float = 0.25, noise_var: float = 1e-4,
                 min_leaf: int = 1, alpha: float = 1e-3) -> Workload:
    """Tiny random problem for unit and brute-force tests."""
    npts = np.atleast_1d(np.asarray(npts, np.int64))
    if npts.size == 1:
        npts = np.repeat(npts, dim)
    X = _rng(seed, 1).random((m, dim))
    y = np.sin(3.0 * X.sum(1)) + 0.1 * _rng(seed, 3).standard_normal(m)
    return Workload(f"small{dim}d", dim, kind, signal_var, _pad3([ell] * dim, 1.0), noise_var, X, y,
                    _pad3([0.0] * dim, 0.0), _pad3([1.0] * dim, 0.0),
                    np.concatenate([npts, np.ones(3 - dim, np.int64)]),
                    float(np.median(y)), alpha, min_leaf, _zbank(seed, n_samples, dim), seed)


def make(name: str, seed: int = 0, **kw) -> Workload:
    """Named workloads: cfg1_2d, cfg2_3d, cfg3_128, cfg3_256 and reduced variants."""
    if name == "cfg1_2d":
        return field2d_bumps(seed, **kw)
    if name == "cfg2_3d":
        return field3d_aniso(seed, **kw)
    if name == "cfg3_128":
        return field3d_trig(seed, npts=128, **kw)
    if name == "cfg3_256":
        return field3d_trig(seed, npts=256, **kw)
    if name.startswith("sgpr"):        # sgpr<m>_<npts>, e.g. sgpr500_128
        mm, nn = name[4:].split("_")
        return sgpr_field(seed, m=int(mm), npts=int(nn), **kw)
    if name.startswith("cfg3_"):
        return field3d_trig(seed, npts=int(name.split("_")[1]), **kw)
    raise KeyError(name)
