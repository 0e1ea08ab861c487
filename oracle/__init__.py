"""FP64 CPU oracle for the LCP hot path -- test infrastructure only.

Thin ctypes binding over oracle/orc.c.  Only the tests, the smoke check and the
bench's CPU-baseline leg use this package; the GPU library never imports it.
All arrays are numpy float64 unless stated.  See orc.c for the paper passages
each routine follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None

ORC_OK, ORC_ENOTPD, ORC_ECAP, ORC_ENOMEM = 0, 2, 3, 4


class Model(C.Structure):
    _fields_ = [("kind", C.c_int), ("dim", C.c_int), ("m", C.c_int), ("s2", C.c_double),
                ("ell", C.c_double * 3), ("noise", C.c_double), ("X", C.c_void_p),
                ("L", C.c_void_p), ("a", C.c_void_p), ("A", C.c_void_p), ("muM", C.c_void_p),
                ("y", C.c_void_p)]


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("n", C.c_int64 * 3)]


class Adapt(C.Structure):
    _fields_ = [("alpha", C.c_double), ("min_leaf", C.c_int), ("bound_at_max_depth", C.c_int),
                ("steps", C.c_int), ("bound_kind", C.c_int), ("split", C.c_int), ("beta", C.c_double),
                ("edge_bound", C.c_int)]


BOUND_SEARCH, BOUND_CERTIFIED, BOUND_LOCAL = 0, 1, 2
SPLIT_OCTREE, SPLIT_KD = 0, 1


class NodeRec(C.Structure):
    _fields_ = [("key", C.c_uint64), ("level", C.c_int32), ("n_obs", C.c_int32), ("p1", C.c_double),
                ("p2", C.c_double), ("path", C.c_int32), ("subdivide", C.c_int32), ("gmin", C.c_double),
                ("ub", C.c_double), ("lattice_gap", C.c_double), ("d", C.c_int64), ("n_local", C.c_int64),
                ("eb", C.c_double)]


NODE_DTYPE = np.dtype([("key", "<u8"), ("level", "<i4"), ("n_obs", "<i4"), ("p1", "<f8"), ("p2", "<f8"),
                       ("path", "<i4"), ("subdivide", "<i4"), ("gmin", "<f8"), ("ub", "<f8"),
                       ("lattice_gap", "<f8"), ("d", "<i8"), ("n_local", "<i8"), ("eb", "<f8")])
assert NODE_DTYPE.itemsize == C.sizeof(NodeRec)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(
                os.path.join(os.path.dirname(LIB), "orc.c")):
            build()
        _lib = C.CDLL(LIB)
        P = C.c_void_p
        _lib.orc_kernel.restype = C.c_double
        _lib.orc_kernel.argtypes = [C.c_int, C.c_int, C.c_double, P, P, P]
        _lib.orc_kernel_grad.argtypes = [C.c_int, C.c_int, C.c_double, P, P, P, P]
        _lib.orc_fit.argtypes = [C.c_int, C.c_int, C.c_double, P, C.c_double, C.c_int, P, P, P, P]
        _lib.orc_posterior.argtypes = [P, C.c_int64, P, P, P, P]
        _lib.orc_posterior_grad.argtypes = [P, P, P, P, P, P]
        _lib.orc_kernel_dlogell.argtypes = [C.c_int, C.c_int, C.c_double, P, P, P, P]
        _lib.orc_posterior_backward.argtypes = [P, C.c_int64, P, P, P, P, P]
        _lib.orc_sov_lcp.restype = C.c_double
        _lib.orc_sov_lcp.argtypes = [C.c_int, P, P, C.c_double, C.c_int, P]
        _lib.orc_sov_lcp_grad.restype = C.c_double
        _lib.orc_sov_lcp_grad.argtypes = [C.c_int, P, P, C.c_double, C.c_int, P, P, P]
        _lib.orc_chol_sd_rev.argtypes = [C.c_int, P, P, P]
        _lib.orc_lcp_sov_cells.argtypes = [P, P, C.c_double, C.c_int, P, P]
        _lib.orc_lcp_backward.argtypes = [P, P, C.c_double, C.c_int, P, P, P, P]
        _lib.orc_grid_posterior.argtypes = [P, P, P, P]
        _lib.orc_chol_sd.argtypes = [C.c_int, P, P, C.c_double]
        _lib.orc_mc_count.restype = C.c_int64
        _lib.orc_mc_count.argtypes = [C.c_int, P, P, C.c_double, C.c_int, P]
        _lib.orc_lcp_cells.argtypes = [P, P, C.c_double, C.c_int, P, C.c_int64, C.c_int64, P]
        _lib.orc_cell_moments.argtypes = [P, P, P, P, P]
        _lib.orc_upper_bound.restype = C.c_double
        _lib.orc_upper_bound.argtypes = [C.c_double, C.c_int64]
        _lib.orc_bound.argtypes = [P, C.c_double, C.c_double, P, P, C.c_int, P, P]
        _lib.orc_curv3_env.restype = C.c_double
        _lib.orc_curv3_env.argtypes = [C.c_int, C.c_double]
        _lib.orc_kernel_hess.argtypes = [C.c_int, C.c_int, C.c_double, P, P, P, P]
        _lib.orc_bound_certified.argtypes = [P, P, P, P]
        _lib.orc_certified_margin.restype = C.c_double
        _lib.orc_certified_margin.argtypes = [C.c_double, C.c_double, P]
        _lib.orc_local_posterior.restype = C.c_int64
        _lib.orc_local_posterior.argtypes = [P, P, P, C.c_double, C.c_int, C.c_int64, P, P, P]
        _lib.orc_octree_shape.argtypes = [P, C.c_int, P, P]
        _lib.orc_adaptive.argtypes = [P, P, C.c_double, P, P, C.c_int64, P, P, C.c_int64, P, P,
                                      C.c_int64, P]
        _lib.orc_lcp_leaves.argtypes = [P, P, C.c_double, C.c_int, P, C.c_int64, P, C.c_int64, P]
        _lib.orc_level_field.argtypes = [P, C.c_int64, P, C.c_int64, P]
        _lib.orc_level_field_kd.argtypes = [P, C.c_int64, P, C.c_int64, P]
        _lib.orc_num_threads.restype = C.c_int
        _lib.orc_edge_cross.restype = C.c_double
        _lib.orc_edge_cross.argtypes = [C.c_double] * 6
        _lib.orc_node_edge_bound.restype = C.c_double
        _lib.orc_node_edge_bound.argtypes = [P, P, P, P, C.c_double]
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def kernel(kind, dim, s2, ell, x, z):
    ell = _f64(np.resize(np.asarray(ell, float), 3))
    return lib().orc_kernel(kind, dim, s2, _p(ell), _p(_f64(x)), _p(_f64(z)))


def kernel_grad(kind, dim, s2, ell, x, z):
    ell = _f64(np.resize(np.asarray(ell, float), 3))
    g = np.zeros(dim)
    lib().orc_kernel_grad(kind, dim, s2, _p(ell), _p(_f64(x)), _p(_f64(z)), _p(g))
    return g


class FitModel:
    """Factored GP model (exact-GP form of eq. (sgp)): L, a and the ctypes struct."""

    def __init__(self, kind, dim, s2, ell, noise, X, y):
        self.X = _f64(X).reshape(-1, dim)
        self.y = _f64(y)
        m = self.X.shape[0]
        self.ell = _f64(np.resize(np.asarray(ell, float), 3))
        self.L = np.zeros((m, m))
        self.a = np.zeros(m)
        rc = lib().orc_fit(kind, dim, s2, _p(self.ell), noise, m, _p(self.X), _p(self.y), _p(self.L),
                           _p(self.a))
        self.rc = rc
        self.s = Model(kind, dim, m, s2, (C.c_double * 3)(*self.ell), noise, self.X.ctypes.data,
                       self.L.ctypes.data, self.a.ctypes.data, None, None, self.y.ctypes.data)
        self.kind, self.dim, self.m, self.s2, self.noise = kind, dim, m, s2, noise
        self.A = None
        self.vwidth = m


class SparseModel(FitModel):
    """General eq. (sgp): inducing points Z with stored N(mu_M, A_M); K_MM + jitter I."""

    def __init__(self, kind, dim, s2, ell, jitter, Z, mu_M, A_M):
        super().__init__(kind, dim, s2, ell, jitter, Z, mu_M)
        self.A = _f64(A_M).reshape(self.m, self.m)
        self.s.A = self.A.ctypes.data
        self.s.muM = self.y.ctypes.data
        self.s.y = None
        self.vwidth = 3 * self.m


def fit(W):
    """Factor the model of a workloads.Workload (sparse when it carries A_M)."""
    if getattr(W, "A_M", None) is not None:
        M = SparseModel(W.kind, W.dim, W.signal_var, W.lengthscale, W.noise_var, W.X, W.y, W.A_M)
    else:
        M = FitModel(W.kind, W.dim, W.signal_var, W.lengthscale, W.noise_var, W.X, W.y)
    if M.rc != ORC_OK:
        raise np.linalg.LinAlgError(f"oracle fit failed with status {M.rc}")
    return M


def grid_of(W) -> Grid:
    return Grid(W.dim, (C.c_double * 3)(*W.lo), (C.c_double * 3)(*W.hi), (C.c_int64 * 3)(*W.npts))


def posterior(M: FitModel, P, want_v=False):
    P = _f64(P).reshape(-1, M.dim)
    n = P.shape[0]
    mean, var = np.zeros(n), np.zeros(n)
    V = np.zeros((n, M.vwidth)) if want_v else None
    rc = lib().orc_posterior(C.byref(M.s), n, _p(P), _p(mean), _p(var), _p(V))
    assert rc == ORC_OK
    return (mean, var, V) if want_v else (mean, var)


def posterior_grad(M: FitModel, x):
    x = _f64(x)
    mean, var = C.c_double(), C.c_double()
    dm, dv = np.zeros(M.dim), np.zeros(M.dim)
    lib().orc_posterior_grad(C.byref(M.s), _p(x), C.byref(mean), C.byref(var), _p(dm), _p(dv))
    return mean.value, var.value, dm, dv


def posterior_backward(M: FitModel, P, gmean=None, gvar=None):
    """Adjoint of the posterior at points P: (dL/dy, dL/dlog(ell)) for upstream dL/dmean, dL/dvar."""
    P = _f64(P).reshape(-1, M.dim)
    n = P.shape[0]
    gm = None if gmean is None else _f64(gmean)
    gv = None if gvar is None else _f64(gvar)
    dy, dl = np.zeros(M.m), np.zeros(M.dim)
    rc = lib().orc_posterior_backward(C.byref(M.s), n, _p(P), _p(gm), _p(gv), _p(dy), _p(dl))
    assert rc == ORC_OK, rc
    return dy, dl


def kernel_dlogell(kind, dim, s2, ell, x, z):
    ell = _f64(np.resize(np.asarray(ell, float), 3))
    g = np.zeros(dim)
    lib().orc_kernel_dlogell(kind, dim, s2, _p(ell), _p(_f64(x)), _p(_f64(z)), _p(g))
    return g


def grid_posterior(M: FitModel, W):
    n = W.n_vertices
    mean, var = np.zeros(n), np.zeros(n)
    g = grid_of(W)
    assert lib().orc_grid_posterior(C.byref(M.s), C.byref(g), _p(mean), _p(var)) == ORC_OK
    return mean, var


def chol_sd(S, tau=1e-12):
    S = _f64(S)
    n = S.shape[0]
    Cm = np.zeros_like(S)
    r = lib().orc_chol_sd(n, _p(S), _p(Cm), tau)
    return Cm, r


def mc_count(mu, Cm, theta, zb):
    mu, Cm, zb = _f64(mu), _f64(Cm), _f64(zb)
    n = mu.shape[0]
    assert zb.shape[1] == n
    return int(lib().orc_mc_count(n, _p(mu), _p(Cm), theta, zb.shape[0], _p(zb)))


def cell_lcp(mu, S, theta, zb):
    """Monte Carlo LCP of one cell from its corner mean and covariance."""
    Cm, _ = chol_sd(S)
    return mc_count(mu, Cm, theta, zb) / zb.shape[0]


def cell_moments(M: FitModel, W, cell):
    g = grid_of(W)
    nc = 1 << W.dim
    mu, S = np.zeros(nc), np.zeros((nc, nc))
    c = np.zeros(3, np.int64)
    c[: W.dim] = cell
    assert lib().orc_cell_moments(C.byref(M.s), C.byref(g), _p(c), _p(mu), _p(S)) == ORC_OK
    return mu, S


def lcp_dense(M: FitModel, W, c0=0, c1=None):
    """Dense LCP field; cells of slowest-axis layers [c0, c1), shape (layers, ..., nx-1)."""
    g = grid_of(W)
    sa = W.dim - 1
    if c1 is None:
        c1 = int(W.npts[sa]) - 1
    shape = [c1 - c0] + [int(W.npts[d]) - 1 for d in range(sa - 1, -1, -1)]
    out = np.zeros(int(np.prod(shape)))
    zb = _f64(W.zbank)
    rc = lib().orc_lcp_cells(C.byref(M.s), C.byref(g), W.theta, zb.shape[0], _p(zb), c0, c1, _p(out))
    assert rc == ORC_OK
    return out.reshape(shape)


def sov_lcp(mu, Cm, theta, zb):
    """Smooth (separation-of-variables) LCP of one cell from its mean and factor."""
    mu, Cm, zb = _f64(mu), _f64(Cm), _f64(zb)
    return lib().orc_sov_lcp(mu.shape[0], _p(mu), _p(Cm), theta, zb.shape[0], _p(zb))


def sov_lcp_grad(mu, Cm, theta, zb):
    mu, Cm, zb = _f64(mu), _f64(Cm), _f64(zb)
    n = mu.shape[0]
    gmu, gC = np.zeros(n), np.zeros((n, n))
    v = lib().orc_sov_lcp_grad(n, _p(mu), _p(Cm), theta, zb.shape[0], _p(zb), _p(gmu), _p(gC))
    return v, gmu, gC


def chol_sd_rev(Cm, gC):
    Cm, gC = _f64(Cm), _f64(gC)
    gS = np.zeros_like(Cm)
    lib().orc_chol_sd_rev(Cm.shape[0], _p(Cm), _p(gC), _p(gS))
    return gS


def lcp_sov_dense(M: FitModel, W):
    """Smooth LCP of every cell (cell-array shape)."""
    g = grid_of(W)
    out = np.zeros(W.n_cells)
    zb = _f64(W.zbank)
    assert lib().orc_lcp_sov_cells(C.byref(M.s), C.byref(g), W.theta, zb.shape[0], _p(zb), _p(out)) == ORC_OK
    return out.reshape(W.cell_shape)


def lcp_backward(M: FitModel, W, gl):
    """Adjoint of the smooth LCP field: (dL/dy, dL/dlog(ell)) for upstream dL/dLCP per cell."""
    g = grid_of(W)
    zb = _f64(W.zbank)
    gl = _f64(gl).reshape(-1)
    dy, dl = np.zeros(M.m), np.zeros(M.dim)
    rc = lib().orc_lcp_backward(C.byref(M.s), C.byref(g), W.theta, zb.shape[0], _p(zb), _p(gl), _p(dy), _p(dl))
    assert rc == ORC_OK, rc
    return dy, dl


def upper_bound(gmin, d):
    return lib().orc_upper_bound(float(gmin), int(d))


def bound(M: FitModel, theta, side, blo, bhi, steps=4):
    gmin, gap = C.c_double(), C.c_double()
    lib().orc_bound(C.byref(M.s), theta, float(side), _p(_f64(blo)), _p(_f64(bhi)), steps, C.byref(gmin),
                    C.byref(gap))
    return gmin.value, gap.value


def curv3_env(kind, r2):
    """Sup over scaled distances >= sqrt(r2) of the largest third directional derivative of
    the kernel along a unit scaled direction (unit signal variance)."""
    return lib().orc_curv3_env(int(kind), float(r2))


def kernel_hess(kind, dim, s2, ell, x, z):
    ell = _f64(np.resize(np.asarray(ell, float), 3))
    Hm = np.zeros(dim * dim)
    lib().orc_kernel_hess(kind, dim, s2, _p(ell), _p(_f64(x)), _p(_f64(z)), _p(Hm))
    return Hm.reshape(dim, dim)


def bound_certified(M: FitModel, blo, bhi):
    """Certified box bounds: (mu(centre), mu_lo, mu_hi, var_hi) over the box [blo, bhi]."""
    out = np.zeros(4)
    rc = lib().orc_bound_certified(C.byref(M.s), _p(_f64(blo)), _p(_f64(bhi)), _p(out))
    assert rc == ORC_OK, rc
    return out


def certified_margin(side, theta, cb):
    return lib().orc_certified_margin(float(side), float(theta), _p(_f64(cb)))


def octree_shape(W, min_leaf=None):
    g = grid_of(W)
    S0, L = C.c_int64(), C.c_int()
    lib().orc_octree_shape(C.byref(g), int(min_leaf or W.min_leaf), C.byref(S0), C.byref(L))
    return S0.value, L.value


def adaptive(M: FitModel, W, alpha=None, min_leaf=None, bound_at_max_depth=1, steps=4, cap=1 << 22,
             bound_kind=BOUND_SEARCH, split=SPLIT_OCTREE, beta=6.0, edge_bound=0):
    """Alg. 1: returns (leaves, skipped, node records), each sorted by key.  With the K-D
    tree, records and skipped keys carry the depth (0 .. dim Lmax); leaves keep the octree
    key of the finest level.  BOUND_LOCAL runs the region test on the local model of
    Sec. 5.2 (box enlarged by beta lengthscales).  edge_bound=1 emits a deepest-level node
    only if its edge-crossing union bound (record field eb) exceeds alpha."""
    g = grid_of(W)
    A = Adapt(float(alpha if alpha is not None else W.alpha), int(min_leaf or W.min_leaf),
              int(bound_at_max_depth), int(steps), int(bound_kind), int(split), float(beta), int(edge_bound))
    leaves = np.zeros(cap, np.uint64)
    skipped = np.zeros(cap, np.uint64)
    recs = np.zeros(cap, NODE_DTYPE)
    nl, ns, nr = C.c_int64(), C.c_int64(), C.c_int64()
    rc = lib().orc_adaptive(C.byref(M.s), C.byref(g), W.theta, C.byref(A), _p(leaves), cap, C.byref(nl),
                            _p(skipped), cap, C.byref(ns), _p(recs), cap, C.byref(nr))
    assert rc == ORC_OK, rc
    return leaves[: nl.value].copy(), skipped[: ns.value].copy(), recs[: nr.value].copy()


def local_posterior(M: FitModel, blo, bhi, beta, P, whole=False):
    """Posterior of the local model M' of Sec. 5.2 for the box [blo, bhi] at points P:
    (mean, var, |M'|)."""
    P = _f64(P).reshape(-1, M.dim)
    n = P.shape[0]
    mean, var = np.zeros(n), np.zeros(n)
    ml = lib().orc_local_posterior(C.byref(M.s), _p(_f64(blo)), _p(_f64(bhi)), float(beta), int(whole), n, _p(P),
                                   _p(mean), _p(var))
    assert ml >= 0, ml
    return mean, var, int(ml)


def lcp_leaves(M: FitModel, W, leaves, min_leaf=None):
    """LCP on the cells of the given leaves, zero elsewhere (shape = cell grid)."""
    g = grid_of(W)
    S0, _ = octree_shape(W, min_leaf)
    out = np.zeros(W.n_cells)
    zb = _f64(W.zbank)
    keys = np.ascontiguousarray(leaves, np.uint64)
    rc = lib().orc_lcp_leaves(C.byref(M.s), C.byref(g), W.theta, zb.shape[0], _p(zb), S0, _p(keys),
                              keys.shape[0], _p(out))
    assert rc == ORC_OK
    return out.reshape(W.cell_shape)


def level_field(W, keys, min_leaf=None):
    g = grid_of(W)
    S0, _ = octree_shape(W, min_leaf)
    out = np.full(W.n_cells, 255, np.uint8)
    k = np.ascontiguousarray(keys, np.uint64)
    lib().orc_level_field(C.byref(g), S0, _p(k), k.shape[0], _p(out))
    return out.reshape(W.cell_shape)


def kd_leaf_keys(W, leaves, min_leaf=None):
    """Leaves (octree keys of the finest level) as K-D tree keys of depth dim * Lmax."""
    _, L = octree_shape(W, min_leaf)
    mask = np.uint64((1 << 58) - 1)
    return (np.asarray(leaves, np.uint64) & mask) | np.uint64((W.dim * L) << 58)


def level_field_kd(W, keys, min_leaf=None):
    """Depth at which each cell's K-D tree node stopped, from K-D keys."""
    g = grid_of(W)
    S0, _ = octree_shape(W, min_leaf)
    out = np.full(W.n_cells, 255, np.uint8)
    k = np.ascontiguousarray(keys, np.uint64)
    lib().orc_level_field_kd(C.byref(g), S0, _p(k), k.shape[0], _p(out))
    return out.reshape(W.cell_shape)


def num_threads():
    return int(lib().orc_num_threads())


def edge_cross(mua, mub, va, vb, c, theta):
    """P(edge crossed) for the bivariate normal of the two end values (Sec. 9 reading)."""
    return lib().orc_edge_cross(float(mua), float(mub), float(va), float(vb), float(c), float(theta))


def node_edge_bound(M: FitModel, W, vlo, vhi):
    """Edge-crossing union bound of the node spanning vertices vlo .. vhi (inclusive)."""
    g = grid_of(W)
    lo = np.zeros(3, np.int64)
    hi = np.zeros(3, np.int64)
    lo[: W.dim], hi[: W.dim] = vlo, vhi
    return lib().orc_node_edge_bound(C.byref(M.s), C.byref(g), _p(lo), _p(hi), W.theta)
