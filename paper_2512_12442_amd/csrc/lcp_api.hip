// Host side of the C ABI declared in include/lcp.h: argument validation, workspace
// carving and the order in which the kernels of the hot path are enqueued.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "lcp_internal.h"

struct lcp_model : lcp::Model {};

struct lcp_model_batch {
    std::vector<lcp_model> models;
    char* scratch;            // factor descriptors and statuses (end of the model memory)
};

using namespace lcp;

namespace {

thread_local char g_err[512] = "";

int fail(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return status;
}

int ok()
{
    g_err[0] = 0;
    return LCP_OK;
}

int dev_fail(hipError_t e, const char* where)
{
    return fail(LCP_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255) == 0; }
bool is_finite(double x) { return isfinite(x) != 0; }

int check_prec(int prec)
{
    if (prec != LCP_FP64 && prec != LCP_FP32 && prec != LCP_MIXED_BF16X3 && prec != LCP_MIXED_F16X3)
        return fail(LCP_EINVAL, "unknown precision %d", prec);
    return LCP_OK;
}

int check_kernel(const lcp_kernel* k, int m)
{
    if (k->dim != 2 && k->dim != 3) return fail(LCP_EINVAL, "dim must be 2 or 3 (got %d)", k->dim);
    if (k->kind != LCP_KERNEL_SE && k->kind != LCP_KERNEL_MATERN52) return fail(LCP_EINVAL, "unknown kernel %d", k->kind);
    if (!(k->signal_var > 0.0) || !is_finite(k->signal_var)) return fail(LCP_EINVAL, "signal_var must be finite and > 0");
    if (!(k->noise_var >= 0.0) || !is_finite(k->noise_var)) return fail(LCP_EINVAL, "noise_var must be finite and >= 0");
    for (int d = 0; d < k->dim; ++d)
        if (!(k->lengthscale[d] > 0.0) || !is_finite(k->lengthscale[d]))
            return fail(LCP_EINVAL, "lengthscale[%d] must be finite and > 0", d);
    if (m < 1 || m > kMaxM) return fail(LCP_EINVAL, "m = %d outside 1..%d", m, kMaxM);
    return LCP_OK;
}

void init_model(Model& M, const lcp_kernel& k, int m, void* mem)
{
    M.k = k;
    M.dim = k.dim;
    M.m = m;
    M.m_pad = (m + 127) / 128 * 128;
    M.nrb = (m + 15) / 16;
    M.kp.kind = k.kind;
    M.kp.dim = k.dim;
    M.kp.s2 = k.signal_var;
    for (int d = 0; d < 3; ++d) M.kp.inv_ell[d] = d < k.dim ? 1.0 / k.lengthscale[d] : 0.0;
    M.X = (double*)mem;
    if (hipGetDevice(&M.device) != hipSuccess) M.device = -1;
}

int check_grid(const lcp_model* M, const lcp_grid* g, GridP* out)
{
    if (!g) return fail(LCP_EINVAL, "grid is NULL");
    if (g->dim != M->dim) return fail(LCP_EINVAL, "grid dim %d differs from model dim %d", g->dim, M->dim);
    GridP p{};
    p.dim = g->dim;
    int64_t nv = 1;
    for (int d = 0; d < 3; ++d) {
        if (d < g->dim) {
            if (g->npts[d] < 2) return fail(LCP_EINVAL, "npts[%d] = %lld < 2", d, (long long)g->npts[d]);
            if (g->npts[d] > (1 << 20)) return fail(LCP_EINVAL, "npts[%d] too large", d);
            if (!is_finite(g->lo[d]) || !is_finite(g->hi[d]) || !(g->hi[d] > g->lo[d]))
                return fail(LCP_EINVAL, "grid axis %d needs finite lo < hi", d);
            p.lo[d] = g->lo[d];
            p.h[d] = (g->hi[d] - g->lo[d]) / (double)(g->npts[d] - 1);
            p.n[d] = g->npts[d];
            p.nc[d] = g->npts[d] - 1;
        } else {
            p.lo[d] = 0.0;
            p.h[d] = 0.0;
            p.n[d] = 1;
            p.nc[d] = 1;
        }
        nv *= p.n[d];
    }
    if (nv > ((int64_t)1 << 31) - 1) return fail(LCP_EINVAL, "grid has more than 2^31 - 1 vertices");
    *out = p;
    return LCP_OK;
}

int check_mc(const lcp_model* M, const lcp_mc* mc)
{
    if (!mc) return fail(LCP_EINVAL, "mc is NULL");
    if (mc->n_samples < 1 || mc->n_samples > (1 << 24)) return fail(LCP_EINVAL, "n_samples = %d", mc->n_samples);
    if (!mc->zbank) return fail(LCP_EINVAL, "zbank is NULL");
    if (mc->estimator != LCP_EST_COUNT && mc->estimator != LCP_EST_SOV)
        return fail(LCP_EINVAL, "estimator = %d", mc->estimator);
    (void)M;
    return LCP_OK;
}

int ndir(int D) { return D == 3 ? 13 : 4; }

size_t dense_ws(const lcp_model* M, const GridP& g, int prec, int ns)
{
    const int64_t nv = g.n[0] * g.n[1] * g.n[2];
    const size_t vb = prec == LCP_FP64 ? 8 : 4;
    size_t b = 0;
    b += align256(sizeof(double) * nv);                      // mean
    b += align256(sizeof(double) * nv);                      // var
    b += align256(vb * (size_t)nv * M->m_pad);               // V
    b += align256(sizeof(double) * (size_t)nv * ndir(g.dim)); // cross
    b += zbank32_bytes(ns, g.dim);                           // FP32 z-bank and split records
    b += align256(sizeof(double) * ((size_t)ns * (1 << g.dim) + 1)); // uniforms of the smooth estimator, max |z|
    b += cells_scratch_bytes(g.nc[0] * g.nc[1] * g.nc[2]);   // Monte Carlo work list
    return b;
}

void octree_shape(const GridP& g, int min_leaf, int64_t* S0, int* Lmax)
{
    int64_t mx = 1;
    for (int d = 0; d < g.dim; ++d)
        if (g.nc[d] > mx) mx = g.nc[d];
    int64_t s = 1;
    while (s < mx) s <<= 1;
    int l = 0;
    while ((s >> l) > min_leaf) ++l;
    *S0 = s;
    *Lmax = l;
}

int check_adapt(const Model& M, const lcp_adapt* A)
{
    if (!A) return fail(LCP_EINVAL, "adapt is NULL");
    if (!(A->alpha > 0.0 && A->alpha < 0.5)) return fail(LCP_EINVAL, "alpha must lie in (0, 0.5)");
    if (A->min_leaf_cells < 1 || (A->min_leaf_cells & (A->min_leaf_cells - 1)))
        return fail(LCP_EINVAL, "min_leaf_cells must be a power of two >= 1");
    if (A->bound_at_max_depth != 0 && A->bound_at_max_depth != 1)
        return fail(LCP_EINVAL, "bound_at_max_depth must be 0 or 1");
    if (A->descent_steps < 0 || A->descent_steps > 16) return fail(LCP_EINVAL, "descent_steps must be in 0..16");
    if (A->bound_kind != LCP_BOUND_SEARCH && A->bound_kind != LCP_BOUND_CERTIFIED && A->bound_kind != LCP_BOUND_LOCAL)
        return fail(LCP_EINVAL, "bound_kind must be LCP_BOUND_SEARCH, LCP_BOUND_CERTIFIED or LCP_BOUND_LOCAL");
    if (A->bound_kind == LCP_BOUND_LOCAL) {
        if (!(is_finite(A->beta) && A->beta >= 0.0)) return fail(LCP_EINVAL, "beta must be finite and >= 0");
    }
    if (A->split != LCP_SPLIT_OCTREE && A->split != LCP_SPLIT_KD)
        return fail(LCP_EINVAL, "split must be LCP_SPLIT_OCTREE or LCP_SPLIT_KD");
    if (A->edge_bound != 0 && A->edge_bound != 1) return fail(LCP_EINVAL, "edge_bound must be 0 or 1");
    return LCP_OK;
}

}  // namespace

extern "C" {

const char* lcp_status_str(int status)
{
    switch (status) {
    case LCP_OK: return "ok";
    case LCP_EINVAL: return "invalid argument";
    case LCP_ENOTPD: return "covariance matrix is not positive definite";
    case LCP_ECAPACITY: return "output capacity too small";
    case LCP_ENOMEM: return "model memory or workspace too small";
    case LCP_EDEVICE: return "HIP runtime error";
    case LCP_ENOTSUPPORTED: return "not supported";
    default: return "unknown status";
    }
}

const char* lcp_last_error(void) { return g_err; }

size_t lcp_model_bytes(int m, int dim)
{
    (void)dim;
    if (m < 1 || m > kMaxM) return 0;
    return model_bytes(m);
}

int gp_fit_factor(const lcp_kernel* k, int m, const double* X, const double* y, void* model_mem, size_t model_bytes_,
                  void* stream, lcp_model** out)
{
    if (!k || !out) return fail(LCP_EINVAL, "kernel and out must not be NULL");
    *out = nullptr;
    if (int r = check_kernel(k, m)) return r;
    if (!X || !y || !model_mem) return fail(LCP_EINVAL, "X, y and model_mem must not be NULL");
    if (!aligned256(model_mem)) return fail(LCP_EINVAL, "model_mem must be 256-byte aligned");
    if (model_bytes_ < model_bytes(m)) return fail(LCP_ENOMEM, "model memory %zu < %zu bytes", model_bytes_, model_bytes(m));
    lcp_model* M = new (std::nothrow) lcp_model();
    if (!M) return fail(LCP_ENOMEM, "host allocation failed");
    init_model(*M, *k, m, model_mem);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_factor(*M, X, y, s);
    if (e != hipSuccess) { delete M; return dev_fail(e, "factor"); }
    int info = 0;
    e = hipMemcpyAsync(&info, M->info, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { delete M; return dev_fail(e, "factor status"); }
    if (info != 0) {
        delete M;
        return fail(LCP_ENOTPD, "Cholesky pivot %d is not above m * eps * max K_ii", info);
    }
    e = launch_factor_finish(*M, s);
    if (e != hipSuccess) { delete M; return dev_fail(e, "factor finish"); }
    *out = M;
    return ok();
}

int gp_fit_sgpr(const lcp_kernel* k, int m, const double* Z, const double* mu_M, const double* A_M,
                void* model_mem, size_t model_bytes_, void* stream, double* shift, lcp_model** out)
{
    if (!k || !out) return fail(LCP_EINVAL, "kernel and out must not be NULL");
    *out = nullptr;
    if (shift) *shift = 0.0;
    if (int r = check_kernel(k, m)) return r;
    if (!Z || !mu_M || !A_M || !model_mem) return fail(LCP_EINVAL, "Z, mu_M, A_M and model_mem must not be NULL");
    if (!aligned256(model_mem)) return fail(LCP_EINVAL, "model_mem must be 256-byte aligned");
    if (model_bytes_ < model_bytes(m)) return fail(LCP_ENOMEM, "model memory %zu < %zu bytes", model_bytes_, model_bytes(m));
    lcp_model* M = new (std::nothrow) lcp_model();
    if (!M) return fail(LCP_ENOMEM, "host allocation failed");
    init_model(*M, *k, m, model_mem);
    hipStream_t s = (hipStream_t)stream;
    auto status = [&](int idx, int* info) {
        hipError_t e = hipMemcpyAsync(info, M->info + idx, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    };
    hipError_t e = launch_factor(*M, Z, mu_M, s);
    int info = 0;
    if (e == hipSuccess) e = status(0, &info);
    if (e != hipSuccess) { delete M; return dev_fail(e, "sparse factor"); }
    if (info != 0) {
        delete M;
        return fail(LCP_ENOTPD, "K_MM + jitter I: Cholesky pivot %d is not above m * eps * max K_ii", info);
    }
    // E = I - L^-1 A_M L^-T is PSD when A_M <= K_MM + jitter I; a pivot at rounding level is
    // met by factoring E + delta I, delta from 16 m eps up to 1e-6 in steps of 100.
    double delta = 0.0;
    for (;;) {
        e = launch_sparse_e(*M, A_M, delta, delta == 0.0, s);
        if (e == hipSuccess) e = status(1, &info);
        if (e != hipSuccess) { delete M; return dev_fail(e, "sparse factor"); }
        if (info == 0) break;
        if (delta >= 1e-6) {
            delete M;
            return fail(LCP_ENOTPD, "A_M is not below K_MM + jitter I: I - L^-1 A_M L^-T has pivot %d at or "
                        "below m * eps even when shifted by 1e-6", info);
        }
        delta = delta == 0.0 ? 16.0 * m * 2.220446049250313e-16 : fmin(delta * 100.0, 1e-6);
    }
    e = launch_sparse_finish(*M, s);
    if (e != hipSuccess) { delete M; return dev_fail(e, "sparse factor finish"); }
    M->sparse = 1;
    if (shift) *shift = delta;
    *out = M;
    return ok();
}

void gp_model_free(lcp_model* model) { delete model; }

int lcp_posterior_workspace(const lcp_model* M, int64_t n, int prec, size_t* bytes)
{
    if (!M || !bytes) return fail(LCP_EINVAL, "model and bytes must not be NULL");
    if (n < 0) return fail(LCP_EINVAL, "n < 0");
    if (check_prec(prec)) return LCP_EINVAL;
    *bytes = 0;
    return ok();
}

int lcp_dense_workspace(const lcp_model* M, const lcp_grid* grid, int prec, int n_samples, size_t* bytes)
{
    if (!M || !bytes) return fail(LCP_EINVAL, "model and bytes must not be NULL");
    if (check_prec(prec)) return LCP_EINVAL;
    if (n_samples < 1) return fail(LCP_EINVAL, "n_samples < 1");
    GridP g;
    if (int r = check_grid(M, grid, &g)) return r;
    *bytes = dense_ws(M, g, prec, n_samples);
    return ok();
}

int lcp_adaptive_workspace(const lcp_model* M, const lcp_grid* grid, const lcp_adapt* A, int prec, int n_samples,
                           size_t* bytes)
{
    if (!M || !bytes) return fail(LCP_EINVAL, "model and bytes must not be NULL");
    if (check_prec(prec)) return LCP_EINVAL;
    if (n_samples < 1) return fail(LCP_EINVAL, "n_samples < 1");
    GridP g;
    if (int r = check_grid(M, grid, &g)) return r;
    if (int r = check_adapt(*M, A)) return r;
    int64_t S0;
    int Lmax;
    octree_shape(g, A->min_leaf_cells, &S0, &Lmax);
    if (Lmax > 7) return fail(LCP_EINVAL, "octree deeper than 8 levels (raise min_leaf_cells)");
    *bytes = adaptive_workspace(*M, g, S0, Lmax, prec, n_samples, *A);
    return ok();
}

int gp_posterior(const lcp_model* M, int64_t n, const double* Xq, int prec, double* mean, double* var, void* ws,
                 size_t ws_bytes, void* stream)
{
    (void)ws;
    (void)ws_bytes;
    if (!M) return fail(LCP_EINVAL, "model is NULL");
    if (n < 0) return fail(LCP_EINVAL, "n < 0");
    if (check_prec(prec)) return LCP_EINVAL;
    if (n == 0) return ok();
    if (!Xq || !mean || !var) return fail(LCP_EINVAL, "Xq, mean and var must not be NULL");
    PostTask t{};
    t.mode = COL_POINTS;
    t.group = 1;
    t.count = nullptr;
    t.n_points = n;
    t.pts = Xq;
    t.pstride = M->dim;
    t.mean = mean;
    t.var = var;
    t.stage = ST_POSTERIOR;
    hipError_t e = launch_posterior(*M, prec, t, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "gp_posterior");
    return ok();
}

int gp_posterior_backward_workspace(const lcp_model* M, int64_t n, int prec, size_t* bytes)
{
    if (!M || !bytes) return fail(LCP_EINVAL, "model and bytes must not be NULL");
    if (n < 0) return fail(LCP_EINVAL, "n < 0");
    if (prec != LCP_FP64 && prec != LCP_FP32) return fail(LCP_EINVAL, "prec must be LCP_FP64 or LCP_FP32");
    *bytes = posterior_backward_ws(*M, n, prec);
    return ok();
}

int gp_posterior_backward(const lcp_model* M, int64_t n, const double* Xq, int prec, const double* dL_dmean,
                          const double* dL_dvar, double* dL_dy, double* dL_dloglen, void* ws, size_t ws_bytes,
                          void* stream)
{
    if (!M) return fail(LCP_EINVAL, "model is NULL");
    if (M->sparse) return fail(LCP_ENOTSUPPORTED, "gp_posterior_backward: the model comes from gp_fit_sgpr");
    if (n < 0) return fail(LCP_EINVAL, "n < 0");
    if (prec != LCP_FP64 && prec != LCP_FP32) return fail(LCP_EINVAL, "prec must be LCP_FP64 or LCP_FP32");
    if (!dL_dy || !dL_dloglen) return fail(LCP_EINVAL, "dL_dy and dL_dloglen must not be NULL");
    if (n > 0 && !Xq) return fail(LCP_EINVAL, "Xq must not be NULL");
    const size_t need = posterior_backward_ws(*M, n, prec);
    if (!ws || !aligned256(ws)) return fail(LCP_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < need) return fail(LCP_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    hipError_t e = launch_posterior_backward(*M, n, Xq, prec, n > 0 ? dL_dmean : nullptr, n > 0 ? dL_dvar : nullptr,
                                             dL_dy, dL_dloglen, (char*)ws, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "gp_posterior_backward");
    return ok();
}

namespace {

struct MomentsWs {
    int32_t* vmask;
    int32_t* voff;
    int32_t* slot;
    int32_t* vlist;
    int64_t* count;
    char* scan;
    double* mean;
    double* var;
    void* V;
    double* cross;
};

// Workspace of lcp_cell_moments: per-vertex flags, offsets and slots over the whole grid,
// then posterior, V (quad-major) and cross terms for at most min(n 2^D, vertices) slots.
size_t moments_ws(const lcp_model* M, const GridP& g, int64_t n, int prec, MomentsWs* w, char* p)
{
    const int64_t nv = g.n[0] * g.n[1] * g.n[2];
    int64_t cap = n << g.dim;
    if (cap > nv) cap = nv;
    if (cap < 1) cap = 1;
    const size_t vb = prec == LCP_FP64 ? 8 : 4;
    const size_t sizes[10] = {4 * (size_t)nv, 4 * (size_t)nv, 4 * (size_t)nv, 4 * (size_t)cap, 8,
                              scan_workspace(nv), 8 * (size_t)cap, 8 * (size_t)cap, vb * (size_t)cap * M->m_pad,
                              8 * (size_t)cap * ndir(g.dim)};
    size_t o = 0;
    void* ptrs[10];
    for (int i = 0; i < 10; ++i) {
        ptrs[i] = p ? p + o : nullptr;
        o += align256(sizes[i]);
    }
    if (w) {
        w->vmask = (int32_t*)ptrs[0];
        w->voff = (int32_t*)ptrs[1];
        w->slot = (int32_t*)ptrs[2];
        w->vlist = (int32_t*)ptrs[3];
        w->count = (int64_t*)ptrs[4];
        w->scan = (char*)ptrs[5];
        w->mean = (double*)ptrs[6];
        w->var = (double*)ptrs[7];
        w->V = ptrs[8];
        w->cross = (double*)ptrs[9];
    }
    return o;
}

}  // namespace

int lcp_cell_moments_workspace(const lcp_model* M, const lcp_grid* grid, int64_t n, int prec, size_t* bytes)
{
    if (!M || !bytes) return fail(LCP_EINVAL, "model and bytes must not be NULL");
    if (n < 0) return fail(LCP_EINVAL, "n < 0");
    if (check_prec(prec)) return LCP_EINVAL;
    GridP g;
    if (int r = check_grid(M, grid, &g)) return r;
    *bytes = moments_ws(M, g, n, prec, nullptr, nullptr);
    return ok();
}

int lcp_cell_moments(const lcp_model* M, const lcp_grid* grid, int64_t n, const int64_t* cells, int prec,
                     double* mean, double* cov, void* ws, size_t ws_bytes, void* stream)
{
    if (!M) return fail(LCP_EINVAL, "model is NULL");
    if (n < 0) return fail(LCP_EINVAL, "n < 0");
    if (check_prec(prec)) return LCP_EINVAL;
    GridP g;
    if (int r = check_grid(M, grid, &g)) return r;
    if (n == 0) return ok();
    if (!cells || !mean || !cov || !ws) return fail(LCP_EINVAL, "cells, mean, cov and ws must not be NULL");
    if (!aligned256(ws)) return fail(LCP_EINVAL, "workspace must be 256-byte aligned");
    MomentsWs w;
    const size_t need = moments_ws(M, g, n, prec, &w, (char*)ws);
    if (ws_bytes < need) return fail(LCP_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    const int64_t nv = g.n[0] * g.n[1] * g.n[2];
    int64_t cap = n << g.dim;
    if (cap > nv) cap = nv;
    hipError_t e = launch_fill_i32(w.vmask, 0, nv, s);
    if (e == hipSuccess) e = launch_mark_cells(g, cells, n, w.vmask, s);
    if (e == hipSuccess) e = launch_scan(w.vmask, w.voff, nv, nullptr, w.count, w.scan, s);
    if (e == hipSuccess) e = launch_vertex_slots(w.vmask, w.voff, nv, w.slot, w.vlist, s);
    if (e != hipSuccess) return dev_fail(e, "lcp_cell_moments: vertex slots");
    PostTask t{};
    t.mode = COL_GRID;
    t.group = 1;
    t.count = w.count;
    t.n_points = cap;
    t.grid = g;
    t.vlist = w.vlist;
    t.mean = w.mean;
    t.var = w.var;
    t.V = w.V;
    t.stage = ST_POSTERIOR;
    e = launch_posterior(*M, prec, t, s);
    if (e == hipSuccess) e = launch_cross(*M, prec, g, w.vlist, w.count, cap, w.slot, w.V, w.cross, s);
    if (e == hipSuccess) e = launch_cell_moments(g, cells, n, w.slot, w.mean, w.var, w.cross, mean, cov, s);
    if (e != hipSuccess) return dev_fail(e, "lcp_cell_moments");
    return ok();
}

int lcp_bound_workspace(const lcp_model* M, int64_t n, size_t* bytes)
{
    if (!M || !bytes) return fail(LCP_EINVAL, "model and bytes must not be NULL");
    if (n < 0) return fail(LCP_EINVAL, "n < 0");
    *bytes = bound_certified_ws(*M, n);
    return ok();
}

int lcp_bound_certified(const lcp_model* M, int64_t n, const double* boxes, double* out, void* ws, size_t ws_bytes,
                        void* stream)
{
    if (!M) return fail(LCP_EINVAL, "model is NULL");
    if (n < 0) return fail(LCP_EINVAL, "n < 0");
    if (n > 0 && (!boxes || !out)) return fail(LCP_EINVAL, "boxes and out must not be NULL");
    const size_t need = bound_certified_ws(*M, n);
    if (!ws || !aligned256(ws)) return fail(LCP_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < need) return fail(LCP_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    hipError_t e = launch_bound_certified(*M, n, boxes, out, (char*)ws, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "lcp_bound_certified");
    return ok();
}

namespace {

// Workspace of one dense evaluation (layout of dense_ws).
struct DenseWs {
    double* mean;
    double* var;
    void* V;
    double* cross;
    float* zb32;
    double* wb;
    int32_t* work;
    int64_t* wcount;
    double* zmax;
};

DenseWs carve_dense(const lcp_model* M, const GridP& g, int prec, int ns, char* p)
{
    DenseWs w;
    const int64_t nv = g.n[0] * g.n[1] * g.n[2];
    const size_t vb = prec == LCP_FP64 ? 8 : 4;
    w.mean = (double*)p;
    p += align256(sizeof(double) * nv);
    w.var = (double*)p;
    p += align256(sizeof(double) * nv);
    w.V = p;
    p += align256(vb * (size_t)nv * M->m_pad);
    w.cross = (double*)p;
    p += align256(sizeof(double) * (size_t)nv * ndir(g.dim));
    w.zb32 = (float*)p;
    p += zbank32_bytes(ns, g.dim);
    w.wb = (double*)p;
    p += align256(sizeof(double) * ((size_t)ns * (1 << g.dim) + 1));
    const int64_t ncells = g.nc[0] * g.nc[1] * g.nc[2];
    w.work = (int32_t*)p;
    p += align256(4 * (size_t)ncells);
    w.wcount = (int64_t*)p;
    w.zmax = (double*)(p + 64);
    return w;
}

PostTask dense_task(const GridP& g, const DenseWs& w)
{
    PostTask t{};
    t.mode = COL_GRID;
    t.group = 1;
    t.count = nullptr;
    t.n_points = g.n[0] * g.n[1] * g.n[2];
    t.grid = g;
    t.vlist = nullptr;
    t.mean = w.mean;
    t.var = w.var;
    t.V = w.V;
    t.stage = ST_POSTERIOR;
    return t;
}

// Cross-covariances and cell Monte Carlo of a dense evaluation whose posterior (mean, var, V)
// is in w; zb32 is the FP32 z-bank (unused for binary64).
int dense_cells(const lcp_model* M, const GridP& g, double theta, const lcp_mc* mc, int prec, const DenseWs& w,
                const float* zb32, float* lcp, hipStream_t s)
{
    const int64_t nv = g.n[0] * g.n[1] * g.n[2];
    hipError_t e = launch_cross(*M, prec, g, nullptr, nullptr, nv, nullptr, w.V, w.cross, s);
    if (e != hipSuccess) return dev_fail(e, "cross");
    CellTask ct{};
    ct.grid = g;
    ct.prec = prec;
    ct.theta = theta;
    ct.ns = mc->n_samples;
    ct.zb64 = mc->zbank;
    ct.zb32 = zb32;
    ct.mean = w.mean;
    ct.var = w.var;
    ct.cross = w.cross;
    ct.slot = nullptr;
    ct.leaves = nullptr;
    ct.lcp = lcp;
    ct.work = w.work;
    ct.wcount = w.wcount;
    ct.zmax = w.zmax;
    if (mc->estimator == LCP_EST_SOV) {
        e = launch_cells_sov(ct, w.wb, s);
    } else {
        e = launch_cells(ct, g.nc[0] * g.nc[1] * g.nc[2], s);
    }
    if (e != hipSuccess) return dev_fail(e, "cells");
    return LCP_OK;
}

}  // namespace

int lcp_dense(const lcp_model* M, const lcp_grid* grid, double theta, const lcp_mc* mc, int prec, float* lcp, void* ws,
              size_t ws_bytes, void* stream)
{
    if (!M) return fail(LCP_EINVAL, "model is NULL");
    if (check_prec(prec)) return LCP_EINVAL;
    GridP g;
    if (int r = check_grid(M, grid, &g)) return r;
    if (int r = check_mc(M, mc)) return r;
    if (!is_finite(theta)) return fail(LCP_EINVAL, "theta must be finite");
    if (!lcp || !ws) return fail(LCP_EINVAL, "lcp and ws must not be NULL");
    if (!aligned256(ws)) return fail(LCP_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = dense_ws(M, g, prec, mc->n_samples);
    if (ws_bytes < need) return fail(LCP_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    const DenseWs w = carve_dense(M, g, prec, mc->n_samples, (char*)ws);
    hipError_t e;
    if (prec != LCP_FP64) {
        e = launch_zbank32(mc->zbank, w.zb32, mc->n_samples, g.dim, s);
        if (e != hipSuccess) return dev_fail(e, "z-bank");
    }
    e = launch_posterior(*M, prec, dense_task(g, w), s);
    if (e != hipSuccess) return dev_fail(e, "posterior");
    if (int r = dense_cells(M, g, theta, mc, prec, w, w.zb32, lcp, s)) return r;
    return ok();
}

int lcp_adaptive(const lcp_model* M, const lcp_grid* grid, double theta, const lcp_adapt* A, const lcp_mc* mc, int prec,
                 float* lcp, uint64_t* leaves, int64_t leaf_cap, int64_t* n_leaves, uint8_t* level_field, void* ws,
                 size_t ws_bytes, void* stream)
{
    if (!M) return fail(LCP_EINVAL, "model is NULL");
    if (check_prec(prec)) return LCP_EINVAL;
    GridP g;
    if (int r = check_grid(M, grid, &g)) return r;
    if (int r = check_mc(M, mc)) return r;
    if (mc->estimator != LCP_EST_COUNT) return fail(LCP_ENOTSUPPORTED, "lcp_adaptive: counting estimator only");
    if (int r = check_adapt(*M, A)) return r;
    if (!is_finite(theta)) return fail(LCP_EINVAL, "theta must be finite");
    if (!lcp || !ws || !n_leaves) return fail(LCP_EINVAL, "lcp, n_leaves and ws must not be NULL");
    if (leaf_cap < 0 || (leaf_cap > 0 && !leaves)) return fail(LCP_EINVAL, "leaves must hold leaf_cap >= 0 keys");
    if (!aligned256(ws)) return fail(LCP_EINVAL, "workspace must be 256-byte aligned");
    int64_t S0;
    int Lmax;
    octree_shape(g, A->min_leaf_cells, &S0, &Lmax);
    if (Lmax > 7) return fail(LCP_EINVAL, "octree deeper than 8 levels (raise min_leaf_cells)");
    const size_t need = adaptive_workspace(*M, g, S0, Lmax, prec, mc->n_samples, *A);
    if (ws_bytes < need) return fail(LCP_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    hipError_t e = run_adaptive(*M, g, theta, *A, S0, Lmax, prec, mc->n_samples, mc->zbank, lcp, leaves, leaf_cap,
                                n_leaves, level_field, (char*)ws, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "lcp_adaptive");
    return ok();
}

int lcp_backward_workspace(const lcp_model* M, const lcp_grid* grid, int prec, int n_samples, size_t* bytes)
{
    if (!M || !bytes) return fail(LCP_EINVAL, "model and bytes must not be NULL");
    if (check_prec(prec)) return LCP_EINVAL;
    if (n_samples < 1) return fail(LCP_EINVAL, "n_samples < 1");
    GridP g;
    if (int r = check_grid(M, grid, &g)) return r;
    *bytes = lcp_backward_ws(*M, g, prec, n_samples);
    return ok();
}

int lcp_backward(const lcp_model* M, const lcp_grid* grid, double theta, const lcp_mc* mc, int prec,
                 const double* dL_dlcp, double* dL_dy, double* dL_dloglen, void* ws, size_t ws_bytes, void* stream)
{
    if (!M) return fail(LCP_EINVAL, "model is NULL");
    if (M->sparse) return fail(LCP_ENOTSUPPORTED, "lcp_backward: the model comes from gp_fit_sgpr");
    if (check_prec(prec)) return LCP_EINVAL;
    GridP g;
    if (int r = check_grid(M, grid, &g)) return r;
    if (int r = check_mc(M, mc)) return r;
    if (mc->estimator != LCP_EST_SOV)
        return fail(LCP_ENOTSUPPORTED, "lcp_backward: the counting estimator is piecewise constant (use LCP_EST_SOV)");
    if (!is_finite(theta)) return fail(LCP_EINVAL, "theta must be finite");
    if (!dL_dlcp || !dL_dy || !dL_dloglen || !ws) return fail(LCP_EINVAL, "dL_dlcp, dL_dy, dL_dloglen and ws must not be NULL");
    if (!aligned256(ws)) return fail(LCP_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = lcp_backward_ws(*M, g, prec, mc->n_samples);
    if (ws_bytes < need) return fail(LCP_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    hipError_t e = launch_lcp_backward(*M, g, theta, mc->n_samples, mc->zbank, prec, dL_dlcp, dL_dy, dL_dloglen,
                                       (char*)ws, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "lcp_backward");
    return ok();
}

}  // extern "C"

// ------------------------------------------------------ allocation-free dense evaluation

namespace {

// Scratch of lcp_dense_noalloc: a file-scope device array that every call on a device
// shares (each device holds its own copy for the life of the process).  Host code must
// not pass `scratch` itself to a kernel: its host-side name is not a device address.
// The device address comes from hipGetSymbolAddress, once per device, with that device
// current, and only that address is used.
constexpr size_t kNoallocBytes = LCP_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dev_fail(e, "lcp_dense_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(LCP_EDEVICE, "lcp_dense_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return dev_fail(e, "lcp_dense_noalloc: hipGetSymbolAddress");
        if (!p || !aligned256(p)) return fail(LCP_EDEVICE, "lcp_dense_noalloc: scratch address not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LCP_OK;
}

}  // namespace

extern "C" int lcp_dense_noalloc(const lcp_model* M, const lcp_grid* grid, double theta, const lcp_mc* mc, int prec,
                                 float* lcp, void* stream)
{
    if (!M) return fail(LCP_EINVAL, "model is NULL");
    if (check_prec(prec)) return LCP_EINVAL;
    GridP g;
    if (int r = check_grid(M, grid, &g)) return r;
    if (int r = check_mc(M, mc)) return r;
    if (M->device >= 0) {
        int dev = -1;
        if (hipGetDevice(&dev) == hipSuccess && dev != M->device)
            return fail(LCP_EINVAL, "lcp_dense_noalloc: the model lives on device %d, device %d is current", M->device,
                        dev);
    }
    const size_t need = dense_ws(M, g, prec, mc->n_samples);
    if (need > kNoallocBytes)
        return fail(LCP_ENOMEM, "lcp_dense_noalloc: this grid needs %zu bytes of scratch, the fixed maximum is %zu",
                    need, kNoallocBytes);
    void* ws = nullptr;
    if (int r = scratch_of_current_device(&ws)) return r;
    return lcp_dense(M, grid, theta, mc, prec, lcp, ws, kNoallocBytes, stream);
}

// ---------------------------------------------------------------- batches of models

namespace {

size_t batch_model_layout(int nb, const int* m, std::vector<size_t>* off)
{
    size_t o = 0;
    for (int b = 0; b < nb; ++b) {
        if (off) off->push_back(o);
        o += align256(model_bytes(m[b]));
    }
    return o + align256(factor_batch_scratch(nb));
}

}  // namespace

size_t lcp_batch_model_bytes(int nb, const int* m, int dim)
{
    (void)dim;
    if (nb < 1 || !m) return 0;
    for (int b = 0; b < nb; ++b)
        if (m[b] < 1 || m[b] > kMaxM) return 0;
    return batch_model_layout(nb, m, nullptr);
}

int gp_fit_factor_batch(int nb, const lcp_kernel* k, const int* m, const double* X, const double* y, void* model_mem,
                        size_t model_bytes_, void* stream, lcp_model_batch** out)
{
    if (!k || !m || !out) return fail(LCP_EINVAL, "k, m and out must not be NULL");
    *out = nullptr;
    if (nb < 1) return fail(LCP_EINVAL, "nb = %d < 1", nb);
    for (int b = 0; b < nb; ++b) {
        if (int r = check_kernel(&k[b], m[b])) {
            char msg[512];
            snprintf(msg, sizeof msg, "%s", g_err);
            return fail(r, "model %d: %s", b, msg);
        }
        if (k[b].dim != k[0].dim) return fail(LCP_EINVAL, "model %d: dim %d differs from model 0", b, k[b].dim);
    }
    if (!X || !y || !model_mem) return fail(LCP_EINVAL, "X, y and model_mem must not be NULL");
    if (!aligned256(model_mem)) return fail(LCP_EINVAL, "model_mem must be 256-byte aligned");
    std::vector<size_t> off;
    const size_t need = batch_model_layout(nb, m, &off);
    if (model_bytes_ < need) return fail(LCP_ENOMEM, "model memory %zu < %zu bytes", model_bytes_, need);
    lcp_model_batch* B = new (std::nothrow) lcp_model_batch();
    if (!B) return fail(LCP_ENOMEM, "host allocation failed");
    B->models.resize(nb);
    B->scratch = (char*)model_mem + need - align256(factor_batch_scratch(nb));
    std::vector<Model*> Ms(nb);
    std::vector<const double*> Xb(nb), yb(nb);
    int64_t mo = 0;
    const int dim = k[0].dim;
    for (int b = 0; b < nb; ++b) {
        init_model(B->models[b], k[b], m[b], (char*)model_mem + off[b]);
        Ms[b] = &B->models[b];
        Xb[b] = X + mo * dim;
        yb[b] = y + mo;
        mo += m[b];
    }
    hipStream_t s = (hipStream_t)stream;
    int* info_dev = (int*)(B->scratch + align256(factor_batch_scratch(nb)) - align256(sizeof(int) * (size_t)nb));
    hipError_t e = launch_factor_batch(Ms.data(), nb, Xb.data(), yb.data(), B->scratch, info_dev, s);
    std::vector<int> info(nb, 0);
    if (e == hipSuccess) e = hipMemcpyAsync(info.data(), info_dev, sizeof(int) * nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { delete B; return dev_fail(e, "batched factor"); }
    for (int b = 0; b < nb; ++b)
        if (info[b] != 0) {
            delete B;
            return fail(LCP_ENOTPD, "model %d: Cholesky pivot %d is not above m * eps * max K_ii", b, info[b]);
        }
    e = launch_factor_batch_finish(Ms.data(), nb, B->scratch, s);
    if (e != hipSuccess) { delete B; return dev_fail(e, "batched factor finish"); }
    *out = B;
    return ok();
}

void gp_model_batch_free(lcp_model_batch* batch) { delete batch; }

namespace {

int batch_grids(const lcp_model_batch* B, const lcp_grid* grids, std::vector<GridP>* gs)
{
    if (!B) return fail(LCP_EINVAL, "batch is NULL");
    if (!grids) return fail(LCP_EINVAL, "grids is NULL");
    const int nb = (int)B->models.size();
    gs->resize(nb);
    for (int b = 0; b < nb; ++b)
        if (int r = check_grid(&B->models[b], &grids[b], &(*gs)[b])) {
            char msg[512];
            snprintf(msg, sizeof msg, "%s", g_err);
            return fail(r, "grid %d: %s", b, msg);
        }
    return LCP_OK;
}

// Per model a dense workspace (in that model's precision), then the batch records
// (posterior, cross, cells) and one Monte Carlo work list for all models' cells.
size_t batch_dense_ws(const lcp_model_batch* B, const std::vector<GridP>& gs, const int* prec, int ns,
                      std::vector<size_t>* off)
{
    const int nb = (int)gs.size();
    size_t o = 0;
    int64_t cells = 0;
    for (int b = 0; b < nb; ++b) {
        if (off) off->push_back(o);
        o += dense_ws(&B->models[b], gs[b], prec[b], ns);
        cells += gs[b].nc[0] * gs[b].nc[1] * gs[b].nc[2];
    }
    if (off) off->push_back(o);
    o += align256(posterior_batch_scratch(nb));
    if (off) off->push_back(o);
    o += align256(cross_batch_scratch(nb));
    if (off) off->push_back(o);
    o += align256(cells_batch_scratch(nb));
    if (off) off->push_back(o);
    return o + cells_scratch_bytes(cells);
}

int check_batch_precs(int nb, const int* prec)
{
    if (!prec) return fail(LCP_EINVAL, "prec is NULL");
    for (int b = 0; b < nb; ++b)
        if (check_prec(prec[b])) return fail(LCP_EINVAL, "prec[%d] = %d is not an lcp_precision", b, prec[b]);
    return LCP_OK;
}

// lcp_dense on every model of the batch, model b in precision prec[b]: the posterior, cross
// and cells passes each run as one launch per precision present.
int dense_batch(const lcp_model_batch* B, const lcp_grid* grids, const double* theta, const lcp_mc* mc,
                const int* prec, float* lcp, void* ws, size_t ws_bytes, void* stream)
{
    std::vector<GridP> gs;
    if (int r = batch_grids(B, grids, &gs)) return r;
    const int nb = (int)gs.size();
    if (int r = check_batch_precs(nb, prec)) return r;
    if (!theta) return fail(LCP_EINVAL, "theta is NULL");
    for (int b = 0; b < nb; ++b) {
        if (int r = check_mc(&B->models[b], mc)) return r;
        if (mc->estimator != LCP_EST_COUNT) return fail(LCP_ENOTSUPPORTED, "lcp_dense_batch: counting estimator only");
        if (!is_finite(theta[b])) return fail(LCP_EINVAL, "theta[%d] must be finite", b);
    }
    if (!lcp || !ws) return fail(LCP_EINVAL, "lcp and ws must not be NULL");
    if (!aligned256(ws)) return fail(LCP_EINVAL, "workspace must be 256-byte aligned");
    std::vector<size_t> off;
    const size_t need = batch_dense_ws(B, gs, prec, mc->n_samples, &off);
    if (ws_bytes < need) return fail(LCP_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    std::vector<DenseWs> w(nb);
    std::vector<PostTask> tasks(nb);
    bool reduced = false;
    for (int b = 0; b < nb; ++b) {
        w[b] = carve_dense(&B->models[b], gs[b], prec[b], mc->n_samples, (char*)ws + off[b]);
        tasks[b] = dense_task(gs[b], w[b]);
        reduced = reduced || prec[b] != LCP_FP64;
    }
    hipError_t e;
    if (reduced) {
        e = launch_zbank32(mc->zbank, w[0].zb32, mc->n_samples, gs[0].dim, s);
        if (e != hipSuccess) return dev_fail(e, "z-bank");
    }
    char* base = (char*)ws;
    // one work list for every model's cells
    int64_t cells = 0;
    for (int b = 0; b < nb; ++b) cells += gs[b].nc[0] * gs[b].nc[1] * gs[b].nc[2];
    char* list = base + off[nb + 3];
    int32_t* work = (int32_t*)list;
    int64_t* wcount = (int64_t*)(list + align256(4 * (size_t)cells));
    double* zmax = (double*)((char*)wcount + 64);
    std::vector<int64_t> cell0(nb + 1, 0);
    for (int b = 0; b < nb; ++b) cell0[b + 1] = cell0[b] + gs[b].nc[0] * gs[b].nc[1] * gs[b].nc[2];
    for (int p = LCP_FP64; p <= LCP_MIXED_F16X3; ++p) {
        std::vector<int> idx;
        for (int b = 0; b < nb; ++b)
            if (prec[b] == p) idx.push_back(b);
        if (idx.empty()) continue;
        const int n = (int)idx.size();
        std::vector<const Model*> Ms(n);
        std::vector<PostTask> ts(n);
        std::vector<GridP> gg(n);
        std::vector<const void*> Vs(n);
        std::vector<double*> crosses(n);
        std::vector<CellTask> cts(n);
        for (int i = 0; i < n; ++i) {
            const int b = idx[i];
            Ms[i] = &B->models[b];
            ts[i] = tasks[b];
            gg[i] = gs[b];
            Vs[i] = w[b].V;
            crosses[i] = w[b].cross;
            CellTask& ct = cts[i];
            ct = CellTask{};
            ct.grid = gs[b];
            ct.prec = p;
            ct.theta = theta[b];
            ct.ns = mc->n_samples;
            ct.zb64 = mc->zbank;
            ct.zb32 = w[0].zb32;
            ct.mean = w[b].mean;
            ct.var = w[b].var;
            ct.cross = w[b].cross;
            ct.slot = nullptr;
            ct.leaves = nullptr;
            ct.lcp = lcp + cell0[b];
            ct.work = work;
            ct.wcount = wcount;
            ct.zmax = zmax;
        }
        e = launch_posterior_batch(Ms.data(), ts.data(), n, p, base + off[nb], s);
        if (e != hipSuccess) return dev_fail(e, "batched posterior");
        e = launch_cross_batch(Ms.data(), gg.data(), Vs.data(), crosses.data(), n, p, base + off[nb + 1], s);
        if (e != hipSuccess) return dev_fail(e, "batched cross");
        e = launch_cells_batch(cts.data(), n, base + off[nb + 2], s);
        if (e != hipSuccess) return dev_fail(e, "batched cells");
    }
    return ok();
}

}  // namespace

int lcp_dense_batch_workspace(const lcp_model_batch* B, const lcp_grid* grids, int prec, int n_samples, size_t* bytes)
{
    if (!bytes) return fail(LCP_EINVAL, "bytes must not be NULL");
    if (check_prec(prec)) return LCP_EINVAL;
    if (n_samples < 1) return fail(LCP_EINVAL, "n_samples must be >= 1");
    std::vector<GridP> gs;
    if (int r = batch_grids(B, grids, &gs)) return r;
    const std::vector<int> precs(gs.size(), prec);
    *bytes = batch_dense_ws(B, gs, precs.data(), n_samples, nullptr);
    return ok();
}

int lcp_dense_batch(const lcp_model_batch* B, const lcp_grid* grids, const double* theta, const lcp_mc* mc, int prec,
                    float* lcp, void* ws, size_t ws_bytes, void* stream)
{
    if (check_prec(prec)) return LCP_EINVAL;
    if (!B) return fail(LCP_EINVAL, "batch is NULL");
    const std::vector<int> precs(B->models.size(), prec);
    return dense_batch(B, grids, theta, mc, precs.data(), lcp, ws, ws_bytes, stream);
}

int lcp_dense_batch_mixed_workspace(const lcp_model_batch* B, const lcp_grid* grids, const int* prec, int n_samples,
                                    size_t* bytes)
{
    if (!bytes) return fail(LCP_EINVAL, "bytes must not be NULL");
    if (n_samples < 1) return fail(LCP_EINVAL, "n_samples must be >= 1");
    std::vector<GridP> gs;
    if (int r = batch_grids(B, grids, &gs)) return r;
    if (int r = check_batch_precs((int)gs.size(), prec)) return r;
    *bytes = batch_dense_ws(B, gs, prec, n_samples, nullptr);
    return ok();
}

int lcp_dense_batch_mixed(const lcp_model_batch* B, const lcp_grid* grids, const double* theta, const lcp_mc* mc,
                          const int* prec, float* lcp, void* ws, size_t ws_bytes, void* stream)
{
    return dense_batch(B, grids, theta, mc, prec, lcp, ws, ws_bytes, stream);
}

int lcp_batch_precision(const lcp_model_batch* B, int reduced, double kappa_max, int* prec, double* kappa,
                        void* stream)
{
    if (!B) return fail(LCP_EINVAL, "batch is NULL");
    if (!prec) return fail(LCP_EINVAL, "prec must not be NULL");
    if (check_prec(reduced)) return LCP_EINVAL;
    if (!(kappa_max == kappa_max)) return fail(LCP_EINVAL, "kappa_max is NaN");
    if (kappa_max <= 0.0) {
        // measured for binary32 (24 bits): 8; scaled by the unit roundoff of the other forms
        const double unit = reduced == LCP_MIXED_BF16X3 ? 0x1p-16 : reduced == LCP_MIXED_F16X3 ? 0x1p-22 : 0x1p-24;
        kappa_max = reduced == LCP_FP64 ? INFINITY : 8.0 * 0x1p-24 / unit;
    }
    const int nb = (int)B->models.size();
    std::vector<double> amax(nb);
    hipStream_t s = (hipStream_t)stream;
    for (int b = 0; b < nb; ++b) {
        hipError_t e = hipMemcpyAsync(&amax[b], B->models[b].amax, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return dev_fail(e, "lcp_batch_precision");
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dev_fail(e, "lcp_batch_precision");
    for (int b = 0; b < nb; ++b) {
        const double k = sqrt(B->models[b].k.signal_var) * amax[b];
        if (kappa) kappa[b] = k;
        prec[b] = k <= kappa_max ? reduced : LCP_FP64;
    }
    return ok();
}

int lcp_batch_tiles(int prec, int size_class, int nt, int nw)
{
    if (check_prec(prec)) return LCP_EINVAL;
    if (size_class < 0 || size_class >= kMaxM / 128) return fail(LCP_EINVAL, "size_class must lie in 0..%d", kMaxM / 128 - 1);
    if (set_batch_tiles(prec, size_class, nt, nw))
        return fail(LCP_EINVAL, "tiles %d x %d waves: not a candidate, or the B tile exceeds LDS at m_pad = %d", nt, nw,
                    128 * (size_class + 1));
    return ok();
}

int lcp_batch_tiles_get(int prec, int size_class, int* nt, int* nw)
{
    if (check_prec(prec)) return LCP_EINVAL;
    if (size_class < 0 || size_class >= kMaxM / 128) return fail(LCP_EINVAL, "size_class must lie in 0..%d", kMaxM / 128 - 1);
    if (!nt || !nw) return fail(LCP_EINVAL, "nt and nw must not be NULL");
    get_batch_tiles(prec, size_class, nt, nw);
    return ok();
}
