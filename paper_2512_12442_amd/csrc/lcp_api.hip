// Host side of the C ABI declared in include/lcp.h: argument validation, workspace
// carving and the order in which the kernels of the hot path are enqueued.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "lcp_internal.h"

struct lcp_model : lcp::Model {};

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
    b += align256(sizeof(float) * (size_t)ns * (1 << g.dim)); // FP32 z-bank
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

int check_adapt(const lcp_adapt* A)
{
    if (!A) return fail(LCP_EINVAL, "adapt is NULL");
    if (!(A->alpha > 0.0 && A->alpha < 0.5)) return fail(LCP_EINVAL, "alpha must lie in (0, 0.5)");
    if (A->min_leaf_cells < 1 || (A->min_leaf_cells & (A->min_leaf_cells - 1)))
        return fail(LCP_EINVAL, "min_leaf_cells must be a power of two >= 1");
    if (A->bound_at_max_depth != 0 && A->bound_at_max_depth != 1)
        return fail(LCP_EINVAL, "bound_at_max_depth must be 0 or 1");
    if (A->descent_steps < 0 || A->descent_steps > 16) return fail(LCP_EINVAL, "descent_steps must be in 0..16");
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
    if (k->dim != 2 && k->dim != 3) return fail(LCP_EINVAL, "dim must be 2 or 3 (got %d)", k->dim);
    if (k->kind != LCP_KERNEL_SE && k->kind != LCP_KERNEL_MATERN52) return fail(LCP_EINVAL, "unknown kernel %d", k->kind);
    if (!(k->signal_var > 0.0) || !is_finite(k->signal_var)) return fail(LCP_EINVAL, "signal_var must be finite and > 0");
    if (!(k->noise_var >= 0.0) || !is_finite(k->noise_var)) return fail(LCP_EINVAL, "noise_var must be finite and >= 0");
    for (int d = 0; d < k->dim; ++d)
        if (!(k->lengthscale[d] > 0.0) || !is_finite(k->lengthscale[d]))
            return fail(LCP_EINVAL, "lengthscale[%d] must be finite and > 0", d);
    if (m < 1 || m > kMaxM) return fail(LCP_EINVAL, "m = %d outside 1..%d", m, kMaxM);
    if (!X || !y || !model_mem) return fail(LCP_EINVAL, "X, y and model_mem must not be NULL");
    if (!aligned256(model_mem)) return fail(LCP_EINVAL, "model_mem must be 256-byte aligned");
    if (model_bytes_ < model_bytes(m)) return fail(LCP_ENOMEM, "model memory %zu < %zu bytes", model_bytes_, model_bytes(m));
    lcp_model* M = new (std::nothrow) lcp_model();
    if (!M) return fail(LCP_ENOMEM, "host allocation failed");
    M->k = *k;
    M->dim = k->dim;
    M->m = m;
    M->m_pad = (m + 127) / 128 * 128;
    M->nrb = (m + 15) / 16;
    M->kp.kind = k->kind;
    M->kp.dim = k->dim;
    M->kp.s2 = k->signal_var;
    for (int d = 0; d < 3; ++d) M->kp.inv_ell[d] = d < k->dim ? 1.0 / k->lengthscale[d] : 0.0;
    M->X = (double*)model_mem;
    if (hipGetDevice(&M->device) != hipSuccess) M->device = -1;
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
    if (int r = check_adapt(A)) return r;
    int64_t S0;
    int Lmax;
    octree_shape(g, A->min_leaf_cells, &S0, &Lmax);
    if (Lmax > 7) return fail(LCP_EINVAL, "octree deeper than 8 levels (raise min_leaf_cells)");
    *bytes = adaptive_workspace(*M, g, S0, Lmax, prec, n_samples);
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
    const int64_t nv = g.n[0] * g.n[1] * g.n[2];
    const size_t vb = prec == LCP_FP64 ? 8 : 4;
    char* p = (char*)ws;
    double* mean = (double*)p;
    p += align256(sizeof(double) * nv);
    double* var = (double*)p;
    p += align256(sizeof(double) * nv);
    void* V = p;
    p += align256(vb * (size_t)nv * M->m_pad);
    double* cross = (double*)p;
    p += align256(sizeof(double) * (size_t)nv * ndir(g.dim));
    float* zb32 = (float*)p;
    p += align256(sizeof(float) * (size_t)mc->n_samples * (1 << g.dim));
    const int64_t ncells = g.nc[0] * g.nc[1] * g.nc[2];
    int32_t* work = (int32_t*)p;
    p += align256(4 * (size_t)ncells);
    int64_t* wcount = (int64_t*)p;
    double* zmax = (double*)(p + 64);
    hipError_t e;
    if (prec != LCP_FP64) {
        e = launch_zbank32(mc->zbank, zb32, (int64_t)mc->n_samples << g.dim, s);
        if (e != hipSuccess) return dev_fail(e, "z-bank");
    }
    PostTask t{};
    t.mode = COL_GRID;
    t.group = 1;
    t.count = nullptr;
    t.n_points = nv;
    t.grid = g;
    t.vlist = nullptr;
    t.mean = mean;
    t.var = var;
    t.V = V;
    t.stage = ST_POSTERIOR;
    e = launch_posterior(*M, prec, t, s);
    if (e != hipSuccess) return dev_fail(e, "posterior");
    e = launch_cross(*M, prec, g, nullptr, nullptr, nv, nullptr, V, cross, s);
    if (e != hipSuccess) return dev_fail(e, "cross");
    CellTask ct{};
    ct.grid = g;
    ct.prec = prec;
    ct.theta = theta;
    ct.ns = mc->n_samples;
    ct.zb64 = mc->zbank;
    ct.zb32 = zb32;
    ct.mean = mean;
    ct.var = var;
    ct.cross = cross;
    ct.slot = nullptr;
    ct.leaves = nullptr;
    ct.lcp = lcp;
    ct.work = work;
    ct.wcount = wcount;
    ct.zmax = zmax;
    e = launch_cells(ct, ncells, s);
    if (e != hipSuccess) return dev_fail(e, "cells");
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
    if (int r = check_adapt(A)) return r;
    if (!is_finite(theta)) return fail(LCP_EINVAL, "theta must be finite");
    if (!lcp || !ws || !n_leaves) return fail(LCP_EINVAL, "lcp, n_leaves and ws must not be NULL");
    if (leaf_cap < 0 || (leaf_cap > 0 && !leaves)) return fail(LCP_EINVAL, "leaves must hold leaf_cap >= 0 keys");
    if (!aligned256(ws)) return fail(LCP_EINVAL, "workspace must be 256-byte aligned");
    int64_t S0;
    int Lmax;
    octree_shape(g, A->min_leaf_cells, &S0, &Lmax);
    if (Lmax > 7) return fail(LCP_EINVAL, "octree deeper than 8 levels (raise min_leaf_cells)");
    const size_t need = adaptive_workspace(*M, g, S0, Lmax, prec, mc->n_samples);
    if (ws_bytes < need) return fail(LCP_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    hipError_t e = run_adaptive(*M, g, theta, *A, S0, Lmax, prec, mc->n_samples, mc->zbank, lcp, leaves, leaf_cap,
                                n_leaves, level_field, (char*)ws, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "lcp_adaptive");
    return ok();
}

int lcp_backward(const lcp_model* M, const lcp_grid* grid, double theta, const lcp_mc* mc, const float* dL_dlcp,
                 double* dL_dy, double* dL_dloglen, void* ws, size_t ws_bytes, void* stream)
{
    (void)M; (void)grid; (void)theta; (void)mc; (void)dL_dlcp; (void)dL_dy; (void)dL_dloglen; (void)ws;
    (void)ws_bytes; (void)stream;
    return fail(LCP_ENOTSUPPORTED, "lcp_backward: the Monte Carlo LCP estimator is piecewise constant; no adjoint");
}

}  // extern "C"
