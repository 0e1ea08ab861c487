// Internal declarations of the gfx950 LCP library: device helpers, the model layout
// in device memory, and the launchers each kernel file provides to the host API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/lcp.h"

namespace lcp {

constexpr int kMaxM = 1024;           // largest supported number of observations
constexpr int kWave = 64;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// Covariance parameters as the kernels read them.
struct KParams {
    int kind;        // lcp_kernel_kind
    int dim;
    double s2;       // signal variance
    double inv_ell[3];
};

// Regular grid: vertex i on axis d is lo[d] + i * h[d] with h = (hi - lo) / (npts - 1).
struct GridP {
    int dim;
    double lo[3];
    double h[3];
    int64_t n[3];    // vertices per axis (1 beyond dim)
    int64_t nc[3];   // cells per axis (1 beyond dim)
};

// Coordinate of vertex i on axis d, rounded exactly as lo + i * h with two roundings
// (no fused multiply-add), so every part of the library agrees on box corners.
__device__ __forceinline__ double vertex_coord(const GridP& g, int d, int64_t i)
{
#pragma clang fp contract(off)
    return g.lo[d] + (double)i * g.h[d];
}

// x * y rounded once, never fused into a following addition.
__device__ __forceinline__ double mul_rn(double x, double y)
{
#pragma clang fp contract(off)
    return x * y;
}

__device__ __forceinline__ double kernel_r2(const KParams& p, const double* x, const double* z)
{
    double r2 = 0.0;
    for (int d = 0; d < p.dim; ++d) {
        double t = (x[d] - z[d]) * p.inv_ell[d];
        r2 = fma(t, t, r2);
    }
    return r2;
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one int per thread (sh: 65 ints of LDS, at most 16 waves);
// returns the block total in *total.
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int* total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int inc = wave_incl_scan(v);
    if (lane == 63) sh[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        int w = lane < nw ? sh[lane] : 0;
        int wi = wave_incl_scan(w);
        if (lane < nw) sh[lane] = wi - w;
        if (lane == nw - 1) sh[64] = wi;
    }
    __syncthreads();
    int ex = inc - v + sh[wave];
    *total = sh[64];
    __syncthreads();
    return ex;
}

// Region bound (Sec. 5.1): the node's margin g = side (theta - mu) / sigma at a point, and
// the bound 1 - B^d = -expm1(d log1p(-t)), t = Phi(-g_min), of eq. (upper_bound) over the
// node's d grid points.
__device__ __forceinline__ double margin(double side, double theta, double mu, double var)
{
    double num = side * (theta - mu);
    if (var > 0.0) return num / sqrt(var);
    if (num > 0.0) return __builtin_inf();
    if (num < 0.0) return -__builtin_inf();
    return 0.0;
}

__device__ __forceinline__ double upper_bound(double gmin, int64_t dp)
{
    double t;
    if (gmin == __builtin_inf()) t = 0.0;
    else if (gmin == -__builtin_inf()) t = 1.0;
    else t = 0.5 * erfc(gmin / 1.41421356237309504880168872421);
    return t >= 1.0 ? 1.0 : -expm1((double)dp * log1p(-t));
}

// e^x for x <= 0 in binary64: Cody-Waite reduction x = n ln2 + r (ln2 split so that n * hi
// is exact for |n| < 2^21), |r| <= ln2 / 2, then the degree-12 Taylor polynomial of e^r
// (truncation below 2e-16 relative) and the exact scaling by 2^n; x < -745 gives 0.
__device__ __forceinline__ double exp_nonpos(double x)
{
    x = fmax(x, -746.0);
    const double n = rint(x * 1.4426950408889634);
    double r = fma(n, -0.6931471803691238, x);
    r = fma(n, -1.9082149292705877e-10, r);
    double p = 2.08767569878681e-09;
    p = fma(p, r, 2.505210838544172e-08);
    p = fma(p, r, 2.755731922398589e-07);
    p = fma(p, r, 2.7557319223985893e-06);
    p = fma(p, r, 2.48015873015873e-05);
    p = fma(p, r, 0.0001984126984126984);
    p = fma(p, r, 0.001388888888888889);
    p = fma(p, r, 0.008333333333333333);
    p = fma(p, r, 0.041666666666666664);
    p = fma(p, r, 0.16666666666666666);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}

// sqrt(x) for x >= 0 in binary64 (x = 0 gives 0).  Goldschmidt's coupled iteration for
// s -> sqrt(x) and h -> 1 / (2 sqrt(x)) (R. E. Goldschmidt, "Applications of division by
// convergence", MIT, 1964; in the form of P. Markstein, "IA-64 and Elementary Functions",
// 2000, ch. 9): start from the hardware reciprocal square root y, s = x y, h = y / 2; each
// step forms e = 1/2 - h s and sets s += s e, h += h e, which doubles the correct bits.
// Two steps from the ~23-bit seed, then one Newton correction s += (x - s^2) h from the
// exact residual (fma), which rounds to within an ulp.
__device__ __forceinline__ double sqrt_nonneg(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y, h = 0.5 * y;
    double e = fma(-h, s, 0.5);
    s = fma(s, e, s);
    h = fma(h, e, h);
    e = fma(-h, s, 0.5);
    s = fma(s, e, s);
    h = fma(h, e, h);
    const double d = fma(-s, s, x);
    s = fma(d, h, s);
    return x > 0.0 ? s : 0.0;
}

// k(x, z) for the squared-exponential and Matern-5/2 covariances.
__device__ __forceinline__ double kernel_val(const KParams& p, double r2)
{
    if (p.kind == LCP_KERNEL_SE) return p.s2 * exp_nonpos(-0.5 * r2);
    const double s5 = 2.23606797749978969640917366873;
    const double r = sqrt_nonneg(r2);
    return p.s2 * fma(5.0 / 3.0, r2, fma(s5, r, 1.0)) * exp_nonpos(-s5 * r);
}

// k in binary32 for the reduced-precision operand paths (binary32 and split 16-bit MFMA
// products carry 22-24 significant bits, which this evaluation matches): hardware exp2 and
// square root, r2 already scaled by the lengthscales.
// Branch-free in the kernel kind, so generation loops stay single basic blocks:
// SE: s2 exp(-r2 / 2); Matern-5/2: s2 (1 + t + t^2 / 3) exp(-t) with t = sqrt(5 r2).
__device__ __forceinline__ float kernel_val32(int kind, float s2, float r2)
{
    constexpr float kLog2e = 1.44269504088896341f;
    const bool se = kind == LCP_KERNEL_SE;
    const float t = 2.23606797749978970f * __builtin_amdgcn_sqrtf(r2);
    const float u = se ? 0.5f * r2 : t;
    const float poly = se ? 1.0f : fmaf(t, fmaf(t, 1.0f / 3.0f, 1.0f), 1.0f);
    return s2 * poly * __builtin_amdgcn_exp2f(-kLog2e * u);
}

// d k(x, z) / d x_d = f(r) * (x_d - z_d) / ell_d^2; returns f(r).
__device__ __forceinline__ double kernel_dfac(const KParams& p, double r2)
{
    if (p.kind == LCP_KERNEL_SE) return -p.s2 * exp_nonpos(-0.5 * r2);
    const double s5 = 2.23606797749978969640917366873;
    const double r = sqrt_nonneg(r2);
    return -(5.0 / 3.0) * p.s2 * fma(s5, r, 1.0) * exp_nonpos(-s5 * r);
}

// Value and derivative factor sharing one exponential.
__device__ __forceinline__ void kernel_val_dfac(const KParams& p, double r2, double* k, double* f)
{
    if (p.kind == LCP_KERNEL_SE) {
        const double e = p.s2 * exp_nonpos(-0.5 * r2);
        *k = e;
        *f = -e;
        return;
    }
    const double s5 = 2.23606797749978969640917366873;
    const double r = sqrt_nonneg(r2);
    const double e = p.s2 * exp_nonpos(-s5 * r);
    const double a = fma(s5, r, 1.0);
    *k = fma(5.0 / 3.0, r2, a) * e;
    *f = -(5.0 / 3.0) * a * e;
}

// ------------------------------------------------------------- posterior GEMM (K1)
//
// V = L^-1 B with B_jc = k(x_j, p_c) (or a derivative of it) generated on the fly.
// Columns come in groups of `group` (1: value only; 4: value + d/dx_0..2 of one point).

enum ColMode { COL_GRID = 0, COL_POINTS = 1 };

struct PostTask {
    int mode;                 // ColMode
    int group;                // 1 or 4 (gradient probes)
    const int64_t* count;     // device count of POINTS (groups); null -> n_points
    int64_t n_points;         // host upper bound of the number of points
    // COL_GRID: vertex id = vlist ? vlist[p] : p
    GridP grid;
    const int32_t* vlist;
    // COL_POINTS: n x dim points, row stride = pstride doubles
    const double* pts;
    int pstride;
    // outputs (per point p): mean[p], var[p]; for group 4: dmean[p*3+d], dvar[p*3+d]
    double* mean;
    double* var;
    double* dmean;
    double* dvar;
    void* V;                  // optional: V per point (value column only), quad-major with
                              // n_points columns: rows 4q..4q+3 of column p at (q * n_points + p) * 4
    int stage;                // stage-timer stage of this launch
    int64_t vld;              // > 0: V column-major instead, column p at p * vld (vld >= m_pad)
    int dense;                // 1: the operand is a full (not lower-triangular) m_pad x m_pad matrix
    // Region-search epilogue of the binary64 group-4 probes of descent candidates (COL_POINTS,
    // the points are the candidates' current positions): EPI_STEP runs projected gradient step
    // epi_step of each candidate and updates its point in place.
    int epi;
    int epi_step;
    double theta;
    int32_t* cand_done;         // per candidate: 1 = the descent stopped
    double* cand_rec;           // per candidate: node box lo[3], hi[3], side, minimum of g so far
    // Small binary64 launches of the region search may share each tile among work-groups:
    // kSplitGrid x 64 doubles of partial products and kSplitGrid tile counters (zero before
    // the first launch; every launch leaves them zero).  Null: one work-group per tile.
    double* sp_part;
    int32_t* sp_cnt;
};

constexpr int kSplitGrid = 256;   // work-groups of a shared-tile launch (one per CU)

enum { EPI_NONE = 0, EPI_STEP = 1 };

struct Model;  // defined below

hipError_t launch_posterior(const Model& M, int prec, const PostTask& t, hipStream_t s);
// The values the model was fitted to (device, m): y of an exact GP, mu_M of a sparse model.
const double* model_values(const Model& M);
// Value columns against another operand in the fragment order of the binary64 (prec
// LCP_FP64) or binary32 (LCP_FP32) posterior: A0 = m_pad x m_pad in 16 x 16 x 4 fragments.
hipError_t launch_posterior_operand(const Model& M, int prec, const PostTask& t, const void* A0, hipStream_t s);
// The same with the FP16 split product (value columns): Hhi, Hlo = the operand times amax[1]
// (a power of two) split into FP16 halves in 16 x 16 x 32 fragment order.
hipError_t launch_posterior_operand_f16x3(const Model& M, const PostTask& t, const void* Hhi, const void* Hlo,
                                          const double* amax, hipStream_t s);

// ------------------------------------------------------------------- cells (K3)

struct CellTask {
    GridP grid;
    int prec;                 // lcp_precision of the Monte Carlo loop
    double theta;
    int ns;                   // samples
    const double* zb64;       // ns x 2^dim
    const float* zb32;        // ns x 2^dim (FP32 copy)
    const double* mean;       // per slot
    const double* var;        // per slot
    const double* cross;      // per slot x ndir
    const int32_t* slot;      // vertex id -> slot (null: slot = vertex id)
    // cell enumeration: dense (leaves == null) or the cells of leaf keys
    const uint64_t* leaves;
    const int64_t* n_leaves;  // device count
    int64_t leaf_cap;
    int64_t S0;               // root edge in cells
    int Lmax;
    int leaf_edge;            // cells per leaf edge
    float* lcp;               // whole cell field
    // scratch (device): Monte Carlo work list of enumeration indices, its count, max ||z||
    int32_t* work;            // >= ncells_cap entries
    int64_t* wcount;
    double* zmax;
};

// Scratch bytes launch_cells needs for ncells_cap enumerated cells.
inline size_t cells_scratch_bytes(int64_t ncells_cap) { return ((4 * (size_t)ncells_cap + 255) & ~size_t(255)) + 256; }

// V: quad-major with nv_cap columns (as written by the posterior kernel).
hipError_t launch_cross(const Model& M, int prec, const GridP& g, const int32_t* vlist, const int64_t* nv_dev,
                        int64_t nv_cap, const int32_t* slot, const void* V, double* cross, hipStream_t s);
hipError_t launch_cells(const CellTask& t, int64_t ncells_cap, hipStream_t s);
// Smooth (separation-of-variables) LCP of every cell of a dense grid; wb: ns x 2^D + 1 doubles;
// t.work / t.wcount: a work list of >= cells entries and its counter (binary32 path).
hipError_t launch_cells_sov(const CellTask& t, double* wb, hipStream_t s);
// Its adjoint for upstream gl (per cell): per-cell gradients gout (2^D + 2^D (2^D + 1) / 2
// doubles each), then per vertex gmean, gvar and gcross (13 / 4 directions).  Same work list.
hipError_t launch_cells_sov_grad(const CellTask& t, double* wb, const double* gl, double* gout, double* gmean,
                                 double* gvar, double* gcross, hipStream_t s);
// Dense cells of nb tasks in one pass; every task's work/wcount/zmax must point to one
// shared list (>= total cells), count and zmax; scratch holds cells_batch_scratch(nb) bytes.
size_t cells_batch_scratch(int nb);
// Dense cross-covariances of nb models in one launch (V quad-major with nv_b columns).
size_t cross_batch_scratch(int nb);
hipError_t launch_cross_batch(const Model* const* Ms, const GridP* grids, const void* const* V, double* const* cross,
                              int nb, int prec, char* scratch, hipStream_t s);
hipError_t launch_cells_batch(const CellTask* tasks, int nb, char* scratch, hipStream_t s);
// Reduced-precision z-bank region (zbank32_bytes): the binary32 copy of the ns x 2^dim bank,
// then (3D) the split FP16 sample records of the matrix-core Monte Carlo loop.
hipError_t launch_zbank32(const double* zb, float* zb32, int64_t ns, int dim, hipStream_t s);
// Corner moments of listed cells (linear cell index, x fastest): flag their corner vertices,
// number the flagged vertices (slot, vlist from an exclusive scan of vmask), then gather each
// cell's 2^D means and 2^D x 2^D covariance from the per-slot posterior and cross terms.
hipError_t launch_mark_cells(const GridP& g, const int64_t* cells, int64_t n, int32_t* vmask, hipStream_t s);
hipError_t launch_vertex_slots(const int32_t* vmask, const int32_t* off, int64_t nv, int32_t* slot, int32_t* vlist,
                               hipStream_t s);
hipError_t launch_cell_moments(const GridP& g, const int64_t* cells, int64_t n, const int32_t* slot,
                               const double* mean, const double* var, const double* cross, double* mu_out,
                               double* cov_out, hipStream_t s);

// --------------------------------------------------------------- model (K2)

struct Model {
    lcp_kernel k;
    KParams kp;
    int m, m_pad, nrb, dim;
    int sparse;       // 1: factored by gp_fit_sgpr (T = F L^-1 stored in place of L^-1)
    double* X;        // m_pad x 4 (zero padded)
    double* a;        // m_pad
    double* U;        // m_pad x m_pad, upper factor L^T (row-major); scratch K before factoring
    double* Linv;     // m_pad x m_pad row-major lower, zero padded
    double* A64;      // Linv in 16x16x4 MFMA fragment order (binary64)
    float* A32;       // Linv in 16x16x4 MFMA fragment order (binary32)
    __bf16* Ahi;      // Linv split, 16x16x32 fragment order, high part
    __bf16* Alo;      //   low part
    _Float16* Hhi;    // (Linv * sA) split into FP16 halves, 16x16x32 fragment order
    _Float16* Hlo;
    double* amax;     // [0] max |Linv|, [1] sA (power of two), device
    double* Q64;      // Q = L^-T L^-1 (T^T T for a sparse model) in 16x16x4 fragment order, binary64,
    float* Q32;       //   and binary32: the certified bound's operand, formed by the single-model fits
    double* obs_mu;   // m
    double* obs_var;  // m
    double* AM;       // sparse model: A_M (m_pad x m_pad, zero padded), kept for local models
    double* Xs;       // m_pad x 4: x_jd / l_d (d < dim, else 0) and a_j, for the split-product
                      // posterior's generation (zero rows past m)
    int* info;
    int device;
};

size_t model_bytes(int m);
hipError_t launch_factor(Model& M, const double* X, const double* y, hipStream_t s);
hipError_t launch_factor_finish(Model& M, hipStream_t s);
// Sparse model of eq. (sgp), after launch_factor on K_MM + jitter I with mu_M as y.
hipError_t launch_sparse_e(Model& M, const double* A, double delta, bool first, hipStream_t s);
hipError_t launch_sparse_finish(Model& M, hipStream_t s);
// Adjoint of the posterior at n points (binary64 or binary32 W); ws of posterior_backward_ws bytes.
size_t posterior_backward_ws(const Model& M, int64_t n, int prec);
hipError_t launch_posterior_backward(const Model& M, int64_t n, const double* Xq, int prec, const double* gm,
                                     const double* gv, double* dy, double* dlogell, char* ws, hipStream_t s);
// Adjoint of the smooth LCP field of a dense grid (upstream gl per cell).
size_t lcp_backward_ws(const Model& M, const GridP& g, int prec, int ns);
hipError_t launch_lcp_backward(const Model& M, const GridP& g, double theta, int ns, const double* zb, int prec,
                               const double* gl, double* dy, double* dlogell, char* ws, hipStream_t s);
// K^-1 = Linv^T Linv (row-major) and its 16 x 16 x 4 fragment copies (binary64, binary32).
hipError_t launch_kinv_frag(const Model& M, double* Kinv, double* F64, float* F32, hipStream_t s);
// Certified region bound (k_bound.hip).  w = Q k(c) for box centres against the model's operand
// Q (Model::Q64, F64 below), 3 doubles per point, device count or cap, W column b at
// b * m_pad; then per box (lo[dim], hi[dim]) the bounds mu(c), mu_lo, mu_hi, var_hi.
hipError_t launch_cert_w(const Model& M, const double* F64, const double* pts, const int64_t* count, int64_t cap,
                         double* W, double* mean, double* var, hipStream_t s);
hipError_t launch_cert(const Model& M, const double* box, const int64_t* count, int64_t cap, const double* W,
                       double* out, hipStream_t s);
size_t bound_certified_ws(const Model& M, int64_t n);
hipError_t launch_bound_certified(const Model& M, int64_t n, const double* box, double* out, char* ws, hipStream_t s);
size_t factor_batch_scratch(int nb);
hipError_t launch_factor_batch(Model* const* Ms, int nb, const double* const* X, const double* const* y, char* scratch,
                               int* info_dev, hipStream_t s);
hipError_t launch_factor_batch_finish(Model* const* Ms, int nb, char* scratch, hipStream_t s);
// Value columns of many models in one launch: KArgs-equivalent records built from tasks[b]
// (COL_GRID or COL_POINTS, no device count) into scratch (posterior_batch_scratch bytes).
size_t posterior_batch_scratch(int nb);
// Tile configuration of the batched posterior for precision prec and size class cls
// (m_pad = 128 (cls + 1)): set (nt = 0 restores the tuned default; -1 if the pair is not
// a candidate or its B tile exceeds LDS) and read back.
int set_batch_tiles(int prec, int cls, int nt, int nw);
void get_batch_tiles(int prec, int cls, int* nt, int* nw);
hipError_t launch_posterior_batch(const Model* const* Ms, const PostTask* tasks, int nb, int prec, char* scratch,
                                  hipStream_t s);

// ------------------------------------------------------------- octree (K4/K5)

size_t adaptive_workspace(const Model& M, const GridP& g, int64_t S0, int Lmax, int prec, int ns, const lcp_adapt& A);
hipError_t run_adaptive(const Model& M, const GridP& g, double theta, const lcp_adapt& A, int64_t S0, int Lmax,
                        int prec, int ns, const double* zb, float* lcp, uint64_t* leaves, int64_t leaf_cap,
                        int64_t* n_leaves, uint8_t* level_field, char* ws, hipStream_t s);

// ------------------------------------------------------------------ utilities

hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);

// Exclusive scan of n int32 flags (device count or host n) into offsets, total into *total.
size_t scan_workspace(int64_t n);
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, const int64_t* n_dev, int64_t* total,
                       char* ws, hipStream_t s);

// Stages of the stage timer (bit positions of the lcp_profile_begin mask).
enum Stage {
    ST_FACTOR = 0,      // model factorisation
    ST_POSTERIOR = 1,   // posterior GEMM at grid vertices / query points
    ST_BOUND = 2,       // binary64 posterior probes of the region bound
    ST_CROSS = 3,       // neighbour cross-covariances
    ST_CELLS = 4,       // cell factor + Monte Carlo
    ST_OCTREE = 5,      // node tests, prefix sums, emission, leaf enumeration
    ST_MISC = 6         // fills and conversions
};

// Brackets the launches issued during its lifetime with events when the stage is profiled.
class StageScope {
public:
    StageScope(hipStream_t s, int stage);
    ~StageScope();
    StageScope(const StageScope&) = delete;
    StageScope& operator=(const StageScope&) = delete;

private:
    hipStream_t s_;
    int idx_;
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes of the reduced-precision z-bank region: the binary32 copy, then 48-byte split FP16
// records of the samples padded to a multiple of 32 (read by the 3D Monte Carlo loop).
constexpr int kZrecBytes = 48;
inline size_t zbank32_bytes(int64_t ns, int dim)
{
    return align256(sizeof(float) * ((size_t)ns << dim)) + align256(kZrecBytes * (size_t)((ns + 31) / 32 * 32));
}
inline const void* zbank_records(const float* zb32, int64_t ns, int dim)
{
    return (const char*)zb32 + align256(sizeof(float) * ((size_t)ns << dim));
}

}  // namespace lcp
