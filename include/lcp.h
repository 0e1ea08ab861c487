/*
 * lcp.h -- C ABI of the MI355X (gfx950) level-crossing-probability library.
 *
 * Implements the hot path of Li, Michaud, Biswas, Shen, "Efficient Level-Crossing
 * Probability Calculation for Gaussian Process Modeled Data" (arXiv 2512.12442):
 * the GP posterior at grid vertices (Sec. 3, eq. (sgp) in its exact-GP form), the
 * per-cell level-crossing probability by Monte Carlo (Sec. 4), and the regional
 * upper bound of eq. (upper_bound) driving the octree query of Alg. 1 (Sec. 5.1,
 * 5.3), with reconstruction only inside the emitted nodes (end of Sec. 5.3).
 *
 * Conventions
 *  - Every pointer argument is a DEVICE pointer unless its comment says "host".
 *  - Floating-point inputs are IEEE binary64.  Arrays are dense and row-major;
 *    grid vertices and cells are ordered with x fastest, then y, then z.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All work is enqueued
 *    on it; only the gp_fit_* calls synchronise it (to read the factorisation
 *    status).  Calls that share a model or workspace must not run concurrently.
 *  - The library never allocates device memory: the caller passes the model
 *    memory and a workspace, sized by lcp_model_bytes / lcp_*_workspace, and
 *    keeps them alive while any enqueued work may still use them.  The one fixed
 *    device array the library holds serves lcp_dense_noalloc only.
 *  - Every call returns an lcp_status.  Arguments are validated on the host before
 *    anything is enqueued; on error nothing is enqueued and lcp_last_error()
 *    describes the problem (thread-local string, valid until the next call).
 */
#ifndef LCP_H
#define LCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LCP_OK = 0,
    LCP_EINVAL = 1,          /* invalid argument (sizes, pointers, parameters) */
    LCP_ENOTPD = 2,          /* K + noise I is numerically singular (Cholesky pivot <= m eps max K_ii) */
    LCP_ECAPACITY = 3,       /* an output list is smaller than the result; *count holds the true size */
    LCP_ENOMEM = 4,          /* model memory or workspace smaller than required */
    LCP_EDEVICE = 5,         /* a HIP runtime call failed */
    LCP_ENOTSUPPORTED = 6    /* operation not provided by this library */
} lcp_status;

typedef enum {
    LCP_KERNEL_SE = 0,       /* squared exponential s2 exp(-r^2/2), Sec. 3 (the paper's RBF, ARD allowed) */
    LCP_KERNEL_MATERN52 = 1  /* Matern-5/2 s2 (1 + sqrt5 r + 5 r^2/3) exp(-sqrt5 r), textbook form */
} lcp_kernel_kind;           /* r^2 = sum_d ((x_d - z_d) / lengthscale_d)^2 */

typedef enum {
    LCP_FP64 = 0,            /* every step in binary64 */
    LCP_FP32 = 1,            /* K* in binary32; V = L^-1 K*^T on FP32 MFMA; mean sums, norms, cell factor
                                in FP64; MC in FP32.  Region bound of lcp_adaptive always FP64 */
    LCP_MIXED_BF16X3 = 2,    /* as LCP_FP32 with V on BF16 MFMA as a 3-term split product
                                (hi*hi + hi*lo + lo*hi) with FP32 accumulation */
    LCP_MIXED_F16X3 = 3      /* as LCP_MIXED_BF16X3 with FP16 halves (22-bit split) on power-of-two scaled
                                operands; about FP32 accuracy at 16-bit MFMA rate */
} lcp_precision;

typedef struct {
    int kind;                /* lcp_kernel_kind */
    int dim;                 /* 2 or 3 */
    double signal_var;       /* s2 > 0 */
    double lengthscale[3];   /* > 0; entries beyond dim are ignored */
    double noise_var;        /* observation-noise variance >= 0 */
} lcp_kernel;

typedef struct {
    int dim;                 /* 2 or 3 (must equal the model's) */
    double lo[3], hi[3];     /* domain box; vertex i on axis d sits at lo + i (hi - lo) / (npts - 1) */
    int64_t npts[3];         /* vertices per axis, >= 2 for d < dim; cells per axis = npts - 1 */
} lcp_grid;

typedef struct {
    double alpha;            /* skip threshold of Alg. 1, 0 < alpha < 0.5 (the paper uses 1e-3, Sec. 7.3) */
    int min_leaf_cells;      /* finest node edge in cells, a power of two >= 1 (max depth of Alg. 1);
                                the octree may have at most 8 levels (root edge / min_leaf_cells <= 128) */
    int bound_at_max_depth;  /* 1: region test at the finest level too (Alg. 1 as printed); 0: emit */
    int descent_steps;       /* projected-gradient steps of the bound search after the 3^D lattice, 0..16 */
    int bound_kind;          /* lcp_bound_kind (0 = the paper's search) */
    int split;               /* lcp_split (0 = the octree of Alg. 1) */
    double beta;             /* LCP_BOUND_LOCAL only: box enlargement of the local model, in
                                lengthscales per axis, finite and >= 0 (Sec. 7.3 recommends 6) */
    int edge_bound;          /* 1: the tighter bound from edge crossings that Sec. 9 proposes: a
                                finest-level node the region test emits is kept only if the union
                                bound sum_e P(edge e crossed) over a spanning tree of its vertices
                                exceeds alpha (the event "some cell crossed" is "some tree edge
                                crossed"); its edge terms use the bivariate posterior of the edge's
                                ends.  0: Alg. 1 as printed */
} lcp_adapt;

typedef enum {
    LCP_SPLIT_OCTREE = 0,    /* Alg. 1: every node splits all axes at once (2^dim children) */
    LCP_SPLIT_KD = 1         /* K-D tree (Sec. 9): a node halves one axis, z, y, x in turn (2 children),
                                so depth dim * l holds the octree nodes of level l and the same finest
                                nodes; leaves keep the octree key of the finest level, and level_field
                                reports the depth (0 .. dim * levels) */
} lcp_split;

typedef enum {
    LCP_BOUND_SEARCH = 0,    /* B from a bounded search of F_M over the node (Sec. 5.1; the paper's
                                L-BFGS-B replaced by the 3^D lattice and descent_steps steps) */
    LCP_BOUND_CERTIFIED = 1, /* B from certified box bounds of mean and variance (lcp_bound_certified):
                                a node is skipped only if every point of it satisfies the bound, the
                                guarantee Sec. 9 leaves open; more nodes are refined than with the
                                search, and every leaf of the search is also a leaf here */
    LCP_BOUND_LOCAL = 2      /* the search of LCP_BOUND_SEARCH on the local model M' of Sec. 5.2 (Alg. 1):
                                the points of M inside the node box enlarged by beta * lengthscale_d
                                along axis d (the root keeps all).  Exact GP: the GP conditioned on
                                those observations alone; sparse model: eq. (sgp) with mu_M and A_M
                                restricted to them.  Factored per node in binary64; an approximation
                                of F_M that approaches it as beta grows.  A node whose local factor
                                is not positive definite is refined */
} lcp_bound_kind;

typedef enum {
    LCP_EST_COUNT = 0,       /* the paper's estimate (Sec. 4): fraction of samples mu + C z that cross */
    LCP_EST_SOV = 1          /* the same probability by Genz's separation of variables, with uniforms
                                Phi(z) from the first 2^dim - 1 normals of each row: smooth in the
                                cell's mean and covariance, so it has an adjoint (lcp_backward);
                                lcp_dense only; binary64 samples for LCP_FP64, binary32 samples
                                with binary64 sums otherwise */
} lcp_estimator;

typedef struct {
    int n_samples;           /* N_s >= 1 (the paper uses 1600, Sec. 6.4) */
    const double* zbank;     /* n_samples x 2^dim standard normals, shared by every cell (device) */
    int estimator;           /* lcp_estimator (0 = the paper's counting estimate) */
} lcp_mc;

typedef struct lcp_model lcp_model;   /* opaque host handle over caller-owned device memory */

/* Status text and the thread's last error message. */
const char* lcp_status_str(int status);
const char* lcp_last_error(void);

/* Bytes of device memory a model with m observations needs. */
size_t lcp_model_bytes(int m, int dim);

/*
 * gp_fit_factor -- factor the GP model (Sec. 3; the inducing set of eq. (sgp) is the
 * observation set, so mu_M and A_M are the latent posterior at the observations).
 * Builds K = k(X, X) + noise I in binary64, its Cholesky factor L, the explicit
 * inverse L^-1 (binary64, plus FP32 and split-BF16 copies), a = K^-1 y, the
 * posterior mean and variance at each observation (used by the preliminary node
 * test of Alg. 1), and K^-1 = L^-T L^-1 in the matrix-core fragment order (the
 * operand of the certified region bound).
 *   k        (host) kernel description
 *   m        number of observations, 1 <= m <= 1024
 *   X        m x dim observation locations (device, binary64)
 *   y        m observation values (device, binary64)
 *   model_mem, model_bytes   caller-owned device memory of >= lcp_model_bytes(m, dim)
 *            bytes, 256-byte aligned; it holds every device array of the model and must
 *            outlive the handle
 *   out      (host) receives the handle; free it with gp_model_free
 * Synchronises `stream` once.  Returns LCP_ENOTPD if a pivot is not above
 * m * eps * max_i K_ii (no jitter is added).
 */
int gp_fit_factor(const lcp_kernel* k, int m, const double* X, const double* y, void* model_mem,
                  size_t model_bytes, void* stream, lcp_model** out);

/*
 * gp_fit_sgpr -- factor a sparse GP model as eq. (sgp) gives it: inducing points M and the
 * Gaussian N(mu_M, A_M) of the inducing values stored after SGPR fitting (Sec. 3).  The
 * posterior at a set I is then mu = K_IM K_MM^-1 mu_M and
 * Sigma = K_II - K_IM K_MM^-1 K_MI + K_IM K_MM^-1 A_M K_MM^-1 K_MI, and the preliminary
 * node test of Alg. 1 reads the marginals N(mu_M_i, A_M_ii) (Sec. 5.3).
 *   k        (host) kernel; k->noise_var is the jitter added to the diagonal of K_MM
 *   m        number of inducing points, 1 <= m <= 1024
 *   Z        m x dim inducing locations (device, binary64)
 *   mu_M     m inducing means (device, binary64)
 *   A_M      m x m inducing covariance, row-major, symmetric (device, binary64); only
 *            read during the call
 *   model_mem, model_bytes, out   as for gp_fit_factor (same lcp_model_bytes)
 *   shift    (host, may be NULL) receives delta below
 * The third term is folded into the stored factor: with K_MM + jitter I = L L^T and
 * E = I - L^-1 A_M L^-T = F^T F (F lower), the model keeps T = F L^-1 in place of L^-1,
 * so every LCP routine applies unchanged.  E is PSD whenever A_M <= K_MM + jitter I (a
 * posterior covariance never exceeds its prior).  If a pivot of E is not above m eps the
 * factorisation is repeated on E + delta I, delta = 16 m eps and then 100 times larger
 * up to 1e-6; this raises each variance by delta ||L^-1 k*||^2 <= delta s2 and each
 * covariance by delta (L^-1 k_p).(L^-1 k_q).  Synchronises `stream` once per attempt.
 * Returns LCP_ENOTPD if K_MM + jitter I is numerically singular or E is not PSD to 1e-6.
 */
int gp_fit_sgpr(const lcp_kernel* k, int m, const double* Z, const double* mu_M, const double* A_M,
                void* model_mem, size_t model_bytes, void* stream, double* shift, lcp_model** out);

void gp_model_free(lcp_model* model);

/* Size queries of the workspace of each operation (host results); the workspace must be
 * 256-byte aligned.  n_samples is the Monte Carlo sample count the call will use.  With
 * LCP_BOUND_LOCAL the adaptive workspace also holds one binary64 slot of
 * m_pad^2 + 128 m_pad doubles (m_pad = m rounded up to 128) per work-group of the
 * local-model kernel resident on the current device: its occupancy for the model's LDS use
 * times the CU count, at most 1024 (4 per CU at m = 500 on a 256-CU device: 2.7 GB; 2 per
 * CU at m = 1024).  The query and the call must run on the same device. */
int lcp_posterior_workspace(const lcp_model* model, int64_t n, int prec, size_t* bytes);
int lcp_dense_workspace(const lcp_model* model, const lcp_grid* grid, int prec, int n_samples, size_t* bytes);
int lcp_adaptive_workspace(const lcp_model* model, const lcp_grid* grid, const lcp_adapt* adapt, int prec,
                           int n_samples, size_t* bytes);

/*
 * gp_posterior -- latent posterior mean and variance at n query points (eq. (sgp),
 * exact-GP form): mean = k*^T a, var = max(0, s2 - ||L^-1 k*||^2).
 *   Xq    n x dim query points; mean, var: n outputs (binary64).
 *   prec  lcp_precision of V = L^-1 k*^T (mean is always accumulated in binary64).
 */
int gp_posterior(const lcp_model* model, int64_t n, const double* Xq, int prec, double* mean, double* var,
                 void* ws, size_t ws_bytes, void* stream);

/*
 * lcp_dense -- the dense baseline of Sec. 4: posterior at every grid vertex, the
 * 2^dim-corner covariance of every cell, its (semidefinite) Cholesky factor C and the
 * Monte Carlo estimate LCP = #{s : not all corners below theta and not all above} / N_s
 * with corner values mu + C z_s.  A sample equal to theta counts as crossed.
 *   lcp   prod(npts - 1) cells (binary32, x fastest).
 */
int lcp_dense(const lcp_model* model, const lcp_grid* grid, double theta, const lcp_mc* mc, int prec,
              float* lcp, void* ws, size_t ws_bytes, void* stream);

/*
 * lcp_adaptive -- Alg. 1 (octree adaptive query) on the full model (or its local models) followed by the
 * reconstruction of Sec. 5.3's last paragraph: cells inside the emitted nodes get the
 * same Monte Carlo LCP as lcp_dense (same precision, same z-bank); all other cells get 0.
 * The region test (preliminary decision on the observations inside the closed node box,
 * then the bound 1 - B^d of eq. (upper_bound) with B from a bounded search of F_M, from
 * certified box bounds when adapt->bound_kind is LCP_BOUND_CERTIFIED, or from the search on
 * the node's local model when it is LCP_BOUND_LOCAL) runs in binary64
 * regardless of `prec`.
 *   lcp          prod(npts - 1) cells (binary32)
 *   leaves       leaf_cap keys of the emitted nodes, key = level << 58 | Morton(node), ascending
 *   n_leaves     (device) receives the number of emitted nodes
 *   level_field  optional (may be NULL): per cell, the octree level (K-D tree: depth) at which
 *                its node stopped
 * If the emitted set exceeds leaf_cap, the first leaf_cap keys are written, *n_leaves
 * receives the true count, and the reconstruction is not performed (LCP stays zero); the
 * caller sees this after synchronising the stream.
 */
int lcp_adaptive(const lcp_model* model, const lcp_grid* grid, double theta, const lcp_adapt* adapt,
                 const lcp_mc* mc, int prec, float* lcp, uint64_t* leaves, int64_t leaf_cap, int64_t* n_leaves,
                 uint8_t* level_field, void* ws, size_t ws_bytes, void* stream);

/*
 * lcp_cell_moments -- the 2^dim-corner Gaussian of listed cells (Sec. 4: the corner values
 * of a cell follow a multivariate normal whose mean and covariance come from eq. (sgp)),
 * computed by the same kernels as lcp_dense and lcp_adaptive in precision `prec`: posterior
 * mean and variance at the corner vertices and the neighbour cross-covariances
 * k(x_p, x_q) - v_p . v_q.  For inspection and error reporting; no Monte Carlo.
 *   cells  n linear cell indices (device, int64; cell (i, j, k) = i + nc0 (j + nc1 k), x
 *          fastest, nc = npts - 1); an index outside [0, prod(nc)) gives NaN outputs
 *   mean   n x 2^dim corner means (device, binary64); corner q is at offset
 *          (q & 1, (q >> 1) & 1, (q >> 2) & 1)
 *   cov    n x 2^dim x 2^dim corner covariances, row-major per cell (device, binary64)
 *   ws     lcp_cell_moments_workspace bytes (grid-sized flags plus the corners' posterior)
 * Asynchronous on `stream`.
 */
int lcp_cell_moments_workspace(const lcp_model* model, const lcp_grid* grid, int64_t n, int prec, size_t* bytes);
int lcp_cell_moments(const lcp_model* model, const lcp_grid* grid, int64_t n, const int64_t* cells, int prec,
                     double* mean, double* cov, void* ws, size_t ws_bytes, void* stream);

/*
 * lcp_bound_certified -- box bounds of the latent posterior that hold at every point of
 * each box, which make the region bound of eq. (upper_bound) guaranteed (the bounded search
 * of Sec. 5.1 can miss the minimum, Sec. 9).  For box b with centre c and half-widths h:
 *   out[4b + 0] = mu(c)
 *   out[4b + 1], out[4b + 2] = lower and upper bound of mu over the box
 *   out[4b + 3] = upper bound of var over the box (within [0, s2])
 * from a second-order Taylor model at c with a third-order remainder bound: mu = a^T k and
 * nu = w^T k with w = Q k(c) (Q = (K + noise I)^-1, or K^-1 - K^-1 A_M K^-1 for a sparse
 * model), using var(x) <= s2 - nu(c) - 2 (nu(x) - nu(c)) (convexity of k^T Q k).  The bounds
 * hold in exact arithmetic for the stored model; the binary64 rounding of their own sums is
 * not bounded.
 *   boxes  n x (2 dim): lo[0..dim-1], hi[0..dim-1] per box (device, binary64); lo <= hi on
 *          every axis is required and not checked (the device data is not read on the host):
 *          otherwise the results are unspecified
 *   out    n x 4 (device, binary64)
 *   ws     lcp_bound_workspace bytes
 */
int lcp_bound_workspace(const lcp_model* model, int64_t n, size_t* bytes);
int lcp_bound_certified(const lcp_model* model, int64_t n, const double* boxes, double* out, void* ws,
                        size_t ws_bytes, void* stream);

/*
 * Batches of independent models (local GP models of subdomains, each with its own
 * observations, kernel and grid, as the local models M' of Sec. 5.1 generalise): every
 * model's Cholesky factor runs in one launch (a work-group each), and the posterior GEMMs
 * of all models run in one launch that walks the batch's tiles, so small models share the
 * GPU with large ones.
 *
 * lcp_batch_model_bytes -- device memory for nb models with m[b] observations (host array);
 *   0 if nb < 1 or some m[b] is outside 1..1024.
 *
 * gp_fit_factor_batch -- gp_fit_factor for each model of the batch.
 *   k, m     (host) nb kernel descriptions (same dim) and observation counts
 *   X, y     (device) the models' observations concatenated in model order: model b's
 *            m[b] x dim rows of X (and m[b] values of y) follow model b - 1's
 *   model_mem, model_bytes   caller-owned device memory of >= lcp_batch_model_bytes bytes,
 *            256-byte aligned, alive as long as the handle
 *   out      (host) receives the batch handle; free it with gp_model_batch_free
 * Synchronises `stream` once.  LCP_ENOTPD if any model's K + noise I is numerically
 * singular (lcp_last_error names the first).  The posterior at the observations that
 * lcp_adaptive uses is not computed: a batch serves lcp_dense_batch.
 */
typedef struct lcp_model_batch lcp_model_batch;   /* opaque host handle */

size_t lcp_batch_model_bytes(int nb, const int* m, int dim);
int gp_fit_factor_batch(int nb, const lcp_kernel* k, const int* m, const double* X, const double* y,
                        void* model_mem, size_t model_bytes, void* stream, lcp_model_batch** out);
void gp_model_batch_free(lcp_model_batch* batch);

/*
 * lcp_dense_batch -- lcp_dense for every model of the batch on its own grid (grids[b],
 * host array) and iso-value (theta[b], host array), with one shared z-bank.
 *   lcp   the models' cell fields concatenated in model order (each x fastest, binary32)
 * The workspace size comes from lcp_dense_batch_workspace.  Synchronises `stream` once
 * (upload of the per-model descriptors).
 */
int lcp_dense_batch_workspace(const lcp_model_batch* batch, const lcp_grid* grids, int prec, int n_samples,
                              size_t* bytes);
int lcp_dense_batch(const lcp_model_batch* batch, const lcp_grid* grids, const double* theta, const lcp_mc* mc,
                    int prec, float* lcp, void* ws, size_t ws_bytes, void* stream);

/*
 * Precision per model.  In a reduced precision the error of V = L^-1 K*^T grows with the
 * conditioning of the model: a binary32 V carries about eps32 |L^-1| |k*|, and the binary32
 * kernel values alone bound what any refinement of V in the same precision can recover.  On
 * batches of models with noise / s2 = 1e-4 and up to 1024 dense observations this reaches an
 * LCP RMSE of several 1e-3, against a target of 1e-4 (Sec. 6.2's accuracy metric).
 *
 * lcp_batch_precision -- prec[b] = `reduced` if kappa_b = sqrt(s2_b) max|L_b^-1| <= kappa_max,
 *   else LCP_FP64.  kappa_max <= 0 takes the library's default: 8 for LCP_FP32 (the largest
 *   kappa at which binary32 stayed below an LCP RMSE of 1e-4 on every measured model), scaled
 *   by the unit roundoff for the split forms (2 for LCP_MIXED_F16X3, 1/32 for
 *   LCP_MIXED_BF16X3).  kappa (host, may be NULL) receives kappa_b.  Reads max|L_b^-1| from
 *   the device: synchronises `stream` once.
 *   prec  (host) nb entries
 * lcp_dense_batch_mixed -- lcp_dense_batch with model b in precision prec[b] (host array);
 *   each pass runs as one launch per precision present.  Workspace from
 *   lcp_dense_batch_mixed_workspace.
 */
int lcp_batch_precision(const lcp_model_batch* batch, int reduced, double kappa_max, int* prec, double* kappa,
                        void* stream);

/*
 * lcp_batch_tiles -- tile width nt (16 or 32 columns per work-group) and waves nw (4, 8 or 16)
 * of the batched posterior for models of precision `prec` with m_pad = 128 (size_class + 1)
 * (m_pad = m rounded up to 128; size_class 0..7).  The library's defaults come from the
 * project's autotuner (paper_2512_12442_amd/autotune.py), which times every candidate on the
 * batched workload and writes the winners into the compiled table (csrc/tune_table.inc);
 * nt = 0 restores them.  LCP_EINVAL if the pair is not a candidate or its tile exceeds the
 * LDS.  Process-wide and not synchronised:
 * set it before launches that other threads may issue.
 * lcp_batch_tiles_get -- the current setting.
 */
int lcp_batch_tiles(int prec, int size_class, int nt, int nw);
int lcp_batch_tiles_get(int prec, int size_class, int* nt, int* nw);
int lcp_dense_batch_mixed_workspace(const lcp_model_batch* batch, const lcp_grid* grids, const int* prec,
                                    int n_samples, size_t* bytes);
int lcp_dense_batch_mixed(const lcp_model_batch* batch, const lcp_grid* grids, const double* theta, const lcp_mc* mc,
                          const int* prec, float* lcp, void* ws, size_t ws_bytes, void* stream);

/*
 * gp_posterior_backward -- adjoint of gp_posterior (Sec. 3, eq. (sgp) in its exact-GP form)
 * with respect to the observation values y and the log-lengthscales log(ell_d).  Given
 * upstream gradients g = dL/dmean and h = dL/dvar at n query points, with K = k(X, X) +
 * noise I, a = K^-1 y and w_p = K^-1 k*_p:
 *   dL/dy          = sum_p g_p w_p
 *   dL/dlog(ell_d) = sum_p g_p (dk*_p,d . a - w_p^T dK_d a) + h_p (-2 dk*_p,d . w_p + w_p^T dK_d w_p)
 * where dk*_d, dK_d are derivatives of k* and K with respect to log(ell_d).  K* is
 * regenerated, never stored; W = K^-1 K*^T runs on MFMA in `prec` (LCP_FP64 or LCP_FP32,
 * FP64 sums either way).
 *   model      from gp_fit_factor (LCP_ENOTSUPPORTED for a gp_fit_sgpr model)
 *   n, Xq      n >= 0 query points, n x dim binary64 (device)
 *   dL_dmean, dL_dvar   n binary64 each (device); either may be NULL (zero)
 *   dL_dy      m binary64 (device), overwritten
 *   dL_dloglen dim binary64 (device), overwritten
 *   ws, ws_bytes   256-byte aligned workspace of gp_posterior_backward_workspace bytes
 *                  (about n * m_pad * 8 (FP64) or 4 (FP32) bytes plus O(m^2))
 * Results are reproducible bit for bit (every sum runs in a fixed order).  Enqueued only.
 */
int gp_posterior_backward_workspace(const lcp_model* model, int64_t n, int prec, size_t* bytes);
int gp_posterior_backward(const lcp_model* model, int64_t n, const double* Xq, int prec, const double* dL_dmean,
                          const double* dL_dvar, double* dL_dy, double* dL_dloglen, void* ws, size_t ws_bytes,
                          void* stream);

/*
 * lcp_backward -- adjoint of the smooth LCP field of lcp_dense (estimator LCP_EST_SOV) with
 * respect to the observation values y and the log-lengthscales, for upstream gradients
 * dL_dlcp (one per cell, x fastest).  The counting estimate of Sec. 4 is piecewise constant
 * in the model; the separation-of-variables estimate of the same probability is smooth, and
 * this call differentiates it exactly (for the fixed z-bank): the cell's gradient with
 * respect to its corner means and factor, the factor's adjoint, then eq. (sgp) through the
 * vertex means, variances and neighbour covariances (the posterior adjoint with
 * neighbour terms; K* regenerated, never stored).
 *   model   from gp_fit_factor (LCP_ENOTSUPPORTED for a gp_fit_sgpr model)
 *   grid, theta, mc   as for lcp_dense; mc->estimator must be LCP_EST_SOV
 *   prec    LCP_FP64 or LCP_FP32: precision of V, W = K^-1 K*^T and the estimator's samples
 *           (cell factors, their adjoint and every sum are binary64); LCP_MIXED_F16X3 or
 *           LCP_MIXED_BF16X3: V by that split product (as in lcp_dense), the rest as LCP_FP32
 *   dL_dlcp cells binary64 (device)
 *   dL_dy   m binary64 (device), overwritten;  dL_dloglen  dim binary64 (device), overwritten
 *   ws, ws_bytes   256-byte aligned, >= lcp_backward_workspace bytes (about 4 n m_pad
 *                  elements of prec for n grid vertices, plus O(cells + m^2))
 * Reproducible bit for bit.  Enqueued only.
 */
int lcp_backward_workspace(const lcp_model* model, const lcp_grid* grid, int prec, int n_samples, size_t* bytes);
int lcp_backward(const lcp_model* model, const lcp_grid* grid, double theta, const lcp_mc* mc, int prec,
                 const double* dL_dlcp, double* dL_dy, double* dL_dloglen, void* ws, size_t ws_bytes,
                 void* stream);

/*
 * lcp_dense_noalloc -- lcp_dense without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Arguments and results are those of lcp_dense; the workspace is
 * a fixed device array inside the library of LCP_NOALLOC_SCRATCH_BYTES bytes per device,
 * held from library load until the process ends.  Nothing is allocated or freed: the call
 * takes the array's device address once per device (on its first call there, with that
 * device current) and then only enqueues work.
 *   Limit: grids whose lcp_dense_workspace size exceeds LCP_NOALLOC_SCRATCH_BYTES return
 *   LCP_ENOMEM before anything is enqueued (with FP32 operands and m = 500: about 31^3
 *   vertices).  The model must live on the current device (LCP_EINVAL otherwise).
 *   Every call on one device shares that device's array and leaves its contents behind;
 *   the call itself clears what it needs at zero.  Calls that overlap on one device (two
 *   streams, or two host threads) race on the array and give undefined results: order them
 *   on one stream or serialise them.
 */
#define LCP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int lcp_dense_noalloc(const lcp_model* model, const lcp_grid* grid, double theta, const lcp_mc* mc, int prec,
                      float* lcp, void* stream);

/*
 * Stage timer (tracing).  lcp_profile_begin(mask) enables it for the stages whose bit is
 * set: 0 model factorisation, 1 posterior GEMM at vertices / query points, 2 binary64
 * posterior probes of the region bound, 3 neighbour cross-covariances, 4 cell factor and
 * Monte Carlo, 5 octree tests / prefix sums / emission, 6 fills and conversions.  Each
 * launch of an enabled stage is bracketed by hipEvents recorded on the launch stream.
 * lcp_profile_end(ms, launches, n_stages) waits for those events, disables the timer and
 * writes per stage the summed elapsed milliseconds and the number of bracketed launches
 * (host arrays of n_stages entries, either may be NULL).  Process-wide; calls from several
 * threads while it is enabled share one record list.
 */
int lcp_profile_begin(unsigned stage_mask);
int lcp_profile_end(double* ms, int64_t* launches, int n_stages);

#ifdef __cplusplus
}
#endif

#endif /* LCP_H */
