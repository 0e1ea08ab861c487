/*
 * Oracle for the level-crossing-probability (LCP) hot path -- TEST INFRASTRUCTURE.
 *
 * A plain, slow, FP64 CPU implementation of what the GPU library computes, written
 * from the paper (Li, Michaud, Biswas, Shen, "Efficient Level-Crossing Probability
 * Calculation for Gaussian Process Modeled Data", arXiv 2512.12442).  Only the test
 * suite, the smoke check and the bench's CPU-baseline leg load this library; the
 * product path never does.  It shares no code with the HIP library.
 *
 * Every loop runs in the order of the definition it implements; OpenMP only
 * distributes independent points, cells or octree nodes over threads.
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see oracle/build.py).
 *
 * Readings of the paper taken here (all listed in the design notes):
 *  - GP model: the exact-GP special case of eq. (sgp) (inducing set = observations),
 *    so mu(x) = k*^T (K + s_n^2 I)^-1 y and var(x) = k(x,x) - ||L^-1 k*||^2, latent f;
 *    or the general eq. (sgp) with stored mu_M and A_M, K_MM taking the model's noise
 *    term as a diagonal jitter.  The preliminary node test of Alg. 1 then reads the
 *    inducing marginals N(mu_M_i, A_M_ii) directly (Sec. 5.3).
 *  - F_M uses the standard deviation, not the variance (Sec. 5.1 prints Sigma).
 *  - Cell covariance is factored with a semidefinite Cholesky (tolerance 1e-12 of the
 *    largest diagonal entry); a sample equal to the iso-value counts as crossed.
 *  - The L-BFGS-B search of Sec. 5.1 is replaced by a fixed-budget bounded search:
 *    a {lo,mid,hi}^D lattice followed by T normalised projected-gradient steps.
 *  - Alg. 1 runs on the full model F_M, or (bound_kind 2) with the local model M' of
 *    Sec. 5.2 in the region test (its box rule and per-model reading are stated at
 *    local_build); p = alpha counts as "not larger than alpha"; a node without
 *    observations takes its side from the sign of theta - mu(box centre) under the
 *    model of its region test.
 *  - The certified variant of the region bound (guaranteed in exact arithmetic, which
 *    Sec. 9 leaves open) bounds mu and var over the whole box instead of searching.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOTPD 2
#define ORC_ECAP 3
#define ORC_ENOMEM 4

typedef struct {
    int kind;          /* 0: squared exponential (Sec. 3), 1: Matern-5/2 (textbook) */
    int dim;           /* 2 or 3 */
    int m;             /* number of observations */
    double s2;         /* signal variance */
    double ell[3];     /* per-axis lengthscales */
    double noise;      /* observation-noise variance */
    const double* X;  /* m x dim observation locations, row-major */
    const double* L;  /* m x m lower Cholesky factor of K + noise I, row-major */
    const double* a;  /* m: (K + noise I)^-1 y */
    const double* A;  /* NULL: exact GP.  Else the sparse model of eq. (sgp): X are the
                         inducing points M, L factors K_MM (+ jitter I, the field noise),
                         a = K_MM^-1 mu_M, and A is the m x m covariance A_M of the
                         inducing values */
    const double* muM; /* sparse model only: the m inducing means mu_M */
    const double* y;   /* exact GP: the m observed values (the local model of Sec. 5.2 refits
                          on a subset of them); may be NULL when no local model is built */
} orc_model;

typedef struct {
    int dim;
    double lo[3];
    double hi[3];
    int64_t n[3];      /* vertices per axis; x is the fastest axis */
} orc_grid;

typedef struct {
    double alpha;
    int min_leaf;           /* finest node edge in cells (power of two) */
    int bound_at_max_depth; /* 1: Alg. 1 as printed (region test at every level) */
    int steps;              /* projected-gradient steps after the lattice */
    int bound_kind;         /* 0: bounded search (lattice + steps), 1: certified box bounds */
    int split;              /* 0: octree (Alg. 1), 1: K-D tree splitting the axes in turn (Sec. 9) */
    double beta;            /* bound_kind 2: box enlargement of the local model, in lengthscales */
    int edge_bound;         /* 1: a deepest-level node the region test would emit is emitted only if
                               its edge-crossing union bound exceeds alpha (orc_node_edge_bound) */
} orc_adapt;

typedef struct {
    uint64_t key;      /* level << 58 | Morton code of the node coordinates */
    int32_t level;
    int32_t n_obs;     /* |M~| : observations inside the closed node box */
    double p1, p2;     /* max P(Y_i < theta), max P(Y_i > theta) over M~ */
    int32_t path;      /* 0 prelim subdivide, 1 bound below, 2 bound above, 3 max depth w/o bound */
    int32_t subdivide;
    double gmin;       /* minimum of the standardised margin found by the search */
    double ub;         /* 1 - B^d */
    double lattice_gap;/* second-smallest minus smallest lattice value */
    int64_t d;         /* grid vertices inside the node */
    int64_t n_local;   /* bound_kind 2: |M'| of the local model (-1: no region test) */
    double eb;         /* edge_bound: the node's edge-crossing union bound (NaN: not evaluated) */
} orc_node_rec;

/* ---------------------------------------------------------------- kernels -- */

static double scaled_r2(int dim, const double* ell, const double* x, const double* z)
{
    double r2 = 0.0;
    for (int d = 0; d < dim; ++d) {
        double t = (x[d] - z[d]) / ell[d];
        r2 += t * t;
    }
    return r2;
}

/* k(x, z): squared exponential s2 exp(-r^2/2) (Sec. 3), Matern-5/2 s2 (1 + sqrt5 r + 5r^2/3) exp(-sqrt5 r). */
double orc_kernel(int kind, int dim, double s2, const double* ell, const double* x, const double* z)
{
    double r2 = scaled_r2(dim, ell, x, z);
    if (kind == 0) return s2 * exp(-0.5 * r2);
    double r = sqrt(r2);
    return s2 * (1.0 + sqrt(5.0) * r + 5.0 * r2 / 3.0) * exp(-sqrt(5.0) * r);
}

/* Gradient of k(x, z) with respect to x. */
void orc_kernel_grad(int kind, int dim, double s2, const double* ell, const double* x, const double* z,
                     double* g)
{
    double r2 = scaled_r2(dim, ell, x, z);
    double f;
    if (kind == 0) {
        f = -s2 * exp(-0.5 * r2);
    } else {
        double r = sqrt(r2);
        f = -(5.0 / 3.0) * s2 * (1.0 + sqrt(5.0) * r) * exp(-sqrt(5.0) * r);
    }
    for (int d = 0; d < dim; ++d) g[d] = f * (x[d] - z[d]) / (ell[d] * ell[d]);
}

/* ---------------------------------------------------------- model factor -- */

/* Per-point vector kept for the cross-covariances: v = L^-1 k* (m) for the exact GP; for
 * the sparse model [k*, w = K_MM^-1 k*, A_M w] (3m). */
static int vwidth(const orc_model* M) { return M->A ? 3 * M->m : M->m; }

/* Solve L v = b by forward substitution (L row-major lower, m x m). */
static void forward_sub(int m, const double* L, const double* b, double* v)
{
    for (int i = 0; i < m; ++i) {
        double s = b[i];
        for (int j = 0; j < i; ++j) s -= L[(int64_t)i * m + j] * v[j];
        v[i] = s / L[(int64_t)i * m + i];
    }
}

/* Solve L^T v = b by backward substitution. */
static void backward_sub_t(int m, const double* L, const double* b, double* v)
{
    for (int i = m - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < m; ++j) s -= L[(int64_t)j * m + i] * v[j];
        v[i] = s / L[(int64_t)i * m + i];
    }
}

/*
 * Factor the model (Sec. 3, exact-GP form of eq. (sgp)): K_ij = k(x_i,x_j) + noise d_ij,
 * K = L L^T by Cholesky-Banachiewicz without pivoting or jitter, a = L^-T L^-1 y.
 * Returns ORC_ENOTPD if a pivot is not above m * eps * max_i K_ii (numerically singular K).
 */
int orc_fit(int kind, int dim, double s2, const double* ell, double noise, int m,
            const double* X, const double* y, double* L, double* a)
{
    double* K = (double*)malloc(sizeof(double) * (size_t)m * m);
    double* w = (double*)malloc(sizeof(double) * (size_t)m);
    if (!K || !w) { free(K); free(w); return ORC_ENOMEM; }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            K[(int64_t)i * m + j] = orc_kernel(kind, dim, s2, ell, X + (int64_t)i * dim, X + (int64_t)j * dim)
                                    + (i == j ? noise : 0.0);
    memset(L, 0, sizeof(double) * (size_t)m * m);
    /* A pivot at or below m * eps * max_i K_ii is rounding noise: K is numerically singular. */
    double kmax = 0.0;
    for (int i = 0; i < m; ++i) if (K[(int64_t)i * m + i] > kmax) kmax = K[(int64_t)i * m + i];
    double piv_min = (double)m * 2.220446049250313e-16 * kmax;
    int rc = ORC_OK;
    for (int i = 0; i < m && rc == ORC_OK; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = K[(int64_t)i * m + j];
            for (int k = 0; k < j; ++k) s -= L[(int64_t)i * m + k] * L[(int64_t)j * m + k];
            if (i == j) {
                if (!(s > piv_min)) { rc = ORC_ENOTPD; break; }
                L[(int64_t)i * m + i] = sqrt(s);
            } else {
                L[(int64_t)i * m + j] = s / L[(int64_t)j * m + j];
            }
        }
    }
    if (rc == ORC_OK) {
        forward_sub(m, L, y, w);
        backward_sub_t(m, L, w, a);
    }
    free(K);
    free(w);
    return rc;
}

/* ------------------------------------------------------------- posterior -- */

/* Posterior of the latent field at one point: mean, variance (clamped at 0), v = L^-1 k*. */
static void posterior_point(const orc_model* M, const double* x, double* mean, double* var,
                            double* kbuf, double* v)
{
    int m = M->m;
    if (M->A) {
        /* eq. (sgp): mu = K_IM K_MM^-1 mu_M, Sigma = K_II - K_IM K_MM^-1 K_MI
         *                                            + K_IM K_MM^-1 A_M K_MM^-1 K_MI */
        double* k = v;
        double* w = v + m;
        double* Aw = v + 2 * m;
        for (int j = 0; j < m; ++j) k[j] = orc_kernel(M->kind, M->dim, M->s2, M->ell, M->X + (int64_t)j * M->dim, x);
        double mu = 0.0;
        for (int j = 0; j < m; ++j) mu += k[j] * M->a[j];
        forward_sub(m, M->L, k, kbuf);
        backward_sub_t(m, M->L, kbuf, w);
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += M->A[(int64_t)i * m + j] * w[j];
            Aw[i] = s;
        }
        double t1 = 0.0, t2 = 0.0;
        for (int j = 0; j < m; ++j) t1 += k[j] * w[j];
        for (int j = 0; j < m; ++j) t2 += w[j] * Aw[j];
        double s = M->s2 - t1 + t2;
        *mean = mu;
        *var = s > 0.0 ? s : 0.0;
        return;
    }
    for (int j = 0; j < m; ++j) kbuf[j] = orc_kernel(M->kind, M->dim, M->s2, M->ell, M->X + (int64_t)j * M->dim, x);
    double mu = 0.0;
    for (int j = 0; j < m; ++j) mu += kbuf[j] * M->a[j];
    forward_sub(m, M->L, kbuf, v);
    double nv = 0.0;
    for (int j = 0; j < m; ++j) nv += v[j] * v[j];
    double s = M->s2 - nv;
    *mean = mu;
    *var = s > 0.0 ? s : 0.0;
}

/* Posterior mean and variance at n points; optionally the per-point vector of vwidth
 * entries (v = L^-1 k* for the exact GP) per point. */
int orc_posterior(const orc_model* M, int64_t n, const double* P, double* mean, double* var, double* V)
{
    int m = M->m;
    int rc = ORC_OK;
#pragma omp parallel
    {
        double* kb = (double*)malloc(sizeof(double) * (size_t)m);
        double* vb = (double*)malloc(sizeof(double) * (size_t)vwidth(M));
        if (!kb || !vb) {
#pragma omp atomic write
            rc = ORC_ENOMEM;
        } else {
#pragma omp for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                double* v = V ? V + i * vwidth(M) : vb;
                posterior_point(M, P + i * M->dim, &mean[i], &var[i], kb, v);
            }
        }
        free(kb);
        free(vb);
    }
    return rc;
}

/* Posterior mean/variance and their gradients at one point (used by the region bound). */
static void posterior_grad_point(const orc_model* M, const double* x, double* mean, double* var,
                                 double* dmean, double* dvar, double* kb, double* dkb, double* v, double* w)
{
    int m = M->m, D = M->dim;
    posterior_point(M, x, mean, var, kb, v);
    for (int j = 0; j < m; ++j) {
        double g[3];
        orc_kernel_grad(M->kind, D, M->s2, M->ell, x, M->X + (int64_t)j * D, g);
        for (int d = 0; d < D; ++d) dkb[(int64_t)d * m + j] = g[d];
    }
    if (M->A) {
        /* d Sigma / dx_d = -2 dk^T w + 2 dk^T K_MM^-1 A_M w = -2 dk^T (w - K_MM^-1 A_M w) */
        const double* wv = v + m;
        forward_sub(m, M->L, v + 2 * m, kb);
        backward_sub_t(m, M->L, kb, w);
        for (int d = 0; d < D; ++d) {
            double dm = 0.0, s = 0.0;
            for (int j = 0; j < m; ++j) dm += dkb[(int64_t)d * m + j] * M->a[j];
            for (int j = 0; j < m; ++j) s += dkb[(int64_t)d * m + j] * (wv[j] - w[j]);
            dmean[d] = dm;
            dvar[d] = -2.0 * s;
        }
        return;
    }
    for (int d = 0; d < D; ++d) {
        double dm = 0.0;
        for (int j = 0; j < m; ++j) dm += dkb[(int64_t)d * m + j] * M->a[j];
        dmean[d] = dm;
        forward_sub(m, M->L, dkb + (int64_t)d * m, w);
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += v[j] * w[j];
        dvar[d] = -2.0 * s;
    }
}

/* d k(x, z) / d log(ell_d): with r^2 = sum_d (x_d - z_d)^2 / ell_d^2, d r^2 / d log(ell_d) =
 * -2 (x_d - z_d)^2 / ell_d^2, times dk/d(r^2) (-k/2 for SE, -(5/6) s2 (1 + sqrt5 r) e^(-sqrt5 r)
 * for Matern-5/2). */
void orc_kernel_dlogell(int kind, int dim, double s2, const double* ell, const double* x, const double* z,
                        double* g)
{
    double r2 = scaled_r2(dim, ell, x, z);
    double dk_dr2;
    if (kind == 0) {
        dk_dr2 = -0.5 * s2 * exp(-0.5 * r2);
    } else {
        double r = sqrt(r2);
        dk_dr2 = -(5.0 / 6.0) * s2 * (1.0 + sqrt(5.0) * r) * exp(-sqrt(5.0) * r);
    }
    for (int d = 0; d < dim; ++d) {
        double t = (x[d] - z[d]) / ell[d];
        g[d] = dk_dr2 * (-2.0 * t * t);
    }
}

/*
 * Adjoint of the exact-GP posterior (eq. (sgp) with the inducing set equal to the
 * observations) at n query points, for upstream gradients gm = dL/dmean and gv = dL/dvar
 * (either may be NULL for zero).  With K = k(X, X) + noise I, a = K^-1 y, w = K^-1 k*:
 *   dmean/dy = w,                       dvar/dy = 0,
 *   dmean/dlog(ell_d) = dk*_d . a - w^T dK_d a,
 *   dvar/dlog(ell_d)  = -2 dk*_d . w + w^T dK_d w,
 * where dk*_d and dK_d are the derivatives of k* and K with respect to log(ell_d).
 * Point by point, in that form; dy (m) and dlogell (dim) receive the sums.
 */
int orc_posterior_backward(const orc_model* M, int64_t n, const double* P, const double* gm, const double* gv,
                           double* dy, double* dlogell)
{
    if (M->A) return ORC_EINVAL;
    int m = M->m, D = M->dim;
    double* dK = (double*)malloc(sizeof(double) * (size_t)D * m * m);
    double* dKa = (double*)malloc(sizeof(double) * (size_t)D * m);
    double* k = (double*)malloc(sizeof(double) * (size_t)m);
    double* t = (double*)malloc(sizeof(double) * (size_t)m);
    double* w = (double*)malloc(sizeof(double) * (size_t)m);
    double* dk = (double*)malloc(sizeof(double) * (size_t)D * m);
    if (!dK || !dKa || !k || !t || !w || !dk) {
        free(dK); free(dKa); free(k); free(t); free(w); free(dk);
        return ORC_ENOMEM;
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            double g[3];
            orc_kernel_dlogell(M->kind, D, M->s2, M->ell, M->X + (int64_t)i * D, M->X + (int64_t)j * D, g);
            for (int d = 0; d < D; ++d) dK[((int64_t)d * m + i) * m + j] = g[d];
        }
    for (int d = 0; d < D; ++d)
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += dK[((int64_t)d * m + i) * m + j] * M->a[j];
            dKa[(int64_t)d * m + i] = s;
        }
    for (int j = 0; j < m; ++j) dy[j] = 0.0;
    for (int d = 0; d < D; ++d) dlogell[d] = 0.0;
    for (int64_t p = 0; p < n; ++p) {
        const double* x = P + p * D;
        double g1 = gm ? gm[p] : 0.0, g2 = gv ? gv[p] : 0.0;
        for (int j = 0; j < m; ++j) {
            const double* xj = M->X + (int64_t)j * D;
            double g[3];
            k[j] = orc_kernel(M->kind, D, M->s2, M->ell, x, xj);
            orc_kernel_dlogell(M->kind, D, M->s2, M->ell, x, xj, g);
            for (int d = 0; d < D; ++d) dk[(int64_t)d * m + j] = g[d];
        }
        forward_sub(m, M->L, k, t);
        backward_sub_t(m, M->L, t, w);
        for (int j = 0; j < m; ++j) dy[j] += g1 * w[j];
        for (int d = 0; d < D; ++d) {
            const double* dkd = dk + (int64_t)d * m;
            const double* dKd = dK + (int64_t)d * m * m;
            double dka = 0.0, wdKa = 0.0, dkw = 0.0, wdKw = 0.0;
            for (int j = 0; j < m; ++j) dka += dkd[j] * M->a[j];
            for (int j = 0; j < m; ++j) wdKa += w[j] * dKa[(int64_t)d * m + j];
            for (int j = 0; j < m; ++j) dkw += dkd[j] * w[j];
            for (int i = 0; i < m; ++i) {
                double s = 0.0;
                for (int j = 0; j < m; ++j) s += dKd[(int64_t)i * m + j] * w[j];
                wdKw += w[i] * s;
            }
            dlogell[d] += g1 * (dka - wdKa) + g2 * (-2.0 * dkw + wdKw);
        }
    }
    free(dK); free(dKa); free(k); free(t); free(w); free(dk);
    return ORC_OK;
}

int orc_posterior_grad(const orc_model* M, const double* x, double* mean, double* var, double* dmean, double* dvar)
{
    int m = M->m;
    double* buf = (double*)malloc(sizeof(double) * ((size_t)m * 5 + (size_t)vwidth(M)));
    if (!buf) return ORC_ENOMEM;
    posterior_grad_point(M, x, mean, var, dmean, dvar, buf, buf + m, buf + 5 * (size_t)m, buf + 4 * (size_t)m);
    free(buf);
    return ORC_OK;
}

/* ------------------------------------------------------------ cell LCP -- */

/* Semidefinite Cholesky S = C C^T (n x n, row-major, C lower).  A column whose pivot
 * is not above tau * max_q S_qq is set to zero.  Returns the number of kept columns. */
int orc_chol_sd(int n, const double* S, double* C, double tau)
{
    double mx = 0.0;
    for (int q = 0; q < n; ++q) if (S[q * n + q] > mx) mx = S[q * n + q];
    memset(C, 0, sizeof(double) * (size_t)n * n);
    int rank = 0;
    for (int k = 0; k < n; ++k) {
        double d = S[k * n + k];
        for (int j = 0; j < k; ++j) d -= C[k * n + j] * C[k * n + j];
        if (!(mx > 0.0) || d <= tau * mx) continue;
        double ckk = sqrt(d);
        C[k * n + k] = ckk;
        for (int i = k + 1; i < n; ++i) {
            double s = S[i * n + k];
            for (int j = 0; j < k; ++j) s -= C[i * n + j] * C[k * n + j];
            C[i * n + k] = s / ckk;
        }
        ++rank;
    }
    return rank;
}

/* Monte Carlo count of crossed samples (Sec. 4, cell LCP): y = mu + C z_s; a sample is
 * crossed unless all corners are below theta or all are above theta. */
int64_t orc_mc_count(int n, const double* mu, const double* C, double theta, int ns, const double* zb)
{
    int64_t cnt = 0;
    for (int s = 0; s < ns; ++s) {
        int below = 1, above = 1;
        for (int q = 0; q < n; ++q) {
            double yq = mu[q];
            for (int r = 0; r <= q; ++r) yq += C[q * n + r] * zb[(int64_t)s * n + r];
            if (!(yq < theta)) below = 0;
            if (!(yq > theta)) above = 0;
        }
        if (!below && !above) ++cnt;
    }
    return cnt;
}

/* ------------------------------------------- smooth cell LCP and its adjoint -- */

/*
 * The Monte Carlo estimate of Sec. 4 counts crossings, so it is piecewise constant in the
 * cell's mean and covariance.  For differentiation the same probability,
 * LCP = 1 - P(all Y_q < theta) - P(all Y_q > theta), is estimated by Genz's separation of
 * variables (Genz 1992): with the factor C of the corner covariance and uniforms
 * w_i = Phi(z_i) from the first n - 1 normals of each z-bank row, each orthant probability
 * is a product of conditional probabilities, smooth in the mean and in C.
 */
static double norm_cdf(double t) { return 0.5 * erfc(-t / sqrt(2.0)); }
static double norm_pdf(double t) { return exp(-0.5 * t * t) * 0.39894228040143267794; }

/* Phi^-1 by Newton's method on Phi from the rational start of Abramowitz-Stegun 26.2.23. */
static double norm_inv(double u)
{
    if (u < 1e-300) u = 1e-300;
    if (u > 1.0 - 1e-16) u = 1.0 - 1e-16;
    double q = u < 0.5 ? u : 1.0 - u;
    double t = sqrt(-2.0 * log(q));
    double x = t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                   (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t);
    if (u < 0.5) x = -x;
    for (int it = 0; it < 6; ++it) {
        double f = norm_pdf(x);
        if (!(f > 0.0)) break;
        x -= (norm_cdf(x) - u) / f;
    }
    return x;
}

/* One sample of one orthant: upper = 0 estimates P(all Y < theta), 1 P(all Y > theta).
 * Y = mu + C y with y standard normal; factor i is the probability of the orthant for
 * Y_i given y_0 .. y_{i-1}, and y_i is drawn inside it by inversion of w_i.  Zero pivots
 * (C_ii = 0) make factor i a step.  t, e, y receive the per-step values (for the adjoint). */
static double sov_sample(int n, const double* mu, const double* C, double theta, int upper, const double* w,
                         double* t, double* e, double* y)
{
    double f = 1.0;
    for (int i = 0; i < n; ++i) {
        double si = 0.0;
        for (int j = 0; j < i; ++j) si += C[i * n + j] * y[j];
        double r = theta - mu[i] - si;
        double cii = C[i * n + i];
        if (cii > 0.0) {
            t[i] = r / cii;
            e[i] = upper ? norm_cdf(-t[i]) : norm_cdf(t[i]);
        } else {
            t[i] = 0.0;
            e[i] = upper ? (r < 0.0 ? 1.0 : 0.0) : (r > 0.0 ? 1.0 : 0.0);
        }
        f *= e[i];
        y[i] = 0.0;
        if (i < n - 1 && cii > 0.0) {
            double u = upper ? 1.0 - e[i] + w[i] * e[i] : w[i] * e[i];
            y[i] = norm_inv(u);
        }
    }
    return f;
}

/* Smooth LCP of one cell (n corners, factor C) over ns samples of the z-bank. */
double orc_sov_lcp(int n, const double* mu, const double* C, double theta, int ns, const double* zb)
{
    double t[8], e[8], y[8], w[8], acc = 0.0;
    for (int s = 0; s < ns; ++s) {
        for (int i = 0; i < n; ++i) w[i] = norm_cdf(zb[(int64_t)s * n + i]);
        acc += sov_sample(n, mu, C, theta, 0, w, t, e, y) + sov_sample(n, mu, C, theta, 1, w, t, e, y);
    }
    return 1.0 - acc / (double)ns;
}

/* Reverse pass of one orthant sample: adds d f / d mu to gmu and d f / d C (lower) to gC,
 * each times scale.  With r_i = theta - mu_i - sum_j C_ij y_j and t_i = r_i / C_ii,
 * e_i = Phi(t_i) (lower orthant) or Phi(-t_i) (upper), y_i = Phi^-1(u_i(e_i)). */
static void sov_sample_rev(int n, const double* C, int upper, const double* w, const double* t, const double* e,
                           const double* y, double scale, double* gmu, double* gC)
{
    double pre[9], suf[9], ybar[8];
    pre[0] = 1.0;
    for (int i = 0; i < n; ++i) pre[i + 1] = pre[i] * e[i];
    suf[n] = 1.0;
    for (int i = n - 1; i >= 0; --i) suf[i] = suf[i + 1] * e[i];
    for (int i = 0; i < n; ++i) ybar[i] = 0.0;
    for (int i = n - 1; i >= 0; --i) {
        double cii = C[i * n + i];
        if (!(cii > 0.0)) continue;                       /* a step: no gradient */
        double ebar = scale * pre[i] * suf[i + 1];        /* d f / d e_i */
        if (i < n - 1) {
            /* y_i = Phi^-1(u), u = w e_i (lower) or 1 - e_i + w e_i (upper) */
            double du = upper ? (w[i] - 1.0) : w[i];
            double py = norm_pdf(y[i]);
            if (py > 0.0) ebar += ybar[i] * du / py;
        }
        double tbar = ebar * norm_pdf(t[i]) * (upper ? -1.0 : 1.0);
        double rbar = tbar / cii;
        gC[i * n + i] += -tbar * t[i] / cii;
        gmu[i] += -rbar;
        for (int j = 0; j < i; ++j) {
            gC[i * n + j] += -rbar * y[j];
            ybar[j] += -rbar * C[i * n + j];
        }
    }
}

/* Smooth cell LCP and its gradient with respect to the mean and the factor C (lower). */
double orc_sov_lcp_grad(int n, const double* mu, const double* C, double theta, int ns, const double* zb,
                        double* gmu, double* gC)
{
    double t[8], e[8], y[8], w[8], acc = 0.0;
    for (int i = 0; i < n; ++i) gmu[i] = 0.0;
    for (int i = 0; i < n * n; ++i) gC[i] = 0.0;
    for (int s = 0; s < ns; ++s) {
        for (int i = 0; i < n; ++i) w[i] = norm_cdf(zb[(int64_t)s * n + i]);
        for (int up = 0; up < 2; ++up) {
            acc += sov_sample(n, mu, C, theta, up, w, t, e, y);
            sov_sample_rev(n, C, up, w, t, e, y, -1.0 / (double)ns, gmu, gC);
        }
    }
    return 1.0 - acc / (double)ns;
}

/* Reverse pass of orc_chol_sd: from dL/dC (lower) to dL/dS for the entries the factor
 * reads (the lower triangle, diagonal included).  Columns the factorisation zeroed are
 * locally constant: they pass no gradient. */
void orc_chol_sd_rev(int n, const double* C, const double* gC_in, double* gS)
{
    double gC[64];
    for (int i = 0; i < n * n; ++i) { gC[i] = gC_in[i]; gS[i] = 0.0; }
    for (int k = n - 1; k >= 0; --k) {
        double ckk = C[k * n + k];
        if (!(ckk > 0.0)) continue;
        /* C_ik = (S_ik - sum_{j<k} C_ij C_kj) / C_kk, i > k (computed after the diagonal) */
        for (int i = n - 1; i > k; --i) {
            double g = gC[i * n + k];
            gS[i * n + k] += g / ckk;
            for (int j = 0; j < k; ++j) {
                gC[i * n + j] -= g * C[k * n + j] / ckk;
                gC[k * n + j] -= g * C[i * n + j] / ckk;
            }
            gC[k * n + k] -= g * C[i * n + k] / ckk;
        }
        /* C_kk = sqrt(S_kk - sum_{j<k} C_kj^2) */
        double g = gC[k * n + k];
        gS[k * n + k] += g / (2.0 * ckk);
        for (int j = 0; j < k; ++j) gC[k * n + j] -= g * C[k * n + j] / ckk;
    }
}

static double vertex_coord(const orc_grid* G, int d, int64_t i)
{
    return G->lo[d] + (double)i * ((G->hi[d] - G->lo[d]) / (double)(G->n[d] - 1));
}

/* Cell covariance of the 2^D corners from per-vertex posterior data. */
static void cell_cov(const orc_model* M, int nc, const double* xc, const double* varc, const double* const* vc,
                     double* S)
{
    int m = M->m, D = M->dim;
    for (int p = 0; p < nc; ++p) {
        S[p * nc + p] = varc[p];
        for (int q = 0; q < p; ++q) {
            double c = orc_kernel(M->kind, D, M->s2, M->ell, xc + p * D, xc + q * D);
            if (M->A) {
                /* eq. (sgp) off the diagonal: - k_p^T K_MM^-1 k_q + k_p^T K_MM^-1 A_M K_MM^-1 k_q */
                double t1 = 0.0, t2 = 0.0;
                for (int j = 0; j < m; ++j) t1 += vc[p][j] * vc[q][m + j];
                for (int j = 0; j < m; ++j) t2 += vc[p][2 * m + j] * vc[q][m + j];
                c = c - t1 + t2;
            } else {
                double dot = 0.0;
                for (int j = 0; j < m; ++j) dot += vc[p][j] * vc[q][j];
                c -= dot;
            }
            S[p * nc + q] = c;
            S[q * nc + p] = c;
        }
    }
}

/* Corner mean vector and covariance of one cell from vertex arrays of a box of vertices
 * (vertex (i,j,k) of the box at offset i + bx*(j + by*k)). */
/* Corner means and covariance of one cell from the posterior of a vertex box. */
static void cell_mu_cov(const orc_model* M, const orc_grid* G, const int64_t* cell, const int64_t* box_lo,
                        const int64_t* box_n, const double* bmean, const double* bvar, const double* bV,
                        double* mu, double* S)
{
    int D = G->dim, nc = 1 << D;
    double var[8], xc[24];
    const double* vc[8];
    for (int q = 0; q < nc; ++q) {
        int64_t idx = 0, stride = 1;
        for (int d = 0; d < D; ++d) {
            int64_t vi = cell[d] + ((q >> d) & 1);
            xc[q * D + d] = vertex_coord(G, d, vi);
            idx += (vi - box_lo[d]) * stride;
            stride *= box_n[d];
        }
        mu[q] = bmean[idx];
        var[q] = bvar[idx];
        vc[q] = bV + idx * vwidth(M);
    }
    cell_cov(M, nc, xc, var, vc, S);
}

static int64_t cell_count(const orc_model* M, const orc_grid* G, double theta, int ns, const double* zb,
                          const int64_t* cell, const int64_t* box_lo, const int64_t* box_n,
                          const double* bmean, const double* bvar, const double* bV)
{
    int D = G->dim, nc = 1 << D;
    double mu[8], var[8], xc[24], S[64], C[64];
    const double* vc[8];
    for (int q = 0; q < nc; ++q) {
        int64_t idx = 0, stride = 1;
        for (int d = 0; d < D; ++d) {
            int64_t vi = cell[d] + ((q >> d) & 1);
            xc[q * D + d] = vertex_coord(G, d, vi);
            idx += (vi - box_lo[d]) * stride;
            stride *= box_n[d];
        }
        mu[q] = bmean[idx];
        var[q] = bvar[idx];
        vc[q] = bV + idx * vwidth(M);
    }
    cell_cov(M, nc, xc, var, vc, S);
    orc_chol_sd(nc, S, C, 1e-12);
    return orc_mc_count(nc, mu, C, theta, ns, zb);
}

/* Posterior at every vertex of a box [box_lo, box_lo + box_n) of grid vertices. */
static int box_posterior(const orc_model* M, const orc_grid* G, const int64_t* box_lo, const int64_t* box_n,
                         double** mean, double** var, double** V, int64_t* nv_out)
{
    int D = G->dim;
    int64_t nv = 1;
    for (int d = 0; d < D; ++d) nv *= box_n[d];
    double* P = (double*)malloc(sizeof(double) * (size_t)nv * D);
    *mean = (double*)malloc(sizeof(double) * (size_t)nv);
    *var = (double*)malloc(sizeof(double) * (size_t)nv);
    *V = (double*)malloc(sizeof(double) * (size_t)nv * vwidth(M));
    if (!P || !*mean || !*var || !*V) { free(P); return ORC_ENOMEM; }
    for (int64_t t = 0; t < nv; ++t) {
        int64_t r = t;
        for (int d = 0; d < D; ++d) {
            P[t * D + d] = vertex_coord(G, d, box_lo[d] + r % box_n[d]);
            r /= box_n[d];
        }
    }
    int rc = orc_posterior(M, nv, P, *mean, *var, *V);
    free(P);
    *nv_out = nv;
    return rc;
}

/* Per-vertex posterior mean and variance for the whole grid (x fastest). */
int orc_grid_posterior(const orc_model* M, const orc_grid* G, double* mean, double* var)
{
    int D = G->dim;
    int64_t nv = 1;
    for (int d = 0; d < D; ++d) nv *= G->n[d];
    double* P = (double*)malloc(sizeof(double) * (size_t)nv * D);
    if (!P) return ORC_ENOMEM;
    for (int64_t t = 0; t < nv; ++t) {
        int64_t r = t;
        for (int d = 0; d < D; ++d) { P[t * D + d] = vertex_coord(G, d, r % G->n[d]); r /= G->n[d]; }
    }
    int rc = orc_posterior(M, nv, P, mean, var, NULL);
    free(P);
    return rc;
}

/* Dense LCP (Sec. 4 baseline) for the cells whose slowest-axis index lies in [c0, c1).
 * lcp receives those cells in x-fastest order. */
int orc_lcp_cells(const orc_model* M, const orc_grid* G, double theta, int ns, const double* zb,
                  int64_t c0, int64_t c1, double* lcp)
{
    int D = G->dim, sa = D - 1;
    int64_t box_lo[3] = {0, 0, 0}, box_n[3] = {1, 1, 1};
    for (int d = 0; d < D; ++d) { box_lo[d] = 0; box_n[d] = G->n[d]; }
    box_lo[sa] = c0;
    box_n[sa] = c1 - c0 + 1;
    double *mean = NULL, *var = NULL, *V = NULL;
    int64_t nv;
    int rc = box_posterior(M, G, box_lo, box_n, &mean, &var, &V, &nv);
    if (rc == ORC_OK) {
        int64_t ncell = 1;
        int64_t cn[3] = {1, 1, 1};
        for (int d = 0; d < D; ++d) { cn[d] = G->n[d] - 1; }
        cn[sa] = c1 - c0;
        for (int d = 0; d < D; ++d) ncell *= cn[d];
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t t = 0; t < ncell; ++t) {
            int64_t cell[3], r = t;
            for (int d = 0; d < D; ++d) { cell[d] = r % cn[d]; r /= cn[d]; }
            cell[sa] += c0;
            int64_t cnt = cell_count(M, G, theta, ns, zb, cell, box_lo, box_n, mean, var, V);
            lcp[t] = (double)cnt / (double)ns;
        }
    }
    free(mean);
    free(var);
    free(V);
    return rc;
}

/* Smooth (separation-of-variables) LCP of every cell, x fastest. */
int orc_lcp_sov_cells(const orc_model* M, const orc_grid* G, double theta, int ns, const double* zb, double* lcp)
{
    int D = G->dim, nc = 1 << D;
    int64_t box_lo[3] = {0, 0, 0}, box_n[3] = {1, 1, 1}, cn[3] = {1, 1, 1}, ncell = 1;
    for (int d = 0; d < D; ++d) { box_n[d] = G->n[d]; cn[d] = G->n[d] - 1; ncell *= cn[d]; }
    double *mean = NULL, *var = NULL, *V = NULL;
    int64_t nv;
    int rc = box_posterior(M, G, box_lo, box_n, &mean, &var, &V, &nv);
    if (rc == ORC_OK) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < ncell; ++t) {
            int64_t cell[3] = {0, 0, 0}, r = t;
            for (int d = 0; d < D; ++d) { cell[d] = r % cn[d]; r /= cn[d]; }
            double mu[8], S[64], C[64];
            cell_mu_cov(M, G, cell, box_lo, box_n, mean, var, V, mu, S);
            orc_chol_sd(nc, S, C, 1e-12);
            lcp[t] = orc_sov_lcp(nc, mu, C, theta, ns, zb);
        }
    }
    free(mean);
    free(var);
    free(V);
    return rc;
}

/*
 * Adjoint of the smooth LCP field with respect to the observation values and the
 * log-lengthscales, for upstream gradients gl (one per cell).  Cell by cell: the cell's
 * gradient with respect to its corner means and covariance (factor adjoint included),
 * then through eq. (sgp) corner by corner with w_q = K^-1 k_q:
 *   dmu_q / dy = w_q,   dmu_q / dlog(ell_d) = dk_q . a - w_q^T dK a,
 *   dS_qr / dlog(ell_d) = dk(x_q, x_r) - dk_q . w_r - dk_r . w_q + w_q^T dK w_r.
 * Exact GP only.
 */
int orc_lcp_backward(const orc_model* M, const orc_grid* G, double theta, int ns, const double* zb,
                     const double* gl, double* dy, double* dlogell)
{
    if (M->A) return ORC_EINVAL;
    int D = G->dim, nc = 1 << D, m = M->m;
    int64_t box_lo[3] = {0, 0, 0}, box_n[3] = {1, 1, 1}, cn[3] = {1, 1, 1}, ncell = 1;
    for (int d = 0; d < D; ++d) { box_n[d] = G->n[d]; cn[d] = G->n[d] - 1; ncell *= cn[d]; }
    double *mean = NULL, *var = NULL, *V = NULL;
    int64_t nv;
    int rc = box_posterior(M, G, box_lo, box_n, &mean, &var, &V, &nv);
    double* dK = (double*)malloc(sizeof(double) * (size_t)D * m * m);
    double* dKa = (double*)malloc(sizeof(double) * (size_t)D * m);
    double* w = (double*)malloc(sizeof(double) * (size_t)nc * m);
    double* dk = (double*)malloc(sizeof(double) * (size_t)nc * D * m);
    double* tmp = (double*)malloc(sizeof(double) * (size_t)m);
    double* kq = (double*)malloc(sizeof(double) * (size_t)m);
    if (rc != ORC_OK || !dK || !dKa || !w || !dk || !tmp || !kq) {
        free(mean); free(var); free(V); free(dK); free(dKa); free(w); free(dk); free(tmp); free(kq);
        return rc != ORC_OK ? rc : ORC_ENOMEM;
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            double g[3];
            orc_kernel_dlogell(M->kind, D, M->s2, M->ell, M->X + (int64_t)i * D, M->X + (int64_t)j * D, g);
            for (int d = 0; d < D; ++d) dK[((int64_t)d * m + i) * m + j] = g[d];
        }
    for (int d = 0; d < D; ++d)
        for (int i = 0; i < m; ++i) {
            double sum = 0.0;
            for (int j = 0; j < m; ++j) sum += dK[((int64_t)d * m + i) * m + j] * M->a[j];
            dKa[(int64_t)d * m + i] = sum;
        }
    for (int j = 0; j < m; ++j) dy[j] = 0.0;
    for (int d = 0; d < D; ++d) dlogell[d] = 0.0;
    for (int64_t t = 0; t < ncell; ++t) {
        if (gl[t] == 0.0) continue;
        int64_t cell[3] = {0, 0, 0}, r = t;
        for (int d = 0; d < D; ++d) { cell[d] = r % cn[d]; r /= cn[d]; }
        double mu[8], S[64], C[64], gmu[8], gC[64], gS[64], xc[24];
        cell_mu_cov(M, G, cell, box_lo, box_n, mean, var, V, mu, S);
        orc_chol_sd(nc, S, C, 1e-12);
        orc_sov_lcp_grad(nc, mu, C, theta, ns, zb, gmu, gC);
        orc_chol_sd_rev(nc, C, gC, gS);
        for (int q = 0; q < nc; ++q) {
            for (int d = 0; d < D; ++d) xc[q * D + d] = vertex_coord(G, d, cell[d] + ((q >> d) & 1));
            for (int j = 0; j < m; ++j) {
                double g[3];
                kq[j] = orc_kernel(M->kind, D, M->s2, M->ell, xc + q * D, M->X + (int64_t)j * D);
                orc_kernel_dlogell(M->kind, D, M->s2, M->ell, xc + q * D, M->X + (int64_t)j * D, g);
                for (int d = 0; d < D; ++d) dk[((int64_t)q * D + d) * m + j] = g[d];
            }
            forward_sub(m, M->L, kq, tmp);
            backward_sub_t(m, M->L, tmp, w + (int64_t)q * m);
        }
        const double up = gl[t];
        for (int q = 0; q < nc; ++q) {
            const double* wq = w + (int64_t)q * m;
            for (int j = 0; j < m; ++j) dy[j] += up * gmu[q] * wq[j];
            for (int d = 0; d < D; ++d) {
                const double* dkq = dk + ((int64_t)q * D + d) * m;
                double dka = 0.0, wdKa = 0.0;
                for (int j = 0; j < m; ++j) dka += dkq[j] * M->a[j];
                for (int j = 0; j < m; ++j) wdKa += wq[j] * dKa[(int64_t)d * m + j];
                dlogell[d] += up * gmu[q] * (dka - wdKa);
            }
            for (int rr = 0; rr <= q; ++rr) {
                double gs = gS[q * nc + rr];
                if (gs == 0.0) continue;
                const double* wr = w + (int64_t)rr * m;
                double g2[3];
                orc_kernel_dlogell(M->kind, D, M->s2, M->ell, xc + q * D, xc + rr * D, g2);
                for (int d = 0; d < D; ++d) {
                    const double* dkq = dk + ((int64_t)q * D + d) * m;
                    const double* dkr = dk + ((int64_t)rr * D + d) * m;
                    const double* dKd = dK + (int64_t)d * m * m;
                    double a1 = 0.0, a2 = 0.0, quad = 0.0;
                    for (int j = 0; j < m; ++j) a1 += dkq[j] * wr[j];
                    for (int j = 0; j < m; ++j) a2 += dkr[j] * wq[j];
                    for (int i = 0; i < m; ++i) {
                        double sum = 0.0;
                        for (int j = 0; j < m; ++j) sum += dKd[(int64_t)i * m + j] * wr[j];
                        quad += wq[i] * sum;
                    }
                    dlogell[d] += up * gs * (g2[d] - a1 - a2 + quad);
                }
            }
        }
    }
    free(mean); free(var); free(V); free(dK); free(dKa); free(w); free(dk); free(tmp); free(kq);
    return ORC_OK;
}

/* Corner mean and covariance of one cell (exposed for the tests). */
int orc_cell_moments(const orc_model* M, const orc_grid* G, const int64_t* cell, double* mu, double* S)
{
    int D = G->dim, nc = 1 << D;
    int64_t box_lo[3] = {0, 0, 0}, box_n[3] = {1, 1, 1};
    for (int d = 0; d < D; ++d) { box_lo[d] = cell[d]; box_n[d] = 2; }
    double *mean = NULL, *var = NULL, *V = NULL;
    int64_t nv;
    int rc = box_posterior(M, G, box_lo, box_n, &mean, &var, &V, &nv);
    if (rc == ORC_OK) {
        double xc[24], vr[8];
        const double* vc[8];
        for (int q = 0; q < nc; ++q) {
            for (int d = 0; d < D; ++d) xc[q * D + d] = vertex_coord(G, d, cell[d] + ((q >> d) & 1));
            mu[q] = mean[q];
            vr[q] = var[q];
            vc[q] = V + (int64_t)q * vwidth(M);
        }
        cell_cov(M, nc, xc, vr, vc, S);
    }
    free(mean);
    free(var);
    free(V);
    return rc;
}

/* ------------------------------------------------------- region bound -- */

/* Standardised margin g = side (theta - mu) / sigma; its minimum over a region gives
 * B = Phi(g_min) = min F_M (side +1) or min (1 - F_M) (side -1), Sec. 5.1. */
static double margin(double side, double theta, double mu, double var)
{
    double num = side * (theta - mu);
    if (var > 0.0) return num / sqrt(var);
    if (num > 0.0) return INFINITY;
    if (num < 0.0) return -INFINITY;
    return 0.0;
}

typedef struct {
    const orc_model* M;
    double theta;
    double* kb;
    double* dkb;
    double* v;
    double* w;
} bound_ws;

static double margin_at(bound_ws* B, double side, const double* x)
{
    double mu, var;
    posterior_point(B->M, x, &mu, &var, B->kb, B->v);
    return margin(side, B->theta, mu, var);
}

/* Margin and its gradient; returns 0 if the gradient is not usable (sigma = 0). */
static int margin_grad_at(bound_ws* B, double side, const double* x, double* g, double* grad)
{
    int D = B->M->dim;
    double mu, var, dmu[3], dvar[3];
    posterior_grad_point(B->M, x, &mu, &var, dmu, dvar, B->kb, B->dkb, B->v, B->w);
    *g = margin(side, B->theta, mu, var);
    if (!(var > 0.0)) return 0;
    double sd = sqrt(var);
    for (int d = 0; d < D; ++d) {
        double dsd = dvar[d] / (2.0 * sd);
        grad[d] = side * (-dmu[d] * sd - (B->theta - mu) * dsd) / var;
    }
    return 1;
}

/* Fixed-budget search for the minimum of g over the box [blo, bhi]: the 3^D lattice
 * {lo, mid, hi}^D (lowest index wins ties), then `steps` projected steps of length
 * 2^-(k+1) of the box width along the normalised, box-scaled negative gradient. */
static double bound_search(bound_ws* B, double side, const double* blo, const double* bhi, int steps,
                           double* gap_out)
{
    int D = B->M->dim;
    int npt = 1;
    for (int d = 0; d < D; ++d) npt *= 3;
    double best = INFINITY, second = INFINITY, xbest[3];
    for (int i = 0; i < npt; ++i) {
        double x[3];
        int r = i;
        for (int d = 0; d < D; ++d) {
            int digit = r % 3;
            r /= 3;
            x[d] = digit == 0 ? blo[d] : (digit == 1 ? 0.5 * (blo[d] + bhi[d]) : bhi[d]);
        }
        double g = margin_at(B, side, x);
        if (g < best) {
            second = best;
            best = g;
            memcpy(xbest, x, sizeof(double) * D);
        } else if (g < second) {
            second = g;
        }
    }
    if (gap_out) *gap_out = second - best;
    double gmin = best, x[3], w[3];
    memcpy(x, xbest, sizeof(double) * D);
    for (int d = 0; d < D; ++d) w[d] = bhi[d] - blo[d];
    double eta = 0.5;
    for (int k = 0; k < steps; ++k, eta *= 0.5) {
        double g, grad[3];
        if (!margin_grad_at(B, side, x, &g, grad)) break;
        double u[3], nrm = 0.0;
        for (int d = 0; d < D; ++d) { u[d] = w[d] * grad[d]; nrm += u[d] * u[d]; }
        nrm = sqrt(nrm);
        if (!(nrm > 0.0) || !isfinite(nrm)) break;
        for (int d = 0; d < D; ++d) {
            double xn = x[d] - eta * w[d] * u[d] / nrm;
            x[d] = xn < blo[d] ? blo[d] : (xn > bhi[d] ? bhi[d] : xn);
        }
        double gn = margin_at(B, side, x);
        if (gn < gmin) gmin = gn;
    }
    return gmin;
}

/* Upper bound 1 - B^d of eq. (upper_bound) for one side, with B = Phi(g_min), computed as
 * -expm1(d log1p(-t)) with the tail t = erfc(g_min / sqrt2) / 2. */
double orc_upper_bound(double gmin, int64_t d)
{
    double t;
    if (gmin == INFINITY) t = 0.0;
    else if (gmin == -INFINITY) t = 1.0;
    else t = 0.5 * erfc(gmin / sqrt(2.0));
    if (t >= 1.0) return 1.0;
    return -expm1((double)d * log1p(-t));
}

int orc_bound(const orc_model* M, double theta, double side, const double* blo, const double* bhi, int steps,
              double* gmin, double* gap)
{
    int m = M->m;
    double* buf = (double*)malloc(sizeof(double) * ((size_t)m * 5 + (size_t)vwidth(M) + 1));
    if (!buf) return ORC_ENOMEM;
    bound_ws B = {M, theta, buf, buf + m, buf + 5 * (size_t)m, buf + 4 * (size_t)m};
    *gmin = bound_search(&B, side, blo, bhi, steps, gap);
    free(buf);
    return ORC_OK;
}

/* ---------------------------------------------------- local model (Sec. 5.2) -- */
/*
 * The region test of a node may use a local model M' instead of M: the points of M inside
 * the node box enlarged by beta lengthscales along every axis (Alg. 1 passes each child the
 * points of its parent's set inside the child box enlarged by the distance threshold; the
 * enlarged child box lies inside the enlarged parent box, so that is M intersected with the
 * child's enlarged box; the root keeps all of M).  The threshold is a distance; with a
 * lengthscale per axis it is beta ell_d along axis d (Sec. 7.3 measures it in units of ell).
 *  - exact GP: the GP with the same hyperparameters conditioned on the local observations
 *    alone, L' = chol(K_M'M' + noise I), a' = (K_M'M' + noise I)^-1 y_M';
 *  - sparse model: eq. (sgp) with mu_M and A_M restricted to M' (the marginal of the
 *    inducing values), K_M'M' + jitter I.
 * Points keep their order in M.  With every point selected the local model is M itself,
 * bit for bit.
 */
typedef struct {
    orc_model M;
    double *X, *L, *a, *rhs, *A;
} orc_local;

static void local_free(orc_local* P)
{
    free(P->X); free(P->L); free(P->a); free(P->rhs); free(P->A);
    memset(P, 0, sizeof *P);
}

static int local_build(const orc_model* M, const double* blo, const double* bhi, double beta, int whole,
                       orc_local* P)
{
    int D = M->dim, m = M->m;
    memset(P, 0, sizeof *P);
    int* idx = (int*)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    if (!idx) return ORC_ENOMEM;
    int n = 0;
    for (int i = 0; i < m; ++i) {
        int in = 1;
        for (int d = 0; d < D && !whole; ++d) {
            double xi = M->X[(int64_t)i * D + d];
            double r = beta * M->ell[d];
            if (!(xi >= blo[d] - r && xi <= bhi[d] + r)) in = 0;
        }
        if (in) idx[n++] = i;
    }
    const double* src = M->A ? M->muM : M->y;
    size_t nn = (size_t)(n > 0 ? n : 1);
    P->X = (double*)malloc(sizeof(double) * nn * D);
    P->L = (double*)malloc(sizeof(double) * nn * nn);
    P->a = (double*)malloc(sizeof(double) * nn);
    P->rhs = (double*)malloc(sizeof(double) * nn);
    if (M->A) P->A = (double*)malloc(sizeof(double) * nn * nn);
    if (!src || !P->X || !P->L || !P->a || !P->rhs || (M->A && !P->A)) {
        free(idx);
        local_free(P);
        return src ? ORC_ENOMEM : ORC_ENOTPD;
    }
    for (int j = 0; j < n; ++j) {
        for (int d = 0; d < D; ++d) P->X[(int64_t)j * D + d] = M->X[(int64_t)idx[j] * D + d];
        P->rhs[j] = src[idx[j]];
        if (M->A)
            for (int k = 0; k < n; ++k) P->A[(int64_t)j * n + k] = M->A[(int64_t)idx[j] * m + idx[k]];
    }
    free(idx);
    int rc = n > 0 ? orc_fit(M->kind, D, M->s2, M->ell, M->noise, n, P->X, P->rhs, P->L, P->a) : ORC_OK;
    if (rc != ORC_OK) { local_free(P); return rc; }
    P->M = *M;
    P->M.m = n;
    P->M.X = P->X;
    P->M.L = P->L;
    P->M.a = P->a;
    P->M.A = P->A;
    P->M.muM = M->A ? P->rhs : NULL;
    P->M.y = M->A ? NULL : P->rhs;
    return ORC_OK;
}

/* Posterior of the local model of the box [blo, bhi] at n points; returns |M'| (or a
 * negative status). */
int64_t orc_local_posterior(const orc_model* M, const double* blo, const double* bhi, double beta, int whole,
                            int64_t n, const double* P, double* mean, double* var)
{
    orc_local LM;
    int rc = local_build(M, blo, bhi, beta, whole, &LM);
    if (rc != ORC_OK) return -rc;
    rc = orc_posterior(&LM.M, n, P, mean, var, NULL);
    int64_t ml = LM.M.m;
    local_free(&LM);
    return rc == ORC_OK ? ml : -rc;
}

/* ------------------------------------------ certified region bound -- */
/*
 * Box bounds of the posterior that hold for every point of the box, so that the bound of
 * eq. (upper_bound) is guaranteed rather than found by a search (the search of Sec. 5.1 can
 * miss the minimum; Sec. 9 leaves a guaranteed bound as future work).  They hold in exact
 * arithmetic for the stored model; the binary64 rounding of the sums below is not bounded.
 *
 * Second-order Taylor model with the Lagrange remainder.  For the box with centre c and
 * half-widths h, u = x - c, v = u / ell (scaled), |v|^2 <= H = sum_d (h_d / ell_d)^2, and r_i
 * the scaled distance from x_i to the box: for any weights b, the function
 * phi(x) = sum_i b_i k_i(x) satisfies
 *   phi(x) = phi(c) + grad.u + u^T Hess u / 2 + R,  |R| <= s2 H^(3/2) sum_i |b_i| C3(r_i) / 6,
 * where s2 C3(r) bounds the third directional derivative of k along a unit scaled direction
 * at every scaled distance >= r (curv3_env); gradient and Hessian are taken at c, where
 * the cancellations of the weights are exact.  Over the box the quadratic part lies within
 * sum_d [min, max of grad_d u_d + Hess_dd u_d^2 / 2] -/+ sum_{d != e} |Hess_de| h_d h_e / 2.
 *  - mean: phi = mu (b = a).
 *  - variance: var(x) = s2 - q(k(x)) with q(k) = k^T Q k, Q = K^-1 (exact GP) or
 *    K^-1 - K^-1 A_M K^-1 (sparse model; positive semidefinite when A_M <= K).  q is convex,
 *    so with w = Q k(c):  q(k(x)) >= q(k(c)) + 2 w^T (k(x) - k(c)).  With nu(x) = w^T k(x)
 *    (b = w) and q(k(c)) = nu(c):  var(x) <= s2 - nu(c) - 2 min_box (nu(x) - nu(c)),
 *    clamped to [0, s2].
 */

/* Hessian of k(x, z) in x (dim x dim, row-major).  With t = (x - z) / ell, r = |t| and
 * k = s2 f(r):  d2k / dx_d dx_e = s2 (g delta_de + gam t_d t_e) / (ell_d ell_e), where g = f'/r
 * and gam = (f'/r)' / r:  SE: g = -e^(-r^2/2), gam = e^(-r^2/2);  Matern-5/2:
 * g = -(5/3) (1 + sqrt5 r) e^(-sqrt5 r), gam = (25/3) e^(-sqrt5 r). */
void orc_kernel_hess(int kind, int dim, double s2, const double* ell, const double* x, const double* z,
                     double* Hm)
{
    double t[3], r2 = scaled_r2(dim, ell, x, z), g, gam;
    for (int d = 0; d < dim; ++d) t[d] = (x[d] - z[d]) / ell[d];
    if (kind == 0) {
        double e = exp(-0.5 * r2);
        g = -e;
        gam = e;
    } else {
        double r = sqrt(r2), e = exp(-sqrt(5.0) * r);
        g = -(5.0 / 3.0) * (1.0 + sqrt(5.0) * r) * e;
        gam = (25.0 / 3.0) * e;
    }
    for (int d = 0; d < dim; ++d)
        for (int f = 0; f < dim; ++f)
            Hm[d * dim + f] = s2 * ((d == f ? g : 0.0) + gam * t[d] * t[f]) / (ell[d] * ell[f]);
}

/* kappa3(rho) = max over unit v of |D^3 f[v, v, v]| at scaled distance rho (s2 = 1).  With
 * p = v . t / rho in [-1, 1]:  D^3 f = 3 g' p + rho^2 (g'/rho)' p^3 (g = f'/rho).
 * SE: e^(-rho^2/2) (3 s - s^3), s = rho p: the maximum of |3 s - s^3| over |s| <= rho is
 *   3 rho - rho^3 (rho <= 1), 2 (rho <= 2), rho^3 - 3 rho.
 * Matern-5/2, t = sqrt5 rho: (5 sqrt5 / 3) e^-t (3 t p - t^2 p^3), whose maximum over p is
 *   3 t - t^2 (t <= 1), 2 sqrt t (t <= 4), t^2 - 3 t. */
static double kappa3(int kind, double rho)
{
    if (kind == 0) {
        double e = exp(-0.5 * rho * rho);
        if (rho <= 1.0) return e * (3.0 * rho - rho * rho * rho);
        if (rho <= 2.0) return 2.0 * e;
        return e * (rho * rho * rho - 3.0 * rho);
    }
    double t = sqrt(5.0) * rho, c = (5.0 * sqrt(5.0) / 3.0) * exp(-t);
    if (t <= 1.0) return c * (3.0 * t - t * t);
    if (t <= 4.0) return c * 2.0 * sqrt(t);
    return c * (t * t - 3.0 * t);
}

/* C3(r) = sup over rho >= r of kappa3(rho).  kappa3 rises to a peak, falls, rises to a
 * second, lower peak and then falls for good:
 *   SE: peaks at rho^2 = 3 - sqrt6 and 3 + sqrt6 (stationary points of e^(-rho^2/2)(3rho - rho^3)
 *       and of e^(-rho^2/2)(rho^3 - 3rho)); the middle piece 2 e^(-rho^2/2) falls.
 *   Matern-5/2: peaks at t = (5 -/+ sqrt13) / 2 (stationary points of e^-t (3t - t^2) and of
 *       e^-t (t^2 - 3t)); the middle piece 2 sqrt t e^-t falls for t > 1/2. */
static double curv3_env(int kind, double r2)
{
    double rho = sqrt(r2);
    double p1, p2, q1, q2;   /* peak positions (in rho) and values */
    if (kind == 0) {
        p1 = sqrt(3.0 - sqrt(6.0));
        p2 = sqrt(3.0 + sqrt(6.0));
    } else {
        p1 = (5.0 - sqrt(13.0)) / 2.0 / sqrt(5.0);
        p2 = (5.0 + sqrt(13.0)) / 2.0 / sqrt(5.0);
    }
    q1 = kappa3(kind, p1);
    q2 = kappa3(kind, p2);
    if (rho <= p1) return q1;
    if (rho >= p2) return kappa3(kind, rho);
    double k = kappa3(kind, rho);
    return k > q2 ? k : q2;
}

double orc_curv3_env(int kind, double r2) { return curv3_env(kind, r2); }

/* Range [lo, hi] over |u| <= h of g u + q u^2 / 2 (ends, and the vertex when inside). */
static void quad_range(double g, double q, double h, double* lo, double* hi)
{
    double a = -g * h + 0.5 * q * h * h, b = g * h + 0.5 * q * h * h;
    *lo = a < b ? a : b;
    *hi = a > b ? a : b;
    if (q != 0.0 && fabs(g) <= fabs(q) * h) {
        double v = -0.5 * g * g / q;
        if (v < *lo) *lo = v;
        if (v > *hi) *hi = v;
    }
}

/* Range of the second-order model of phi over the box, relative to phi(c). */
static void model_range(int D, const double* g, const double* Hm, const double* h, double R, double* lo,
                        double* hi)
{
    double l = -R, u = R;
    for (int d = 0; d < D; ++d) {
        double a, b;
        quad_range(g[d], Hm[d * D + d], h[d], &a, &b);
        l += a;
        u += b;
        for (int e = 0; e < D; ++e) {
            if (e == d) continue;
            double x = 0.5 * fabs(Hm[d * D + e]) * h[d] * h[e];
            l -= x;
            u += x;
        }
    }
    *lo = l;
    *hi = u;
}

/* out[0] = mu(c), out[1] = lower bound of mu, out[2] = upper bound of mu, out[3] = upper
 * bound of var over the closed box [blo, bhi]. */
int orc_bound_certified(const orc_model* M, const double* blo, const double* bhi, double* out)
{
    const int m = M->m, D = M->dim;
    double* buf = (double*)malloc(sizeof(double) * 5 * (size_t)m);
    if (!buf) return ORC_ENOMEM;
    double *k = buf, *t = buf + m, *w = buf + 2 * m, *u = buf + 3 * m, *v = buf + 4 * m;
    double c[3], h[3], H = 0.0;
    for (int d = 0; d < D; ++d) {
        c[d] = 0.5 * (blo[d] + bhi[d]);
        h[d] = 0.5 * (bhi[d] - blo[d]);
        H += (h[d] / M->ell[d]) * (h[d] / M->ell[d]);
    }
    for (int i = 0; i < m; ++i) k[i] = orc_kernel(M->kind, D, M->s2, M->ell, c, M->X + (int64_t)i * D);
    /* w = Q k(c) */
    forward_sub(m, M->L, k, t);
    backward_sub_t(m, M->L, t, M->A ? u : w);
    if (M->A) {
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += M->A[(int64_t)i * m + j] * u[j];
            v[i] = s;
        }
        forward_sub(m, M->L, v, t);
        backward_sub_t(m, M->L, t, v);
        for (int i = 0; i < m; ++i) w[i] = u[i] - v[i];
    }
    double mu = 0.0, nu = 0.0, gmu[3] = {0, 0, 0}, gnu[3] = {0, 0, 0}, Ra = 0.0, Rw = 0.0;
    double Hmu[9] = {0}, Hnu[9] = {0};
    for (int i = 0; i < m; ++i) {
        const double* xi = M->X + (int64_t)i * D;
        double g[3], Hk[9], r2 = 0.0;
        orc_kernel_grad(M->kind, D, M->s2, M->ell, c, xi, g);
        orc_kernel_hess(M->kind, D, M->s2, M->ell, c, xi, Hk);
        for (int d = 0; d < D; ++d) {
            double e = blo[d] - xi[d];
            if (xi[d] - bhi[d] > e) e = xi[d] - bhi[d];
            if (e < 0.0) e = 0.0;
            r2 += (e / M->ell[d]) * (e / M->ell[d]);
        }
        double C3 = curv3_env(M->kind, r2);
        mu += M->a[i] * k[i];
        nu += w[i] * k[i];
        for (int d = 0; d < D; ++d) {
            gmu[d] += M->a[i] * g[d];
            gnu[d] += w[i] * g[d];
        }
        for (int q = 0; q < D * D; ++q) {
            Hmu[q] += M->a[i] * Hk[q];
            Hnu[q] += w[i] * Hk[q];
        }
        Ra += fabs(M->a[i]) * C3;
        Rw += fabs(w[i]) * C3;
    }
    const double r3 = M->s2 * H * sqrt(H) / 6.0;
    double mlo, mhi, nlo, nhi;
    model_range(D, gmu, Hmu, h, r3 * Ra, &mlo, &mhi);
    model_range(D, gnu, Hnu, h, r3 * Rw, &nlo, &nhi);
    double vhi = M->s2 - nu - 2.0 * nlo;
    if (vhi > M->s2) vhi = M->s2;
    if (vhi < 0.0) vhi = 0.0;
    out[0] = mu;
    out[1] = mu + mlo;
    out[2] = mu + mhi;
    out[3] = vhi;
    free(buf);
    return ORC_OK;
}

/* Lower bound of the standardised margin side (theta - mu(x)) / sigma(x) over the box from
 * the certified box bounds: num / sigma_hi when num = side (theta - mu) at the box's worst
 * mean is >= 0, else -infinity (no lower bound of sigma is kept). */
double orc_certified_margin(double side, double theta, const double* cb)
{
    double mu = side > 0 ? cb[2] : cb[1];
    double num = side * (theta - mu);
    if (num < 0.0) return -INFINITY;
    return margin(side, theta, mu, cb[3]);
}

/* ---------------------------------------------------- octree (Alg. 1) -- */

/* -------------------------------------------- edge-crossing region bound (Sec. 9) -- */
/*
 * Sec. 9 names a tighter region bound from the crossing probabilities of grid edges as
 * future work.  The event "some cell of a node is crossed" (Sec. 4: not all corner values
 * on one side of theta) equals "the vertex values of the node are not all on one side",
 * which equals "some edge of a spanning tree of the node's vertices joins values on the two
 * sides".  By the union bound, P(node crossed) <= sum over the tree's edges of
 * P(edge crossed), and every cell's LCP is at most P(node crossed).  The edge terms use the
 * joint bivariate posterior of the two end vertices (eq. (sgp)), so strong neighbour
 * correlation keeps them small where the marginal bound of eq. (upper_bound) is not.
 */

/* Integrand of Plackett's identity: with rho = sin t,
 *   P(Za < h, Zb < k) = Phi(h) Phi(k) + (1 / 2pi) int_0^{asin rho} f(t) dt,
 *   f(t) = exp(-(h^2 - 2 h k sin t + k^2) / (2 cos^2 t)),
 * since d/drho P = phi2(h, k; rho) and drho = cos t dt.  The exponent is rewritten as
 * -(h - k)^2 / (2 cos^2 t) - h k / (1 + sin t) (using 1 - sin t = cos^2 t / (1 + sin t)),
 * which stays exact as cos t -> 0 and gives 0 < f <= 1. */
static double plackett_f(double h, double k, double t)
{
    double c = cos(t), s = sin(t);
    double e = -h * k / (1.0 + s);
    if (h != k) e -= (h - k) * (h - k) / (2.0 * c * c);
    return exp(e);
}

/* Adaptive Simpson quadrature (Kuncir 1962; Richardson-corrected on acceptance). */
static double simpson_step(double h, double k, double a, double b, double fa, double fm, double fb, double whole,
                           double tol, int depth)
{
    double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
    double flm = plackett_f(h, k, lm), frm = plackett_f(h, k, rm);
    double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
    double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
    double diff = left + right - whole;
    if (depth <= 0 || !(fabs(diff) > 15.0 * tol)) return left + right + diff / 15.0;
    return simpson_step(h, k, a, m, fa, flm, fm, left, 0.5 * tol, depth - 1) +
           simpson_step(h, k, m, b, fm, frm, fb, right, 0.5 * tol, depth - 1);
}

static double plackett_integral(double h, double k, double t1)
{
    double fa = plackett_f(h, k, 0.0), fb = plackett_f(h, k, t1), fm = plackett_f(h, k, 0.5 * t1);
    double whole = t1 / 6.0 * (fa + 4.0 * fm + fb);
    return simpson_step(h, k, 0.0, t1, fa, fm, fb, whole, 1e-15, 40);
}

static double norm_sf(double t) { return 0.5 * erfc(t / sqrt(2.0)); }

/* P(edge crossed) for the bivariate normal of its end values X, Y (means mua, mub,
 * variances va, vb, covariance c): P(not both < theta and not both > theta), a value equal
 * to theta counting as crossed (Sec. 4's cell rule on two vertices). */
double orc_edge_cross(double mua, double mub, double va, double vb, double c, double theta)
{
    double sa = sqrt(va > 0.0 ? va : 0.0), sb = sqrt(vb > 0.0 ? vb : 0.0);
    if (sa == 0.0 && sb == 0.0) {
        int below = mua < theta && mub < theta, above = mua > theta && mub > theta;
        return (below || above) ? 0.0 : 1.0;
    }
    if (sa == 0.0 || sb == 0.0) {
        /* one end is a constant: crossed unless the random end falls on its side */
        double mc = sa == 0.0 ? mua : mub, mr = sa == 0.0 ? mub : mua, sr = sa == 0.0 ? sb : sa;
        if (mc == theta) return 1.0;
        double hr = (theta - mr) / sr;                 /* P(random end < theta) = Phi(hr) */
        return mc < theta ? norm_sf(hr) : norm_cdf(hr);
    }
    double h = (theta - mua) / sa, k = (theta - mub) / sb;
    double rho = c / (sa * sb);
    if (rho >= 1.0) return fabs(norm_cdf(h) - norm_cdf(k));        /* Y = mub + sb Za */
    if (rho <= -1.0) return 1.0 - fabs(norm_cdf(h) - norm_cdf(-k)); /* Y = mub - sb Za */
    /* A negative correlation is reflected (Zb -> -Zb, k -> -k turns "crossed" into "not
     * crossed"), so the integral below runs over t in [0, pi / 2) only. */
    int reflect = rho < 0.0;
    if (reflect) {
        rho = -rho;
        k = -k;
    }
    /* P = Phi(h) + Phi(k) - 2 P(both < theta)
     *   = Phi(h) Q(k) + Phi(k) Q(h) - (1 / pi) int_0^{asin rho} f */
    double p = norm_cdf(h) * norm_sf(k) + norm_cdf(k) * norm_sf(h) -
               plackett_integral(h, k, asin(rho)) / 3.14159265358979323846;
    if (reflect) p = 1.0 - p;
    return p > 0.0 ? (p < 1.0 ? p : 1.0) : 0.0;
}

/* The edge-crossing union bound of the node whose vertices are [clo, chi] (inclusive) on
 * every axis.  Spanning tree: every x-edge; the y-edges of the first x column of each
 * z-plane; the z-edges of the first (x, y) column.  Summed in that order. */
double orc_node_edge_bound(const orc_model* M, const orc_grid* G, const int64_t* clo, const int64_t* chi,
                           double theta)
{
    int D = G->dim;
    int64_t box_n[3] = {1, 1, 1}, nv;
    for (int d = 0; d < D; ++d) box_n[d] = chi[d] - clo[d] + 1;
    double *mean, *var, *V;
    if (box_posterior(M, G, clo, box_n, &mean, &var, &V, &nv) != ORC_OK) return NAN;
    int64_t nx = box_n[0], ny = box_n[1], nz = D == 3 ? box_n[2] : 1;
    double eb = 0.0;
    for (int pass = 0; pass < 3; ++pass) {
        int64_t ei = pass == 0, ej = pass == 1, ek = pass == 2;
        if (pass == 2 && D < 3) break;
        for (int64_t k = 0; k < nz - ek; ++k)
            for (int64_t j = 0; j < (pass == 2 ? 1 : ny - ej); ++j)
                for (int64_t i = 0; i < (pass == 0 ? nx - 1 : 1); ++i) {
                    int64_t a = i + nx * (j + ny * k), b = (i + ei) + nx * ((j + ej) + ny * (k + ek));
                    double xc[6], vv[2] = {var[a], var[b]}, S[4];
                    const double* vc[2] = {V + a * vwidth(M), V + b * vwidth(M)};
                    int64_t ia[3] = {clo[0] + i, clo[1] + j, clo[2] + k};
                    int64_t ib[3] = {ia[0] + ei, ia[1] + ej, ia[2] + ek};
                    for (int d = 0; d < D; ++d) {
                        xc[d] = vertex_coord(G, d, ia[d]);
                        xc[D + d] = vertex_coord(G, d, ib[d]);
                    }
                    cell_cov(M, 2, xc, vv, vc, S);
                    eb += orc_edge_cross(mean[a], mean[b], S[0], S[3], S[1], theta);
                }
    }
    free(mean);
    free(var);
    free(V);
    return eb;
}

static uint64_t morton(int D, const int64_t* c, int level)
{
    uint64_t key = 0;
    for (int b = 0; b < level; ++b)
        for (int d = 0; d < D; ++d)
            key |= (uint64_t)((c[d] >> b) & 1) << (b * D + d);
    return key;
}

/*
 * K-D tree variant (Sec. 9 proposes splitting the axes in turn instead of all at once).
 * The split at depth L halves axis D - 1 - (L mod D): z, then y, then x in 3D, so after D
 * splits a node is an octree child and, at depth D l, a node is the octree node of level l
 * with the same Morton code.  A node at depth L has had kd_splits(D, L, d) halvings along
 * axis d, and its code lists the split bits in split order (the first split is the most
 * significant bit).
 */
static int kd_axis(int D, int L) { return D - 1 - L % D; }

static int kd_splits(int D, int L, int d) { return L / D + (d >= D - L % D ? 1 : 0); }

static uint64_t kd_code(int D, const int64_t* c, int L)
{
    uint64_t code = 0;
    for (int j = 0; j < L; ++j) {
        int a = kd_axis(D, j);
        int bit = (int)((c[a] >> (kd_splits(D, L, a) - 1 - j / D)) & 1);
        code = (code << 1) | (uint64_t)bit;
    }
    return code;
}

typedef struct {
    const orc_model* M;
    const orc_grid* G;
    const orc_adapt* A;
    double theta;
    const double* qlo;   /* P(Y_i < theta) per observation */
    const double* qhi;   /* P(Y_i > theta) per observation */
    int64_t S0;          /* root edge in cells (power of two) */
    int Lmax;            /* octree levels below the root */
    int kd;              /* K-D tree: depths 0 .. D Lmax */
    int Ldepth;          /* deepest level: Lmax (octree) or D Lmax (K-D tree) */
    int rc;              /* first failure of a local model fit */
    omp_lock_t lock;
    uint64_t* leaves; int64_t leaf_cap; int64_t n_leaves;
    uint64_t* skipped; int64_t skip_cap; int64_t n_skipped;
    orc_node_rec* recs; int64_t rec_cap; int64_t n_recs;
} octree_ctx;

static void push(octree_ctx* T, uint64_t* arr, int64_t cap, int64_t* n, uint64_t key)
{
    omp_set_lock(&T->lock);
    if (*n < cap) arr[*n] = key;
    ++*n;
    omp_unset_lock(&T->lock);
}

static void octree_node(octree_ctx* T, int level, const int64_t* c)
{
    const orc_model* M = T->M;
    const orc_grid* G = T->G;
    int D = G->dim;
    int64_t clo[3], chi[3];
    double blo[3], bhi[3];
    int64_t d_pts = 1;
    for (int d = 0; d < D; ++d) {
        int64_t s = T->S0 >> (T->kd ? kd_splits(D, level, d) : level);
        clo[d] = c[d] * s;
        chi[d] = (c[d] + 1) * s;
        if (chi[d] > G->n[d] - 1) chi[d] = G->n[d] - 1;
        blo[d] = vertex_coord(G, d, clo[d]);
        bhi[d] = vertex_coord(G, d, chi[d]);
        d_pts *= chi[d] - clo[d] + 1;
    }
    orc_node_rec rec;
    memset(&rec, 0, sizeof rec);
    rec.key = ((uint64_t)level << 58) | (T->kd ? kd_code(D, c, level) : morton(D, c, level));
    rec.level = level;
    rec.d = d_pts;
    rec.gmin = NAN;
    rec.ub = NAN;
    rec.lattice_gap = NAN;
    rec.n_local = -1;
    rec.eb = NAN;

    int subdivide = 0;
    if (level == T->Ldepth && !T->A->bound_at_max_depth) {
        rec.path = 3;
        subdivide = 1;
    } else {
        /* M~: observations inside the closed node box; p1, p2 over M~. */
        int nobs = 0;
        double p1 = 0.0, p2 = 0.0;
        for (int i = 0; i < M->m; ++i) {
            int in = 1;
            for (int d = 0; d < D; ++d) {
                double xi = M->X[(int64_t)i * D + d];
                if (!(xi >= blo[d] && xi <= bhi[d])) { in = 0; break; }
            }
            if (!in) continue;
            if (nobs == 0 || T->qlo[i] > p1) p1 = T->qlo[i];
            if (nobs == 0 || T->qhi[i] > p2) p2 = T->qhi[i];
            ++nobs;
        }
        rec.n_obs = nobs;
        rec.p1 = p1;
        rec.p2 = p2;
        double alpha = T->A->alpha;
        if (nobs > 0 && p1 > alpha && p2 > alpha) {
            rec.path = 0;
            subdivide = 1;
        } else {
            /* the region test runs on M, or on the local model M' of Sec. 5.2 */
            orc_local LM;
            const orc_model* Mb = M;
            int local_failed = 0;
            if (T->A->bound_kind == 2) {
                int rc = local_build(M, blo, bhi, T->A->beta, level == 0, &LM);
                if (rc == ORC_ENOTPD) {
                    local_failed = 1;   /* no local model, no bound: the node is refined */
                } else if (rc != ORC_OK) {
                    omp_set_lock(&T->lock);
                    if (!T->rc) T->rc = rc;
                    omp_unset_lock(&T->lock);
                    return;
                } else {
                    Mb = &LM.M;
                    rec.n_local = Mb->m;
                }
            }
            double side;
            if (local_failed) {
                side = (nobs > 0 && p2 <= alpha) ? 1.0 : -1.0;
            } else if (nobs > 0) {
                side = (p2 <= alpha) ? 1.0 : -1.0;
            } else {
                double xc[3], mu, var;
                double* kb = (double*)malloc(sizeof(double) * ((size_t)Mb->m + (size_t)vwidth(Mb) + 1));
                for (int d = 0; d < D; ++d) xc[d] = 0.5 * (blo[d] + bhi[d]);
                posterior_point(Mb, xc, &mu, &var, kb, kb + Mb->m);
                free(kb);
                side = (mu < T->theta) ? 1.0 : -1.0;
            }
            rec.path = side > 0 ? 1 : 2;
            if (local_failed) {
                rec.gmin = -INFINITY;
            } else if (T->A->bound_kind == 1) {
                double cb[4];
                orc_bound_certified(M, blo, bhi, cb);
                rec.gmin = orc_certified_margin(side, T->theta, cb);
            } else {
                double gap;
                orc_bound(Mb, T->theta, side, blo, bhi, T->A->steps, &rec.gmin, &gap);
                rec.lattice_gap = gap;
            }
            if (Mb != M) local_free(&LM);
            rec.ub = orc_upper_bound(rec.gmin, d_pts);
            subdivide = rec.ub > alpha;
        }
    }
    if (subdivide && level == T->Ldepth && T->A->edge_bound) {
        /* the edge-crossing union bound may still show that no cell of the node exceeds alpha */
        int64_t vlo[3] = {clo[0], clo[1], D == 3 ? clo[2] : 0}, vhi[3] = {chi[0], chi[1], D == 3 ? chi[2] : 0};
        rec.eb = orc_node_edge_bound(M, G, vlo, vhi, T->theta);
        subdivide = rec.eb > T->A->alpha;
    }
    rec.subdivide = subdivide;
    omp_set_lock(&T->lock);
    if (T->recs && T->n_recs < T->rec_cap) T->recs[T->n_recs] = rec;
    ++T->n_recs;
    omp_unset_lock(&T->lock);

    if (!subdivide) {
        push(T, T->skipped, T->skip_cap, &T->n_skipped, rec.key);
        return;
    }
    if (level == T->Ldepth) {
        /* leaves keep the octree key (level Lmax); the K-D code at depth D Lmax is the same */
        push(T, T->leaves, T->leaf_cap, &T->n_leaves, ((uint64_t)T->Lmax << 58) | (rec.key & ((1ull << 58) - 1)));
        return;
    }
    if (T->kd) {
        int a = kd_axis(D, level);
        int64_t hs = T->S0 >> kd_splits(D, level + 1, a);
        for (int i = 0; i < 2; ++i) {
            int64_t cc[3] = {c[0], c[1], c[2]};
            cc[a] = 2 * c[a] + i;
            if (cc[a] * hs >= G->n[a] - 1) continue;
#pragma omp task firstprivate(cc) if (level < 12)
            octree_node(T, level + 1, cc);
        }
        return;
    }
    int64_t s = T->S0 >> level;
    int nchild = 1 << D;
    for (int i = 0; i < nchild; ++i) {
        int64_t cc[3] = {0, 0, 0};
        int empty = 0;
        for (int d = 0; d < D; ++d) {
            cc[d] = 2 * c[d] + ((i >> d) & 1);
            if (cc[d] * (s >> 1) >= G->n[d] - 1) empty = 1;
        }
        if (empty) continue;
#pragma omp task firstprivate(cc) if (level < 4)
        octree_node(T, level + 1, cc);
    }
}

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y);
}

static int cmp_rec(const void* a, const void* b)
{
    uint64_t x = ((const orc_node_rec*)a)->key, y = ((const orc_node_rec*)b)->key;
    return x < y ? -1 : (x > y);
}

/* Root edge S0 = smallest power of two >= max_d (n_d - 1) cells; L_max = log2(S0 / min_leaf). */
void orc_octree_shape(const orc_grid* G, int min_leaf, int64_t* S0, int* Lmax)
{
    int64_t mx = 1;
    for (int d = 0; d < G->dim; ++d) if (G->n[d] - 1 > mx) mx = G->n[d] - 1;
    int64_t s = 1;
    while (s < mx) s <<= 1;
    int l = 0;
    while ((s >> l) > min_leaf) ++l;
    *S0 = s;
    *Lmax = l;
}

/*
 * Alg. 1 (octree adaptive query) from the root.  Observation tail probabilities are
 * P(Y_i < theta) and P(Y_i > theta) under N(mu_i, A_ii), the latent posterior at x_i.
 * Leaves (set S) and skipped nodes are returned sorted by key; recs (optional) receives
 * one record per visited node, sorted by key.  Returns ORC_ECAP if a list overflowed
 * (counts are still exact).
 */
int orc_adaptive(const orc_model* M, const orc_grid* G, double theta, const orc_adapt* A,
                 uint64_t* leaves, int64_t leaf_cap, int64_t* n_leaves,
                 uint64_t* skipped, int64_t skip_cap, int64_t* n_skipped,
                 orc_node_rec* recs, int64_t rec_cap, int64_t* n_recs)
{
    int m = M->m;
    double* qlo = (double*)malloc(sizeof(double) * (size_t)m);
    double* qhi = (double*)malloc(sizeof(double) * (size_t)m);
    double* mu = (double*)malloc(sizeof(double) * (size_t)m);
    double* var = (double*)malloc(sizeof(double) * (size_t)m);
    if (!qlo || !qhi || !mu || !var) { free(qlo); free(qhi); free(mu); free(var); return ORC_ENOMEM; }
    if (M->A) {
        /* Sec. 5.3: the inducing values are N(mu_M, A_M); their marginals are stored */
        for (int i = 0; i < m; ++i) {
            mu[i] = M->muM[i];
            var[i] = M->A[(int64_t)i * m + i] > 0.0 ? M->A[(int64_t)i * m + i] : 0.0;
        }
    } else {
        orc_posterior(M, m, M->X, mu, var, NULL);
    }
    for (int i = 0; i < m; ++i) {
        if (var[i] > 0.0) {
            double z = (theta - mu[i]) / sqrt(var[i]);
            qlo[i] = 0.5 * erfc(-z / sqrt(2.0));
            qhi[i] = 0.5 * erfc(z / sqrt(2.0));
        } else {
            qlo[i] = mu[i] < theta ? 1.0 : 0.0;
            qhi[i] = mu[i] > theta ? 1.0 : 0.0;
        }
    }
    octree_ctx T;
    memset(&T, 0, sizeof T);
    T.M = M; T.G = G; T.A = A; T.theta = theta; T.qlo = qlo; T.qhi = qhi;
    orc_octree_shape(G, A->min_leaf, &T.S0, &T.Lmax);
    T.kd = A->split == 1;
    T.Ldepth = T.kd ? G->dim * T.Lmax : T.Lmax;
    T.leaves = leaves; T.leaf_cap = leaf_cap;
    T.skipped = skipped; T.skip_cap = skip_cap;
    T.recs = recs; T.rec_cap = rec_cap;
    omp_init_lock(&T.lock);
    int64_t root[3] = {0, 0, 0};
#pragma omp parallel
#pragma omp single
    octree_node(&T, 0, root);
    omp_destroy_lock(&T.lock);
    int64_t nl = T.n_leaves < leaf_cap ? T.n_leaves : leaf_cap;
    int64_t ns = T.n_skipped < skip_cap ? T.n_skipped : skip_cap;
    int64_t nr = T.n_recs < rec_cap ? T.n_recs : rec_cap;
    if (leaves) qsort(leaves, (size_t)nl, sizeof(uint64_t), cmp_u64);
    if (skipped) qsort(skipped, (size_t)ns, sizeof(uint64_t), cmp_u64);
    if (recs) qsort(recs, (size_t)nr, sizeof(orc_node_rec), cmp_rec);
    *n_leaves = T.n_leaves;
    *n_skipped = T.n_skipped;
    if (n_recs) *n_recs = T.n_recs;
    free(qlo); free(qhi); free(mu); free(var);
    if (T.rc) return T.rc;
    if (T.n_leaves > leaf_cap || T.n_skipped > skip_cap || (recs && T.n_recs > rec_cap)) return ORC_ECAP;
    return ORC_OK;
}

static void key_decode(int D, uint64_t key, int* level, int64_t* c)
{
    *level = (int)(key >> 58);
    uint64_t mc = key & ((1ull << 58) - 1);
    for (int d = 0; d < D; ++d) c[d] = 0;
    for (int b = 0; b < *level; ++b)
        for (int d = 0; d < D; ++d)
            c[d] |= (int64_t)((mc >> (b * D + d)) & 1) << b;
}

/* LCP of every cell inside the given leaves (end of Sec. 5.3: only these are reconstructed); each
 * cell is computed exactly as in the dense path.  lcp covers the whole cell grid and
 * is written only inside leaves. */
int orc_lcp_leaves(const orc_model* M, const orc_grid* G, double theta, int ns, const double* zb,
                   int64_t S0, const uint64_t* keys, int64_t nkeys, double* lcp)
{
    int D = G->dim;
    int rc = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nkeys; ++t) {
        int level;
        int64_t c[3], clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0}, box_n[3] = {1, 1, 1};
        key_decode(D, keys[t], &level, c);
        int64_t s = S0 >> level;
        for (int d = 0; d < D; ++d) {
            clo[d] = c[d] * s;
            chi[d] = (c[d] + 1) * s;
            if (chi[d] > G->n[d] - 1) chi[d] = G->n[d] - 1;
            box_n[d] = chi[d] - clo[d] + 1;
        }
        double *mean = NULL, *var = NULL, *V = NULL;
        int64_t nv;
        if (box_posterior(M, G, clo, box_n, &mean, &var, &V, &nv) != ORC_OK) {
#pragma omp atomic write
            rc = ORC_ENOMEM;
        } else {
            int64_t cn[3] = {1, 1, 1}, ncell = 1;
            for (int d = 0; d < D; ++d) { cn[d] = chi[d] - clo[d]; ncell *= cn[d]; }
            for (int64_t u = 0; u < ncell; ++u) {
                int64_t cell[3], r = u, lin = 0, stride = 1;
                for (int d = 0; d < D; ++d) { cell[d] = clo[d] + r % cn[d]; r /= cn[d]; }
                for (int d = 0; d < D; ++d) { lin += cell[d] * stride; stride *= G->n[d] - 1; }
                int64_t cnt = cell_count(M, G, theta, ns, zb, cell, clo, box_n, mean, var, V);
                lcp[lin] = (double)cnt / (double)ns;
            }
        }
        free(mean); free(var); free(V);
    }
    return rc;
}

/* Octree level at which each cell's node stopped (leaf level for cells in S). */
void orc_level_field(const orc_grid* G, int64_t S0, const uint64_t* keys, int64_t nkeys, uint8_t* field)
{
    int D = G->dim;
    for (int64_t t = 0; t < nkeys; ++t) {
        int level;
        int64_t c[3], clo[3] = {0, 0, 0}, chi[3] = {1, 1, 1};
        key_decode(D, keys[t], &level, c);
        int64_t s = S0 >> level;
        for (int d = 0; d < D; ++d) {
            clo[d] = c[d] * s;
            chi[d] = (c[d] + 1) * s;
            if (chi[d] > G->n[d] - 1) chi[d] = G->n[d] - 1;
        }
        for (int64_t k = clo[2]; k < (D > 2 ? chi[2] : 1); ++k)
            for (int64_t j = clo[1]; j < chi[1]; ++j)
                for (int64_t i = clo[0]; i < chi[0]; ++i)
                    field[i + (G->n[0] - 1) * (j + (G->n[1] - 1) * k)] = (uint8_t)level;
    }
}

/* Depth at which each cell's node stopped, for K-D tree keys (depth L << 58 | code). */
void orc_level_field_kd(const orc_grid* G, int64_t S0, const uint64_t* keys, int64_t nkeys, uint8_t* field)
{
    int D = G->dim;
    for (int64_t t = 0; t < nkeys; ++t) {
        int L = (int)(keys[t] >> 58);
        uint64_t code = keys[t] & ((1ull << 58) - 1);
        int64_t c[3] = {0, 0, 0}, clo[3] = {0, 0, 0}, chi[3] = {1, 1, 1};
        for (int j = 0; j < L; ++j) {
            int a = kd_axis(D, j);
            c[a] = 2 * c[a] + (int64_t)((code >> (L - 1 - j)) & 1);
        }
        for (int d = 0; d < D; ++d) {
            int64_t s = S0 >> kd_splits(D, L, d);
            clo[d] = c[d] * s;
            chi[d] = (c[d] + 1) * s;
            if (chi[d] > G->n[d] - 1) chi[d] = G->n[d] - 1;
        }
        for (int64_t k = clo[2]; k < (D > 2 ? chi[2] : 1); ++k)
            for (int64_t j = clo[1]; j < chi[1]; ++j)
                for (int64_t i = clo[0]; i < chi[0]; ++i)
                    field[i + (G->n[0] - 1) * (j + (G->n[1] - 1) * k)] = (uint8_t)L;
    }
}

int orc_num_threads(void)
{
    return omp_get_max_threads();
}
