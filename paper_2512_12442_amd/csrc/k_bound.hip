// Certified region bound: box bounds of the posterior mean and variance that hold at every
// point of a box, so that the bound 1 - B^d of eq. (upper_bound) is guaranteed instead of
// found by a bounded search (the search of Sec. 5.1 can miss the minimum; Sec. 9 leaves a
// guaranteed bound open).  The bounds hold in exact arithmetic for the stored model.
//
// Second-order Taylor model with the Lagrange remainder around the box centre c.  For
// phi(x) = sum_i b_i k(x, x_i), u = x - c, H = sum_d (h_d / ell_d)^2 (h the half-widths):
//   phi(c + u) = phi(c) + grad.u + u^T Hess u / 2 + R,  |R| <= s2 H^(3/2) sum_i |b_i| C3(r_i) / 6,
// with r_i the scaled distance from x_i to the box and s2 C3(r) the supremum, beyond r, of
// the kernel's third derivative along a unit scaled direction.  The mean takes b = a.  The
// variance var = s2 - q(k), q(k) = k^T Q k convex (Q = L^-T L^-1, or T^T T for a sparse
// model), obeys var(x) <= s2 - nu(c) - 2 min_box (nu(x) - nu(c)) with nu(x) = w^T k(x) and
// w = Q k(c), so it takes b = w.
//
// Per box: w on MFMA (the binary64 posterior kernel run against the full operand Q, with
// k(c) generated on the fly), then one wave per box accumulates the 22 moments (value,
// gradient, Hessian and remainder weight for a and for w) over the observations, lanes
// striding the observations, and reduces them by a fixed butterfly.
#include "lcp_internal.h"

namespace lcp {

namespace {

// kappa3(rho): max over unit v of |D^3 f[v, v, v]| at scaled distance rho (s2 = 1).
//  SE: e^(-rho^2/2) max over |s| <= rho of |3 s - s^3|.
//  Matern-5/2, t = sqrt5 rho: (5 sqrt5 / 3) e^-t max over |p| <= 1 of |3 t p - t^2 p^3|.
__device__ __forceinline__ double kappa3(int kind, double rho)
{
    if (kind == LCP_KERNEL_SE) {
        const double e = exp_nonpos(-0.5 * rho * rho);
        if (rho <= 1.0) return e * (3.0 * rho - rho * rho * rho);
        if (rho <= 2.0) return 2.0 * e;
        return e * (rho * rho * rho - 3.0 * rho);
    }
    const double t = 2.23606797749978969640917366873 * rho;
    const double c = 3.72677996249964981 * exp_nonpos(-t);   // 5 sqrt5 / 3
    if (t <= 1.0) return c * (3.0 * t - t * t);
    if (t <= 4.0) return c * 2.0 * sqrt_nonneg(t);
    return c * (t * t - 3.0 * t);
}

// C3(r) = sup over rho >= r of kappa3: kappa3 rises to a first peak, falls, rises to a
// second, lower peak and then falls.  Peaks (rho, value):
//   SE: rho^2 = 3 -/+ sqrt6;  Matern-5/2: t = (5 -/+ sqrt13) / 2.
__device__ __forceinline__ double curv3_env(int kind, double r2)
{
    const bool se = kind == LCP_KERNEL_SE;
    const double p1 = se ? 0.741963784302726 : 0.3118082139200399;
    const double p2 = se ? 2.3344142183389773 : 1.9242597635797498;
    const double q1 = se ? 1.3801190461607493 : 2.979595011595829;
    const double q2 = se ? 0.3748969288392891 : 0.2826704205128165;
    const double rho = sqrt_nonneg(r2);
    if (rho <= p1) return q1;
    const double k = kappa3(kind, rho);
    if (rho >= p2) return k;
    return k > q2 ? k : q2;
}

// Range over |u| <= h of g u + q u^2 / 2: the two ends, and the vertex when it lies inside.
__device__ __forceinline__ void quad_range(double g, double q, double h, double& lo, double& hi)
{
    const double a = -g * h + 0.5 * q * h * h, b = g * h + 0.5 * q * h * h;
    lo = a < b ? a : b;
    hi = a > b ? a : b;
    if (q != 0.0 && fabs(g) <= fabs(q) * h) {
        const double v = -0.5 * g * g / q;
        lo = v < lo ? v : lo;
        hi = v > hi ? v : hi;
    }
}

// Symmetric 3 x 3 stored as (00, 01, 02, 11, 12, 22).
__device__ __forceinline__ int sym(int d, int e)
{
    const int i = d < e ? d : e, j = d < e ? e : d;
    return i == 0 ? j : (i == 1 ? 2 + j : 5);
}

// Range of the second-order model relative to phi(c): g[3], Hs[6], remainder R.
template <int D>
__device__ __forceinline__ void model_range(const double* g, const double* Hs, const double* h, double R,
                                            double& lo, double& hi)
{
    lo = -R;
    hi = R;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double a, b;
        quad_range(g[d], Hs[sym(d, d)], h[d], a, b);
        lo += a;
        hi += b;
#pragma unroll
        for (int e = 0; e < D; ++e) {
            if (e == d) continue;
            const double x = 0.5 * fabs(Hs[sym(d, e)]) * h[d] * h[e];
            lo -= x;
            hi += x;
        }
    }
}

constexpr int kMom = 11;   // value, gradient (3), Hessian (6), remainder weight

// One wave per box.  box: lo[D], hi[D] per box; W: column b at b * ldw; out: mu(c), mu_lo,
// mu_hi, var_hi per box.
template <int D>
__global__ void __launch_bounds__(256) k_cert(KParams kp, const double* __restrict__ X, const double* __restrict__ a,
                                              int m, const double* __restrict__ W, int64_t ldw,
                                              const double* __restrict__ box, const int64_t* __restrict__ count,
                                              int64_t cap, double* __restrict__ out)
{
    int64_t n = count ? *count : cap;
    if (n > cap) n = cap;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= n) return;   // uniform over the wave
    const int lane = threadIdx.x & 63;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, c[3] = {0, 0, 0}, h[3] = {0, 0, 0}, H = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = box[b * 2 * D + d];
        hi[d] = box[b * 2 * D + D + d];
        c[d] = 0.5 * (lo[d] + hi[d]);
        h[d] = 0.5 * (hi[d] - lo[d]);
        const double t = h[d] * kp.inv_ell[d];
        H += t * t;
    }
    const double* wcol = W + b * ldw;
    double acc[2 * kMom];
#pragma unroll
    for (int q = 0; q < 2 * kMom; ++q) acc[q] = 0.0;
    const double s5 = 2.23606797749978969640917366873;
    for (int i = lane; i < m; i += 64) {
        double t[3] = {0, 0, 0}, r2 = 0.0, e2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double xi = X[(int64_t)i * 4 + d];
            t[d] = (c[d] - xi) * kp.inv_ell[d];
            r2 += t[d] * t[d];
            double e = lo[d] - xi;
            e = xi - hi[d] > e ? xi - hi[d] : e;
            e = e > 0.0 ? e * kp.inv_ell[d] : 0.0;
            e2 += e * e;
        }
        double k, g, gam;
        if (kp.kind == LCP_KERNEL_SE) {
            const double E = kp.s2 * exp_nonpos(-0.5 * r2);
            k = E;
            g = -E;
            gam = E;
        } else {
            const double r = sqrt_nonneg(r2);
            const double E = kp.s2 * exp_nonpos(-s5 * r);
            k = fma(5.0 / 3.0, r2, fma(s5, r, 1.0)) * E;
            g = -(5.0 / 3.0) * fma(s5, r, 1.0) * E;
            gam = (25.0 / 3.0) * E;
        }
        const double C3 = curv3_env(kp.kind, e2);
        double mom[kMom];
        mom[0] = k;
        for (int d = 0; d < 3; ++d) mom[1 + d] = d < D ? g * t[d] * kp.inv_ell[d] : 0.0;
        for (int d = 0; d < 3; ++d)
            for (int e = d; e < 3; ++e)
                mom[4 + sym(d, e)] = (d < D && e < D)
                                         ? ((d == e ? g : 0.0) + gam * t[d] * t[e]) * kp.inv_ell[d] * kp.inv_ell[e]
                                         : 0.0;
        mom[10] = C3;
        const double ai = a[i], wi = wcol[i];
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            acc[q] = fma(ai, mom[q], acc[q]);
            acc[kMom + q] = fma(wi, mom[q], acc[kMom + q]);
        }
        acc[10] = fma(fabs(ai), C3, acc[10]);
        acc[kMom + 10] = fma(fabs(wi), C3, acc[kMom + 10]);
    }
#pragma unroll
    for (int q = 0; q < 2 * kMom; ++q)
        for (int o = 32; o >= 1; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
    if (lane != 0) return;
    const double r3 = kp.s2 * H * sqrt_nonneg(H) / 6.0;
    double mlo, mhi, nlo, nhi;
    model_range<D>(acc + 1, acc + 4, h, r3 * acc[10], mlo, mhi);
    model_range<D>(acc + kMom + 1, acc + kMom + 4, h, r3 * acc[kMom + 10], nlo, nhi);
    double vhi = kp.s2 - acc[kMom] - 2.0 * nlo;
    vhi = vhi > kp.s2 ? kp.s2 : vhi;
    vhi = vhi < 0.0 ? 0.0 : vhi;
    out[b * 4 + 0] = acc[0];
    out[b * 4 + 1] = acc[0] + mlo;
    out[b * 4 + 2] = acc[0] + mhi;
    out[b * 4 + 3] = vhi;
}

// Box centres (3 doubles per box) for the operand pass.
__global__ void k_box_centres(const double* __restrict__ box, int D, int64_t n, double* __restrict__ pts)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    for (int d = 0; d < 3; ++d) pts[b * 3 + d] = d < D ? 0.5 * (box[b * 2 * D + d] + box[b * 2 * D + D + d]) : 0.0;
}

struct CertLayout {
    size_t pts, w, mean, var, total;
};

CertLayout cert_layout(const Model& M, int64_t n)
{
    CertLayout L{};
    const size_t mp = (size_t)M.m_pad, nn = (size_t)(n > 0 ? n : 1);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
    L.pts = take(24 * nn);
    L.w = take(8 * mp * nn);
    L.mean = take(8 * nn);
    L.var = take(8 * nn);
    L.total = o;
    return L;
}

}  // namespace

hipError_t launch_cert_w(const Model& M, const double* F64, const double* pts, const int64_t* count, int64_t cap,
                         double* W, double* mean, double* var, hipStream_t s)
{
    PostTask t{};
    t.mode = COL_POINTS;
    t.group = 1;
    t.count = count;
    t.n_points = cap;
    t.pts = pts;
    t.pstride = 3;
    t.mean = mean;
    t.var = var;
    t.V = W;
    t.vld = M.m_pad;
    t.dense = 1;
    t.stage = ST_BOUND;
    return launch_posterior_operand(M, LCP_FP64, t, F64, s);
}

hipError_t launch_cert(const Model& M, const double* box, const int64_t* count, int64_t cap, const double* W,
                       double* out, hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    StageScope sc(s, ST_BOUND);
    if (M.dim == 3)
        hipLaunchKernelGGL(k_cert<3>, dim3((unsigned)ceil_div(cap, 4)), dim3(256), 0, s, M.kp, M.X, M.a, M.m, W,
                           (int64_t)M.m_pad, box, count, cap, out);
    else
        hipLaunchKernelGGL(k_cert<2>, dim3((unsigned)ceil_div(cap, 4)), dim3(256), 0, s, M.kp, M.X, M.a, M.m, W,
                           (int64_t)M.m_pad, box, count, cap, out);
    return hipGetLastError();
}

size_t bound_certified_ws(const Model& M, int64_t n) { return cert_layout(M, n).total; }

hipError_t launch_bound_certified(const Model& M, int64_t n, const double* box, double* out, char* ws, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const CertLayout L = cert_layout(M, n);
    const double* F64 = M.Q64;   // the operand Q, formed by the fit
    hipError_t e;
    double* pts = (double*)(ws + L.pts);
    double* W = (double*)(ws + L.w);
    {
        StageScope sc(s, ST_BOUND);
        hipLaunchKernelGGL(k_box_centres, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, box, M.dim, n, pts);
    }
    e = launch_cert_w(M, F64, pts, nullptr, n, W, (double*)(ws + L.mean), (double*)(ws + L.var), s);
    if (e != hipSuccess) return e;
    return launch_cert(M, box, nullptr, n, W, out, s);
}

}  // namespace lcp
