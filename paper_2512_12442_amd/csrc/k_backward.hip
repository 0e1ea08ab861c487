// Adjoint of the posterior (exact-GP form of eq. (sgp)) with respect to the observation
// values y and the log-lengthscales.  With K = k(X, X) + noise I, a = K^-1 y, w_p = K^-1 k*_p
// and upstream gradients g_p = dL/dmean_p, h_p = dL/dvar_p at n query points:
//
//   dL/dy             = b = sum_p g_p w_p
//   dL/dlog(ell_d)    = sum_p sum_j dk_pj,d (g_p a_j - 2 h_p w_pj)            (T_d)
//                     + sum_jl dK_d[j][l] (G[j][l] - b_j a_l)                  (P_d)
//   G                 = sum_p h_p w_p w_p^T
//
// where dk and dK are derivatives with respect to log(ell_d).  The pass runs:
//   1. K^-1 = L^-T L^-1 (binary64) in the posterior kernel's fragment order;
//   2. W = K^-1 K*^T for all points on MFMA (the posterior kernel with a full operand,
//      K* generated on the fly and never stored), W column-major;
//   3. per point chunk: T_d partials and b partials, kernel derivatives recomputed;
//   4. G by a binary64 symmetric rank-n product over point splits (upper blocks);
//   5. P_d over all (j, l) pairs, then the ordered sums of every partial.
// Every sum runs in a fixed order, so results are reproducible bit for bit.
//
// The adjoint of the smooth LCP field adds, per grid vertex p, the gradient c_p,e with
// respect to the cross-covariance of p and its neighbour p + e (canonical directions e).
// With cross = k(p, q) - k_p^T K^-1 k_q and z_p = sum over neighbours q of c_pq w_q (both
// directions), the same passes apply with
//   T_d  += -sum_p dk_p,d . z_p + sum_(p,e) c_p,e dk(x_p, x_p+e)/dlog(ell_d)   (direct term)
//   G    += (1/2) sum_p w_p z_p^T,
// so the rank-n product runs on U_p = h_p w_p + z_p / 2 in place of h_p w_p.
#include "lcp_internal.h"

namespace lcp {

namespace {

constexpr int kBwdChunk = 64;       // points per chunk of the points pass
constexpr int kBwdGridP = 1024;     // work-groups of the points pass (partials)
constexpr int kBwdGridQ = 1024;     // work-groups of the pairs pass (partials)
constexpr int kBwdSplitPts = 4096;  // points per split of the rank-n product
constexpr int kBwdMaxSplit = 32;

// K^-1[i][j] = sum_k Linv[k][i] Linv[k][j]: a 16 x 16 tile per work-group, k in steps of 64
// through LDS (few dependent load-barrier rounds).  Linv is lower triangular, so the sum
// starts at the first step that reaches row max(i, j); every term it skips is an exact zero
// and the FMAs run in increasing k as over the whole range.
__global__ void __launch_bounds__(256) k_kinv(const double* __restrict__ Li, int mp, double* __restrict__ Ki)
{
    __shared__ double As[16][65], Bs[64][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
    const int kfirst = (16 * (blockIdx.x > blockIdx.y ? blockIdx.x : blockIdx.y)) / 64 * 64;
    double c = 0.0;
    for (int k0 = kfirst; k0 < mp; k0 += 64) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = 16 * q + (threadIdx.x >> 4), r = threadIdx.x & 15;      // 64 x 16 of each, rows coalesced
            const bool in = k0 + kk < mp;
            As[r][kk] = in ? Li[(int64_t)(k0 + kk) * mp + blockIdx.y * 16 + r] : 0.0;   // Linv^T[i][k]
            Bs[kk][r] = in ? Li[(int64_t)(k0 + kk) * mp + blockIdx.x * 16 + r] : 0.0;   // Linv[k][j]
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 64; ++k) c = fma(As[ty][k], Bs[k][tx], c);
        __syncthreads();
    }
    Ki[(int64_t)i * mp + j] = c;
}

// 16 x 16 x 4 fragment order: fragment (i, s), lane l holds X[16 i + l % 16][4 s + l / 16].
__global__ void k_frag_full(const double* __restrict__ Ki, int mp, double* __restrict__ F64, float* __restrict__ F32)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)mp * mp) return;
    const int64_t frag = t / 64;
    const int l = (int)(t % 64);
    const int ks = mp / 4;
    const int i = (int)(frag / ks), s = (int)(frag % ks);
    const double x = Ki[(int64_t)(16 * i + l % 16) * mp + 4 * s + l / 16];
    F64[t] = x;
    F32[t] = (float)x;
}

// Query points: n x dim binary64 coordinates, or the vertices of a grid (x fastest).
struct BwdPts {
    const double* P;
    int dim;
    int grid_mode;
    GridP grid;
    int64_t n;
    __device__ __forceinline__ void at(int64_t p, double& x, double& y, double& z) const
    {
        if (grid_mode) {
            x = vertex_coord(grid, 0, p % grid.n[0]);
            y = vertex_coord(grid, 1, (p / grid.n[0]) % grid.n[1]);
            z = dim > 2 ? vertex_coord(grid, 2, p / (grid.n[0] * grid.n[1])) : 0.0;
        } else {
            x = P[p * dim + 0];
            y = P[p * dim + 1];
            z = dim > 2 ? P[p * dim + 2] : 0.0;
        }
    }
};

struct BwdArgs {
    KParams kp;
    int m, mp, dim;
    const double* X;       // m_pad x 4
    const double* alpha;   // a = K^-1 y
    const void* W;         // column p at p * ldw (binary64 or binary32)
    const void* Z;         // optional, as W: neighbour term z_p
    int64_t ldw;
    BwdPts pts;
    const double* gm;      // dL/dmean (may be null)
    const double* gv;      // dL/dvar (may be null)
    double* bpart;         // [kBwdGridP][mp]
    double* tpart;         // [kBwdGridP][4]
};

__device__ __forceinline__ double block_sum256(double v, double* red)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Each work-group walks point chunks blockIdx.x, blockIdx.x + gridDim.x, ...; thread t owns
// observations j = t, t + 256, ... (m <= 1024) and keeps their b partials in registers.
template <class T>
__global__ void __launch_bounds__(256) k_bwd_points(BwdArgs A)
{
    __shared__ double red[4];
    constexpr int J = 4;
    const int tid = threadIdx.x;
    const T* __restrict__ W = (const T*)A.W;
    const T* __restrict__ Z = (const T*)A.Z;
    const double ie0 = A.kp.inv_ell[0], ie1 = A.kp.inv_ell[1], ie2 = A.kp.inv_ell[2];
    double xj[J][3], aj[J], bacc[J];
#pragma unroll
    for (int u = 0; u < J; ++u) {
        const int j = tid + 256 * u;
        const bool live = j < A.m;
        xj[u][0] = live ? A.X[(size_t)j * 4 + 0] : 0.0;
        xj[u][1] = live ? A.X[(size_t)j * 4 + 1] : 0.0;
        xj[u][2] = live ? A.X[(size_t)j * 4 + 2] : 0.0;
        aj[u] = live ? A.alpha[j] : 0.0;
        bacc[u] = 0.0;
    }
    double tacc[3] = {0.0, 0.0, 0.0};
    const int64_t n = A.pts.n;
    const int64_t nchunks = (n + kBwdChunk - 1) / kBwdChunk;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t p1 = (c + 1) * kBwdChunk < n ? (c + 1) * kBwdChunk : n;
        for (int64_t p = c * kBwdChunk; p < p1; ++p) {
            double px, py, pz;
            A.pts.at(p, px, py, pz);
            const double g1 = A.gm ? A.gm[p] : 0.0, g2 = A.gv ? A.gv[p] : 0.0;
#pragma unroll
            for (int u = 0; u < J; ++u) {
                const int j = tid + 256 * u;
                if (j >= A.m) continue;
                const double t0 = (px - xj[u][0]) * ie0, t1 = (py - xj[u][1]) * ie1, t2 = (pz - xj[u][2]) * ie2;
                const double r2 = fma(t2, t2, fma(t1, t1, t0 * t0));
                double kv, f;
                kernel_val_dfac(A.kp, r2, &kv, &f);
                const double w = (double)W[p * A.ldw + j];
                const double zj = Z ? (double)Z[p * A.ldw + j] : 0.0;
                // dk/dlog(ell_d) = -f t_d^2 (f = 2 dk/d(r^2))
                const double coef = -f * (fma(-2.0 * g2, w, g1 * aj[u]) - zj);
                tacc[0] = fma(coef, t0 * t0, tacc[0]);
                tacc[1] = fma(coef, t1 * t1, tacc[1]);
                tacc[2] = fma(coef, t2 * t2, tacc[2]);
                bacc[u] = fma(g1, w, bacc[u]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < J; ++u) {
        const int j = tid + 256 * u;
        if (j < A.mp) A.bpart[(size_t)blockIdx.x * A.mp + j] = bacc[u];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double s = block_sum256(tacc[d], red);
        if (tid == 0) A.tpart[(size_t)blockIdx.x * 4 + d] = s;
    }
}

// b_j = sum over the points pass's work-groups, in order.
__global__ void k_bwd_reduce_b(const double* __restrict__ bpart, int nparts, int mp, double* __restrict__ b)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= mp) return;
    double s = 0.0;
    for (int q = 0; q < nparts; ++q) s += bpart[(size_t)q * mp + j];
    b[j] = s;
}

// G partial of split blockIdx.y over the upper 64 x 64 block pair blockIdx.x:
// Gpart[s][j][l] = sum_{p in split} h_p W[p][j] W[p][l].
// With U non-null the second operand is U[p][l] instead of h_p W[p][l].
template <class T>
__global__ void __launch_bounds__(256) k_bwd_syrk(const T* __restrict__ W, const T* __restrict__ U, int64_t ldw,
                                                  int64_t n, const double* __restrict__ h, int mp,
                                                  int64_t split_pts, double* __restrict__ Gpart)
{
    __shared__ double As[16][68], Bs[16][68];
    const int nb = mp / 64;
    // block pair index -> (jb, lb), jb <= lb
    int rem = blockIdx.x, jb = 0;
    while (rem >= nb - jb) { rem -= nb - jb; ++jb; }
    const int lb = jb + rem;
    const int j0 = jb * 64, l0 = lb * 64;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int64_t pbeg = (int64_t)blockIdx.y * split_pts;
    const int64_t pend = pbeg + split_pts < n ? pbeg + split_pts : n;
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
    const int lk = tid >> 4, lc = (tid & 15) * 4;     // loader: point row lk, columns lc..lc+3
    for (int64_t p0 = pbeg; p0 < pend; p0 += 16) {
        const int64_t p = p0 + lk;
        const bool live = p < pend;
        const double hp = (live && !U) ? h[p] : 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            As[lk][lc + e] = live ? (double)W[p * ldw + j0 + lc + e] : 0.0;
            Bs[lk][lc + e] = live ? (U ? (double)U[p * ldw + l0 + lc + e] : hp * (double)W[p * ldw + l0 + lc + e])
                                  : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[k][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[k][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
    double* G = Gpart + (size_t)blockIdx.y * mp * mp;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) G[(size_t)(j0 + ty * 4 + r) * mp + l0 + tx * 4 + c] = acc[r][c];
}

// The same partial for binary32 W and U on FP32 MFMA (16 x 16 x 4): the products of each run
// of 256 points are summed in binary32, those sums in binary64.  A 16-point step stages the
// block's W and U rows in LDS; wave w owns the 32 x 32 quarter (w / 2, w % 2) of the block.
__global__ void __launch_bounds__(256) k_bwd_syrk_mfma(const float* __restrict__ W, const float* __restrict__ U,
                                                       int64_t ldw, int64_t n, const double* __restrict__ h, int mp,
                                                       int64_t split_pts, double* __restrict__ Gpart)
{
    __shared__ float As[16][68], Bs[16][68];
    const int nb = mp / 64;
    int rem = blockIdx.x, jb = 0;
    while (rem >= nb - jb) { rem -= nb - jb; ++jb; }
    const int lb = jb + rem;
    const int j0 = jb * 64, l0 = lb * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wj = (wave >> 1) * 32, wl = (wave & 1) * 32;
    const int64_t pbeg = (int64_t)blockIdx.y * split_pts;
    const int64_t pend = pbeg + split_pts < n ? pbeg + split_pts : n;
    f4 acc[2][2];
    double dacc[2][2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            acc[t][u] = f4{0, 0, 0, 0};
#pragma unroll
            for (int r = 0; r < 4; ++r) dacc[t][u][r] = 0.0;
        }
    auto flush = [&]() {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
#pragma unroll
                for (int r = 0; r < 4; ++r) dacc[t][u][r] += (double)acc[t][u][r];
                acc[t][u] = f4{0, 0, 0, 0};
            }
    };
    const int lk = tid >> 4, lc = (tid & 15) * 4;     // loader: point row lk, columns lc .. lc + 3
    int steps = 0;
    for (int64_t p0 = pbeg; p0 < pend; p0 += 16) {
        const int64_t p = p0 + lk;
        const bool live = p < pend;
        f4 a = f4{0, 0, 0, 0}, b = f4{0, 0, 0, 0};
        if (live) {
            a = *(const f4*)(W + p * ldw + j0 + lc);
            b = U ? *(const f4*)(U + p * ldw + l0 + lc) : (float)h[p] * *(const f4*)(W + p * ldw + l0 + lc);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            As[lk][lc + e] = a[e];
            Bs[lk][lc + e] = b[e];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            const int k = kk + (lane >> 4);
            const float av0 = As[k][wj + (lane & 15)], av1 = As[k][wj + 16 + (lane & 15)];
            const float bv0 = Bs[k][wl + (lane & 15)], bv1 = Bs[k][wl + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av0, bv0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av0, bv1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av1, bv0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av1, bv1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
        if (++steps == 16) {
            flush();
            steps = 0;
        }
    }
    flush();
    double* G = Gpart + (size_t)blockIdx.y * mp * mp;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                G[(size_t)(j0 + wj + 16 * t + 4 * (lane >> 4) + r) * mp + l0 + wl + 16 * u + (lane & 15)] = dacc[t][u][r];
}

// P_d partials over all (j, l): dK_d[j][l] (G[j][l] - b_j a_l).
__global__ void __launch_bounds__(256) k_bwd_pairs(KParams kp, int m, int mp, const double* __restrict__ X,
                                                   const double* __restrict__ alpha, const double* __restrict__ b,
                                                   const double* __restrict__ Gpart, int nsplit,
                                                   double* __restrict__ ppart)
{
    __shared__ double red[4];
    double pacc[3] = {0.0, 0.0, 0.0};
    const int64_t npairs = (int64_t)m * m;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < npairs; t += (int64_t)gridDim.x * 256) {
        const int j = (int)(t / m), l = (int)(t % m);
        const double t0 = (X[j * 4 + 0] - X[l * 4 + 0]) * kp.inv_ell[0];
        const double t1 = (X[j * 4 + 1] - X[l * 4 + 1]) * kp.inv_ell[1];
        const double t2 = (X[j * 4 + 2] - X[l * 4 + 2]) * kp.inv_ell[2];
        const double r2 = fma(t2, t2, fma(t1, t1, t0 * t0));
        double kv, f;
        kernel_val_dfac(kp, r2, &kv, &f);
        // G is stored in the upper block pairs only
        const size_t gi = (j / 64 <= l / 64) ? (size_t)j * mp + l : (size_t)l * mp + j;
        double g = 0.0;
        for (int s = 0; s < nsplit; ++s) g += Gpart[(size_t)s * mp * mp + gi];
        const double coef = -f * fma(-b[j], alpha[l], g);
        pacc[0] = fma(coef, t0 * t0, pacc[0]);
        pacc[1] = fma(coef, t1 * t1, pacc[1]);
        pacc[2] = fma(coef, t2 * t2, pacc[2]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double s = block_sum256(pacc[d], red);
        if (threadIdx.x == 0) ppart[(size_t)blockIdx.x * 4 + d] = s;
    }
}

__global__ void k_bwd_finish(const double* __restrict__ b, int m, const double* __restrict__ tpart, int ntp,
                             const double* __restrict__ ppart, int npp, const double* __restrict__ dpart, int ndp,
                             int dim, double* __restrict__ dy, double* __restrict__ dlogell)
{
    for (int j = threadIdx.x; j < m; j += blockDim.x) dy[j] = b[j];
    if (threadIdx.x < dim) {
        const int d = threadIdx.x;
        double t = 0.0, p = 0.0, q2 = 0.0;
        for (int q = 0; q < ntp; ++q) t += tpart[(size_t)q * 4 + d];
        for (int q = 0; q < npp; ++q) p += ppart[(size_t)q * 4 + d];
        for (int q = 0; q < ndp; ++q) q2 += dpart[(size_t)q * 4 + d];
        dlogell[d] = (t + p) + q2;
    }
}

// Neighbour terms of the LCP adjoint over grid vertices (W, Z, U column-major, ld m_pad):
// z_p = sum_e c_p,e w_p+e + c_p-e,e w_p-e and U_p = h_p w_p + z_p / 2.
// One wave owns 64 consecutive observation rows of one x-line of vertices (fixed y, z), so
// every load and store of a column is 64 consecutive elements.  The wave walks the line in
// x with the W columns of the 3^D neighbourhood in registers: each step loads the column at
// x + 2 of the 3^(D-1) neighbouring lines, and the coefficients c (the same for all lanes)
// come through scalar loads.  Consecutive waves take neighbouring lines of the same rows,
// so the columns they share are served from L2.
constexpr int kStRows = 64;
__host__ __device__ inline int64_t stencil_lines(const GridP& g) { return g.n[1] * (g.dim == 3 ? g.n[2] : 1); }

// Direction e: offset with last non-zero component +1 (codes 14..26 of {-1,0,1}^3 in base 3,
// x fastest; 5..8 of {-1,0,1}^2).
template <int D>
__device__ __forceinline__ void stencil_offset(int e, int* off)
{
    if (D == 3) { off[0] = (e + 14) % 3 - 1; off[1] = ((e + 14) / 3) % 3 - 1; off[2] = (e + 14) / 9 - 1; }
    else { off[0] = (e + 5) % 3 - 1; off[1] = (e + 5) / 3 - 1; off[2] = 0; }
}

template <class T, int D>
__global__ void __launch_bounds__(256) k_bwd_stencil(GridP g, int mp, const T* __restrict__ W,
                                                     const double* __restrict__ gvar,
                                                     const double* __restrict__ gcross, T* __restrict__ Z,
                                                     T* __restrict__ U)
{
    constexpr int NDIR = D == 3 ? 13 : 4;
    constexpr int NL = D == 3 ? 9 : 3;              // neighbouring lines (dy, dz) in {-1,0,1}^(D-1)
    const int lane = threadIdx.x & 63;
    const int64_t nlines = stencil_lines(g);
    const int64_t wv = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wv >= nlines * (mp / kStRows)) return;      // uniform over the wave
    const int64_t line = wv % nlines;
    const int j = (int)(wv / nlines) * kStRows + lane;
    const int64_t y = line % g.n[1], z = D == 3 ? line / g.n[1] : 0;
    const int64_t n0 = g.n[0];
    // line l = (dy + 1) + 3 (dz + 1) (2D: dy + 1): its first vertex, or -1 outside the grid
    int64_t base[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const int64_t yy = y + l % 3 - 1, zz = z + (D == 3 ? l / 3 - 1 : 0);
        base[l] = (yy >= 0 && yy < g.n[1] && zz >= 0 && zz < g.n[2]) ? n0 * (yy + g.n[1] * zz) : -1;
    }
    auto col = [&](int l, int64_t x) -> T {
        return (base[l] >= 0 && x >= 0 && x < n0) ? W[(size_t)(base[l] + x) * mp + j] : T(0);
    };
    T win[NL][3];                                   // columns at x - 1, x, x + 1
    T pf[NL];                                       // column x + 2, loaded a step ahead
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        win[l][0] = T(0);
        win[l][1] = col(l, 0);
        win[l][2] = col(l, 1);
        pf[l] = col(l, 2);
    }
    // The coefficients of a vertex (the same for all lanes) come through vector loads one
    // vertex ahead: lane e < NDIR holds the forward c_p,e, lane 16 + e the backward
    // c_p-e,e (zero where the neighbour is outside the grid), read out with readlane.
    const int ce = lane & 15;
    const bool cfw = lane < 16;
    int coff[3] = {0, 0, 0};
    if (ce < NDIR) stencil_offset<D>(ce, coff);
    auto coef = [&](int64_t x) -> double {
        if (ce >= NDIR || lane >= 32) return 0.0;
        const int sg = cfw ? 1 : -1;
        const int64_t b[3] = {x + sg * coff[0], y + sg * coff[1], z + sg * coff[2]};
        if (!(b[0] >= 0 && b[0] < n0 && b[1] >= 0 && b[1] < g.n[1] && b[2] >= 0 && b[2] < g.n[2])) return 0.0;
        const int64_t q = cfw ? base[NL / 2] + x : b[0] + n0 * (b[1] + g.n[1] * b[2]);
        return gcross[(size_t)q * NDIR + ce];
    };
    auto bcast = [](double v, int l) -> double {
        const long long u = __builtin_bit_cast(long long, v);
        const int lo = __builtin_amdgcn_readlane((int)u, l), hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
        return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
    };
    double cv = coef(0);
    for (int64_t x = 0; x < n0; ++x) {
        T next[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            next[l] = pf[l];
            pf[l] = col(l, x + 3);
        }
        const double cvn = coef(x + 1 < n0 ? x + 1 : x);
        const int64_t p = base[NL / 2] + x;
        double zz = 0.0;
#pragma unroll
        for (int e = 0; e < NDIR; ++e) {
            int off[3];
            stencil_offset<D>(e, off);
            zz = fma(bcast(cv, e), (double)win[(off[1] + 1) + (D == 3 ? 3 * (off[2] + 1) : 0)][off[0] + 1], zz);
        }
#pragma unroll
        for (int e = 0; e < NDIR; ++e) {
            int off[3];
            stencil_offset<D>(e, off);
            zz = fma(bcast(cv, 16 + e), (double)win[(1 - off[1]) + (D == 3 ? 3 * (1 - off[2]) : 0)][1 - off[0]], zz);
        }
        const double w = (double)win[NL / 2][1];
        Z[(size_t)p * mp + j] = (T)zz;
        U[(size_t)p * mp + j] = (T)fma(gvar[p], w, 0.5 * zz);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            win[l][0] = win[l][1];
            win[l][1] = win[l][2];
            win[l][2] = next[l];
        }
        cv = cvn;
    }
}

// Direct term of the LCP adjoint, sum_e c_p,e dk(x_p, x_p+e)/dlog(ell_d): one thread per
// vertex, one partial per work-group.
constexpr int kDirectThreads = 256;
__host__ __device__ inline int64_t direct_parts(const GridP& g)
{
    return (g.n[0] * g.n[1] * g.n[2] + kDirectThreads - 1) / kDirectThreads;
}

template <int D>
__global__ void __launch_bounds__(kDirectThreads) k_bwd_direct(KParams kp, GridP g, const double* __restrict__ gcross,
                                                               double* __restrict__ dpart)
{
    constexpr int NDIR = D == 3 ? 13 : 4;
    __shared__ double red[4];
    const int64_t p = (int64_t)blockIdx.x * kDirectThreads + threadIdx.x;
    const int64_t nv = g.n[0] * g.n[1] * g.n[2];
    double dacc[3] = {0.0, 0.0, 0.0};
    if (p < nv) {
        const int64_t v[3] = {p % g.n[0], (p / g.n[0]) % g.n[1], p / (g.n[0] * g.n[1])};
        for (int e = 0; e < NDIR; ++e) {
            int off[3];
            stencil_offset<D>(e, off);
            const int64_t a[3] = {v[0] + off[0], v[1] + off[1], v[2] + off[2]};
            const bool fw = a[0] >= 0 && a[0] < g.n[0] && a[1] >= 0 && a[1] < g.n[1] && a[2] >= 0 && a[2] < g.n[2];
            const double cf = fw ? gcross[(size_t)p * NDIR + e] : 0.0;
            if (cf == 0.0) continue;
            double t[3];
            for (int d = 0; d < 3; ++d)
                t[d] = (off[d] == 0 || d >= D) ? 0.0 : (vertex_coord(g, d, a[d]) - vertex_coord(g, d, v[d])) * kp.inv_ell[d];
            const double r2 = fma(t[2], t[2], fma(t[1], t[1], t[0] * t[0]));
            double kv, f;
            kernel_val_dfac(kp, r2, &kv, &f);
            for (int d = 0; d < 3; ++d) dacc[d] = fma(-f * cf, t[d] * t[d], dacc[d]);
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double sres = block_sum256(dacc[d], red);
        if (threadIdx.x == 0) dpart[(size_t)blockIdx.x * 4 + d] = sres;
    }
}

struct BwdLayout {
    size_t kinv, f64, f32, w, mean, var, bpart, tpart, b, gpart, ppart, total;
    size_t hhi, hlo, kamax;   // FP16 split operand (LCP_MIXED_F16X3 only)
    // LCP adjoint only
    size_t V, cross, wbank, gout, gmean, gvar, gcross, z, u, dpart, work;
    int nsplit;
};

// lcp: also the forward moments, the cell and vertex gradients and the neighbour terms of
// a dense grid with n vertices, ncell cells and ns samples.
BwdLayout bwd_layout(const Model& M, int64_t n, int prec, bool lcp, int D, int64_t ncell, int ns, int64_t ntiles)
{
    BwdLayout L{};
    const size_t mp = (size_t)M.m_pad;
    const size_t es = prec == LCP_FP64 ? 8 : 4;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    L.nsplit = (int)((n + kBwdSplitPts - 1) / kBwdSplitPts);
    if (L.nsplit > kBwdMaxSplit) L.nsplit = kBwdMaxSplit;
    if (L.nsplit < 1) L.nsplit = 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
    L.kinv = take(8 * mp * mp);
    L.f64 = take(8 * mp * mp);
    L.f32 = take(4 * mp * mp);
    L.w = take(es * mp * nn);
    L.mean = take(8 * nn);
    L.var = take(8 * nn);
    L.bpart = take(8 * mp * kBwdGridP);
    L.tpart = take(8 * 4 * kBwdGridP);
    L.b = take(8 * mp);
    L.gpart = take(8 * mp * mp * (size_t)L.nsplit);
    L.ppart = take(8 * 4 * kBwdGridQ);
    if (prec == LCP_MIXED_F16X3) {
        L.hhi = take(2 * mp * mp);
        L.hlo = take(2 * mp * mp);
        L.kamax = take(8 * 2);
    }
    if (lcp) {
        const int N = 1 << D, ndir = D == 3 ? 13 : 4;
        L.V = take(es * mp * nn);
        L.cross = take(8 * (size_t)ndir * nn);
        L.wbank = take(8 * ((size_t)ns * N + 1));
        L.gout = take(8 * (size_t)(N + N * (N + 1) / 2) * (size_t)(ncell > 0 ? ncell : 1));
        L.gmean = take(8 * nn);
        L.gvar = take(8 * nn);
        L.gcross = take(8 * (size_t)ndir * nn);
        L.z = take(es * mp * nn);
        L.u = take(es * mp * nn);
        L.dpart = take(8 * 4 * (size_t)(ntiles > 0 ? ntiles : 1));
        L.work = take(4 * (size_t)(ncell > 0 ? ncell : 1) + 256);
    }
    L.total = o;
    return L;
}

// Largest |K^-1| and the power-of-two scale that brings it to [2^14, 2^15) (one work-group).
__global__ void __launch_bounds__(1024) k_kinv_amax(const double* __restrict__ Ki, int mp, double* __restrict__ amax)
{
    __shared__ double wmax[16];
    double mx = 0.0;
    for (int64_t t = threadIdx.x; t < (int64_t)mp * mp; t += 1024) mx = fmax(mx, fabs(Ki[t]));
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < 16; ++w) mx = fmax(mx, wmax[w]);
        int e;
        frexp(mx, &e);
        amax[0] = mx;
        amax[1] = ldexp(1.0, 15 - e);
    }
}

// 16 x 16 x 32 fragment order: fragment (i, s), lane l holds X[16 i + l % 16][32 s + 8 (l / 16) + e],
// e = 0..7; x * amax[1] split into FP16 halves hi = fp16(x sA), lo = fp16(x sA - hi).
__global__ void k_kinv_split16(const double* __restrict__ Ki, int mp, const double* __restrict__ amax,
                               _Float16* __restrict__ hi, _Float16* __restrict__ lo)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)mp * mp) return;
    const int64_t frag = t / 512;
    const int rem = (int)(t % 512);
    const int l = rem / 8, e = rem % 8;
    const int ks = mp / 32;
    const int i = (int)(frag / ks), s = (int)(frag % ks);
    const double xs = Ki[(int64_t)(16 * i + l % 16) * mp + 32 * s + 8 * (l / 16) + e] * amax[1];
    const _Float16 h = (_Float16)xs;
    hi[t] = h;
    lo[t] = (_Float16)(xs - (double)h);
}

}  // namespace

hipError_t launch_kinv_frag(const Model& M, double* Kinv, double* F64, float* F32, hipStream_t s)
{
    const int mp = M.m_pad;
    const int64_t n2 = (int64_t)mp * mp;
    StageScope sc(s, ST_FACTOR);
    hipLaunchKernelGGL(k_kinv, dim3((unsigned)(mp / 16), (unsigned)(mp / 16)), dim3(256), 0, s, M.Linv, mp, Kinv);
    hipLaunchKernelGGL(k_frag_full, dim3((unsigned)ceil_div(n2, 256)), dim3(256), 0, s, Kinv, mp, F64, F32);
    return hipGetLastError();
}

namespace {

// K^-1 fragments, then W = K^-1 K*^T for the points (plain columns of m_pad).
hipError_t bwd_w(const Model& M, const BwdLayout& L, const BwdPts& P, int prec, char* ws, hipStream_t s)
{
    const int mp = M.m_pad;
    double* Kinv = (double*)(ws + L.kinv);
    double* F64 = (double*)(ws + L.f64);
    float* F32 = (float*)(ws + L.f32);
    hipError_t e = launch_kinv_frag(M, Kinv, F64, F32, s);
    if (e != hipSuccess) return e;
    if (prec == LCP_MIXED_F16X3) {
        StageScope sc(s, ST_FACTOR);
        const int64_t n2 = (int64_t)mp * mp;
        hipLaunchKernelGGL(k_kinv_amax, dim3(1), dim3(1024), 0, s, Kinv, mp, (double*)(ws + L.kamax));
        hipLaunchKernelGGL(k_kinv_split16, dim3((unsigned)ceil_div(n2, 256)), dim3(256), 0, s, Kinv, mp,
                           (const double*)(ws + L.kamax), (_Float16*)(ws + L.hhi), (_Float16*)(ws + L.hlo));
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (P.n <= 0) return hipSuccess;
    PostTask t{};
    t.group = 1;
    t.n_points = P.n;
    if (P.grid_mode) {
        t.mode = COL_GRID;
        t.grid = P.grid;
    } else {
        t.mode = COL_POINTS;
        t.pts = P.P;
        t.pstride = P.dim;
    }
    t.mean = (double*)(ws + L.mean);
    t.var = (double*)(ws + L.var);
    t.V = ws + L.w;
    t.vld = mp;
    t.dense = 1;
    t.stage = ST_POSTERIOR;
    if (prec == LCP_MIXED_F16X3)
        return launch_posterior_operand_f16x3(M, t, ws + L.hhi, ws + L.hlo, (const double*)(ws + L.kamax), s);
    // the full operand in binary64 or binary32 (the BF16 split serves V only)
    const int wprec = prec == LCP_FP64 ? LCP_FP64 : LCP_FP32;
    return launch_posterior_operand(M, wprec, t, wprec == LCP_FP64 ? (const void*)F64 : (const void*)F32, s);
}

// Points pass, b, the rank-n product (on U when given), pairs and the final sums.
hipError_t bwd_tail(const Model& M, const BwdLayout& L, const BwdPts& P, int prec, const double* gm, const double* gv,
                    const void* Z, const void* U, const double* dpart, int ndp, double* dy, double* dlogell,
                    char* ws, hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    const int mp = M.m_pad;
    const int64_t n = P.n;
    const void* W = ws + L.w;
    double* bpart = (double*)(ws + L.bpart);
    double* tpart = (double*)(ws + L.tpart);
    double* b = (double*)(ws + L.b);
    double* gpart = (double*)(ws + L.gpart);
    double* ppart = (double*)(ws + L.ppart);
    BwdArgs A{};
    A.kp = M.kp;
    A.m = M.m;
    A.mp = mp;
    A.dim = M.dim;
    A.X = M.X;
    A.alpha = M.a;
    A.W = W;
    A.Z = Z;
    A.ldw = mp;
    A.pts = P;
    A.gm = gm;
    A.gv = gv;
    A.bpart = bpart;
    A.tpart = tpart;
    if (prec == LCP_FP64) hipLaunchKernelGGL(k_bwd_points<double>, dim3(kBwdGridP), dim3(256), 0, s, A);
    else hipLaunchKernelGGL(k_bwd_points<float>, dim3(kBwdGridP), dim3(256), 0, s, A);
    hipLaunchKernelGGL(k_bwd_reduce_b, dim3((unsigned)ceil_div(mp, 256)), dim3(256), 0, s, bpart, kBwdGridP, mp, b);
    const int nb = mp / 64;
    const unsigned npairs_blk = (unsigned)(nb * (nb + 1) / 2);
    const bool rank_n = (gv || U) && n > 0;
    if (rank_n) {
        const int64_t split_pts = (n + L.nsplit - 1) / L.nsplit;
        if (prec == LCP_FP64)
            hipLaunchKernelGGL(k_bwd_syrk<double>, dim3(npairs_blk, (unsigned)L.nsplit), dim3(256), 0, s,
                               (const double*)W, (const double*)U, (int64_t)mp, n, gv, mp, split_pts, gpart);
        else
            hipLaunchKernelGGL(k_bwd_syrk_mfma, dim3(npairs_blk, (unsigned)L.nsplit), dim3(256), 0, s,
                               (const float*)W, (const float*)U, (int64_t)mp, n, gv, mp, split_pts, gpart);
    } else {
        hipError_t e = launch_fill_f64(gpart, 0.0, (int64_t)mp * mp, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_bwd_pairs, dim3(kBwdGridQ), dim3(256), 0, s, M.kp, M.m, mp, M.X, M.a, b, gpart,
                       rank_n ? L.nsplit : 1, ppart);
    hipLaunchKernelGGL(k_bwd_finish, dim3(1), dim3(256), 0, s, b, M.m, tpart, kBwdGridP, ppart, kBwdGridQ, dpart, ndp,
                       M.dim, dy, dlogell);
    return hipGetLastError();
}

}  // namespace

size_t posterior_backward_ws(const Model& M, int64_t n, int prec)
{
    return bwd_layout(M, n, prec, false, M.dim, 0, 0, 0).total;
}

hipError_t launch_posterior_backward(const Model& M, int64_t n, const double* Xq, int prec, const double* gm,
                                     const double* gv, double* dy, double* dlogell, char* ws, hipStream_t s)
{
    const BwdLayout L = bwd_layout(M, n, prec, false, M.dim, 0, 0, 0);
    BwdPts P{};
    P.P = Xq;
    P.dim = M.dim;
    P.n = n;
    hipError_t e = bwd_w(M, L, P, prec, ws, s);
    if (e != hipSuccess) return e;
    return bwd_tail(M, L, P, prec, gm, gv, nullptr, nullptr, nullptr, 0, dy, dlogell, ws, s);
}

size_t lcp_backward_ws(const Model& M, const GridP& g, int prec, int ns)
{
    const int64_t nv = g.n[0] * g.n[1] * g.n[2], nc = g.nc[0] * g.nc[1] * g.nc[2];
    return bwd_layout(M, nv, prec, true, g.dim, nc, ns, direct_parts(g)).total;
}

hipError_t launch_lcp_backward(const Model& M, const GridP& g, double theta, int ns, const double* zb, int prec,
                               const double* gl, double* dy, double* dlogell, char* ws, hipStream_t s)
{
    const int64_t nv = g.n[0] * g.n[1] * g.n[2], nc = g.nc[0] * g.nc[1] * g.nc[2];
    const BwdLayout L = bwd_layout(M, nv, prec, true, g.dim, nc, ns, direct_parts(g));
    // forward moments: mean, variance, V (quad-major) and the neighbour cross-covariances
    PostTask t{};
    t.mode = COL_GRID;
    t.group = 1;
    t.n_points = nv;
    t.grid = g;
    t.mean = (double*)(ws + L.mean);
    t.var = (double*)(ws + L.var);
    t.V = ws + L.V;
    t.stage = ST_POSTERIOR;
    hipError_t e = launch_posterior(M, prec, t, s);
    if (e != hipSuccess) return e;
    double* cross = (double*)(ws + L.cross);
    e = launch_cross(M, prec, g, nullptr, nullptr, nv, nullptr, ws + L.V, cross, s);
    if (e != hipSuccess) return e;
    // cell gradients of the smooth LCP, gathered per vertex
    CellTask ct{};
    ct.grid = g;
    ct.prec = prec;
    ct.theta = theta;
    ct.ns = ns;
    ct.zb64 = zb;
    ct.mean = t.mean;
    ct.var = t.var;
    ct.cross = cross;
    ct.work = (int32_t*)(ws + L.work);
    ct.wcount = (int64_t*)(ws + L.work + align256(4 * (size_t)(nc > 0 ? nc : 1)));
    double* gmean = (double*)(ws + L.gmean);
    double* gvar = (double*)(ws + L.gvar);
    double* gcross = (double*)(ws + L.gcross);
    e = launch_cells_sov_grad(ct, (double*)(ws + L.wbank), gl, (double*)(ws + L.gout), gmean, gvar, gcross, s);
    if (e != hipSuccess) return e;
    // W, the neighbour terms, then the shared tail
    BwdPts P{};
    P.dim = M.dim;
    P.grid_mode = 1;
    P.grid = g;
    P.n = nv;
    e = bwd_w(M, L, P, prec, ws, s);
    if (e != hipSuccess) return e;
    double* dpart = (double*)(ws + L.dpart);
    {
        StageScope sc(s, ST_MISC);
        const int mp = M.m_pad;
        const unsigned nw = (unsigned)ceil_div(stencil_lines(g) * (mp / kStRows), 4);
        const unsigned nd = (unsigned)direct_parts(g);
        if (prec == LCP_FP64) {
            if (g.dim == 3)
                hipLaunchKernelGGL((k_bwd_stencil<double, 3>), dim3(nw), dim3(256), 0, s, g, mp, (const double*)(ws + L.w),
                                   gvar, gcross, (double*)(ws + L.z), (double*)(ws + L.u));
            else
                hipLaunchKernelGGL((k_bwd_stencil<double, 2>), dim3(nw), dim3(256), 0, s, g, mp, (const double*)(ws + L.w),
                                   gvar, gcross, (double*)(ws + L.z), (double*)(ws + L.u));
        } else {
            if (g.dim == 3)
                hipLaunchKernelGGL((k_bwd_stencil<float, 3>), dim3(nw), dim3(256), 0, s, g, mp, (const float*)(ws + L.w),
                                   gvar, gcross, (float*)(ws + L.z), (float*)(ws + L.u));
            else
                hipLaunchKernelGGL((k_bwd_stencil<float, 2>), dim3(nw), dim3(256), 0, s, g, mp, (const float*)(ws + L.w),
                                   gvar, gcross, (float*)(ws + L.z), (float*)(ws + L.u));
        }
        if (g.dim == 3)
            hipLaunchKernelGGL(k_bwd_direct<3>, dim3(nd), dim3(kDirectThreads), 0, s, M.kp, g, gcross, dpart);
        else
            hipLaunchKernelGGL(k_bwd_direct<2>, dim3(nd), dim3(kDirectThreads), 0, s, M.kp, g, gcross, dpart);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return bwd_tail(M, L, P, prec, gmean, gvar, ws + L.z, ws + L.u, dpart, (int)direct_parts(g), dy, dlogell, ws, s);
}

}  // namespace lcp
