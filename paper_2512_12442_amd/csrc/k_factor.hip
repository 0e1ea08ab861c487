// Model factorisation on the GPU (binary64): K = k(X, X) + noise I, its Cholesky factor,
// the explicit inverse L^-1 in the MFMA fragment orders used by the posterior kernel,
// and a = K^-1 y.  Sec. 3 of the paper with the inducing set equal to the observations.
#include <algorithm>
#include <vector>

#include "lcp_internal.h"

namespace lcp {

size_t model_bytes(int m)
{
    int mp = (m + 127) / 128 * 128;
    size_t b = 0;
    b += align256(sizeof(double) * mp * 4);          // X
    b += align256(sizeof(double) * mp);              // a
    b += align256(sizeof(double) * mp);              // y / w scratch
    b += align256(sizeof(double) * (size_t)mp * mp); // U
    b += align256(sizeof(double) * (size_t)mp * mp); // Linv
    b += align256(sizeof(double) * (size_t)mp * mp); // A64
    b += align256(sizeof(float) * (size_t)mp * mp);  // A32
    b += 2 * align256(sizeof(__bf16) * (size_t)mp * mp);  // Ahi, Alo
    b += 2 * align256(sizeof(_Float16) * (size_t)mp * mp); // Hhi, Hlo
    b += 256;                                        // amax, sA
    b += 2 * align256(sizeof(double) * mp);          // obs_mu, obs_var
    b += 256;                                        // info
    b += align256(sizeof(double) * (size_t)mp * mp); // A_M (sparse model)
    b += align256(sizeof(double) * mp * 4);          // Xs
    b += align256(sizeof(double) * (size_t)mp * mp); // Q64: K^-1 (T^T T) fragments, certified bound
    b += align256(sizeof(float) * (size_t)mp * mp);  // Q32
    return b;
}

__global__ void k_pack(const double* __restrict__ X, const double* __restrict__ y, int m, int mp, int dim,
                       double* __restrict__ Xp, double* __restrict__ w)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= mp) return;
    for (int d = 0; d < 4; ++d) Xp[i * 4 + d] = (i < m && d < dim) ? X[(int64_t)i * dim + d] : 0.0;
    w[i] = i < m ? y[i] : 0.0;
}

// Observations scaled by the inverse lengthscales, with a_j in the fourth slot: what the
// split-product posterior reads per row.  Rows past m sit 1e15 lengthscales away on every
// axis with a_j = 0: their binary32 kernel values underflow to exactly 0 (and stay finite
// on the way), as the zero rows of B they stand for.
__global__ void k_scaled_obs(KParams kp, const double* __restrict__ Xp, const double* __restrict__ a, int m, int mp,
                             double* __restrict__ Xs)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= mp) return;
    for (int d = 0; d < 3; ++d)
        Xs[i * 4 + d] = i < m ? (d < kp.dim ? mul_rn(Xp[i * 4 + d], kp.inv_ell[d]) : 0.0) : 1e15;
    Xs[i * 4 + 3] = i < m ? a[i] : 0.0;
}

// Element t of the padded K + noise I (zero outside the m x m block).
__device__ __forceinline__ void build_K_elem(const KParams& kp, const double* __restrict__ Xp, int m, int mp,
                                             double noise, double* __restrict__ K, int64_t t)
{
    int i = (int)(t / mp), j = (int)(t % mp);
    double v = 0.0;
    if (i < m && j < m) {
        v = kernel_val(kp, kernel_r2(kp, Xp + i * 4, Xp + j * 4));
        if (i == j) v += noise;
    }
    K[t] = v;
}

__global__ void k_build_K(KParams kp, const double* __restrict__ Xp, int m, int mp, double noise,
                          double* __restrict__ K)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)mp * mp) return;
    build_K_elem(kp, Xp, m, mp, noise, K, t);
}

// Largest |Linv| and the power-of-two scale sA that brings it to [2^14, 2^15) (FP16 max is 65504).
__device__ __forceinline__ void amax_body(const double* __restrict__ Li, int mp, double* __restrict__ amax)
{
    __shared__ double wmax[16];
    const int tid = threadIdx.x, nt = blockDim.x;
    double mx = 0.0;
    for (int64_t t = tid; t < (int64_t)mp * mp; t += nt) mx = fmax(mx, fabs(Li[t]));
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((tid & 63) == 0) wmax[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < nt / 64; ++w) mx = fmax(mx, wmax[w]);
        mx = fmax(mx, wmax[0]);
        int e;
        frexp(mx, &e);                   // mx = f * 2^e, f in [0.5, 1)
        amax[0] = mx;
        amax[1] = ldexp(1.0, 15 - e);    // mx * sA in [2^14, 2^15)
    }
}


__global__ void __launch_bounds__(1024) k_amax(const double* __restrict__ Li, int mp, double* __restrict__ amax)
{
    amax_body(Li, mp, amax);
}

// a = Linv^T (Linv y): w = Linv y, then a_i = sum_{k >= i} Linv[k][i] w_k.
__device__ __forceinline__ void alpha_body(const double* __restrict__ Li, const double* __restrict__ y,
                                           double* __restrict__ a, int m, int mp)
{
    __shared__ double w[kMaxM];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < m; i += nt) {
        double s = 0.0;
        for (int k = 0; k <= i; ++k) s = fma(Li[(int64_t)i * mp + k], y[k], s);
        w[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < mp; i += nt) {
        double s = 0.0;
        if (i < m)
            for (int k = i; k < m; ++k) s = fma(Li[(int64_t)k * mp + i], w[k], s);
        a[i] = s;
    }
}

__global__ void __launch_bounds__(1024) k_alpha(const double* __restrict__ Li, const double* __restrict__ y,
                                                double* __restrict__ a, int m, int mp)
{
    alpha_body(Li, y, a, m, mp);
}

// ----------------------------------------------------- blocked factorisation (one model)
//
// Right-looking Cholesky in 64 x 64 blocks over the upper triangle (U = L^T, row-major),
// then the blocked inverse of L: the diagonal blocks first, then each block diagonal d from
// the previous ones, Linv_ij = -Linv_ii sum_{k=j}^{i-1} L_ik Linv_kj.  Every block product
// is one work-group of 256 threads with both operands in LDS (4 x 4 outputs per thread).
// Columns >= m (padding) are skipped and left zero.
constexpr int kFB = 64;

// acc[r][c] += sum_k a(ty*4+r, k) * b(k, tx*4+c) over a 64 x 64 block in LDS.
__device__ __forceinline__ void blk_mma(const double (*a)[kFB + 1], const double (*b)[kFB + 1], double (&acc)[4][4],
                                        bool transpose_a)
{
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll 4
    for (int k = 0; k < kFB; ++k) {
        double av[4], bv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) av[r] = transpose_a ? a[k][ty * 4 + r] : a[ty * 4 + r][k];
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[c] = b[k][tx * 4 + c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
    }
}

__device__ __forceinline__ void blk_load(double (*dst)[kFB + 1], const double* __restrict__ src, int mp, int r0, int c0)
{
    for (int t = threadIdx.x; t < kFB * kFB; t += 256) {
        const int r = t / kFB, c = t % kFB;
        dst[r][c] = src[(int64_t)(r0 + r) * mp + c0 + c];
    }
}

// Invert the lower-triangular block lo (in LDS) into inv (in LDS): column by column,
// inv[i][c] = -(sum_{k=c}^{i-1} lo[i][k] inv[k][c]) / lo[i][i]; rows with lo[i][i] = 0
// (padding) stay zero.
__device__ __forceinline__ void blk_trinv(const double (*lo)[kFB + 1], double (*inv)[kFB + 1])
{
    for (int t = threadIdx.x; t < kFB * kFB; t += 256) inv[t / kFB][t % kFB] = 0.0;
    __syncthreads();
    for (int i = 0; i < kFB; ++i) {
        const double lii = lo[i][i];
        for (int c = threadIdx.x; c <= i; c += 256) {
            if (!(lii > 0.0)) continue;
            if (c == i) {
                inv[i][i] = 1.0 / lii;
            } else {
                double sum = 0.0;
                for (int k = c; k < i; ++k) sum = fma(lo[i][k], inv[k][c], sum);
                inv[i][c] = -sum / lii;
            }
        }
        __syncthreads();
    }
}

// Step k, diagonal block: factor A_kk (upper, in U) in LDS, write U_kk and Linv_kk.
__device__ __forceinline__ void chol_diag_body(double* __restrict__ U, int m, int mp, int kb, double piv_min,
                                               int* __restrict__ info, double* __restrict__ Lkk_inv)
{
    __shared__ double a[kFB][kFB + 1], lo[kFB][kFB + 1];
    const int k0 = kb * kFB;
    if (kb == 0 && threadIdx.x == 0) *info = 0;
    blk_load(a, U, mp, k0, k0);
    __syncthreads();
    for (int c = 0; c < kFB; ++c) {
        const bool real = k0 + c < m;
        double d = a[c][c];
        if (real && !(d > piv_min) && threadIdx.x == 0 && *info == 0) *info = k0 + c + 1;
        const double ucc = real && d > 0.0 ? sqrt(d) : 0.0;
        const double inv = ucc > 0.0 ? 1.0 / ucc : 0.0;
        __syncthreads();
        // row c of U_kk, then the trailing update of the block
        for (int j = c + 1 + threadIdx.x; j < kFB; j += 256) a[c][j] *= inv;
        __syncthreads();
        for (int t = threadIdx.x; t < kFB * kFB; t += 256) {
            const int i = t / kFB, j = t % kFB;
            if (i > c && j >= i) a[i][j] = fma(-a[c][i], a[c][j], a[i][j]);
        }
        if (threadIdx.x == 0) a[c][c] = ucc;
        __syncthreads();
    }
    for (int t = threadIdx.x; t < kFB * kFB; t += 256) {
        const int i = t / kFB, j = t % kFB;
        const double u = j >= i ? a[i][j] : 0.0;
        U[(int64_t)(k0 + i) * mp + k0 + j] = u;
        lo[j][i] = u;                                   // L_kk = U_kk^T
    }
    __syncthreads();
    blk_trinv(lo, a);
    for (int t = threadIdx.x; t < kFB * kFB; t += 256) Lkk_inv[t] = a[t / kFB][t % kFB];
}

// Step k, panel: U_kj = Linv_kk A_kj for block column jb > k.
__device__ __forceinline__ void chol_panel_body(double* __restrict__ U, int mp, int kb, int jb,
                                                const double* __restrict__ Lkk_inv)
{
    __shared__ double li[kFB][kFB + 1], b[kFB][kFB + 1];
    for (int t = threadIdx.x; t < kFB * kFB; t += 256) li[t / kFB][t % kFB] = Lkk_inv[t];
    blk_load(b, U, mp, kb * kFB, jb * kFB);
    __syncthreads();
    double acc[4][4] = {};
    blk_mma(li, b, acc, false);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) U[(int64_t)(kb * kFB + ty * 4 + r) * mp + jb * kFB + tx * 4 + c] = acc[r][c];
}

// Step k, trailing update of the upper blocks: A_ij -= U_ki^T U_kj, k < i <= j; upper block
// pair number idx of the T (T + 1) / 2, T = nblk - kb - 1.
__device__ __forceinline__ void chol_update_body(double* __restrict__ U, int mp, int kb, int nblk, int idx)
{
    __shared__ double a[kFB][kFB + 1], b[kFB][kFB + 1];
    const int T = nblk - kb - 1;
    int rem = idx, ii = 0;
    while (rem >= T - ii) { rem -= T - ii; ++ii; }
    const int ib = kb + 1 + ii, jb = ib + rem;
    blk_load(a, U, mp, kb * kFB, ib * kFB);
    blk_load(b, U, mp, kb * kFB, jb * kFB);
    __syncthreads();
    double acc[4][4] = {};
    blk_mma(a, b, acc, true);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double* p = U + (int64_t)(ib * kFB + ty * 4 + r) * mp + jb * kFB + tx * 4 + c;
            *p -= acc[r][c];
        }
}

// Clear the strictly lower part of U (it still holds K) and of the padding.
__global__ void k_clear_lower(double* __restrict__ U, int mp)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)mp * mp) return;
    if (t % mp < t / mp) U[t] = 0.0;
}

// Inverse, diagonal block ib: Linv_ii = L_ii^-1 with L_ii = U_ii^T.
__device__ __forceinline__ void trinv_diag_body(const double* __restrict__ U, double* __restrict__ Li, int mp, int ib)
{
    __shared__ double lo[kFB][kFB + 1], inv[kFB][kFB + 1];
    const int i0 = ib * kFB;
    for (int t = threadIdx.x; t < kFB * kFB; t += 256) {
        const int r = t / kFB, c = t % kFB;
        lo[c][r] = U[(int64_t)(i0 + r) * mp + i0 + c];
    }
    __syncthreads();
    blk_trinv(lo, inv);
    for (int t = threadIdx.x; t < kFB * kFB; t += 256)
        Li[(int64_t)(i0 + t / kFB) * mp + i0 + t % kFB] = inv[t / kFB][t % kFB];
}

// Inverse, block diagonal d: Linv_ij = -Linv_ii sum_{k=j}^{i-1} L_ik Linv_kj, i = j + d.
__device__ __forceinline__ void trinv_off_body(const double* __restrict__ U, double* __restrict__ Li, int mp, int d,
                                               int jb)
{
    __shared__ double a[kFB][kFB + 1], b[kFB][kFB + 1];
    const int ib = jb + d;
    double acc[4][4] = {};
    for (int kb = jb; kb < ib; ++kb) {
        // a = L_ik = (U_ki)^T: load U_ki and use it transposed
        blk_load(a, U, mp, kb * kFB, ib * kFB);
        blk_load(b, Li, mp, kb * kFB, jb * kFB);
        __syncthreads();
        blk_mma(a, b, acc, true);
        __syncthreads();
    }
    // b = the sum, a = Linv_ii; Linv_ij = -a b
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) b[ty * 4 + r][tx * 4 + c] = acc[r][c];
    blk_load(a, Li, mp, ib * kFB, ib * kFB);
    __syncthreads();
    double out[4][4] = {};
    blk_mma(a, b, out, false);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) Li[(int64_t)(ib * kFB + ty * 4 + r) * mp + jb * kFB + tx * 4 + c] = -out[r][c];
}

// One model: a launch per step, one work-group per block.
__global__ void __launch_bounds__(256) k_chol_diag(double* __restrict__ U, int m, int mp, int kb, double piv_min,
                                                   int* __restrict__ info, double* __restrict__ Lkk_inv)
{
    chol_diag_body(U, m, mp, kb, piv_min, info, Lkk_inv);
}
__global__ void __launch_bounds__(256) k_chol_panel(double* __restrict__ U, int mp, int kb,
                                                    const double* __restrict__ Lkk_inv)
{
    chol_panel_body(U, mp, kb, kb + 1 + blockIdx.x, Lkk_inv);
}
__global__ void __launch_bounds__(256) k_chol_update(double* __restrict__ U, int mp, int kb, int nblk)
{
    chol_update_body(U, mp, kb, nblk, blockIdx.x);
}
__global__ void __launch_bounds__(256) k_trinv_diag(const double* __restrict__ U, double* __restrict__ Li, int mp)
{
    trinv_diag_body(U, Li, mp, blockIdx.x);
}
__global__ void __launch_bounds__(256) k_trinv_off(const double* __restrict__ U, double* __restrict__ Li, int mp,
                                                   int d)
{
    trinv_off_body(U, Li, mp, d, blockIdx.x);
}

// A batch: the same block steps for every model in one launch, blockIdx.y = model.  A
// model runs the very arithmetic of its single-model factorisation, so its factor is
// bitwise the one gp_fit_factor computes; work-groups past a model's block count return.
struct FactorDesc {
    const double* Xin;    // model inputs (device): m x dim, m
    const double* yin;
    double* X;            // packed m_pad x 4
    double* w;            // packed values
    double* U;
    double* Linv;
    double* a;
    double* amax;
    int* info;
    double* lkk;          // 64 x 64 scratch: Linv of the current diagonal block
    KParams kp;
    double noise;
    double piv_min;
    int m, mp, dim;
};

__global__ void k_pack_batch(const FactorDesc* __restrict__ D)
{
    const FactorDesc& d = D[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.mp) return;
    for (int c = 0; c < 4; ++c) d.X[i * 4 + c] = (i < d.m && c < d.dim) ? d.Xin[(int64_t)i * d.dim + c] : 0.0;
    d.w[i] = i < d.m ? d.yin[i] : 0.0;
}

__global__ void k_build_K_batch(const FactorDesc* __restrict__ D)
{
    const FactorDesc& d = D[blockIdx.y];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.mp * d.mp) return;
    build_K_elem(d.kp, d.X, d.m, d.mp, d.noise, d.U, t);
}

__global__ void __launch_bounds__(256) k_chol_diag_batch(const FactorDesc* __restrict__ D, int kb)
{
    const FactorDesc& d = D[blockIdx.y];
    if (kb >= d.mp / kFB) return;
    chol_diag_body(d.U, d.m, d.mp, kb, d.piv_min, d.info, d.lkk);
}

__global__ void __launch_bounds__(256) k_chol_panel_batch(const FactorDesc* __restrict__ D, int kb)
{
    const FactorDesc& d = D[blockIdx.y];
    if ((int)blockIdx.x >= d.mp / kFB - kb - 1) return;
    chol_panel_body(d.U, d.mp, kb, kb + 1 + blockIdx.x, d.lkk);
}

__global__ void __launch_bounds__(256) k_chol_update_batch(const FactorDesc* __restrict__ D, int kb)
{
    const FactorDesc& d = D[blockIdx.y];
    const int T = d.mp / kFB - kb - 1;
    if (T <= 0 || (int)blockIdx.x >= T * (T + 1) / 2) return;
    chol_update_body(d.U, d.mp, kb, d.mp / kFB, blockIdx.x);
}

__global__ void k_clear_lower_batch(const FactorDesc* __restrict__ D)
{
    const FactorDesc& d = D[blockIdx.y];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d.mp * d.mp) return;
    if (t % d.mp < t / d.mp) d.U[t] = 0.0;
}

__global__ void k_gather_info(const FactorDesc* __restrict__ D, int nb, int* __restrict__ out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) out[b] = *D[b].info;
}

__global__ void k_zero_linv_batch(const FactorDesc* __restrict__ D)
{
    const FactorDesc& d = D[blockIdx.y];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (int64_t)d.mp * d.mp) d.Linv[t] = 0.0;
}

__global__ void __launch_bounds__(256) k_trinv_diag_batch(const FactorDesc* __restrict__ D)
{
    const FactorDesc& d = D[blockIdx.y];
    if ((int)blockIdx.x >= d.mp / kFB) return;
    trinv_diag_body(d.U, d.Linv, d.mp, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_trinv_off_batch(const FactorDesc* __restrict__ D, int dd)
{
    const FactorDesc& d = D[blockIdx.y];
    if ((int)blockIdx.x + dd >= d.mp / kFB) return;
    trinv_off_body(d.U, d.Linv, d.mp, dd, blockIdx.x);
}

__global__ void __launch_bounds__(1024) k_amax_alpha_batch(const FactorDesc* __restrict__ D)
{
    const FactorDesc& d = D[blockIdx.x];
    amax_body(d.Linv, d.mp, d.amax);
    alpha_body(d.Linv, d.w, d.a, d.m, d.mp);
}

// Fragment orders of Linv.
//  16x16x4 (binary64 and binary32): fragment (i, s), lane l holds Linv[16i + l%16][4s + l/16].
//  16x16x32 bf16: fragment (i, s), lane l holds Linv[16i + l%16][32s + 8(l/16) + e], e = 0..7,
//  split as hi = bf16(x), lo = bf16(x - hi); the FP16 copy splits x * sA the same way.
__global__ void k_frag(const double* __restrict__ Li, int mp, double* __restrict__ A64, float* __restrict__ A32,
                       __bf16* __restrict__ Ahi, __bf16* __restrict__ Alo, _Float16* __restrict__ Hhi,
                       _Float16* __restrict__ Hlo, const double* __restrict__ amax)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)mp * mp) return;
    {
        int64_t frag = t / 64;
        int l = (int)(t % 64);
        int ks = mp / 4;
        int i = (int)(frag / ks), s = (int)(frag % ks);
        double x = Li[(int64_t)(16 * i + l % 16) * mp + 4 * s + l / 16];
        A64[t] = x;
        A32[t] = (float)x;
    }
    {
        int64_t frag = t / 512;
        int rem = (int)(t % 512);
        int l = rem / 8, e = rem % 8;
        int ks = mp / 32;
        int i = (int)(frag / ks), s = (int)(frag % ks);
        double x = Li[(int64_t)(16 * i + l % 16) * mp + 32 * s + 8 * (l / 16) + e];
        __bf16 hi = (__bf16)(float)x;
        __bf16 lo = (__bf16)(float)(x - (double)(float)hi);
        Ahi[t] = hi;
        Alo[t] = lo;
        const double xs = x * amax[1];
        _Float16 h = (_Float16)xs;
        Hhi[t] = h;
        Hlo[t] = (_Float16)(xs - (double)h);
    }
}

// ------------------------------------------------------------ sparse model (eq. (sgp))
//
// The third term of eq. (sgp) folds into the stored factor.  With K = K_MM + jitter I = L L^T,
//   Q = K^-1 - K^-1 A_M K^-1 = L^-T E L^-1,   E = I - L^-1 A_M L^-T,
// and E = F^T F with F lower triangular (the Cholesky factor of E taken in reversed index
// order), Q = T^T T with T = F L^-1, again lower triangular.  The model keeps T where the
// exact GP keeps L^-1, so var = s2 - ||T k*||^2 and the corner covariances
// k(p,q) - (T k_p).(T k_q) come out of the unchanged posterior and cell kernels.

// C = A B over mp x mp operands given by index functors; one 16 x 16 tile per work-group,
// k staged through LDS 16 at a time.  Binary64; runs once per fit.
template <class LA, class LB, class ST>
__global__ void __launch_bounds__(256) k_gemm64(int mp, LA la, LB lb, ST st)
{
    __shared__ double As[16][17], Bs[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
    double c = 0.0;
    for (int k0 = 0; k0 < mp; k0 += 16) {
        As[ty][tx] = la(i, k0 + tx);
        Bs[ty][tx] = lb(k0 + ty, j);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) c = fma(As[ty][k], Bs[k][tx], c);
        __syncthreads();
    }
    st(i, j, c);
}

struct RowMajor {
    const double* p;
    int ld;
    __device__ double operator()(int i, int k) const { return p[(int64_t)i * ld + k]; }
};
struct Transposed {
    const double* p;
    int ld;
    __device__ double operator()(int k, int j) const { return p[(int64_t)j * ld + k]; }
};
// F[i][k] = G[m-1-k][m-1-i] where the array holds G^T (row r = row r of G^T) after the blocked Cholesky.
struct ReversedFactor {
    const double* p;
    int ld, m;
    __device__ double operator()(int i, int k) const
    {
        return (i < m && k < m) ? p[(int64_t)(m - 1 - i) * ld + (m - 1 - k)] : 0.0;
    }
};
struct Store {
    double* p;
    int ld;
    __device__ void operator()(int i, int j, double c) const { p[(int64_t)i * ld + j] = c; }
};
// E + delta I = I + delta I - W stored in reversed index order (zero outside the m x m block).
struct StoreReversedE {
    double* p;
    int ld, m;
    double delta;
    __device__ void operator()(int i, int j, double w) const
    {
        if (i < m && j < m)
            p[(int64_t)(m - 1 - i) * ld + (m - 1 - j)] = (i == j ? 1.0 + delta : 0.0) - w;
        else
            p[(int64_t)i * ld + j] = 0.0;
    }
};

__global__ void k_pack_square(const double* __restrict__ A, int m, int mp, double* __restrict__ dst)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)mp * mp) return;
    int i = (int)(t / mp), j = (int)(t % mp);
    dst[t] = (i < m && j < m) ? A[(int64_t)i * m + j] : 0.0;
}

// Sec. 5.3 with stored inducing values: the node test reads N(mu_M_i, A_M_ii).
__global__ void k_obs_sparse(const double* __restrict__ mu, const double* __restrict__ A, int m,
                             double* __restrict__ obs_mu, double* __restrict__ obs_var)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    obs_mu[i] = mu[i];
    obs_var[i] = fmax(A[(int64_t)i * m + i], 0.0);
}

// Cholesky of the leading m x m block of A (row-major, ld mp): on exit the upper triangle of
// A holds U = L^T and the lower part is zero; info (device) = first failing column + 1 or 0.
// scratch: 64 x 64 doubles.
static void launch_chol_blocked(double* A, int m, int mp, double piv_min, int* info, double* scratch, hipStream_t s)
{
    const int nblk = mp / kFB;
    for (int kb = 0; kb < nblk; ++kb) {
        hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, A, m, mp, kb, piv_min, info, scratch);
        const int T = nblk - kb - 1;
        if (T == 0) break;
        hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)T), dim3(256), 0, s, A, mp, kb, (const double*)scratch);
        hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, s, A, mp, kb, nblk);
    }
    const int64_t n2 = (int64_t)mp * mp;
    hipLaunchKernelGGL(k_clear_lower, dim3((unsigned)ceil_div(n2, 256)), dim3(256), 0, s, A, mp);
}

// Li = (U^T)^-1 (lower, zero above the diagonal) and its scale (amax).
static hipError_t launch_trinv_blocked(const double* U, double* Li, int mp, double* amax, hipStream_t s)
{
    const int nblk = mp / kFB;
    hipError_t e = launch_fill_f64(Li, 0.0, (int64_t)mp * mp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_trinv_diag, dim3((unsigned)nblk), dim3(256), 0, s, U, Li, mp);
    for (int d = 1; d < nblk; ++d)
        hipLaunchKernelGGL(k_trinv_off, dim3((unsigned)(nblk - d)), dim3(256), 0, s, U, Li, mp, d);
    hipLaunchKernelGGL(k_amax, dim3(1), dim3(1024), 0, s, (const double*)Li, mp, amax);
    return hipGetLastError();
}

static void carve(Model& M, char* base)
{
    int mp = M.m_pad;
    size_t o = 0;
    auto take = [&](size_t bytes) { char* p = base + o; o += align256(bytes); return p; };
    M.X = (double*)take(sizeof(double) * mp * 4);
    M.a = (double*)take(sizeof(double) * mp);
    double* w = (double*)take(sizeof(double) * mp);
    (void)w;
    M.U = (double*)take(sizeof(double) * (size_t)mp * mp);
    M.Linv = (double*)take(sizeof(double) * (size_t)mp * mp);
    M.A64 = (double*)take(sizeof(double) * (size_t)mp * mp);
    M.A32 = (float*)take(sizeof(float) * (size_t)mp * mp);
    M.Ahi = (__bf16*)take(sizeof(__bf16) * (size_t)mp * mp);
    M.Alo = (__bf16*)take(sizeof(__bf16) * (size_t)mp * mp);
    M.Hhi = (_Float16*)take(sizeof(_Float16) * (size_t)mp * mp);
    M.Hlo = (_Float16*)take(sizeof(_Float16) * (size_t)mp * mp);
    M.amax = (double*)take(256);
    M.obs_mu = (double*)take(sizeof(double) * mp);
    M.obs_var = (double*)take(sizeof(double) * mp);
    M.info = (int*)take(256);
    M.AM = (double*)take(sizeof(double) * (size_t)mp * mp);
    M.Xs = (double*)take(sizeof(double) * mp * 4);
    M.Q64 = (double*)take(sizeof(double) * (size_t)mp * mp);
    M.Q32 = (float*)take(sizeof(float) * (size_t)mp * mp);
}

static double* ybuf(const Model& M)
{
    return (double*)((char*)M.a + align256(sizeof(double) * M.m_pad));
}

const double* model_values(const Model& M) { return ybuf(M); }

hipError_t launch_factor(Model& M, const double* X, const double* y, hipStream_t s)
{
    carve(M, (char*)M.X);
    StageScope sc(s, ST_FACTOR);
    int mp = M.m_pad;
    double* w = ybuf(M);
    hipLaunchKernelGGL(k_pack, dim3((unsigned)ceil_div(mp, 256)), dim3(256), 0, s, X, y, M.m, mp, M.dim, M.X, w);
    int64_t n2 = (int64_t)mp * mp;
    hipLaunchKernelGGL(k_build_K, dim3((unsigned)ceil_div(n2, 256)), dim3(256), 0, s, M.kp, M.X, M.m, mp,
                       M.k.noise_var, M.U);
    double piv_min = (double)M.m * 2.220446049250313e-16 * (M.k.signal_var + M.k.noise_var);
    launch_chol_blocked(M.U, M.m, mp, piv_min, M.info, (double*)M.A32, s);
    return hipGetLastError();
}

// After the status has been read: inverse, a, fragments, observation posterior.
hipError_t launch_factor_finish(Model& M, hipStream_t s)
{
    StageScope sc(s, ST_FACTOR);
    int mp = M.m_pad;
    int64_t n2 = (int64_t)mp * mp;
    hipError_t e0 = launch_trinv_blocked(M.U, M.Linv, mp, M.amax, s);
    if (e0 != hipSuccess) return e0;
    hipLaunchKernelGGL(k_alpha, dim3(1), dim3(1024), 0, s, M.Linv, ybuf(M), M.a, M.m, mp);
    hipLaunchKernelGGL(k_scaled_obs, dim3((unsigned)ceil_div(mp, 256)), dim3(256), 0, s, M.kp, M.X, M.a, M.m, mp,
                       M.Xs);
    hipLaunchKernelGGL(k_frag, dim3((unsigned)ceil_div(n2, 256)), dim3(256), 0, s, M.Linv, mp, M.A64, M.A32,
                       M.Ahi, M.Alo, M.Hhi, M.Hlo, M.amax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    PostTask t{};
    t.mode = COL_POINTS;
    t.group = 1;
    t.count = nullptr;
    t.n_points = M.m;
    t.pts = M.X;
    t.pstride = 4;
    t.mean = M.obs_mu;
    t.var = M.obs_var;
    e = launch_posterior(M, LCP_FP64, t, s);
    if (e != hipSuccess) return e;
    return launch_kinv_frag(M, M.U, M.Q64, M.Q32, s);   // U (L^T) is free now
}

// Sparse model, after launch_factor (K_MM + jitter I, mu_M in place of y) succeeded:
// L^-1, a = K^-1 mu_M, the inducing marginals, then P = reversed(E + delta I) in A64 and
// its Cholesky factor with status in info[1].
hipError_t launch_sparse_e(Model& M, const double* A, double delta, bool first, hipStream_t s)
{
    StageScope sc(s, ST_FACTOR);
    const int mp = M.m_pad, m = M.m;
    const int64_t n2 = (int64_t)mp * mp;
    const dim3 tiles((unsigned)(mp / 16), (unsigned)(mp / 16));
    if (first) {
        hipError_t e0 = launch_trinv_blocked(M.U, M.Linv, mp, M.amax, s);
        if (e0 != hipSuccess) return e0;
        hipLaunchKernelGGL(k_alpha, dim3(1), dim3(1024), 0, s, M.Linv, ybuf(M), M.a, m, mp);
        hipLaunchKernelGGL(k_scaled_obs, dim3((unsigned)ceil_div(mp, 256)), dim3(256), 0, s, M.kp, M.X, M.a, m, mp,
                           M.Xs);
        hipLaunchKernelGGL(k_obs_sparse, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s, ybuf(M), A, m,
                           M.obs_mu, M.obs_var);
        hipLaunchKernelGGL(k_pack_square, dim3((unsigned)ceil_div(n2, 256)), dim3(256), 0, s, A, m, mp, M.A64);
        hipLaunchKernelGGL(k_pack_square, dim3((unsigned)ceil_div(n2, 256)), dim3(256), 0, s, A, m, mp, M.AM);
        // U <- L^-1 A_M (U held L^T, no longer needed)
        hipLaunchKernelGGL((k_gemm64<RowMajor, RowMajor, Store>), tiles, dim3(256), 0, s, mp,
                           RowMajor{M.Linv, mp}, RowMajor{M.A64, mp}, Store{M.U, mp});
    }
    // A64 <- reversed(I + delta I - (L^-1 A_M) L^-T)
    hipLaunchKernelGGL((k_gemm64<RowMajor, Transposed, StoreReversedE>), tiles, dim3(256), 0, s, mp,
                       RowMajor{M.U, mp}, Transposed{M.Linv, mp}, StoreReversedE{M.A64, mp, m, delta});
    const double piv_min = (double)m * 2.220446049250313e-16;
    launch_chol_blocked(M.A64, m, mp, piv_min, M.info + 1, (double*)M.A32, s);
    return hipGetLastError();
}

// After E factored: T = F L^-1 replaces L^-1, then scale and fragments.
hipError_t launch_sparse_finish(Model& M, hipStream_t s)
{
    StageScope sc(s, ST_FACTOR);
    const int mp = M.m_pad;
    const int64_t n2 = (int64_t)mp * mp;
    const dim3 tiles((unsigned)(mp / 16), (unsigned)(mp / 16));
    hipLaunchKernelGGL((k_gemm64<ReversedFactor, RowMajor, Store>), tiles, dim3(256), 0, s, mp,
                       ReversedFactor{M.A64, mp, M.m}, RowMajor{M.Linv, mp}, Store{M.U, mp});
    hipError_t e = hipMemcpyAsync(M.Linv, M.U, sizeof(double) * (size_t)n2, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_amax, dim3(1), dim3(1024), 0, s, M.Linv, mp, M.amax);
    hipLaunchKernelGGL(k_frag, dim3((unsigned)ceil_div(n2, 256)), dim3(256), 0, s, M.Linv, mp, M.A64, M.A32,
                       M.Ahi, M.Alo, M.Hhi, M.Hlo, M.amax);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_kinv_frag(M, M.U, M.Q64, M.Q32, s);   // Q = T^T T; U (a copy of T) is free now
}

// Descriptors, one 64 x 64 diagonal-block inverse per model, then the statuses (last).
size_t factor_batch_scratch(int nb)
{
    return align256(sizeof(FactorDesc) * (size_t)nb) + align256(sizeof(double) * kFB * kFB * (size_t)nb) +
           align256(sizeof(int) * (size_t)nb);
}

// Batched factorisation, part 1: pack and build K for every model, then the blocked
// Cholesky of all models one block step at a time (three launches per step over the
// largest model's block count); the statuses land in info_dev[b] (0 = positive definite).
// X[b], y[b] are the models' device inputs; scratch holds factor_batch_scratch(nb) bytes.
hipError_t launch_factor_batch(Model* const* Ms, int nb, const double* const* X, const double* const* y, char* scratch,
                               int* info_dev, hipStream_t s)
{
    StageScope sc(s, ST_FACTOR);
    std::vector<FactorDesc> D(nb);
    double* lkk = (double*)(scratch + align256(sizeof(FactorDesc) * (size_t)nb));
    int mpmax = 0;
    for (int b = 0; b < nb; ++b) {
        Model& M = *Ms[b];
        carve(M, (char*)M.X);
        D[b] = FactorDesc{X[b], y[b], M.X, ybuf(M), M.U, M.Linv, M.a, M.amax, M.info, lkk + (size_t)b * kFB * kFB,
                          M.kp, M.k.noise_var, (double)M.m * 2.220446049250313e-16 * (M.k.signal_var + M.k.noise_var),
                          M.m, M.m_pad, M.dim};
        mpmax = std::max(mpmax, M.m_pad);
    }
    FactorDesc* Dd = (FactorDesc*)scratch;
    hipError_t e = hipMemcpyAsync(Dd, D.data(), sizeof(FactorDesc) * nb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);       // pageable source
    if (e != hipSuccess) return e;
    const int64_t n2 = (int64_t)mpmax * mpmax;
    const unsigned ub = (unsigned)nb;
    hipLaunchKernelGGL(k_pack_batch, dim3((unsigned)ceil_div(mpmax, 256), ub), dim3(256), 0, s, Dd);
    hipLaunchKernelGGL(k_build_K_batch, dim3((unsigned)ceil_div(n2, 256), ub), dim3(256), 0, s, Dd);
    const int nblk = mpmax / kFB;
    for (int kb = 0; kb < nblk; ++kb) {
        hipLaunchKernelGGL(k_chol_diag_batch, dim3(1, ub), dim3(256), 0, s, Dd, kb);
        const int T = nblk - kb - 1;
        if (T == 0) break;
        hipLaunchKernelGGL(k_chol_panel_batch, dim3((unsigned)T, ub), dim3(256), 0, s, Dd, kb);
        hipLaunchKernelGGL(k_chol_update_batch, dim3((unsigned)(T * (T + 1) / 2), ub), dim3(256), 0, s, Dd, kb);
    }
    hipLaunchKernelGGL(k_clear_lower_batch, dim3((unsigned)ceil_div(n2, 256), ub), dim3(256), 0, s, Dd);
    hipLaunchKernelGGL(k_gather_info, dim3((unsigned)ceil_div(nb, 256)), dim3(256), 0, s, Dd, nb, info_dev);
    return hipGetLastError();
}

// Part 2 (statuses read): the blocked inverse and a of every model, a block diagonal per
// launch, then the scaled observations and the fragment orders per model.  The observation
// posteriors are not computed (dense use only).
hipError_t launch_factor_batch_finish(Model* const* Ms, int nb, char* scratch, hipStream_t s)
{
    StageScope sc(s, ST_FACTOR);
    const FactorDesc* Dd = (const FactorDesc*)scratch;
    int mpmax = 0;
    for (int b = 0; b < nb; ++b) mpmax = std::max(mpmax, Ms[b]->m_pad);
    const int64_t n2 = (int64_t)mpmax * mpmax;
    const unsigned ub = (unsigned)nb;
    const int nblk = mpmax / kFB;
    hipLaunchKernelGGL(k_zero_linv_batch, dim3((unsigned)ceil_div(n2, 256), ub), dim3(256), 0, s, Dd);
    hipLaunchKernelGGL(k_trinv_diag_batch, dim3((unsigned)nblk, ub), dim3(256), 0, s, Dd);
    for (int d = 1; d < nblk; ++d)
        hipLaunchKernelGGL(k_trinv_off_batch, dim3((unsigned)(nblk - d), ub), dim3(256), 0, s, Dd, d);
    hipLaunchKernelGGL(k_amax_alpha_batch, dim3(ub), dim3(1024), 0, s, Dd);
    for (int b = 0; b < nb; ++b) {
        Model& M = *Ms[b];
        const int64_t m2 = (int64_t)M.m_pad * M.m_pad;
        hipLaunchKernelGGL(k_scaled_obs, dim3((unsigned)ceil_div(M.m_pad, 256)), dim3(256), 0, s, M.kp, M.X, M.a, M.m,
                           M.m_pad, M.Xs);
        hipLaunchKernelGGL(k_frag, dim3((unsigned)ceil_div(m2, 256)), dim3(256), 0, s, M.Linv, M.m_pad, M.A64, M.A32,
                           M.Ahi, M.Alo, M.Hhi, M.Hlo, M.amax);
    }
    return hipGetLastError();
}

}  // namespace lcp
