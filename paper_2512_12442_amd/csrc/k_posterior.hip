// Posterior GEMM (the O(m^2 n) reconstruction of Sec. 3): for a tile of NT columns,
//   B_jc = k(x_j, p_c) (or d/dp k for gradient columns), generated into LDS,
//   mean_c = sum_j B_jc a_j                                    (binary64),
//   V = L^-1 B as a lower-triangular GEMM on MFMA with L^-1 precomputed,
//   dot_c = sum_i V_ic V_i,base(c)  (||v||^2, or v . w_d for gradient columns), binary64 sums,
// and optionally V itself (for the cell cross-covariances).  V is stored per column with
// its 16-row blocks in order; inside a block the rows follow the MFMA result registers,
// a fixed permutation that dot products of V columns do not see.
// Row blocks of 16 are dealt to the four waves in a balanced (snake) order; every column's
// result depends only on that column, so a vertex gets bitwise the same numbers whatever
// tile or launch it is computed in.
#include "lcp_internal.h"

namespace lcp {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = 4;

// Precision traits: operand types, MFMA k-step, fragment arrays and LDS element type.
struct P64 {
    using Acc = d4;
    using Elem = double;
    static constexpr int KS = 4;
    static constexpr int LPAD = 4;   // LDS column stride = m_pad + LPAD elements
    static constexpr bool kScaled = false;
};
struct P32 {
    using Acc = f4;
    using Elem = float;
    static constexpr int KS = 4;
    static constexpr int LPAD = 4;
    static constexpr bool kScaled = false;
};
// 16-bit split product: x = hi + lo in T16, V += lo_A hi_B + hi_A lo_B + hi_A hi_B.
// FP16 operands are scaled by powers of two (sA for L^-1, sB for B) into FP16 range.
template <class T16, bool SCALED>
struct P16 {
    using Acc = f4;
    using Elem = T16;
    using Vec = T16 __attribute__((ext_vector_type(8)));
    static constexpr int KS = 32;
    static constexpr int LPAD = 32;
    static constexpr bool kScaled = SCALED;
};
using PB3 = P16<__bf16, false>;
using PH3 = P16<_Float16, true>;

__device__ __forceinline__ f4 mfma16(bf8 a, bf8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(h8 a, h8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

template <class P>
__device__ __forceinline__ int lds_ld(int mp)
{
    if (P::KS == 32) return (mp + 63) / 64 * 64 + P::LPAD;
    return mp + P::LPAD;
}

template <class P>
__host__ __device__ constexpr int lds_planes()
{
    return P::KS == 32 ? 2 : 1;       // bf16: hi and lo planes
}

struct KArgs {
    KParams kp;
    int m, mp, nrb;
    const double* X;
    const double* a;
    const void* A0;       // fragment array (A64 / A32 / Ahi / Hhi)
    const void* A1;       // low halves for the 16-bit split products
    const double* amax;   // [1] = sA for the FP16 operands
    double sB;            // power-of-two scale of B for the FP16 operands
    PostTask t;
};

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <class P, int NT, int G>
__global__ void __launch_bounds__(kThreads) k_post(KArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    using Elem = typename P::Elem;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mp = A.mp;
    const int ldb = lds_ld<P>(mp);
    Elem* Bt = (Elem*)smem;                                   // [plane][NT][ldb]
    double* red = (double*)(smem + sizeof(Elem) * (size_t)lds_planes<P>() * NT * ldb);  // [kWaves][NT]
    double* mucol = red + kWaves * NT;                        // [NT]
    double* pts = mucol + NT;                                 // [NT/G][3]

    const PostTask& T = A.t;
    int64_t npts = T.count ? *T.count : T.n_points;
    if (npts > T.n_points) npts = T.n_points;
    const int64_t ncols = npts * G;
    const int64_t ntiles = (ncols + NT - 1) / NT;
    const int dim = A.kp.dim;

    // rows of X owned by this thread for B generation (m_pad <= 1024 -> <= 4 rows)
    constexpr int RPT = kMaxM / kThreads;
    double xr[RPT][3], ar[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        int j = tid + r * kThreads;
        bool ok = j < A.m;
        for (int d = 0; d < 3; ++d) xr[r][d] = ok ? A.X[j * 4 + d] : 0.0;
        ar[r] = ok ? A.a[j] : 0.0;
    }

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t col0 = tile * NT;
        __syncthreads();   // previous tile fully consumed
        // ---- point coordinates of this tile
        if (tid < NT / G) {
            int64_t p = col0 / G + tid;
            double x[3] = {0.0, 0.0, 0.0};
            if (p < npts) {
                if (T.mode == COL_GRID) {
                    int64_t v = T.vlist ? (int64_t)T.vlist[p] : p;
                    int64_t i0 = v % T.grid.n[0];
                    int64_t r = v / T.grid.n[0];
                    int64_t i1 = r % T.grid.n[1];
                    int64_t i2 = r / T.grid.n[1];
                    x[0] = vertex_coord(T.grid, 0, i0);
                    x[1] = vertex_coord(T.grid, 1, i1);
                    x[2] = dim > 2 ? vertex_coord(T.grid, 2, i2) : 0.0;
                } else {
                    for (int d = 0; d < dim; ++d) x[d] = T.pts[p * T.pstride + d];
                }
            }
            pts[tid * 3 + 0] = x[0];
            pts[tid * 3 + 1] = x[1];
            pts[tid * 3 + 2] = x[2];
        }
        __syncthreads();
        // ---- generate B (transposed: Bt[c][j]) and the per-column mean partials
        for (int pc = 0; pc < NT / G; ++pc) {
            const int64_t p = col0 / G + pc;
            const bool valid = p < npts;
            const double px = pts[pc * 3 + 0], py = pts[pc * 3 + 1], pz = pts[pc * 3 + 2];
            double part[G];
#pragma unroll
            for (int g = 0; g < G; ++g) part[g] = 0.0;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int j = tid + r * kThreads;
                if (j >= mp) break;
                double b[G];
                double dx[3] = {px - xr[r][0], py - xr[r][1], pz - xr[r][2]};
                double r2 = 0.0;
                for (int d = 0; d < dim; ++d) {
                    double tt = dx[d] * A.kp.inv_ell[d];
                    r2 = fma(tt, tt, r2);
                }
                const bool live = valid && j < A.m;
                if (G == 1) {
                    b[0] = live ? kernel_val(A.kp, r2) : 0.0;
                } else {
                    double kv = 0.0, f = 0.0;
                    if (live) {
                        kv = kernel_val(A.kp, r2);
                        f = kernel_dfac(A.kp, r2);
                    }
                    b[0] = kv;
#pragma unroll
                    for (int d = 0; d < G - 1; ++d)
                        b[d + 1] = (d < dim) ? f * dx[d] * A.kp.inv_ell[d] * A.kp.inv_ell[d] : 0.0;
                }
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    part[g] = fma(b[g], ar[r], part[g]);
                    const int c = pc * G + g;
                    if constexpr (P::KS == 32) {
                        double bs = b[g];
                        if constexpr (P::kScaled) bs *= A.sB;
                        Elem hi = (Elem)(float)bs;
                        Elem lo = (Elem)(float)(bs - (double)(float)hi);
                        Bt[(size_t)c * ldb + j] = hi;
                        Bt[(size_t)(NT + c) * ldb + j] = lo;
                    } else {
                        Bt[(size_t)c * ldb + j] = (Elem)b[g];
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                double s = wave_sum(part[g]);
                if (lane == 0) red[wave * NT + pc * G + g] = s;
            }
        }
        __syncthreads();
        if (tid < NT) {
            double s = 0.0;
            for (int w = 0; w < kWaves; ++w) s += red[w * NT + tid];
            mucol[tid] = s;
        }

        // ---- V = L^-1 B on MFMA, balanced row blocks per wave, fused norm/dot epilogue
        constexpr int NCT = NT / 16;
        double dacc[NCT][4];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) dacc[ct][r] = 0.0;
        const int gl = lane >> 4, cl = lane & 15;
        const int nks_total = mp / P::KS;
        for (int q = 0; q * 8 < A.nrb; ++q) {
            for (int h = 0; h < 2; ++h) {
                const int rb = 8 * q + (h == 0 ? wave : 7 - wave);
                if (rb >= A.nrb) continue;
                const int nks = (16 * (rb + 1) + P::KS - 1) / P::KS;
                typename P::Acc acc[NCT];
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct) acc[ct] = typename P::Acc{0, 0, 0, 0};
                if constexpr (P::KS == 4) {
                    const Elem* Af = (const Elem*)A.A0 + ((size_t)rb * nks_total) * 64 + lane;
#pragma unroll 4
                    for (int s = 0; s < nks; ++s) {
                        Elem av = Af[(size_t)s * 64];
#pragma unroll
                        for (int ct = 0; ct < NCT; ++ct) {
                            Elem bv = Bt[(size_t)(16 * ct + cl) * ldb + 4 * s + gl];
                            if constexpr (sizeof(Elem) == 8)
                                acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);
                            else
                                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[ct], 0, 0, 0);
                        }
                    }
                } else {
                    using Vec = typename P::Vec;
                    const Vec* Ah = (const Vec*)A.A0 + ((size_t)rb * nks_total) * 64 + lane;
                    const Vec* Al = (const Vec*)A.A1 + ((size_t)rb * nks_total) * 64 + lane;
#pragma unroll 2
                    for (int s = 0; s < nks; ++s) {
                        Vec ah = Ah[(size_t)s * 64];
                        Vec al = Al[(size_t)s * 64];
#pragma unroll
                        for (int ct = 0; ct < NCT; ++ct) {
                            const size_t off = (size_t)(16 * ct + cl) * ldb + 32 * s + 8 * gl;
                            Vec bh = *(const Vec*)(Bt + off);
                            Vec bl = *(const Vec*)(Bt + (size_t)NT * ldb + off);
                            acc[ct] = mfma16(al, bh, acc[ct]);
                            acc[ct] = mfma16(ah, bl, acc[ct]);
                            acc[ct] = mfma16(ah, bh, acc[ct]);
                        }
                    }
                }
                // epilogue: one 16-row block of V for columns 16 ct + cl
                if constexpr (P::KS == 32 && P::kScaled) {
                    const float inv = (float)(1.0 / (A.amax[1] * A.sB));   // exact power of two
#pragma unroll
                    for (int ct = 0; ct < NCT; ++ct) acc[ct] *= inv;
                }
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double v = (double)acc[ct][r];
                        double base = (G == 1) ? v : __shfl(v, lane & ~3, 64);
                        dacc[ct][r] = fma(v, base, dacc[ct][r]);
                    }
                    if (G == 1 && T.V) {
                        const int64_t p = col0 + 16 * ct + cl;
                        if (p < npts) {
                            if constexpr (sizeof(Elem) == 8) {
                                double* Vp = (double*)T.V + (size_t)p * mp + 16 * rb + 4 * gl;
                                *(d4*)Vp = acc[ct];
                            } else {
                                float* Vp = (float*)T.V + (size_t)p * mp + 16 * rb + 4 * gl;
                                *(f4*)Vp = f4{(float)acc[ct][0], (float)acc[ct][1], (float)acc[ct][2],
                                              (float)acc[ct][3]};
                            }
                        }
                    }
                }
            }
        }
        // ---- reduce the dot partials: rows within lane, lane groups, waves
        __syncthreads();   // red[] reuse
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            double s = (dacc[ct][0] + dacc[ct][1]) + (dacc[ct][2] + dacc[ct][3]);
            s += __shfl_xor(s, 16, 64);
            s += __shfl_xor(s, 32, 64);
            if (gl == 0) red[wave * NT + 16 * ct + cl] = s;
        }
        __syncthreads();
        if (tid < NT) {
            double dot = 0.0;
            for (int w = 0; w < kWaves; ++w) dot += red[w * NT + tid];
            const int64_t col = col0 + tid;
            const int64_t p = col / G;
            const int comp = (int)(col % G);
            if (p < npts) {
                if (comp == 0) {
                    T.mean[p] = mucol[tid];
                    double v = A.kp.s2 - dot;
                    T.var[p] = v > 0.0 ? v : 0.0;
                } else if (comp - 1 < dim) {
                    T.dmean[p * 3 + comp - 1] = mucol[tid];
                    T.dvar[p * 3 + comp - 1] = -2.0 * dot;
                }
            }
        }
    }
}

template <class P, int NT, int G>
hipError_t launch_t(const Model& M, const PostTask& t, hipStream_t s, const void* A0, const void* A1)
{
    KArgs A;
    A.kp = M.kp;
    A.m = M.m;
    A.mp = M.m_pad;
    A.nrb = (M.m + 15) / 16;
    A.X = M.X;
    A.a = M.a;
    A.A0 = A0;
    A.A1 = A1;
    A.amax = M.amax;
    {
        int e;
        frexp(M.k.signal_var, &e);
        A.sB = ldexp(1.0, 15 - e);          // k* <= s2, so sB * k* < 2^15
    }
    A.t = t;
    int ldb = (P::KS == 32) ? (M.m_pad + 63) / 64 * 64 + P::LPAD : M.m_pad + P::LPAD;
    size_t lds = sizeof(typename P::Elem) * (size_t)lds_planes<P>() * NT * ldb + sizeof(double) * (kWaves * NT + NT + 3 * NT);
    hipError_t e = hipFuncSetAttribute((const void*)k_post<P, NT, G>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    int64_t ncols = t.n_points * G;
    int64_t ntiles = (ncols + NT - 1) / NT;
    int dev_cus = 256;
    int64_t grid = ntiles < (int64_t)dev_cus * 8 ? ntiles : (int64_t)dev_cus * 8;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_post<P, NT, G>), dim3((unsigned)grid), dim3(kThreads), lds, s, A);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_posterior(const Model& M, int prec, const PostTask& t, hipStream_t s)
{
    if (t.n_points <= 0) return hipSuccess;
    StageScope sc(s, t.stage);
    const bool grad = t.group == 4;
    // LDS: binary64 with 32 columns needs 32 * (m_pad + 4) * 8 bytes (<= 160 KB for m_pad <= 608)
    const bool small = M.m_pad <= 576;
    if (prec == LCP_FP64) {
        if (grad) return small ? launch_t<P64, 32, 4>(M, t, s, M.A64, nullptr) : launch_t<P64, 16, 4>(M, t, s, M.A64, nullptr);
        return small ? launch_t<P64, 32, 1>(M, t, s, M.A64, nullptr) : launch_t<P64, 16, 1>(M, t, s, M.A64, nullptr);
    }
    if (prec == LCP_FP32) {
        if (grad) return launch_t<P32, 32, 4>(M, t, s, M.A32, nullptr);
        return launch_t<P32, 32, 1>(M, t, s, M.A32, nullptr);
    }
    if (prec == LCP_MIXED_F16X3) {
        if (grad) return launch_t<PH3, 32, 4>(M, t, s, M.Hhi, M.Hlo);
        return launch_t<PH3, 32, 1>(M, t, s, M.Hhi, M.Hlo);
    }
    if (grad) return launch_t<PB3, 32, 4>(M, t, s, M.Ahi, M.Alo);
    return launch_t<PB3, 32, 1>(M, t, s, M.Ahi, M.Alo);
}

}  // namespace lcp
