// Posterior GEMM (the O(m^2 n) reconstruction of Sec. 3): for a tile of NT columns,
//   B_jc = k(x_j, p_c) (or d/dp k for gradient columns), generated into LDS,
//   mean_c = sum_j B_jc a_j                                    (binary64),
//   V = L^-1 B as a lower-triangular GEMM on MFMA with L^-1 precomputed,
//   dot_c = sum_i V_ic V_i,base(c)  (||v||^2, or v . w_d for gradient columns), binary64 sums,
// and optionally V itself (for the cell cross-covariances).  V is stored quad-major: rows
// 4q .. 4q + 3 of column p sit at (q * n_points + p) * 4, so the 16 lanes of one MFMA
// result quad write 256 B (FP32) or 512 B (binary64) runs, and a consumer reading four
// rows of consecutive columns reads contiguous memory; inside a 16-row block the rows
// follow the MFMA result registers, a fixed permutation that dot products of V columns
// do not see.
// In k_post, row blocks of 16 are dealt to the four waves in a balanced (snake) order; the
// 16-bit split value columns run in k_post_ps (below).  In both, every column's result
// depends only on that column, so a vertex gets bitwise the same numbers whatever tile or
// launch it is computed in.  k_post_sp (the region search's small binary64 launches) may
// share a tile among 2 or 4 work-groups and add their partial dot products in a fixed order:
// its results depend on the launch's tile count as well, and are the same on every run.
// The group-4 launches of the search also take each candidate's descent step in their
// epilogue (search_step).
#include <vector>

#include "lcp_internal.h"

namespace lcp {

namespace {

constexpr int kWaves = 4;

// Precision traits: operand types, MFMA k-step, fragment arrays and LDS element type.
// LDS column stride of B = m_pad + LPAD elements, chosen so the lanes of one LDS pass of the
// B-fragment reads fall on distinct banks (b64: 16 lanes, b32: 32 lanes, b128: 8 lanes).
struct P64 {
    using Acc = d4;
    using Elem = double;
    static constexpr int KS = 4;
    static constexpr int LPAD = 1;
    static constexpr bool kScaled = false;
};
struct P32 {
    using Acc = f4;
    using Elem = float;
    static constexpr int KS = 4;
    static constexpr int LPAD = 2;
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
    static constexpr int LPAD = 8;
    static constexpr bool kScaled = SCALED;
};
using PB3 = P16<__bf16, false>;
using PH3 = P16<_Float16, true>;

// x = hi + lo in 16-bit halves, formed in binary32 with hardware conversions: the
// residual x32 - hi is exact in binary32, so hi + lo carries about 2 x 11 (FP16) or
// 2 x 8 (BF16) significant bits of x.
__device__ __forceinline__ void split16(float f, _Float16& hi, _Float16& lo)
{
    hi = __builtin_amdgcn_cvt_pkrtz(f, 0.0f)[0];
    lo = __builtin_amdgcn_cvt_pkrtz(f - (float)hi, 0.0f)[0];
}
__device__ __forceinline__ void split16(float f, __bf16& hi, __bf16& lo)
{
    hi = (__bf16)f;
    lo = (__bf16)(f - (float)hi);
}

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
    const double* Xs;     // scaled observations and a (Model::Xs), for k_post_ps
    PostTask t;
};

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Region search (Sec. 5.1) in the epilogue of the group-4 probes, wave 0 of a binary64 tile.
// The lane of a candidate's value column gathers its three derivative columns from the next
// lanes.  The value enters g_min from the second step on; then one projected gradient step of
// g = side (theta - mu) / sigma, of length eta = 2^-(k+1) times the box width along the
// normalised direction u_a = w_a dg/dx_a, clamped to the node box.  A zero variance or a zero
// or non-finite direction ends the candidate's descent.
__device__ __forceinline__ void search_step(const KArgs& A, int64_t d, int comp, double dot, double mc, bool live)
{
    const PostTask& T = A.t;
    const int lane = threadIdx.x & 63;
    double dm[3], dv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dm[a] = __shfl(mc, lane + 1 + a, 64);
        dv[a] = -2.0 * __shfl(dot, lane + 1 + a, 64);
    }
    if (!live || comp != 0) return;
    // one round of independent loads: the candidate's record, flag and point
    double* rec = T.cand_rec + d * 8;
    const double2 r01 = *(const double2*)(rec + 0), r23 = *(const double2*)(rec + 2);
    const double2 r45 = *(const double2*)(rec + 4), r67 = *(const double2*)(rec + 6);
    const int done = T.cand_done[d];
    double* x = (double*)T.pts + d * T.pstride;
    const double x0 = x[0], x1 = x[1], x2 = x[2];
    if (done) return;
    const double lo[3] = {r01.x, r01.y, r23.x}, hi[3] = {r23.y, r45.x, r45.y};
    const double xs[3] = {x0, x1, x2};
    const double side = r67.x;
    const double mu = mc;
    const double vr = A.kp.s2 - dot;
    const double var = vr > 0.0 ? vr : 0.0;
    const double g = margin(side, T.theta, mu, var);
    if (T.epi_step >= 1 && g < r67.y) rec[7] = g;
    if (!(var > 0.0)) {
        T.cand_done[d] = 1;
        return;
    }
    const int dim = A.kp.dim;
    const double sd = sqrt(var);
    double u[3] = {0.0, 0.0, 0.0}, nrm = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a < dim) {
            const double dsd = dv[a] / (2.0 * sd);
            const double gr = side * (-dm[a] * sd - (T.theta - mu) * dsd) / var;
            u[a] = (hi[a] - lo[a]) * gr;
            nrm += u[a] * u[a];
        }
    }
    nrm = sqrt(nrm);
    if (!(nrm > 0.0) || !isfinite(nrm)) {
        T.cand_done[d] = 1;
        return;
    }
    double eta = 0.5;
    for (int i = 0; i < T.epi_step; ++i) eta *= 0.5;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a < dim) {
            const double w = hi[a] - lo[a];
            const double xn = xs[a] - eta * w * u[a] / nrm;
            x[a] = xn < lo[a] ? lo[a] : (xn > hi[a] ? hi[a] : xn);
        }
    }
}

// Tiles t_first, t_first + t_stride, ... (below t_limit and the column count) of one model.
// SPLIT (small launches of the region search, T.sp_cnt set): when the tiles are few, W = 2 or
// 4 work-groups share a tile.  Each takes every W-th row-block pair, on its first NW / W waves
// (so one busy wave per SIMD at W = 4), and stores its partial dot products; the last of the
// W to arrive (one atomic per work-group on the tile's counter, which it resets) adds the W
// partials in a fixed order and writes the outputs.  No work-group waits for another.
template <class P, int NT, int G, int NW, bool SPLIT = false>
__device__ __forceinline__ void post_tiles(const KArgs& A, int64_t t_first, int64_t t_stride, int64_t t_limit)
{
    constexpr int kThreads = NW * 64;
    constexpr int kWaves = NW;
    extern __shared__ __align__(16) unsigned char smem[];
    using Elem = typename P::Elem;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform (scalar)
    const int mp = A.mp;
    const int ldb = lds_ld<P>(mp);
    Elem* Bt = (Elem*)smem;                                   // [plane][NT][ldb]
    double* red = (double*)(smem + sizeof(Elem) * (size_t)lds_planes<P>() * NT * ldb);  // [256 / NP][NT]
    double* mucol = red + kThreads * G;                       // [NT]

    const PostTask& T = A.t;
    int64_t npts = T.count ? *T.count : T.n_points;
    if (npts > T.n_points) npts = T.n_points;
    const int64_t ncols = npts * G;
    int64_t ntiles = (ncols + NT - 1) / NT;
    if (ntiles > t_limit) ntiles = t_limit;
    const int dim = A.kp.dim;
    int ways = 1, spart = 0;
    if constexpr (SPLIT) {
        ways = ntiles * 4 <= t_stride ? 4 : (ntiles * 2 <= t_stride ? 2 : 1);   // t_stride: the grid
        spart = (int)(t_first % ways);
        t_first /= ways;
        t_stride /= ways;
    }

    // B generation layout: thread t serves point pc = t % NP of the tile (NP = NT / G points)
    // for the rows j = t / NP + k * (256 / NP); its mean partials cover its own columns only
    // and are combined through LDS once per tile.
    constexpr int NP = NT / G;
    constexpr int RSTEP = kThreads / NP;
    // value columns of the reduced-precision paths generate B in binary32
    constexpr bool kGen32 = G == 1 && sizeof(Elem) < 8;
    const int pc = tid % NP, jg = tid / NP;
    const double ie0 = A.kp.inv_ell[0], ie1 = A.kp.inv_ell[1], ie2 = A.kp.inv_ell[2];

    for (int64_t tile = t_first; tile < ntiles; tile += t_stride) {
        const int64_t col0 = tile * NT;
        __syncthreads();   // previous tile fully consumed
        // ---- this thread's point
        const int64_t p = col0 / G + pc;
        const bool valid = p < npts;
        double px = 0.0, py = 0.0, pz = 0.0;
        if (valid) {
            if (T.mode == COL_GRID) {
                const int64_t v = T.vlist ? (int64_t)T.vlist[p] : p;
                const int64_t i0 = v % T.grid.n[0];
                const int64_t r = v / T.grid.n[0];
                const int64_t i1 = r % T.grid.n[1];
                const int64_t i2 = r / T.grid.n[1];
                px = vertex_coord(T.grid, 0, i0);
                py = vertex_coord(T.grid, 1, i1);
                pz = dim > 2 ? vertex_coord(T.grid, 2, i2) : 0.0;
            } else {
                px = T.pts[p * T.pstride + 0];
                py = T.pts[p * T.pstride + 1];
                pz = dim > 2 ? T.pts[p * T.pstride + 2] : 0.0;
            }
        }
        // ---- generate B (transposed: Bt[c][j]) and the mean partials of this thread's columns
        double part[G];
#pragma unroll
        for (int g = 0; g < G; ++g) part[g] = 0.0;
        if constexpr (kGen32) {
            // binary32 kernel values (binary64 coordinate differences and mean sums)
            const float fie0 = (float)ie0, fie1 = (float)ie1, fie2 = (float)ie2;
            const float fs2 = (float)A.kp.s2;
            const float fsB = (float)A.sB;
            for (int j = jg; j < mp; j += RSTEP) {
                const bool live = valid && j < A.m;
                const double* xj = A.X + (size_t)j * 4;
                const float t0 = (float)(px - xj[0]) * fie0, t1 = (float)(py - xj[1]) * fie1,
                            t2 = (float)(pz - xj[2]) * fie2;
                const float r2 = fmaf(t2, t2, fmaf(t1, t1, t0 * t0));
                const float b = live ? kernel_val32(A.kp.kind, fs2, r2) : 0.0f;
                part[0] = fma((double)b, A.a[j], part[0]);
                if constexpr (P::KS == 32) {
                    Elem hi, lo;
                    split16(P::kScaled ? b * fsB : b, hi, lo);
                    Bt[(size_t)pc * ldb + j] = hi;
                    Bt[(size_t)(NT + pc) * ldb + j] = lo;
                } else {
                    Bt[(size_t)pc * ldb + j] = (Elem)b;
                }
            }
        } else
        for (int j = jg; j < mp; j += RSTEP) {
            const bool live = valid && j < A.m;
            const double* xj = A.X + (size_t)j * 4;
            const double dx = px - xj[0], dy = py - xj[1], dz = pz - xj[2];
            const double t0 = dx * ie0, t1 = dy * ie1, t2 = dz * ie2;
            const double r2 = fma(t2, t2, fma(t1, t1, t0 * t0));
            const double aj = A.a[j];
            double b[G];
            if (G == 1) {
                b[0] = live ? kernel_val(A.kp, r2) : 0.0;
            } else {
                double kv = 0.0, f = 0.0;
                if (live) kernel_val_dfac(A.kp, r2, &kv, &f);
                b[0] = kv;
                const double dd[3] = {dx * ie0 * ie0, dy * ie1 * ie1, dz * ie2 * ie2};
#pragma unroll
                for (int d = 0; d < G - 1; ++d) b[d + 1] = (d < 3) ? f * dd[d] : 0.0;
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                part[g] = fma(b[g], aj, part[g]);
                const int c = pc * G + g;
                if constexpr (P::KS == 32) {
                    double bs = b[g];
                    if constexpr (P::kScaled) bs *= A.sB;
                    Elem hi, lo;
                    split16((float)bs, hi, lo);
                    Bt[(size_t)c * ldb + j] = hi;
                    Bt[(size_t)(NT + c) * ldb + j] = lo;
                } else {
                    Bt[(size_t)c * ldb + j] = (Elem)b[g];
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) red[jg * NT + pc * G + g] = part[g];
        __syncthreads();
        if (tid < NT) {
            double s = 0.0;
            for (int w = 0; w < RSTEP; ++w) s += red[w * NT + tid];
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
        // epilogue of one finished 16-row block: norm / gradient dot partials and V stores
        auto epilogue = [&](int rb, typename P::Acc (&acc)[NCT]) {
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
                    // quad-major V: rows 4 q .. 4 q + 3 of column p at (q * n_points + p) * 4.
                    // The binary64 MFMA leaves row gl + 4 r of the block in register r (binary32:
                    // row 4 gl + r); quad-major binary64 V keeps that order, a permutation of the
                    // rows inside each 16-row block that no dot product of two columns sees.
                    const int64_t p = col0 + 16 * ct + cl;
                    if (p < npts) {
                        const size_t o = T.vld ? (size_t)p * T.vld + 4 * (4 * rb + gl)
                                               : ((size_t)(4 * rb + gl) * T.n_points + p) * 4;
                        if constexpr (sizeof(Elem) == 8) {
                            if (T.vld) {
                                double* c = (double*)T.V + (size_t)p * T.vld + 16 * rb + gl;
#pragma unroll
                                for (int r = 0; r < 4; ++r) c[4 * r] = acc[ct][r];
                            } else {
                                *(d4*)((double*)T.V + o) = acc[ct];
                            }
                        } else {
                            *(f4*)((float*)T.V + o) = f4{(float)acc[ct][0], (float)acc[ct][1], (float)acc[ct][2],
                                                         (float)acc[ct][3]};
                        }
                    }
                }
            }
        };
        // Each wave owns the row-block pair (2NW q + w, 2NW q + 2NW - 1 - w) of every group of
        // 2NW (equal triangular work per wave) and runs both in one k loop, so each B fragment
        // read from LDS feeds both.  k-steps run in groups of U with two fragment buffers in
        // ping-pong: the L^-1 fragments of group g + U are requested before group g is
        // multiplied.  Loop bounds are rounded up to 2U k-steps (m_pad is a multiple of 128,
        // so no group leaves the padded matrix; steps past the diagonal multiply zeros).
        const int wp = wave * ways + spart;            // this wave's pair within each group
        for (int q = 0; q * 2 * NW < A.nrb; ++q) {
            const int ra = 2 * NW * q + wp, rbb = 2 * NW * q + 2 * NW - 1 - wp;
            if (wp >= NW || ra >= A.nrb) continue;     // then rbb >= nrb as well
            const bool hasB = rbb < A.nrb;
            typename P::Acc accA[NCT], accB[NCT];
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
                accA[ct] = typename P::Acc{0, 0, 0, 0};
                accB[ct] = typename P::Acc{0, 0, 0, 0};
            }
            constexpr int U = P::KS == 4 ? 4 : 2;
            bool ra_done = false;
            const int needA = T.dense ? nks_total : (16 * (ra + 1) + P::KS - 1) / P::KS;
            const int needB = T.dense ? nks_total : (16 * (rbb + 1) + P::KS - 1) / P::KS;
            const int gA = (needA + 2 * U - 1) / (2 * U) * (2 * U);
            const int gB = hasB ? (needB + 2 * U - 1) / (2 * U) * (2 * U) : gA;
            const int glast = nks_total - U;
            if constexpr (P::KS == 4) {
                const Elem* AfA = (const Elem*)A.A0 + ((size_t)ra * nks_total) * 64 + lane;
                const Elem* AfB = (const Elem*)A.A0 + ((size_t)(hasB ? rbb : ra) * nks_total) * 64 + lane;
                auto mf = [&](Elem a, Elem b, typename P::Acc c) {
                    if constexpr (sizeof(Elem) == 8) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
                    else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
                };
                auto ld = [&](Elem (&d)[U], const Elem* Af, int g) {
                    g = g < glast ? g : glast;
#pragma unroll
                    for (int u = 0; u < U; ++u) d[u] = Af[(size_t)(g + u) * 64];
                };
                auto mul2 = [&](int g, const Elem (&xa)[U], const Elem (&xb)[U]) {
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int ct = 0; ct < NCT; ++ct) {
                            const Elem bv = Bt[(size_t)(16 * ct + cl) * ldb + 4 * (g + u) + gl];
                            accB[ct] = mf(xb[u], bv, accB[ct]);
                            accA[ct] = mf(xa[u], bv, accA[ct]);
                        }
                };
                auto mul1 = [&](int g, const Elem (&x)[U], typename P::Acc (&acc)[NCT]) {
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int ct = 0; ct < NCT; ++ct) {
                            const Elem bv = Bt[(size_t)(16 * ct + cl) * ldb + 4 * (g + u) + gl];
                            acc[ct] = mf(x[u], bv, acc[ct]);
                        }
                };
                Elem a0[U], a1[U], b0[U], b1[U];
                if (hasB) {
                    ld(a0, AfA, 0);
                    ld(b0, AfB, 0);
                    for (int g = 0; g < gA; g += 2 * U) {
                        ld(a1, AfA, g + U);
                        ld(b1, AfB, g + U);
                        mul2(g, a0, b0);
                        ld(a0, AfA, g + 2 * U);
                        ld(b0, AfB, g + 2 * U);
                        mul2(g + U, a1, b1);
                    }
                    if constexpr (SPLIT && G == 1) {
                        // one busy wave per SIMD: block ra is complete, so its accumulator
                        // takes every other group of rbb's tail (two independent chains; the
                        // group-4 kernel has no registers to spare for it)
                        if (gA < gB) {
                            epilogue(ra, accA);
                            ra_done = true;
#pragma unroll
                            for (int ct = 0; ct < NCT; ++ct) accA[ct] = typename P::Acc{0, 0, 0, 0};
                            for (int g = gA; g < gB; g += 2 * U) {
                                ld(b1, AfB, g + U);
                                mul1(g, b0, accB);
                                ld(b0, AfB, g + 2 * U);
                                mul1(g + U, b1, accA);
                            }
#pragma unroll
                            for (int ct = 0; ct < NCT; ++ct) accB[ct] += accA[ct];
                        }
                    } else {
                        for (int g = gA; g < gB; g += 2 * U) {     // b0 holds group g
                            ld(b1, AfB, g + U);
                            mul1(g, b0, accB);
                            ld(b0, AfB, g + 2 * U);
                            mul1(g + U, b1, accB);
                        }
                    }
                } else {
                    ld(a0, AfA, 0);
                    for (int g = 0; g < gA; g += 2 * U) {
                        ld(a1, AfA, g + U);
                        mul1(g, a0, accA);
                        ld(a0, AfA, g + 2 * U);
                        mul1(g + U, a1, accA);
                    }
                }
            } else {
                using Vec = typename P::Vec;
                const size_t oA = ((size_t)ra * nks_total) * 64 + lane;
                const size_t oB = ((size_t)(hasB ? rbb : ra) * nks_total) * 64 + lane;
                const Vec* AhA = (const Vec*)A.A0 + oA;
                const Vec* AlA = (const Vec*)A.A1 + oA;
                const Vec* AhB = (const Vec*)A.A0 + oB;
                const Vec* AlB = (const Vec*)A.A1 + oB;
                auto ld = [&](Vec (&h)[U], Vec (&l)[U], const Vec* Ah, const Vec* Al, int g) {
                    g = g < glast ? g : glast;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        h[u] = Ah[(size_t)(g + u) * 64];
                        l[u] = Al[(size_t)(g + u) * 64];
                    }
                };
                auto mulg = [&](int g, const Vec (&ha)[U], const Vec (&la)[U], const Vec (&hb)[U],
                                const Vec (&lb)[U], bool doA, bool doB) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        Vec bh[NCT], bl[NCT];
#pragma unroll
                        for (int ct = 0; ct < NCT; ++ct) {
                            const size_t off = (size_t)(16 * ct + cl) * ldb + 32 * (g + u) + 8 * gl;
                            bh[ct] = *(const Vec*)(Bt + off);
                            bl[ct] = *(const Vec*)(Bt + (size_t)NT * ldb + off);
                        }
                        if (doB) {
#pragma unroll
                            for (int ct = 0; ct < NCT; ++ct) {
                                accB[ct] = mfma16(lb[u], bh[ct], accB[ct]);
                                accB[ct] = mfma16(hb[u], bl[ct], accB[ct]);
                                accB[ct] = mfma16(hb[u], bh[ct], accB[ct]);
                            }
                        }
                        if (doA) {
#pragma unroll
                            for (int ct = 0; ct < NCT; ++ct) {
                                accA[ct] = mfma16(la[u], bh[ct], accA[ct]);
                                accA[ct] = mfma16(ha[u], bl[ct], accA[ct]);
                                accA[ct] = mfma16(ha[u], bh[ct], accA[ct]);
                            }
                        }
                    }
                };
                Vec ha0[U], la0[U], hb0[U], lb0[U], ha1[U], la1[U], hb1[U], lb1[U];
                if (hasB) {
                    ld(ha0, la0, AhA, AlA, 0);
                    ld(hb0, lb0, AhB, AlB, 0);
                    for (int g = 0; g < gA; g += 2 * U) {
                        ld(ha1, la1, AhA, AlA, g + U);
                        ld(hb1, lb1, AhB, AlB, g + U);
                        mulg(g, ha0, la0, hb0, lb0, true, true);
                        ld(ha0, la0, AhA, AlA, g + 2 * U);
                        ld(hb0, lb0, AhB, AlB, g + 2 * U);
                        mulg(g + U, ha1, la1, hb1, lb1, true, true);
                    }
                    for (int g = gA; g < gB; g += 2 * U) {
                        ld(hb1, lb1, AhB, AlB, g + U);
                        mulg(g, ha0, la0, hb0, lb0, false, true);
                        ld(hb0, lb0, AhB, AlB, g + 2 * U);
                        mulg(g + U, ha1, la1, hb1, lb1, false, true);
                    }
                } else {
                    ld(ha0, la0, AhA, AlA, 0);
                    for (int g = 0; g < gA; g += 2 * U) {
                        ld(ha1, la1, AhA, AlA, g + U);
                        mulg(g, ha0, la0, hb0, lb0, true, false);
                        ld(ha0, la0, AhA, AlA, g + 2 * U);
                        mulg(g + U, ha1, la1, hb1, lb1, true, false);
                    }
                }
            }
            if (!ra_done) epilogue(ra, accA);
            if (hasB) epilogue(rbb, accB);
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
        if (tid < 64) {   // wave 0: lane c < NT holds column col0 + c
            double dot = 0.0, mc = 0.0;
            const int64_t col = col0 + tid;
            const int64_t p = col / G;
            const int comp = (int)(col % G);
            if (tid < NT)
                for (int w = 0; w < kWaves; ++w) dot += red[w * NT + tid];
            if (SPLIT && ways > 1) {
                double* sp = T.sp_part + ((int64_t)tile * ways) * NT;
                if (tid < NT) __hip_atomic_store(sp + spart * NT + tid, dot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                int last = 0;
                // release this work-group's partials; the last arrival acquires all of them
                if (tid == 0)
                    last = __hip_atomic_fetch_add(T.sp_cnt + tile, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
                                   ways - 1 ? 1 : 0;
                last = __shfl(last, 0, 64);
                if (!last) continue;                   // another work-group of this tile finishes it
                dot = 0.0;
                if (tid < NT)
                    for (int r = 0; r < ways; ++r)
                        dot += __hip_atomic_load(sp + r * NT + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (tid == 0) T.sp_cnt[tile] = 0;
            }
            if (tid < NT) {
                mc = mucol[tid];
                if (p < npts) {
                    if (comp == 0) {
                        T.mean[p] = mc;
                        double v = A.kp.s2 - dot;
                        T.var[p] = v > 0.0 ? v : 0.0;
                    } else if (comp - 1 < dim) {
                        T.dmean[p * 3 + comp - 1] = mc;
                        T.dvar[p * 3 + comp - 1] = -2.0 * dot;
                    }
                }
            }
            if constexpr (std::is_same<P, P64>::value && G == 4) {
                if (T.epi == EPI_STEP) search_step(A, p, comp, dot, mc, tid < NT && p < npts);
            }
        }
    }
}

template <class P, int NT, int G, int NW>
__global__ void __launch_bounds__(NW * 64) k_post(KArgs A)
{
    post_tiles<P, NT, G, NW>(A, blockIdx.x, gridDim.x, INT64_MAX);
}

// Small launches of the region search: a fixed grid, tiles shared by W work-groups when few.
template <class P, int NT, int G, int NW>
__global__ void __launch_bounds__(NW * 64) k_post_sp(KArgs A)
{
    post_tiles<P, NT, G, NW, true>(A, blockIdx.x, gridDim.x, INT64_MAX);
}

// Many models in one launch: model b owns tiles tile_off[b] .. tile_off[b + 1] - 1 of the
// batch; work-groups walk the batch's tiles, so small models share the GPU with large ones.
template <class P, int NT, int NW>
__global__ void __launch_bounds__(NW * 64) k_post_batch(const KArgs* __restrict__ As,
                                                        const int64_t* __restrict__ tile_off, int nb)
{
    const int64_t total = tile_off[nb];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        int lo = 0, hi = nb - 1;                // last b with tile_off[b] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_off[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const int64_t t = item - tile_off[lo];
        post_tiles<P, NT, 1, NW>(As[lo], t, 1, t + 1);
    }
}

// Calls f(integral_constant<int, K>) for K = B .. E - 1 in order.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int kChunk = 32;          // B rows per k-step of the 16-bit split product

// ---------------------------------------------------------------- split-product kernel
//
// Value columns with the 16-bit split operands (the reconstruction's posterior).  A
// work-group owns a tile of NT columns and runs two kinds of waves:
//  - eight consumer waves (two per SIMD) hold V = L^-1 B for the tile in registers, consumer
//    w owning row blocks w + 8 r.  B arrives in chunks of 32 rows (one MFMA k-step) through
//    a double-buffered LDS slice; row block rb takes chunks 0 .. rb / 2, so a consumer runs
//    its chunk loop in phases, with the row blocks r >= K live in phase K (each phase body is
//    one branch-free basic block).  A row block is final at the end of its phase; its
//    epilogue undoes the power-of-two scales, adds the binary64 ||v||^2 partial and stores V.
//    The next chunk's L^-1 fragments are loaded before each barrier, so their L2 latency
//    overlaps the wait and the B fragment reads.
//  - four producer waves (one per SIMD) generate the next chunk of B: binary32 kernel values
//    (the kind is a template parameter, so this is straight-line code), the binary64 mean
//    partials and the 16-bit split.  A producer wave's rows are the same for all its lanes.
//    The observations (pre-scaled by the inverse lengthscales, with a_j) are copied to LDS
//    once per work-group, and a producer issues all of a chunk's broadcast reads before their
//    first use, so it waits for LDS once per chunk (scalar loads of the same rows waited on
//    the scalar cache twice per chunk: 4 % slower).  The FP16 scale sB is folded into the
//    kernel's constants and taken out of the mean at the end (powers of two: exact).
// A SIMD so runs two instruction streams of MFMAs beside one of vector arithmetic, which
// overlap between the per-chunk barriers.  Each column's k-steps accumulate in increasing
// order, three products per step in a fixed order, and its sums run in a fixed order, so a
// vertex gets bitwise the same numbers in any tile or launch.
constexpr int kThreadsPS = 768;
constexpr int kConsPS = 8;        // consumer waves 0..7; producers are waves 8..11

template <int KIND>
__device__ __forceinline__ float kval32_scaled(float r2, float c0, float c1, float c2)
{
    constexpr float kLog2e = 1.44269504088896341f;
    if constexpr (KIND == LCP_KERNEL_SE) {
        (void)c1;
        (void)c2;
        return c0 * __builtin_amdgcn_exp2f(-0.5f * kLog2e * r2);
    } else {
        const float r = __builtin_amdgcn_sqrtf(r2);
        const float poly = fmaf(c1, r, fmaf(c2, r2, c0));          // s2' (1 + sqrt5 r + 5 r^2 / 3)
        return poly * __builtin_amdgcn_exp2f(-2.23606797749978970f * kLog2e * r);
    }
}

template <class P, int NT, int RBW, int KIND>
__global__ void __launch_bounds__(kThreadsPS) k_post_ps(KArgs A)
{
    static_assert(P::KS == 32, "split-product operands");
    using Elem = typename P::Elem;
    using Vec = typename P::Vec;
    constexpr int NCT = NT / 16;
    constexpr int LDC = kChunk + 8;
    constexpr int NPW = 4;                                   // producer waves
    constexpr int RPT = kChunk / NPW;                        // rows per producer lane per chunk
    static_assert(NT == 64 || NT == 32, "tile width");
    __shared__ __align__(16) Elem Bs[2][2][NT][LDC];
    __shared__ double red[kConsPS][NT];
    __shared__ double redm[NPW][NT];
    // the observations of every chunk, pre-scaled, with a_j: 32 bytes per row (row count 32 nch
    // <= 16 kConsPS RBW)
    __shared__ __align__(16) double Xsh[kConsPS * RBW * 16 * 4];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool consumer = wave < kConsPS;
    const int gl = lane >> 4, cl = lane & 15;
    const PostTask& T = A.t;
    int64_t npts = T.count ? *T.count : T.n_points;
    if (npts > T.n_points) npts = T.n_points;
    const int64_t ntiles = (npts + NT - 1) / NT;
    const int dim = A.kp.dim;
    const int nks_total = A.mp / P::KS;
    const int nch = (A.nrb + 1) / 2;

    // producer wave pw serves rows 32 c + RPT pw .. + RPT - 1 of every chunk c (the same for
    // all its lanes) for column gc = lane % NT; with 32-column tiles lanes 32..63 repeat
    // lanes 0..31 and store nothing
    const int pw = wave - kConsPS;
    const int gc = lane & (NT - 1);
    const bool pstore = lane < NT;
    const double ie0 = A.kp.inv_ell[0], ie1 = A.kp.inv_ell[1], ie2 = A.kp.inv_ell[2];
    const double sB = P::kScaled ? A.sB : 1.0;
    const float c0 = (float)(A.kp.s2 * sB);
    const float c1 = (float)(2.23606797749978969640917366873 * A.kp.s2 * sB);
    const float c2 = (float)((5.0 / 3.0) * A.kp.s2 * sB);
    const float inv = P::kScaled ? (float)(1.0 / (A.amax[1] * A.sB)) : 1.0f;   // a power of two
    const Vec* __restrict__ Ahi = (const Vec*)A.A0;
    const Vec* __restrict__ Alo = (const Vec*)A.A1;
    // the chunks' observation rows into LDS, ordered before their first use by the tile barrier
    for (int i = tid; i < kChunk * nch * 4; i += kThreadsPS) Xsh[i] = A.Xs[i];

    const int cw = wave;                                     // consumer wave: row blocks cw + 8 r
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t col0 = tile * NT;
        __syncthreads();                                     // previous tile's LDS reads are complete
        if (!consumer) {
            // ------------------------------------------------------------ producer
            const int64_t p = col0 + gc;
            double px = 0.0, py = 0.0, pz = 0.0;             // an invalid column stays finite
            if (p < npts) {
                if (T.mode == COL_GRID) {
                    const int64_t v = T.vlist ? (int64_t)T.vlist[p] : p;
                    const int64_t i0 = v % T.grid.n[0];
                    const int64_t r = v / T.grid.n[0];
                    px = vertex_coord(T.grid, 0, i0);
                    py = vertex_coord(T.grid, 1, r % T.grid.n[1]);
                    pz = dim > 2 ? vertex_coord(T.grid, 2, r / T.grid.n[1]) : 0.0;
                } else {
                    px = T.pts[p * T.pstride + 0];
                    py = T.pts[p * T.pstride + 1];
                    pz = dim > 2 ? T.pts[p * T.pstride + 2] : 0.0;
                }
            }
            px = mul_rn(px, ie0);
            py = mul_rn(py, ie1);
            pz = mul_rn(pz, ie2);
            double mpart = 0.0;
            auto generate = [&](int c, int b) {
                // rows j0 .. j0 + RPT - 1 < 32 nch <= m_pad (m_pad is a multiple of 128); rows
                // past m sit at 1e15 lengthscales with a_j = 0, so their values are exactly 0
                float kv[RPT];
                // the wave's rows, read by every lane from one LDS address (a broadcast); all
                // reads are issued before the first use
                const double2* Xj = (const double2*)&Xsh[4 * (kChunk * c + RPT * pw)];
                double2 xa[RPT], xb[RPT];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    xa[i] = Xj[2 * i];
                    xb[i] = Xj[2 * i + 1];
                }
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const double x0 = xa[i].x, x1 = xa[i].y, x2 = xb[i].x, aj = xb[i].y;
                    const float t0 = (float)(px - x0), t1 = (float)(py - x1), t2 = (float)(pz - x2);
                    const float r2 = fmaf(t2, t2, fmaf(t1, t1, t0 * t0));
                    kv[i] = kval32_scaled<KIND>(r2, c0, c1, c2);
                    mpart = fma((double)kv[i], aj, mpart);
                }
                typedef Elem EV __attribute__((ext_vector_type(RPT)));
                EV hi, lo;
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    Elem h, l;
                    split16(kv[i], h, l);
                    hi[i] = h;
                    lo[i] = l;
                }
                if (pstore) {
                    *(EV*)&Bs[b][0][gc][RPT * pw] = hi;
                    *(EV*)&Bs[b][1][gc][RPT * pw] = lo;
                }
            };
            generate(0, 0);
            __syncthreads();
            for (int c = 0; c < nch; ++c) {
                if (c + 1 < nch) generate(c + 1, (c + 1) & 1);
                __syncthreads();
            }
            if (pstore) redm[pw][gc] = mpart;
        } else {
            // ------------------------------------------------------------ consumer
            f4 acc[RBW][NCT];
#pragma unroll
            for (int r = 0; r < RBW; ++r)
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct) acc[r][ct] = f4{0, 0, 0, 0};
            double dacc[NCT];
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) dacc[ct] = 0.0;
            Vec ah[RBW], al[RBW];
            auto load_a = [&](auto Kc, int c) {
                constexpr int K = decltype(Kc)::value;
#pragma unroll
                for (int r = K; r < RBW; ++r) {
                    int rb = cw + kConsPS * r;
                    rb = rb < A.nrb ? rb : A.nrb - 1;          // a missing row block is never stored
                    const size_t o = ((size_t)rb * nks_total + c) * 64 + lane;
                    ah[r] = Ahi[o];
                    al[r] = Alo[o];
                }
            };
            auto epilogue = [&](int rb, f4 (&ac)[NCT]) {
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct) {
                    if constexpr (P::kScaled) ac[ct] *= inv;
                    const double v0 = (double)ac[ct][0], v1 = (double)ac[ct][1];
                    const double v2 = (double)ac[ct][2], v3 = (double)ac[ct][3];
                    dacc[ct] += fma(v0, v0, v1 * v1) + fma(v2, v2, v3 * v3);
                    if (T.V) {
                        const int64_t pc = col0 + 16 * ct + cl;
                        if (pc < npts) {
                            const size_t o = T.vld ? (size_t)pc * T.vld + 16 * rb + 4 * gl
                                                   : ((size_t)(4 * rb + gl) * T.n_points + pc) * 4;
                            *(f4*)((float*)T.V + o) = ac[ct];
                        }
                    }
                }
            };
            // chunk c with row blocks r >= K live; then the next chunk's A fragments
            auto body = [&](auto Kc, int c) {
                constexpr int K = decltype(Kc)::value;
                const int b = c & 1;
                Vec bh[NCT], bl[NCT];
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct) {
                    bh[ct] = *(const Vec*)&Bs[b][0][16 * ct + cl][8 * gl];
                    bl[ct] = *(const Vec*)&Bs[b][1][16 * ct + cl][8 * gl];
                }
#pragma unroll
                for (int r = K; r < RBW; ++r)
#pragma unroll
                    for (int ct = 0; ct < NCT; ++ct) {
                        acc[r][ct] = mfma16(al[r], bh[ct], acc[r][ct]);
                        acc[r][ct] = mfma16(ah[r], bl[ct], acc[r][ct]);
                        acc[r][ct] = mfma16(ah[r], bh[ct], acc[r][ct]);
                    }
                load_a(Kc, c + 1 < nch ? c + 1 : nch - 1);
                __syncthreads();
            };
            auto phase = [&](auto Kc, int& c) {
                constexpr int K = decltype(Kc)::value;
                const int rbK = cw + kConsPS * K;
                const int cend = (!T.dense && rbK / 2 < nch - 1) ? rbK / 2 : nch - 1;
                for (; c <= cend; ++c) body(Kc, c);
                if (rbK < A.nrb) epilogue(rbK, acc[K]);
            };
            load_a(std::integral_constant<int, 0>{}, 0);
            __syncthreads();                                 // chunk 0 generated
            int c = 0;
            static_for<0, RBW>([&](auto Kc) { phase(Kc, c); });
            for (; c < nch; ++c) __syncthreads();
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
                double sum = dacc[ct];
                sum += __shfl_xor(sum, 16, 64);
                sum += __shfl_xor(sum, 32, 64);
                if (gl == 0) red[cw][16 * ct + cl] = sum;
            }
        }
        __syncthreads();
        if (tid < NT) {
            double mu = 0.0, dot = 0.0;
            for (int g = 0; g < NPW; ++g) mu += redm[g][tid];
            for (int w = 0; w < kConsPS; ++w) dot += red[w][tid];
            const int64_t pc = col0 + tid;
            if (pc < npts) {
                T.mean[pc] = mu / sB;
                const double v = A.kp.s2 - dot;
                T.var[pc] = v > 0.0 ? v : 0.0;
            }
        }
    }
}

template <class P, int NT, int RBW, int KIND>
hipError_t launch_ps(const Model& M, const PostTask& t, hipStream_t s, const void* A0, const void* A1,
                     const double* amax)
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
    A.amax = amax ? amax : M.amax;
    {
        int e;
        frexp(M.k.signal_var, &e);
        A.sB = ldexp(1.0, 15 - e);          // k* <= s2, so sB * k* < 2^15
    }
    A.Xs = M.Xs;
    A.t = t;
    if (A.nrb > kConsPS * RBW) return hipErrorInvalidValue;
    const int64_t ntiles = (t.n_points + NT - 1) / NT;
    int64_t grid = ntiles < 256 * 8 ? ntiles : 256 * 8;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_post_ps<P, NT, RBW, KIND>), dim3((unsigned)grid), dim3(kThreadsPS), 0, s, A);
    return hipGetLastError();
}

template <class P, int NT, int RBW>
hipError_t launch_ps_kind(const Model& M, const PostTask& t, hipStream_t s, const void* A0, const void* A1,
                          const double* amax)
{
    if (M.kp.kind == LCP_KERNEL_SE) return launch_ps<P, NT, RBW, LCP_KERNEL_SE>(M, t, s, A0, A1, amax);
    return launch_ps<P, NT, RBW, LCP_KERNEL_MATERN52>(M, t, s, A0, A1, amax);
}

template <class P>
hipError_t launch_split(const Model& M, const PostTask& t, hipStream_t s, const void* A0, const void* A1,
                        const double* amax = nullptr)
{
    switch ((M.nrb + kConsPS - 1) / kConsPS) {
    case 1: return launch_ps_kind<P, 64, 1>(M, t, s, A0, A1, amax);
    case 2: return launch_ps_kind<P, 64, 2>(M, t, s, A0, A1, amax);
    case 3: return launch_ps_kind<P, 64, 3>(M, t, s, A0, A1, amax);
    case 4: return launch_ps_kind<P, 64, 4>(M, t, s, A0, A1, amax);
    default: return launch_ps_kind<P, 32, 8>(M, t, s, A0, A1, amax);
    }
}

static KArgs kargs_of(const Model& M, const PostTask& t, const void* A0, const void* A1)
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
    return A;
}

template <class P, int NT, int G, int NW = kWaves>
hipError_t launch_t(const Model& M, const PostTask& t, hipStream_t s, const void* A0, const void* A1)
{
    KArgs A = kargs_of(M, t, A0, A1);
    int ldb = (P::KS == 32) ? (M.m_pad + 63) / 64 * 64 + P::LPAD : M.m_pad + P::LPAD;
    size_t lds = sizeof(typename P::Elem) * (size_t)lds_planes<P>() * NT * ldb + sizeof(double) * (NW * 64 * G + NT);
    if (NW == 16 && t.sp_cnt) {
        // a fixed grid of one work-group per CU; the kernel shares small tile counts among them
        hipError_t e = hipFuncSetAttribute((const void*)k_post_sp<P, NT, G, NW>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_post_sp<P, NT, G, NW>), dim3(kSplitGrid), dim3(NW * 64), lds, s, A);
        return hipGetLastError();
    }
    hipError_t e = hipFuncSetAttribute((const void*)k_post<P, NT, G, NW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    int64_t ncols = t.n_points * G;
    int64_t ntiles = (ncols + NT - 1) / NT;
    int dev_cus = 256;
    int64_t grid = ntiles < (int64_t)dev_cus * 8 ? ntiles : (int64_t)dev_cus * 8;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_post<P, NT, G, NW>), dim3((unsigned)grid), dim3(NW * 64), lds, s, A);
    return hipGetLastError();
}

}  // namespace

// One launch over the listed models (idx) with tiles of NT columns and NW waves.
template <class P, int NT, int NW>
static hipError_t launch_batch_t(const Model* const* Ms, const PostTask* tasks, const std::vector<int>& idx,
                                 char* scratch, hipStream_t s, const void* const* A0, const void* const* A1)
{
    const int nb = (int)idx.size();
    if (nb == 0) return hipSuccess;
    std::vector<KArgs> KA(nb);
    std::vector<int64_t> toff(nb + 1, 0);
    int mpmax = 0;
    for (int i = 0; i < nb; ++i) {
        const int b = idx[i];
        KA[i] = kargs_of(*Ms[b], tasks[b], A0[b], A1[b]);
        toff[i + 1] = toff[i] + (tasks[b].n_points + NT - 1) / NT;
        if (Ms[b]->m_pad > mpmax) mpmax = Ms[b]->m_pad;
    }
    KArgs* KAd = (KArgs*)scratch;
    int64_t* toffd = (int64_t*)(scratch + align256(sizeof(KArgs) * (size_t)nb));
    hipError_t e = hipMemcpyAsync(KAd, KA.data(), sizeof(KArgs) * nb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(toffd, toff.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, s);
    // pageable sources: wait for the copies so the host vectors may go
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (toff[nb] == 0) return hipSuccess;
    const int ldb = (P::KS == 32) ? (mpmax + 63) / 64 * 64 + P::LPAD : mpmax + P::LPAD;
    const size_t lds = sizeof(typename P::Elem) * (size_t)lds_planes<P>() * NT * ldb + sizeof(double) * (NW * 64 + NT);
    e = hipFuncSetAttribute((const void*)k_post_batch<P, NT, NW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
    const int64_t grid = toff[nb] < 256 * 8 ? toff[nb] : 256 * 8;
    hipLaunchKernelGGL((k_post_batch<P, NT, NW>), dim3((unsigned)grid), dim3(NW * 64), lds, s, KAd, toffd, nb);
    return hipGetLastError();
}

// ------------------------------------------------------------- batched posterior tiles
//
// Tile width (columns per work-group) and waves per work-group of the batched posterior,
// per precision and size class c (m_pad = 128 (c + 1)).  The defaults are the autotuner's
// measured choices (paper_2512_12442_amd/autotune.py writes tune_table.inc); lcp_batch_tiles
// overrides them.  Candidates: tile width 16 or 32, 4, 8 or 16 waves, whose B tile fits LDS.
struct TileCfg {
    int nt, nw;
};

constexpr int kSizeClasses = kMaxM / 128;
#include "tune_table.inc"          // static const TileCfg kTunedTiles[4][kSizeClasses]
static TileCfg g_tiles[4][kSizeClasses];
static bool g_tiles_init = false;

static size_t batch_lds_bytes(int prec, int nt, int nw, int mp)
{
    const bool split = prec == LCP_MIXED_F16X3 || prec == LCP_MIXED_BF16X3;
    const int ldb = split ? (mp + 63) / 64 * 64 + 8 : mp + (prec == LCP_FP64 ? 1 : 2);
    const size_t elem = prec == LCP_FP64 ? 8 : (prec == LCP_FP32 ? 4 : 2);
    return elem * (split ? 2 : 1) * (size_t)nt * ldb + sizeof(double) * (nw * 64 + nt);
}

static bool tile_valid(int prec, int cls, int nt, int nw)
{
    return (nt == 16 || nt == 32) && (nw == 4 || nw == 8 || nw == 16) &&
           batch_lds_bytes(prec, nt, nw, 128 * (cls + 1)) <= 160 * 1024;
}

static TileCfg tiles_of(int prec, int cls)
{
    if (!g_tiles_init) {
        for (int p = 0; p < 4; ++p)
            for (int c = 0; c < kSizeClasses; ++c) g_tiles[p][c] = kTunedTiles[p][c];
        g_tiles_init = true;
    }
    return g_tiles[prec][cls];
}

int set_batch_tiles(int prec, int cls, int nt, int nw)
{
    if (prec < 0 || prec > 3 || cls < 0 || cls >= kSizeClasses) return -1;
    tiles_of(prec, cls);
    if (nt == 0) {
        g_tiles[prec][cls] = kTunedTiles[prec][cls];
        return 0;
    }
    if (!tile_valid(prec, cls, nt, nw)) return -1;
    g_tiles[prec][cls] = TileCfg{nt, nw};
    return 0;
}

void get_batch_tiles(int prec, int cls, int* nt, int* nw)
{
    const TileCfg t = tiles_of(prec, cls);
    *nt = t.nt;
    *nw = t.nw;
}

template <class P>
static hipError_t launch_batch_cfg(TileCfg c, const Model* const* Ms, const PostTask* tasks, const std::vector<int>& idx,
                                   char* scratch, hipStream_t s, const void* const* A0, const void* const* A1)
{
    switch (c.nt * 100 + c.nw) {
    case 1604: return launch_batch_t<P, 16, 4>(Ms, tasks, idx, scratch, s, A0, A1);
    case 1608: return launch_batch_t<P, 16, 8>(Ms, tasks, idx, scratch, s, A0, A1);
    case 1616: return launch_batch_t<P, 16, 16>(Ms, tasks, idx, scratch, s, A0, A1);
    case 3204: return launch_batch_t<P, 32, 4>(Ms, tasks, idx, scratch, s, A0, A1);
    case 3208: return launch_batch_t<P, 32, 8>(Ms, tasks, idx, scratch, s, A0, A1);
    case 3216: return launch_batch_t<P, 32, 16>(Ms, tasks, idx, scratch, s, A0, A1);
    default: return hipErrorInvalidValue;
    }
}

size_t posterior_batch_scratch(int nb)
{
    // the records of one launch (the size-class launches reuse them in stream order)
    return align256(sizeof(KArgs) * (size_t)nb) + align256(sizeof(int64_t) * (size_t)(nb + 1));
}

hipError_t launch_posterior_batch(const Model* const* Ms, const PostTask* tasks, int nb, int prec, char* scratch,
                                  hipStream_t s)
{
    if (nb <= 0) return hipSuccess;
    StageScope sc(s, ST_POSTERIOR);
    std::vector<const void*> A0(nb), A1(nb);
    for (int b = 0; b < nb; ++b) {
        const Model& M = *Ms[b];
        A0[b] = prec == LCP_FP64 ? (const void*)M.A64 : prec == LCP_FP32 ? (const void*)M.A32
              : prec == LCP_MIXED_F16X3 ? (const void*)M.Hhi : (const void*)M.Ahi;
        A1[b] = prec == LCP_MIXED_F16X3 ? (const void*)M.Hlo : prec == LCP_MIXED_BF16X3 ? (const void*)M.Alo : nullptr;
    }
    // one launch per size class, with that class's tile configuration
    std::vector<std::vector<int>> cls(kSizeClasses);
    for (int b = 0; b < nb; ++b) cls[Ms[b]->m_pad / 128 - 1].push_back(b);
    for (int c = 0; c < kSizeClasses; ++c) {
        if (cls[c].empty()) continue;
        const TileCfg t = tiles_of(prec, c);
        hipError_t e;
        if (prec == LCP_FP64) e = launch_batch_cfg<P64>(t, Ms, tasks, cls[c], scratch, s, A0.data(), A1.data());
        else if (prec == LCP_FP32) e = launch_batch_cfg<P32>(t, Ms, tasks, cls[c], scratch, s, A0.data(), A1.data());
        else if (prec == LCP_MIXED_F16X3) e = launch_batch_cfg<PH3>(t, Ms, tasks, cls[c], scratch, s, A0.data(), A1.data());
        else e = launch_batch_cfg<PB3>(t, Ms, tasks, cls[c], scratch, s, A0.data(), A1.data());
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_posterior_operand(const Model& M, int prec, const PostTask& t, const void* A0, hipStream_t s)
{
    if (t.n_points <= 0) return hipSuccess;
    StageScope sc(s, t.stage);
    if (t.group != 1) return hipErrorInvalidValue;
    if (prec == LCP_FP64) return launch_t<P64, 16, 1>(M, t, s, A0, nullptr);
    if (prec == LCP_FP32) return launch_t<P32, 32, 1>(M, t, s, A0, nullptr);
    return hipErrorInvalidValue;
}

hipError_t launch_posterior_operand_f16x3(const Model& M, const PostTask& t, const void* Hhi, const void* Hlo,
                                          const double* amax, hipStream_t s)
{
    if (t.n_points <= 0) return hipSuccess;
    StageScope sc(s, t.stage);
    if (t.group != 1) return hipErrorInvalidValue;
    return launch_split<PH3>(M, t, s, Hhi, Hlo, amax);
}

hipError_t launch_posterior(const Model& M, int prec, const PostTask& t, hipStream_t s)
{
    if (t.n_points <= 0) return hipSuccess;
    StageScope sc(s, t.stage);
    const bool grad = t.group == 4;
    // Tile widths keep B at <= 80 KB of LDS (m_pad <= 1024 / 1152), so two work-groups share
    // a CU and one's B generation (VALU) overlaps the other's MFMA sweep.
    if (prec == LCP_FP64) {
        // launches of at most 2048 tiles (the region bound's probes at coarse levels) run
        // sixteen waves per tile: a quarter of the per-tile latency, one tile per CU
        if (t.n_points * t.group <= 2048 * 16) {
            if (grad) return launch_t<P64, 16, 4, 16>(M, t, s, M.A64, nullptr);
            return launch_t<P64, 16, 1, 16>(M, t, s, M.A64, nullptr);
        }
        // larger launches: eight waves per work-group, two work-groups per CU (measured on
        // the region bound at 128^3: 2.35 -> 2.26 ms against four waves; sixteen gave 2.33)
        if (grad) return launch_t<P64, 16, 4, 8>(M, t, s, M.A64, nullptr);
        return launch_t<P64, 16, 1, 8>(M, t, s, M.A64, nullptr);
    }
    if (prec == LCP_FP32) {
        if (grad) return launch_t<P32, 32, 4>(M, t, s, M.A32, nullptr);
        return launch_t<P32, 32, 1>(M, t, s, M.A32, nullptr);
    }
    // 16-bit split value columns: producer/consumer kernel, RBW = ceil(nrb / 8) row blocks per consumer
    if (prec == LCP_MIXED_F16X3) {
        if (grad) return launch_t<PH3, 32, 4>(M, t, s, M.Hhi, M.Hlo);
        return launch_split<PH3>(M, t, s, M.Hhi, M.Hlo);
    }
    if (grad) return launch_t<PB3, 32, 4>(M, t, s, M.Ahi, M.Alo);
    return launch_split<PB3>(M, t, s, M.Ahi, M.Alo);
}

}  // namespace lcp
