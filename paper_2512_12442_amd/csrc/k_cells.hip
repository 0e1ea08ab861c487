// Cell stage of Sec. 4: cross-covariances between neighbouring vertices, the 2^D-corner
// covariance of each cell, its semidefinite Cholesky factor (binary64), and the Monte
// Carlo crossing count over the shared bank of standard normals.
#include <vector>

#include "lcp_internal.h"

namespace lcp {

namespace {

// Neighbour directions: offsets in {-1,0,1}^D whose last non-zero component is +1
// (13 in 3D, 4 in 2D).  Direction index = base-3 code of (offset + 1) minus (origin code + 1).
__device__ __forceinline__ int dir_index(int D, int dx, int dy, int dz)
{
    if (D == 3) return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1) - 14;
    return (dx + 1) + 3 * (dy + 1) - 5;
}

// Neighbour cross-covariances cross[slot][dir] = k(x_p, x_q) - v_p . v_q, q = p + dir.
//
// One wave owns a run of 62 consecutive vertices of the grid flattened with one padding
// vertex at each end of every x-line (index F = (x + 1) + (n0 + 2) * (y + n1 * z)); lanes
// 1..62 are the outputs, lanes 0 and 63 carry the neighbours just outside the run.  Each
// lane streams the V columns of its own vertex and of the vertices at (y+1, z) and
// (y-1..y+1, z+1), four rows at a time; the x +-1 neighbours are the adjacent lanes,
// reached with wavefront DPP shifts of the own value, so every V element is fetched by
// five lanes and no LDS is used.  Dot products accumulate in binary64.
//
// V is quad-major: rows 4q..4q+3 of column s sit at (q * ldv + s) * 4 (rows 16 rb .. 16 rb
// + 15 of each column hold the MFMA result order of that row block, a fixed permutation
// no dot product of two columns depends on).  Padding vertices and vertices without a
// slot read as zero columns; their pairs are written as NaN.
constexpr int kCrossRun = 62;
// Buffer descriptor word 3 for raw (untyped, unswizzled) buffer access on gfx9-family GPUs.
constexpr int kBufferFlags = 0x00020000;
typedef unsigned u4 __attribute__((ext_vector_type(4)));

// Wavefront DPP shifts: lane i receives lane i + 1 (kFromNext) or lane i - 1 (kFromPrev);
// the lane without a source receives 0.
constexpr int kFromNext = 0x130;   // wave_shl:1
constexpr int kFromPrev = 0x138;   // wave_shr:1

template <int CTRL>
__device__ __forceinline__ float lane_shift(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ int32_t slot_at(const GridP& g, const int32_t* slot, int64_t x, int64_t y, int64_t z)
{
    if (x < 0 || x >= g.n[0] || y < 0 || y >= g.n[1] || z < 0 || z >= g.n[2]) return -1;
    const int64_t vid = x + g.n[0] * (y + g.n[1] * z);
    return slot ? slot[vid] : (int32_t)vid;
}

// A cross-covariance task (one model and grid) and the sources of a kernel's waves: one
// task, or a batch whose waves are numbered consecutively (task b owns woff[b] ..).
struct CrossTask {
    KParams kp;
    GridP g;
    int64_t ldv;
    int nquads;
    const int32_t* slot;
    const void* V;
    double* cross;
};

__host__ __device__ inline int64_t cross_waves(const GridP& g)
{
    return ((g.n[0] + 2) * g.n[1] * (g.dim == 3 ? g.n[2] : 1) + kCrossRun - 1) / kCrossRun;
}

struct CrossOne {
    CrossTask c;
    int64_t nw;
    __device__ int64_t total() const { return nw; }
    __device__ const CrossTask& resolve(int64_t w, int64_t& lw) const { lw = w; return c; }
};

struct CrossBatch {
    const CrossTask* tasks;
    const int64_t* woff;
    int nb;
    __device__ int64_t total() const { return woff[nb]; }
    __device__ const CrossTask& resolve(int64_t w, int64_t& lw) const
    {
        int lo = 0, hi = nb - 1;                // last b with woff[b] <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (woff[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        lw = w - woff[lo];
        return tasks[lo];
    }
};

template <class T, int D, class R>
__global__ void __launch_bounds__(256) k_cross(R src)
{
    constexpr int NDIR = D == 3 ? 13 : 4;
    constexpr int NPEN = D == 3 ? 5 : 2;     // own column, (y+1, z), (y-1, z+1), (y, z+1), (y+1, z+1)
    using V4 = T __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nwaves = src.total();
    for (int64_t wg = wave0; wg < nwaves; wg += (int64_t)gridDim.x * 4) {
        int64_t w;
        const CrossTask& ct = src.resolve(wg, w);
        const KParams& kp = ct.kp;
        const GridP& g = ct.g;
        const int64_t ldv = ct.ldv;
        const int nquads = ct.nquads;
        const int32_t* __restrict__ slot = ct.slot;
        const T* __restrict__ V = (const T*)ct.V;
        double* __restrict__ cross = ct.cross;
        const int64_t xw = g.n[0] + 2;
        const int64_t nflat = xw * g.n[1] * (D == 3 ? g.n[2] : 1);
        const int64_t F = w * kCrossRun + lane - 1;
        int64_t x = -1, y = 0, z = 0;
        if (F >= 0 && F < nflat) {
            x = F % xw - 1;
            const int64_t r = F / xw;
            y = r % g.n[1];
            z = r / g.n[1];
        }
        int32_t sl[NPEN];
        sl[0] = slot_at(g, slot, x, y, z);
        sl[1] = slot_at(g, slot, x, y + 1, z);
        if constexpr (D == 3) {
            sl[2] = slot_at(g, slot, x, y - 1, z + 1);
            sl[3] = slot_at(g, slot, x, y, z + 1);
            sl[4] = slot_at(g, slot, x, y + 1, z + 1);
        }
        const bool out = lane >= 1 && lane <= kCrossRun && sl[0] >= 0;
        if (__ballot(out) == 0) continue;        // wave-uniform

        double acc[NDIR];
#pragma unroll
        for (int d = 0; d < NDIR; ++d) acc[d] = 0.0;
        // V through buffer loads: the descriptor covers one quad plane (ldv columns); a
        // missing column gets an offset past its end, which the hardware reads as zeros.
        const unsigned plane = (unsigned)(ldv * 4 * sizeof(T));
        unsigned voff[NPEN];
#pragma unroll
        for (int k = 0; k < NPEN; ++k) voff[k] = sl[k] >= 0 ? (unsigned)sl[k] * (unsigned)(4 * sizeof(T)) : plane;
        auto load = [&](V4 (&b)[NPEN], int q) {
            __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)(V + (size_t)q * ldv * 4), 0,
                                                                          (int)plane, kBufferFlags);
#pragma unroll
            for (int k = 0; k < NPEN; ++k) {
                if constexpr (sizeof(T) == 4) {
                    b[k] = __builtin_bit_cast(V4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff[k], 0, 0));
                } else {
                    const u4 lo = __builtin_amdgcn_raw_buffer_load_b128(rs, voff[k], 0, 0);
                    const u4 hi = __builtin_amdgcn_raw_buffer_load_b128(rs, voff[k] + 16, 0, 0);
                    b[k] = V4{__builtin_bit_cast(double, ((unsigned long long)lo[1] << 32) | lo[0]),
                              __builtin_bit_cast(double, ((unsigned long long)lo[3] << 32) | lo[2]),
                              __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | hi[0]),
                              __builtin_bit_cast(double, ((unsigned long long)hi[3] << 32) | hi[2])};
                }
            }
        };
        // Row i of a quad: the x-neighbour products use the own value shifted by one lane
        // (a(x - 1), a(x + 1)), so lane y accumulates a(y + 1) u(y) for the dx = -1 pair of
        // vertex y + 1 and a(y - 1) u(y) for the dx = +1 pair of vertex y - 1; those sums
        // move back to their owners with one lane shift after the row loop.  Products of
        // binary32 operands are exact in binary64, and every sum is binary64.
        auto accumulate = [&](const V4 (&b)[NPEN]) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const T a32 = b[0][i];
                const double a = (double)a32;
                const double an = (double)lane_shift<kFromNext>(a32), ap = (double)lane_shift<kFromPrev>(a32);
                acc[0] = fma(a, an, acc[0]);                                     // (+1, 0, 0)
#pragma unroll
                for (int k = 1; k < NPEN; ++k) {
                    // pencil k covers directions 1 + 3 (k - 1) + (dx + 1)
                    const double u = (double)b[k][i];
                    const int d0 = 1 + 3 * (k - 1);
                    acc[d0 + 0] = fma(an, u, acc[d0 + 0]);
                    acc[d0 + 1] = fma(a, u, acc[d0 + 1]);
                    acc[d0 + 2] = fma(ap, u, acc[d0 + 2]);
                }
            }
        };
        // nquads is a multiple of 4: pairs of quads, the next one prefetched
        V4 b0[NPEN], b1[NPEN];
        load(b0, 0);
        for (int q = 0; q < nquads; q += 2) {
            load(b1, q + 1);
            accumulate(b0);
            load(b0, q + 2 < nquads ? q + 2 : q + 1);   // the last prefetch re-reads a quad
            accumulate(b1);
        }
#pragma unroll
        for (int k = 1; k < NPEN; ++k) {
            const int d0 = 1 + 3 * (k - 1);
            acc[d0 + 0] = lane_shift<kFromPrev>(acc[d0 + 0]);
            acc[d0 + 2] = lane_shift<kFromNext>(acc[d0 + 2]);
        }

        if (out) {
            const double xp[3] = {vertex_coord(g, 0, x), vertex_coord(g, 1, y), D == 3 ? vertex_coord(g, 2, z) : 0.0};
#pragma unroll
            for (int d = 0; d < NDIR; ++d) {
                // direction d: offset (dx, dy, dz) with last non-zero component +1
                int dx, dy, dz;
                if (d == 0) { dx = 1; dy = 0; dz = 0; }
                else if (d < 4) { dx = d - 2; dy = 1; dz = 0; }
                else { dx = (d - 4) % 3 - 1; dy = (d - 4) / 3 - 1; dz = 1; }
                double res = __builtin_nan("");
                if (slot_at(g, slot, x + dx, y + dy, z + dz) >= 0) {
                    const double xq[3] = {vertex_coord(g, 0, x + dx), vertex_coord(g, 1, y + dy),
                                          D == 3 ? vertex_coord(g, 2, z + dz) : 0.0};
                    res = kernel_val(kp, kernel_r2(kp, xp, xq)) - acc[d];
                }
                cross[(size_t)sl[0] * NDIR + d] = res;
            }
        }
    }
}

// Semidefinite Cholesky of the lower triangle of S (N x N, row-major in registers).
template <int N>
__device__ __forceinline__ void chol_sd(double (&S)[N][N], double (&C)[N][N])
{
    double mx = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) mx = S[q][q] > mx ? S[q][q] : mx;
    const double tol = 1e-12 * mx;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) C[i][j] = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double d = S[k][k];
#pragma unroll
        for (int j = 0; j < k; ++j) d = fma(-C[k][j], C[k][j], d);
        const bool keep = (mx > 0.0) && (d > tol);
        const double ckk = keep ? sqrt(d) : 0.0;
        const double inv = keep ? 1.0 / ckk : 0.0;
        C[k][k] = ckk;
#pragma unroll
        for (int i = k + 1; i < N; ++i) {
            double s = S[i][k];
#pragma unroll
            for (int j = 0; j < k; ++j) s = fma(-C[i][j], C[k][j], s);
            C[i][k] = s * inv;
        }
    }
}

// Cell e of the enumeration (dense: all cells, x fastest; adaptive: leaf by leaf): its
// linear index and the slots of its corners.  Returns 0 (cell outside the domain), 1 (a
// corner has no posterior data: the cell's LCP is NaN) or 2.
template <int D>
__device__ __forceinline__ int cell_corners(const CellTask& t, int64_t e, int64_t& lin, int64_t (&sl)[1 << D])
{
    constexpr int N = 1 << D;
    const GridP& g = t.grid;
    int64_t cell[3] = {0, 0, 0};
    if (t.leaves) {
        int64_t cpl = 1;
        for (int d = 0; d < D; ++d) cpl *= t.leaf_edge;
        const int64_t lf = e / cpl;
        int64_t loc = e % cpl;
        const uint64_t key = t.leaves[lf];
        const int level = (int)(key >> 58);
        const uint64_t mc = key & ((1ull << 58) - 1);
        int64_t nc[3] = {0, 0, 0};
        for (int b = 0; b < level; ++b)
            for (int d = 0; d < D; ++d) nc[d] |= (int64_t)((mc >> (b * D + d)) & 1) << b;
        const int64_t sz = t.S0 >> level;
        bool in = true;
        for (int d = 0; d < D; ++d) {
            cell[d] = nc[d] * sz + loc % t.leaf_edge;
            loc /= t.leaf_edge;
            in = in && cell[d] < g.nc[d];
        }
        if (!in) return 0;
    } else {
        int64_t r = e;
        cell[0] = r % g.nc[0];
        r /= g.nc[0];
        cell[1] = r % g.nc[1];
        cell[2] = r / g.nc[1];
    }
    lin = cell[0] + g.nc[0] * (cell[1] + g.nc[1] * cell[2]);
    bool have = true;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const int64_t vx = cell[0] + (q & 1), vy = cell[1] + ((q >> 1) & 1), vz = cell[2] + ((q >> 2) & 1);
        const int64_t vid = vx + g.n[0] * (vy + g.n[1] * (D == 3 ? vz : 0));
        sl[q] = t.slot ? (int64_t)t.slot[vid] : vid;
        have = have && sl[q] >= 0;
    }
    return have ? 2 : 1;
}

// Corner moments of a cell: mu - theta and the semidefinite Cholesky factor of the corner
// covariance (sl from cell_corners).
template <int D>
__device__ __forceinline__ void cell_factor(const CellTask& t, const int64_t (&sl)[1 << D], double (&mu)[1 << D],
                                            double (&Cd)[1 << D][1 << D])
{
    constexpr int N = 1 << D;
    constexpr int NDIR = D == 3 ? 13 : 4;
    double S[N][N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
        mu[q] = t.mean[sl[q]] - t.theta;
        S[q][q] = t.var[sl[q]];
    }
#pragma unroll
    for (int p = 0; p < N; ++p)
#pragma unroll
        for (int q = p + 1; q < N; ++q) {
            const int dx = (q & 1) - (p & 1), dy = ((q >> 1) & 1) - ((p >> 1) & 1),
                      dz = ((q >> 2) & 1) - ((p >> 2) & 1);
            const double c = t.cross[(size_t)sl[p] * NDIR + dir_index(D, dx, dy, dz)];
            S[q][p] = c;
            S[p][q] = c;
        }
    chol_sd<N>(S, Cd);
}

// Number of enumerated cells (dense grid, or the cells of the emitted leaves).
template <int D>
__device__ __forceinline__ int64_t cell_total(const CellTask& t, int64_t ncells_cap)
{
    int64_t total;
    if (t.leaves) {
        const int64_t nleaf = *t.n_leaves;
        if (nleaf > t.leaf_cap) return 0;          // overflow: reconstruction skipped
        int64_t cpl = 1;
        for (int d = 0; d < D; ++d) cpl *= t.leaf_edge;
        total = nleaf * cpl;
    } else {
        total = t.grid.nc[0] * t.grid.nc[1] * t.grid.nc[2];
    }
    return total < ncells_cap ? total : ncells_cap;
}

// max_s ||z_s||_2 over the z-bank (one work-group).
__global__ void __launch_bounds__(256) k_zmax(const double* __restrict__ zb, int ns, int n, double* __restrict__ out)
{
    __shared__ double red[256];
    double m = 0.0;
    for (int s = threadIdx.x; s < ns; s += 256) {
        double q = 0.0;
        for (int r = 0; r < n; ++r) q = fma(zb[(size_t)s * n + r], zb[(size_t)s * n + r], q);
        m = fmax(m, sqrt(q));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// Where a kernel's cells come from: one task (its enumeration), or a batch of dense tasks
// whose cells are numbered consecutively (task b owns coff[b] .. coff[b + 1] - 1).  Work
// lists hold these global numbers; a batch shares one list, count and zmax (task 0's).
template <int D>
struct CellsOne {
    CellTask t;
    __device__ int64_t total(int64_t cap) const { return cell_total<D>(t, cap); }
    __device__ const CellTask& first() const { return t; }
    __device__ const CellTask& resolve(int64_t e, int64_t& le) const { le = e; return t; }
};

struct CellsBatch {
    const CellTask* tasks;
    const int64_t* coff;
    int nb;
    __device__ int64_t total(int64_t cap) const { return coff[nb] < cap ? coff[nb] : cap; }
    __device__ const CellTask& first() const { return tasks[0]; }
    __device__ const CellTask& resolve(int64_t e, int64_t& le) const
    {
        int lo = 0, hi = nb - 1;                // last b with coff[b] <= e
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (coff[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        le = e - coff[lo];
        return tasks[lo];
    }
};

// Certified skip of the Monte Carlo loop.  Every sample value of corner q is
// y_q = m_q + C_q . z_s with |C_q . z_s| <= ||C_q||_2 ||z_s||_2 <= ||C_q||_2 zmax, so when
// m_q - ||C_q|| zmax > 0 for every corner (or m_q + ||C_q|| zmax < 0 for every corner) no
// sample can cross: the count is exactly 0.  The margin covers the rounding of the Monte
// Carlo loop in its own precision (relative 1e-5 for binary32, 1e-12 for binary64).
// Cells that cannot be certified go to the work list (order immaterial: each cell's
// result depends on that cell only).
template <int D, class TM, class R>
__global__ void __launch_bounds__(256) k_cells_cert(R src, int64_t ncells_cap)
{
    constexpr int N = 1 << D;
    const int64_t total = src.total(ncells_cap);
    const CellTask& t0 = src.first();
    const double zm = *t0.zmax;
    const double rel = std::is_same<TM, double>::value ? 1e-12 : 1e-5;
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = base + threadIdx.x;
        bool work = false;
        if (e < total) {
            int64_t le = 0, lin = 0;
            const CellTask& t = src.resolve(e, le);
            int64_t sl[N];
            const int st = cell_corners<D>(t, le, lin, sl);
            if (st == 1) {
                t.lcp[lin] = __builtin_nanf("");
            } else if (st == 2) {
                // pre-filter on the corner standard deviations (row norms of an exact factor);
                // only cells that pass it are factored for the exact test
                bool above = true, below = true;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    const double m = t.mean[sl[q]] - t.theta;
                    const double b = 1.001 * sqrt(fmax(t.var[sl[q]], 0.0)) * zm;
                    above = above && (m > b);
                    below = below && (m < -b);
                }
                if (above || below) {
                    double mu[N], Cd[N][N];
                    cell_factor<D>(t, sl, mu, Cd);
                    above = below = true;
#pragma unroll
                    for (int q = 0; q < N; ++q) {
                        double rn = 0.0;
#pragma unroll
                        for (int r = 0; r <= q; ++r) rn = fma(Cd[q][r], Cd[q][r], rn);
                        const double b = sqrt(rn) * zm;
                        const double pad = rel * (fabs(mu[q]) + b) + 1e-300;
                        above = above && (mu[q] - b > pad);
                        below = below && (mu[q] + b < -pad);
                    }
                }
                if (above || below) t.lcp[lin] = 0.0f;
                else work = true;
            }
        }
        // wave-aggregated append
        const uint64_t bal = __ballot(work);
        if (bal) {
            int64_t pos = 0;
            if (lane == 0) pos = atomicAdd((unsigned long long*)t0.wcount, (unsigned long long)__popcll(bal));
            pos = __shfl(pos, 0, 64);
            if (work) t0.work[pos + __popcll(bal & ((1ull << lane) - 1))] = (int32_t)e;
        }
    }
}

// Monte Carlo LCP of the listed cells (count = *wcount).
template <int D, class TM, class R>
__global__ void __launch_bounds__(256) k_cells(R src, int64_t ncells_cap)
{
    constexpr int N = 1 << D;
    const CellTask& t0 = src.first();
    int64_t total = *t0.wcount;
    if (total > ncells_cap) total = ncells_cap;
    const TM* zb = std::is_same<TM, double>::value ? (const TM*)t0.zb64 : (const TM*)t0.zb32;
    const int ns = t0.ns;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        int64_t le = 0, lin = 0;
        const CellTask& t = src.resolve(t0.work[it], le);
        int64_t sl[N];
        if (cell_corners<D>(t, le, lin, sl) != 2) continue;
        double mu[N], Cd[N][N];
        cell_factor<D>(t, sl, mu, Cd);
        TM C[N][N], m[N];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            m[q] = (TM)mu[q];
#pragma unroll
            for (int r = 0; r < N; ++r) C[q][r] = (TM)Cd[q][r];
        }
        int cnt = 0;
        for (int s = 0; s < ns; ++s) {
            TM z[N];
#pragma unroll
            for (int r = 0; r < N; ++r) z[r] = zb[(size_t)s * N + r];
            TM ymin, ymax;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                TM y = m[q];
#pragma unroll
                for (int r = 0; r <= q; ++r) y = fma(C[q][r], z[r], y);
                if (q == 0) {
                    ymin = y;
                    ymax = y;
                } else {
                    ymin = fmin(ymin, y);
                    ymax = fmax(ymax, y);
                }
            }
            // crossed unless all corners are below theta (ymax < 0) or all above (ymin > 0)
            cnt += (!(ymax < (TM)0) && !(ymin > (TM)0)) ? 1 : 0;
        }
        t.lcp[lin] = (float)cnt / (float)ns;
    }
}

// ------------------------------------------------------------ matrix-core Monte Carlo
//
// Reduced-precision paths, 3D.  The values y - theta of the 8 corners of 4 cells (32 rows)
// for 32 samples (columns) form one 32 x 32 product.  With s a power of two per cell that
// keeps the operands in FP16 range, row (cell, corner q) of the left operand holds s C_q and
// s (mu_q - theta), each as an FP16 pair hi + lo, and column j of the right operand holds
// z_j as an FP16 pair and a 1:
//   s (mu_q - theta + C_q . z_j) = [C_hi | C_lo] [z_hi; z_hi] + [C_hi | m_hi m_lo 0..] [z_lo; 1 1 0..]
// (two 32x32x16 MFMAs, binary32 accumulation).  The operands are rounded once to binary32;
// hi is their round-toward-zero FP16 value and lo the nearest FP16 value of the exact
// binary32 residual, so hi + lo is within 2^-21 of the operand.  With the dropped C_lo z_lo
// term and the binary32 accumulation of 18 terms, a corner value is within about 2^-19
// (|s (mu - theta)| + sum |s C| |z|) of exact, inside the margin the certificate keeps for
// binary32 loops (1e-5).  The crossing test reads only signs, which s > 0 leaves unchanged.
//
// Row order: the MFMA leaves row r = 8a + 4h + c of the result in register 4a + c of lane
// half h, and row r is corner 2a + (c & 1) of cell 2h + (c >> 1) of the quad, so each lane
// holds all 8 corners of two cells for its sample.

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMcCells = 32;     // cells per wave (8 quads of 4)
constexpr int kMcWaves = 4;

// Split FP16 records of the z-bank, 24 halves per sample: [z_hi (8) | z_lo (8) | 1, 1, 0 x 6],
// z = z_hi + z_lo to within 2^-22 |z|; samples ns .. nspad - 1 are zero.
__global__ void k_zrec(const double* __restrict__ zb, int ns, int nspad, _Float16* __restrict__ rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nspad * 8) return;
    const int64_t smp = i >> 3;
    const int k = (int)(i & 7);
    const double z = smp < ns ? zb[smp * 8 + k] : 0.0;
    const _Float16 hi = (_Float16)(float)z;
    rec[smp * 24 + k] = hi;
    rec[smp * 24 + 8 + k] = (_Float16)(float)(z - (double)hi);
    rec[smp * 24 + 16 + k] = (_Float16)(k < 2 ? 1.0f : 0.0f);
}

// Sign tests on the bit patterns (no NaN canonicalisation): for a non-NaN binary32 y,
// y > 0 iff its bits as a signed integer are > 0, and y < 0 iff its bits as an unsigned
// integer exceed 0x80000000 (-0 is 0x80000000).  So every corner of a cell is above theta
// iff the signed minimum of its 8 values is > 0, and below iff the unsigned minimum is
// > 0x80000000.  Registers o, o+1, o+4, o+5, o+8, o+9, o+12, o+13 hold one cell (o = 0, 2).
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ unsigned umin(unsigned a, unsigned b) { return a < b ? a : b; }
template <int O>
__device__ __forceinline__ int min8_i(const f32x16& a)
{
    const int m0 = imin(imin(__float_as_int(a[O]), __float_as_int(a[O + 1])), __float_as_int(a[O + 4]));
    const int m1 = imin(imin(__float_as_int(a[O + 5]), __float_as_int(a[O + 8])), __float_as_int(a[O + 9]));
    return imin(imin(m0, m1), imin(__float_as_int(a[O + 12]), __float_as_int(a[O + 13])));
}
template <int O>
__device__ __forceinline__ unsigned min8_u(const f32x16& a)
{
    const unsigned m0 = umin(umin(__float_as_uint(a[O]), __float_as_uint(a[O + 1])), __float_as_uint(a[O + 4]));
    const unsigned m1 = umin(umin(__float_as_uint(a[O + 5]), __float_as_uint(a[O + 8])), __float_as_uint(a[O + 9]));
    return umin(umin(m0, m1), umin(__float_as_uint(a[O + 12]), __float_as_uint(a[O + 13])));
}

// Monte Carlo LCP of the listed cells (count = *wcount), 32 cells per wave: lanes 0..31
// factor one cell each in binary64 and stage its scaled FP16 operand rows in LDS; the wave
// then sweeps the sample blocks with the 8 quads' operands in registers and keeps the
// crossing counts in scalar registers.
template <class R>
__global__ void __launch_bounds__(kMcWaves * 64) k_cells_mfma(R src, int64_t ncells_cap, const h8v* __restrict__ zrec)
{
    __shared__ __align__(16) h8v stage[kMcWaves][kMcCells][8][3];   // [cell][corner]: C_hi, C_lo, (m_hi, m_lo, 0..)
    const CellTask& t0 = src.first();
    int64_t total = *t0.wcount;
    if (total > ncells_cap) total = ncells_cap;
    const int ns = t0.ns;
    const int nblk = (ns + 31) >> 5;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, r = lane & 31;
    const int rcell = 2 * ((r >> 2) & 1) + ((r & 3) >> 1), rcorner = 2 * (r >> 3) + (r & 1);
    const int tail = ns - 32 * (nblk - 1);                    // samples of the last block, 1..32
    const uint64_t tm32 = tail == 32 ? 0xffffffffull : ((1ull << tail) - 1);
    const uint64_t tmask = tm32 | (tm32 << 32);               // both lane halves hold the same samples
    h8v (*st)[8][3] = stage[wave];
    for (int64_t base = ((int64_t)blockIdx.x * kMcWaves + wave) * kMcCells; base < total;
         base += (int64_t)gridDim.x * kMcWaves * kMcCells) {
        int64_t lin = -1;
        float* out = nullptr;
        if (lane < kMcCells) {
            double mu[8], Cd[8][8];
            const int64_t it = base + lane;
            if (it < total) {
                int64_t le = 0;
                const CellTask& t = src.resolve(t0.work[it], le);
                int64_t sl[8];
                if (cell_corners<3>(t, le, lin, sl) == 2) {
                    cell_factor<3>(t, sl, mu, Cd);
                    out = t.lcp;
                }
            }
            if (out) {
                double mx = 0.0;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    mx = fmax(mx, fabs(mu[q]));
#pragma unroll
                    for (int k = 0; k <= q; ++k) mx = fmax(mx, fabs(Cd[q][k]));
                }
                int e = 0;
                if (mx > 0.0) frexp(mx, &e);                  // mx < 2^e
                if (e < -1000) e = -1000;
                const double sc = ldexp(1.0, 14 - e);         // every scaled operand below 2^14
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    h8v hi, lo, mm;
                    float f[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) f[k] = k <= q ? (float)(Cd[q][k] * sc) : 0.0f;
#pragma unroll
                    for (int k = 0; k < 8; k += 2) {
                        const auto ph = __builtin_amdgcn_cvt_pkrtz(f[k], f[k + 1]);
                        hi[k] = ph[0];
                        hi[k + 1] = ph[1];
                        lo[k] = (_Float16)(f[k] - (float)ph[0]);
                        lo[k + 1] = (_Float16)(f[k + 1] - (float)ph[1]);
                        mm[k] = (_Float16)0.0f;
                        mm[k + 1] = (_Float16)0.0f;
                    }
                    const float m = (float)(mu[q] * sc);
                    const auto pm = __builtin_amdgcn_cvt_pkrtz(m, 0.0f);
                    mm[0] = pm[0];
                    mm[1] = (_Float16)(m - (float)pm[0]);
                    st[lane][q][0] = hi;
                    st[lane][q][1] = lo;
                    st[lane][q][2] = mm;
                }
            } else {
                const h8v z = {};
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    st[lane][q][0] = z;
                    st[lane][q][1] = z;
                    st[lane][q][2] = z;
                }
            }
        }
        // the staged rows are read by other lanes of this wave
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        h8v A1[8], A2[8];
#pragma unroll
        for (int Q = 0; Q < 8; ++Q) {
            A1[Q] = st[4 * Q + rcell][rcorner][h];            // C_hi | C_lo
            A2[Q] = st[4 * Q + rcell][rcorner][2 * h];        // C_hi | (m_hi, m_lo, 0..)
        }
        uint32_t cnt[8][4];
#pragma unroll
        for (int Q = 0; Q < 8; ++Q)
#pragma unroll
            for (int k = 0; k < 4; ++k) cnt[Q][k] = 0;
        const h8v* zp = zrec + 3 * r;                         // record of sample 32 b + r
        // one block of 32 samples for the 8 quads; quad Q + 1's products are issued before
        // quad Q's sign tests (two result sets)
        auto block = [&](const h8v& B1, const h8v& B2, uint64_t valid) {
            f32x16 acc[2];
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A1[0], B1, f32x16{}, 0, 0, 0);
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A2[0], B2, acc[0], 0, 0, 0);
#pragma unroll
            for (int Q = 0; Q < 8; ++Q) {
                if (Q + 1 < 8) {
                    acc[(Q + 1) & 1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A1[Q + 1], B1, f32x16{}, 0, 0, 0);
                    acc[(Q + 1) & 1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A2[Q + 1], B2, acc[(Q + 1) & 1], 0, 0, 0);
                }
                const f32x16& a = acc[Q & 1];
                // crossed unless every corner is above theta or every corner is below it
                const uint64_t c0 = valid & ~(__ballot(min8_i<0>(a) > 0) | __ballot(min8_u<0>(a) > 0x80000000u));
                const uint64_t c1 = valid & ~(__ballot(min8_i<2>(a) > 0) | __ballot(min8_u<2>(a) > 0x80000000u));
                cnt[Q][0] += __builtin_popcount((uint32_t)c0);
                cnt[Q][2] += __builtin_popcount((uint32_t)(c0 >> 32));
                cnt[Q][1] += __builtin_popcount((uint32_t)c1);
                cnt[Q][3] += __builtin_popcount((uint32_t)(c1 >> 32));
            }
        };
        // two record sets in turn: a block's records are requested one block ahead
        auto ld = [&](int b, h8v& R1, h8v& R2) {
            const size_t o = (size_t)96 * (b < nblk ? b : nblk - 1);
            R1 = zp[o];
            R2 = zp[o + 1 + h];
        };
        const int nfull = ns >> 5;                            // blocks of 32 live samples
        h8v X1, X2, Y1, Y2;
        ld(0, X1, X2);
        int b = 0;
        for (; b + 2 <= nfull; b += 2) {
            ld(b + 1, Y1, Y2);
            block(X1, X2, ~0ull);
            ld(b + 2, X1, X2);
            block(Y1, Y2, ~0ull);
        }
        if (b < nfull) {                                      // odd count of full blocks
            ld(b + 1, Y1, Y2);
            block(X1, X2, ~0ull);
            X1 = Y1;
            X2 = Y2;
        }
        if (nfull < nblk) block(X1, X2, tmask);               // last, partial block
        if (out) {
            uint32_t c = 0;
#pragma unroll
            for (int Q = 0; Q < 8; ++Q)
#pragma unroll
                for (int k = 0; k < 4; ++k) c = lane == 4 * Q + k ? cnt[Q][k] : c;
            out[lin] = (float)c / (float)ns;
        }
    }
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

template <class T>
__global__ void k_fill(T* __restrict__ p, T v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------- smooth cell LCP
//
// For differentiation, the cell probability 1 - P(all Y < theta) - P(all Y > theta) is
// estimated by Genz's separation of variables: with the corner factor C and uniforms
// w_i = Phi(z_i) from the first 2^D - 1 normals of each z-bank row, each orthant is a
// product of conditional probabilities e_i = Phi(+-t_i), t_i = (theta - mu_i - sum_j C_ij
// y_j) / C_ii, and y_i is drawn inside orthant i by inversion.  Smooth in mu and C; a zero
// pivot makes its factor a step.  Binary64 throughout, one lane per cell.

template <class T>
struct SovMath;
template <>
struct SovMath<double> {
    static __device__ __forceinline__ double cdf(double t) { return normcdf(t); }
    static __device__ __forceinline__ double pdf(double t) { return exp(-0.5 * t * t) * 0.39894228040143267794; }
    static __device__ __forceinline__ double inv(double u) { return normcdfinv(fmin(fmax(u, 1e-300), 1.0 - 1e-16)); }
};
template <>
struct SovMath<float> {
    static __device__ __forceinline__ float cdf(float t) { return normcdff(t); }
    static __device__ __forceinline__ float pdf(float t) { return expf(-0.5f * t * t) * 0.398942280f; }
    static __device__ __forceinline__ float inv(float u) { return normcdfinvf(fminf(fmaxf(u, 1e-37f), 1.0f - 1e-7f)); }
};

// Lower-triangular N x N matrices packed by rows: (i, j), j <= i, at i (i + 1) / 2 + j.
template <int N>
constexpr int kTri = N * (N + 1) / 2;
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// One sample of one orthant (upper = 1: all above theta); mt = mu - theta.  T is the
// arithmetic of the sample (binary64, or binary32 for the binary32 paths).
template <int N, class T>
__device__ __forceinline__ T sov_orthant(const T (&mt)[N], const T (&C)[kTri<N>], bool upper,
                                         const double* __restrict__ w, T (&t)[N], T (&e)[N], T (&y)[N])
{
    using M = SovMath<T>;
    T f = 1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T si = 0;
#pragma unroll
        for (int j = 0; j < i; ++j) si = fma(C[tri(i, j)], y[j], si);
        const T r = -mt[i] - si;
        const T cii = C[tri(i, i)];
        if (cii > T(0)) {
            t[i] = r / cii;
            e[i] = M::cdf(upper ? -t[i] : t[i]);
        } else {
            t[i] = 0;
            e[i] = upper ? (r < T(0) ? T(1) : T(0)) : (r > T(0) ? T(1) : T(0));
        }
        f *= e[i];
        y[i] = 0;
        const T wi = (T)w[i];
        if (i < N - 1 && cii > T(0)) y[i] = M::inv(upper ? T(1) - e[i] + wi * e[i] : wi * e[i]);
    }
    return f;
}

// Reverse pass of one orthant sample, scaled: adds d f / d mu to gmu and d f / d C to gC
// (binary64 accumulators).
template <int N, class T>
__device__ __forceinline__ void sov_orthant_rev(const T (&C)[kTri<N>], bool upper, const double* __restrict__ w,
                                                const T (&t)[N], const T (&e)[N], const T (&y)[N], T scale,
                                                double (&gmu)[N], double (&gC)[kTri<N>])
{
    using M = SovMath<T>;
    T suf[N + 1], ybar[N], pre[N];
    suf[N] = 1;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) suf[i] = suf[i + 1] * e[i];
    pre[0] = 1;
#pragma unroll
    for (int i = 1; i < N; ++i) pre[i] = pre[i - 1] * e[i - 1];
#pragma unroll
    for (int i = 0; i < N; ++i) ybar[i] = 0;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        const T cii = C[tri(i, i)];
        if (!(cii > T(0))) continue;
        T ebar = scale * pre[i] * suf[i + 1];
        if (i < N - 1) {
            const T py = M::pdf(y[i]);
            const T wi = (T)w[i];
            if (py > T(0)) ebar += ybar[i] * (upper ? wi - T(1) : wi) / py;
        }
        const T tbar = ebar * M::pdf(t[i]) * (upper ? T(-1) : T(1));
        const T rbar = tbar / cii;
        gC[tri(i, i)] -= (double)(tbar * t[i] / cii);
        gmu[i] -= (double)rbar;
#pragma unroll
        for (int j = 0; j < i; ++j) {
            gC[tri(i, j)] -= (double)(rbar * y[j]);
            ybar[j] -= rbar * C[tri(i, j)];
        }
    }
}

// Reverse pass of the semidefinite Cholesky chol_sd: dL/dC (lower, packed, consumed) to
// dL/dS on the lower triangle the factor reads.  Zeroed columns pass no gradient.
template <int N>
__device__ __forceinline__ void chol_sd_rev(const double (&C)[kTri<N>], double (&gC)[kTri<N>], double (&gS)[kTri<N>])
{
#pragma unroll
    for (int i = 0; i < kTri<N>; ++i) gS[i] = 0.0;
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        const double ckk = C[tri(k, k)];
        if (!(ckk > 0.0)) continue;
        const double inv = 1.0 / ckk;
#pragma unroll
        for (int i = N - 1; i > k; --i) {
            const double g = gC[tri(i, k)] * inv;
            gS[tri(i, k)] += g;
#pragma unroll
            for (int j = 0; j < k; ++j) {
                gC[tri(i, j)] -= g * C[tri(k, j)];
                gC[tri(k, j)] -= g * C[tri(i, j)];
            }
            gC[tri(k, k)] -= g * C[tri(i, k)];
        }
        const double g = gC[tri(k, k)];
        gS[tri(k, k)] += 0.5 * g * inv;
#pragma unroll
        for (int j = 0; j < k; ++j) gC[tri(k, j)] -= g * C[tri(k, j)] * inv;
    }
}

template <int N, class T>
__device__ __forceinline__ void pack_lower(const double (&Cd)[N][N], T (&C)[kTri<N>])
{
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) C[tri(i, j)] = (T)Cd[i][j];
}

__global__ void k_wbank(const double* __restrict__ zb, double* __restrict__ wb, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        wb[i] = normcdf(zb[i]);
}

// Largest |z| of the bank (one work-group of 256 threads) -> out[0].
__global__ void k_zabsmax(const double* __restrict__ zb, int64_t n, double* __restrict__ out)
{
    __shared__ double red[4];
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) mx = fmax(mx, fabs(zb[i]));
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Binary32 samples only: a cell whose corners all lie, with every conditional draw of the
// bank, more than 6.5 conditional standard deviations on one side of theta has every
// lower (or upper) orthant factor equal to 1 in binary32 and the other orthant's product
// below 1e-10: its smooth LCP and gradient are zero at binary32 accuracy and are skipped.
// In that orthant each draw is y_j = Phi^-1(w_j e_j) with e_j >= Phi(6.5), so |y_j| <= the
// bank's largest |z| (ymax, plus a margin), and |sum_j C_ij y_j| <= ymax sum_j |C_ij|.
template <int N>
__device__ __forceinline__ bool sov_far(const double (&md)[N], const double (&Cd)[N][N], double ymax)
{
    bool below = true, above = true;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double r = 0.0;
#pragma unroll
        for (int j = 0; j < i; ++j) r += fabs(Cd[i][j]);
        const double need = 6.5 * Cd[i][i] + ymax * r;
        below = below && (-md[i] > need);
        above = above && (md[i] > need);
    }
    return below || above;
}

// Binary32 smooth estimator: far cells (sov_far) get their zero LCP (lcp non-null) or zero
// gradient (gout non-null) here; the others are appended to the work list, one atomic per
// wave, so the sample loop runs on full waves.
template <int D>
__global__ void __launch_bounds__(256) k_sov_select(CellTask t, int64_t ncell, const double* __restrict__ zabs,
                                                    float* __restrict__ lcp, double* __restrict__ gout,
                                                    int32_t* __restrict__ work, int64_t* __restrict__ wcount)
{
    constexpr int N = 1 << D;
    constexpr int NO = N + kTri<N>;
    const double ymax = zabs[0] + 0.01;
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < ncell; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = base + threadIdx.x;
        bool need = false;
        if (c < ncell) {
            int64_t lin, sl[N];
            const int st = cell_corners<D>(t, c, lin, sl);
            if (st == 1) {
                need = true;                         // the sample kernel writes NaN / zeros
            } else if (st == 2) {
                double md[N], Cd[N][N];
                cell_factor<D>(t, sl, md, Cd);
                if (sov_far<N>(md, Cd, ymax)) {
                    if (lcp) lcp[lin] = 0.0f;
                    if (gout)
#pragma unroll
                        for (int i = 0; i < NO; ++i) gout[(size_t)lin * NO + i] = 0.0;
                } else {
                    need = true;
                }
            }
        }
        const uint64_t bal = __ballot(need);
        if (bal) {
            int64_t pos = 0;
            if (lane == 0) pos = atomicAdd((unsigned long long*)wcount, (unsigned long long)__popcll(bal));
            pos = __shfl(pos, 0, 64);
            if (need) work[pos + __popcll(bal & ((1ull << lane) - 1))] = (int32_t)c;
        }
    }
}

// Smooth LCP of every cell of the dense grid (work == null) or of the listed cells.
template <int D, class T>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 4 : 1) k_cells_sov(CellTask t, const double* __restrict__ wb, int64_t ncell,
                                                   const int32_t* __restrict__ work, const int64_t* __restrict__ wcount)
{
    constexpr int N = 1 << D;
    const int64_t total = work ? *wcount : ncell;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total; it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = work ? (int64_t)work[it] : it;
        int64_t lin, sl[N];
        const int st = cell_corners<D>(t, c, lin, sl);
        if (st == 0) continue;
        if (st == 1) { t.lcp[lin] = __builtin_nanf(""); continue; }
        double md[N], Cd[N][N];
        T mt[N], C[kTri<N>], tt[N], e[N], y[N];
        cell_factor<D>(t, sl, md, Cd);
#pragma unroll
        for (int q = 0; q < N; ++q) mt[q] = (T)md[q];
        pack_lower<N>(Cd, C);
        double acc = 0.0;
        for (int sIdx = 0; sIdx < t.ns; ++sIdx) {
            const double* w = wb + (size_t)sIdx * N;
            acc += (double)sov_orthant<N, T>(mt, C, false, w, tt, e, y);
            acc += (double)sov_orthant<N, T>(mt, C, true, w, tt, e, y);
        }
        t.lcp[lin] = (float)(1.0 - acc / (double)t.ns);
    }
}

// Gradient of gl[cell] * LCP_cell with respect to the cell's corner means (N values) and
// the lower triangle of its corner covariance (N (N + 1) / 2, packed) -> gout[cell].
template <int D, class T>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) k_cells_sov_grad(CellTask t, const double* __restrict__ wb,
                                                        const double* __restrict__ gl, double* __restrict__ gout,
                                                        int64_t ncell, const int32_t* __restrict__ work,
                                                        const int64_t* __restrict__ wcount)
{
    constexpr int N = 1 << D;
    constexpr int NO = N + kTri<N>;
    const int64_t total = work ? *wcount : ncell;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total; it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = work ? (int64_t)work[it] : it;
        int64_t lin, sl[N];
        const int st = cell_corners<D>(t, c, lin, sl);
        if (st == 0) continue;
        double* out = gout + (size_t)lin * NO;
        const double up = gl[lin];
        if (st == 1 || up == 0.0) {
#pragma unroll
            for (int i = 0; i < NO; ++i) out[i] = 0.0;
            continue;
        }
        double gmu[N], gC[kTri<N>];
        T mt[N], C[kTri<N>], tt[N], e[N], y[N];
        {
            double md[N], Cd[N][N];
            cell_factor<D>(t, sl, md, Cd);
#pragma unroll
            for (int q = 0; q < N; ++q) mt[q] = (T)md[q];
            pack_lower<N>(Cd, C);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) gmu[i] = 0.0;
#pragma unroll
        for (int i = 0; i < kTri<N>; ++i) gC[i] = 0.0;
        // LCP = 1 - mean(f_lo + f_hi): each sample's reverse pass runs with weight -1 and the
        // binary64 sums are scaled once at the end
        for (int sIdx = 0; sIdx < t.ns; ++sIdx) {
            const double* w = wb + (size_t)sIdx * N;
            sov_orthant<N, T>(mt, C, false, w, tt, e, y);
            sov_orthant_rev<N, T>(C, false, w, tt, e, y, T(-1), gmu, gC);
            sov_orthant<N, T>(mt, C, true, w, tt, e, y);
            sov_orthant_rev<N, T>(C, true, w, tt, e, y, T(-1), gmu, gC);
        }
        const double scale = up / (double)t.ns;
#pragma unroll
        for (int i = 0; i < N; ++i) gmu[i] *= scale;
#pragma unroll
        for (int i = 0; i < kTri<N>; ++i) gC[i] *= scale;
        // the binary64 factor again (bitwise the same), rather than kept live through the
        // sample loop: the registers go to more resident waves
        double C64[kTri<N>], gS[kTri<N>];
        {
            double md[N], Cd[N][N];
            cell_factor<D>(t, sl, md, Cd);
            pack_lower<N>(Cd, C64);
        }
        chol_sd_rev<N>(C64, gC, gS);
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = gmu[i];
#pragma unroll
        for (int i = 0; i < kTri<N>; ++i) out[N + i] = gS[i];
    }
}

// Per vertex: dL/dmean, dL/dvar and dL/dcross (its canonical directions) gathered from
// the cells that contain it (cell gradients from k_cells_sov_grad).
template <int D>
__global__ void __launch_bounds__(256) k_sov_gather(GridP g, const double* __restrict__ gout,
                                                    double* __restrict__ gmean, double* __restrict__ gvar,
                                                    double* __restrict__ gcross)
{
    constexpr int N = 1 << D;
    constexpr int NO = N + kTri<N>;
    constexpr int NDIR = D == 3 ? 13 : 4;
    const int64_t nv = g.n[0] * g.n[1] * g.n[2];
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x[3] = {v % g.n[0], (v / g.n[0]) % g.n[1], v / (g.n[0] * g.n[1])};
        auto cell_of = [&](int q, int64_t& lin) {
            int64_t c[3] = {0, 0, 0};
            for (int d = 0; d < D; ++d) {
                c[d] = x[d] - ((q >> d) & 1);
                if (c[d] < 0 || c[d] >= g.nc[d]) return false;
            }
            lin = c[0] + g.nc[0] * (c[1] + g.nc[1] * c[2]);
            return true;
        };
        double gm = 0.0, gv = 0.0;
        for (int q = 0; q < N; ++q) {
            int64_t lin;
            if (!cell_of(q, lin)) continue;
            gm += gout[(size_t)lin * NO + q];
            gv += gout[(size_t)lin * NO + N + tri(q, q)];
        }
        gmean[v] = gm;
        gvar[v] = gv;
        for (int dir = 0; dir < NDIR; ++dir) {
            int off[3];
            if (D == 3) { off[0] = (dir + 14) % 3 - 1; off[1] = ((dir + 14) / 3) % 3 - 1; off[2] = (dir + 14) / 9 - 1; }
            else { off[0] = (dir + 5) % 3 - 1; off[1] = (dir + 5) / 3 - 1; off[2] = 0; }
            double gc = 0.0;
            // cells holding v at corner q and v + off at corner r
            for (int q = 0; q < N; ++q) {
                int r = 0;
                bool ok = true;
                for (int d = 0; d < D; ++d) {
                    const int b = ((q >> d) & 1) + off[d];
                    ok = ok && b >= 0 && b <= 1;
                    r |= (b & 1) << d;
                }
                int64_t lin;
                if (!ok || !cell_of(q, lin)) continue;
                gc += gout[(size_t)lin * NO + N + tri(r, q)];   // r > q: the lower entry
            }
            gcross[(size_t)v * NDIR + dir] = gc;
        }
    }
}

inline unsigned grid_for(int64_t n, int per)
{
    int64_t b = (n + per - 1) / per;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

namespace {

template <class R>
void cross_dispatch(R src, int dim, bool f64, unsigned grid, hipStream_t s)
{
    if (f64) {
        if (dim == 3) hipLaunchKernelGGL((k_cross<double, 3, R>), dim3(grid), dim3(256), 0, s, src);
        else hipLaunchKernelGGL((k_cross<double, 2, R>), dim3(grid), dim3(256), 0, s, src);
    } else {
        if (dim == 3) hipLaunchKernelGGL((k_cross<float, 3, R>), dim3(grid), dim3(256), 0, s, src);
        else hipLaunchKernelGGL((k_cross<float, 2, R>), dim3(grid), dim3(256), 0, s, src);
    }
}

bool cross_addressable(int64_t nv_cap, int prec)
{
    // one quad plane of V must stay addressable by a 32-bit buffer offset
    return (double)nv_cap * 4 * (prec == LCP_FP64 ? 8 : 4) < 2147483648.0;
}

}  // namespace

hipError_t launch_cross(const Model& M, int prec, const GridP& g, const int32_t* vlist, const int64_t* nv_dev,
                        int64_t nv_cap, const int32_t* slot, const void* V, double* cross, hipStream_t s)
{
    (void)vlist;
    (void)nv_dev;
    if (nv_cap <= 0) return hipSuccess;
    StageScope sc(s, ST_CROSS);
    if (!cross_addressable(nv_cap, prec)) return hipErrorInvalidValue;
    const int64_t nw = cross_waves(g);
    CrossOne src{CrossTask{M.kp, g, nv_cap, 4 * M.nrb, slot, V, cross}, nw};
    cross_dispatch(src, g.dim, prec == LCP_FP64, grid_for(nw, 4), s);
    return hipGetLastError();
}

size_t cross_batch_scratch(int nb)
{
    return align256(sizeof(CrossTask) * (size_t)nb) + align256(sizeof(int64_t) * (size_t)(nb + 1));
}

hipError_t launch_cross_batch(const Model* const* Ms, const GridP* grids, const void* const* V, double* const* cross,
                              int nb, int prec, char* scratch, hipStream_t s)
{
    if (nb <= 0) return hipSuccess;
    StageScope sc(s, ST_CROSS);
    std::vector<CrossTask> T(nb);
    std::vector<int64_t> woff(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        const GridP& g = grids[b];
        const int64_t nv = g.n[0] * g.n[1] * g.n[2];
        if (!cross_addressable(nv, prec)) return hipErrorInvalidValue;
        T[b] = CrossTask{Ms[b]->kp, g, nv, 4 * Ms[b]->nrb, nullptr, V[b], cross[b]};
        woff[b + 1] = woff[b] + cross_waves(g);
    }
    CrossTask* Td = (CrossTask*)scratch;
    int64_t* wd = (int64_t*)(scratch + align256(sizeof(CrossTask) * (size_t)nb));
    hipError_t e = hipMemcpyAsync(Td, T.data(), sizeof(CrossTask) * nb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(wd, woff.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);       // pageable sources
    if (e != hipSuccess) return e;
    cross_dispatch(CrossBatch{Td, wd, nb}, grids[0].dim, prec == LCP_FP64, grid_for(woff[nb], 4), s);
    return hipGetLastError();
}

namespace {

template <int D, class TM, class R>
void cells_pair(R src, unsigned grid, int64_t cap, const void* zrec, hipStream_t s)
{
    hipLaunchKernelGGL((k_cells_cert<D, TM, R>), dim3(grid), dim3(256), 0, s, src, cap);
    if constexpr (D == 3 && std::is_same<TM, float>::value) {
        const unsigned g = grid_for(cap, kMcWaves * kMcCells);
        hipLaunchKernelGGL((k_cells_mfma<R>), dim3(g < 4096 ? g : 4096), dim3(kMcWaves * 64), 0, s, src, cap,
                           (const h8v*)zrec);
    } else {
        (void)zrec;
        hipLaunchKernelGGL((k_cells<D, TM, R>), dim3(grid), dim3(256), 0, s, src, cap);
    }
}

template <int D, class R>
void cells_dispatch(R src, bool f64, unsigned grid, int64_t cap, const void* zrec, hipStream_t s)
{
    if (f64) cells_pair<D, double>(src, grid, cap, zrec, s);
    else cells_pair<D, float>(src, grid, cap, zrec, s);
}

}  // namespace

namespace {

// Binary64: every cell.  Binary32: far cells first (k_sov_select), then the listed ones.
template <int D>
void sov_dispatch(const CellTask& t, double* wb, const double* gl, double* gout, int32_t* work, int64_t* wcount,
                  hipStream_t s)
{
    const int64_t ncell = t.grid.nc[0] * t.grid.nc[1] * t.grid.nc[2];
    const int64_t nz = (int64_t)t.ns << D;
    double* zabs = wb + nz;
    const unsigned gc = grid_for(ncell, 256);
    hipLaunchKernelGGL(k_wbank, dim3(grid_for(nz, 256)), dim3(256), 0, s, t.zb64, wb, nz);
    if (t.prec == LCP_FP64) {
        if (gl) hipLaunchKernelGGL((k_cells_sov_grad<D, double>), dim3(gc), dim3(256), 0, s, t, wb, gl, gout, ncell,
                                   nullptr, nullptr);
        else hipLaunchKernelGGL((k_cells_sov<D, double>), dim3(gc), dim3(256), 0, s, t, wb, ncell, nullptr, nullptr);
        return;
    }
    hipLaunchKernelGGL(k_zabsmax, dim3(1), dim3(256), 0, s, t.zb64, nz, zabs);
    hipLaunchKernelGGL(k_fill<int64_t>, dim3(1), dim3(64), 0, s, wcount, (int64_t)0, (int64_t)1);
    hipLaunchKernelGGL(k_sov_select<D>, dim3(gc), dim3(256), 0, s, t, ncell, zabs, gl ? nullptr : t.lcp, gout, work,
                       wcount);
    if (gl) hipLaunchKernelGGL((k_cells_sov_grad<D, float>), dim3(gc), dim3(256), 0, s, t, wb, gl, gout, ncell, work,
                               wcount);
    else hipLaunchKernelGGL((k_cells_sov<D, float>), dim3(gc), dim3(256), 0, s, t, wb, ncell, work, wcount);
}

}  // namespace

hipError_t launch_cells_sov(const CellTask& t, double* wb, hipStream_t s)
{
    const int64_t ncell = t.grid.nc[0] * t.grid.nc[1] * t.grid.nc[2];
    if (ncell <= 0) return hipSuccess;
    StageScope sc(s, ST_CELLS);
    if (t.grid.dim == 3) sov_dispatch<3>(t, wb, nullptr, nullptr, t.work, t.wcount, s);
    else sov_dispatch<2>(t, wb, nullptr, nullptr, t.work, t.wcount, s);
    return hipGetLastError();
}

hipError_t launch_cells_sov_grad(const CellTask& t, double* wb, const double* gl, double* gout, double* gmean,
                                 double* gvar, double* gcross, hipStream_t s)
{
    const int D = t.grid.dim;
    const int64_t ncell = t.grid.nc[0] * t.grid.nc[1] * t.grid.nc[2];
    const int64_t nv = t.grid.n[0] * t.grid.n[1] * t.grid.n[2];
    StageScope sc(s, ST_CELLS);
    if (ncell > 0) {
        if (D == 3) sov_dispatch<3>(t, wb, gl, gout, t.work, t.wcount, s);
        else sov_dispatch<2>(t, wb, gl, gout, t.work, t.wcount, s);
    }
    if (D == 3)
        hipLaunchKernelGGL(k_sov_gather<3>, dim3(grid_for(nv, 256)), dim3(256), 0, s, t.grid, gout, gmean, gvar,
                           gcross);
    else
        hipLaunchKernelGGL(k_sov_gather<2>, dim3(grid_for(nv, 256)), dim3(256), 0, s, t.grid, gout, gmean, gvar,
                           gcross);
    return hipGetLastError();
}

hipError_t launch_cells(const CellTask& t, int64_t ncells_cap, hipStream_t s)
{
    if (ncells_cap <= 0) return hipSuccess;
    StageScope sc(s, ST_CELLS);
    hipLaunchKernelGGL(k_zmax, dim3(1), dim3(256), 0, s, t.zb64, t.ns, 1 << t.grid.dim, t.zmax);
    hipLaunchKernelGGL(k_fill<int64_t>, dim3(1), dim3(64), 0, s, t.wcount, (int64_t)0, (int64_t)1);
    const unsigned grid = grid_for(ncells_cap, 256);
    const void* zrec = t.prec == LCP_FP64 ? nullptr : zbank_records(t.zb32, t.ns, t.grid.dim);
    if (t.grid.dim == 3) cells_dispatch<3>(CellsOne<3>{t}, t.prec == LCP_FP64, grid, ncells_cap, zrec, s);
    else cells_dispatch<2>(CellsOne<2>{t}, t.prec == LCP_FP64, grid, ncells_cap, zrec, s);
    return hipGetLastError();
}

size_t cells_batch_scratch(int nb)
{
    return align256(sizeof(CellTask) * (size_t)nb) + align256(sizeof(int64_t) * (size_t)(nb + 1));
}

hipError_t launch_cells_batch(const CellTask* tasks, int nb, char* scratch, hipStream_t s)
{
    if (nb <= 0) return hipSuccess;
    StageScope sc(s, ST_CELLS);
    std::vector<int64_t> coff(nb + 1, 0);
    for (int b = 0; b < nb; ++b) coff[b + 1] = coff[b] + tasks[b].grid.nc[0] * tasks[b].grid.nc[1] * tasks[b].grid.nc[2];
    CellTask* Td = (CellTask*)scratch;
    int64_t* cd = (int64_t*)(scratch + align256(sizeof(CellTask) * (size_t)nb));
    hipError_t e = hipMemcpyAsync(Td, tasks, sizeof(CellTask) * nb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(cd, coff.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);       // pageable sources
    if (e != hipSuccess) return e;
    const CellTask& t = tasks[0];
    hipLaunchKernelGGL(k_zmax, dim3(1), dim3(256), 0, s, t.zb64, t.ns, 1 << t.grid.dim, t.zmax);
    hipLaunchKernelGGL(k_fill<int64_t>, dim3(1), dim3(64), 0, s, t.wcount, (int64_t)0, (int64_t)1);
    const unsigned grid = grid_for(coff[nb], 256);
    const void* zrec = t.prec == LCP_FP64 ? nullptr : zbank_records(t.zb32, t.ns, t.grid.dim);
    if (t.grid.dim == 3) cells_dispatch<3>(CellsBatch{Td, cd, nb}, t.prec == LCP_FP64, grid, coff[nb], zrec, s);
    else cells_dispatch<2>(CellsBatch{Td, cd, nb}, t.prec == LCP_FP64, grid, coff[nb], zrec, s);
    return hipGetLastError();
}

hipError_t launch_zbank32(const double* zb, float* zb32, int64_t ns, int dim, hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    const int64_t n = ns << dim;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, zb, zb32, n);
    if (dim == 3) {
        const int64_t nspad = (ns + 31) / 32 * 32;
        hipLaunchKernelGGL(k_zrec, dim3((unsigned)ceil_div(nspad * 8, 256)), dim3(256), 0, s, zb, (int)ns, (int)nspad,
                           (_Float16*)((char*)zb32 + align256(sizeof(float) * (size_t)n)));
    }
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

// ------------------------------------------------------------ corner moments of listed cells
namespace {

// Cell index e (x fastest) -> its integer coordinates; false when e is out of range.
__device__ __forceinline__ bool cell_of(const GridP& g, int64_t e, int64_t (&c)[3])
{
    const int64_t nc = g.nc[0] * g.nc[1] * g.nc[2];
    if (e < 0 || e >= nc) return false;
    c[0] = e % g.nc[0];
    c[1] = (e / g.nc[0]) % g.nc[1];
    c[2] = e / (g.nc[0] * g.nc[1]);
    return true;
}

// Flag the 2^D corner vertices of every listed cell.
__global__ void k_mark_cells(GridP g, const int64_t* __restrict__ cells, int64_t n, int32_t* __restrict__ vmask)
{
    const int N = 1 << g.dim;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < n * N;
         it += (int64_t)gridDim.x * blockDim.x) {
        int64_t c[3];
        if (!cell_of(g, cells[it / N], c)) continue;
        const int q = (int)(it % N);
        const int64_t vx = c[0] + (q & 1), vy = c[1] + ((q >> 1) & 1), vz = c[2] + ((q >> 2) & 1);
        vmask[vx + g.n[0] * (vy + g.n[1] * (g.dim == 3 ? vz : 0))] = 1;
    }
}

__global__ void k_vertex_slots(const int32_t* __restrict__ vmask, const int32_t* __restrict__ off, int64_t nv,
                               int32_t* __restrict__ slot, int32_t* __restrict__ vlist)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        slot[i] = vmask[i] ? off[i] : -1;
        if (vmask[i]) vlist[off[i]] = (int32_t)i;
    }
}

// Corner mean (2^D) and covariance (2^D x 2^D, row-major) of each listed cell, gathered
// exactly as the Monte Carlo kernels gather them: diagonal = posterior variance, the other
// entries = the neighbour cross-covariances.  An out-of-range cell gets NaN.
template <int D>
__global__ void k_cell_moments(GridP g, const int64_t* __restrict__ cells, int64_t n, const int32_t* __restrict__ slot,
                               const double* __restrict__ mean, const double* __restrict__ var,
                               const double* __restrict__ cross, double* __restrict__ mu_out,
                               double* __restrict__ cov_out)
{
    constexpr int N = 1 << D;
    constexpr int NDIR = D == 3 ? 13 : 4;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t c[3];
        double* mo = mu_out + e * N;
        double* co = cov_out + e * N * N;
        if (!cell_of(g, cells[e], c)) {
            for (int q = 0; q < N; ++q) mo[q] = __builtin_nan("");
            for (int q = 0; q < N * N; ++q) co[q] = __builtin_nan("");
            continue;
        }
        int64_t sl[N];
        for (int q = 0; q < N; ++q) {
            const int64_t vx = c[0] + (q & 1), vy = c[1] + ((q >> 1) & 1), vz = c[2] + ((q >> 2) & 1);
            sl[q] = slot[vx + g.n[0] * (vy + g.n[1] * (D == 3 ? vz : 0))];
            mo[q] = mean[sl[q]];
            co[q * N + q] = var[sl[q]];
        }
        for (int p = 0; p < N; ++p)
            for (int q = p + 1; q < N; ++q) {
                const int dx = (q & 1) - (p & 1), dy = ((q >> 1) & 1) - ((p >> 1) & 1),
                          dz = ((q >> 2) & 1) - ((p >> 2) & 1);
                const double v = cross[(size_t)sl[p] * NDIR + dir_index(D, dx, dy, dz)];
                co[p * N + q] = v;
                co[q * N + p] = v;
            }
    }
}

}  // namespace

hipError_t launch_mark_cells(const GridP& g, const int64_t* cells, int64_t n, int32_t* vmask, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    StageScope sc(s, ST_MISC);
    hipLaunchKernelGGL(k_mark_cells, dim3(grid_for(n << g.dim, 256)), dim3(256), 0, s, g, cells, n, vmask);
    return hipGetLastError();
}

hipError_t launch_vertex_slots(const int32_t* vmask, const int32_t* off, int64_t nv, int32_t* slot, int32_t* vlist,
                               hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    hipLaunchKernelGGL(k_vertex_slots, dim3(grid_for(nv, 256)), dim3(256), 0, s, vmask, off, nv, slot, vlist);
    return hipGetLastError();
}

hipError_t launch_cell_moments(const GridP& g, const int64_t* cells, int64_t n, const int32_t* slot,
                               const double* mean, const double* var, const double* cross, double* mu_out,
                               double* cov_out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    StageScope sc(s, ST_MISC);
    if (g.dim == 3)
        hipLaunchKernelGGL(k_cell_moments<3>, dim3(grid_for(n, 256)), dim3(256), 0, s, g, cells, n, slot, mean, var,
                           cross, mu_out, cov_out);
    else
        hipLaunchKernelGGL(k_cell_moments<2>, dim3(grid_for(n, 256)), dim3(256), 0, s, g, cells, n, slot, mean, var,
                           cross, mu_out, cov_out);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace lcp
