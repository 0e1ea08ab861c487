// Cell stage of Sec. 4: cross-covariances between neighbouring vertices, the 2^D-corner
// covariance of each cell, its semidefinite Cholesky factor (binary64), and the Monte
// Carlo crossing count over the shared bank of standard normals.
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

__device__ __forceinline__ void dir_offset(int D, int dir, int& dx, int& dy, int& dz)
{
    int code = dir + (D == 3 ? 14 : 5);
    dx = code % 3 - 1;
    dy = (code / 3) % 3 - 1;
    dz = D == 3 ? code / 9 - 1 : 0;
}

// Neighbour cross-covariances cross[slot][dir] = k(x_p, x_q) - v_p . v_q, q = p + dir.
// A work-group owns a BX x BY x BZ brick of vertices (one thread each) and stages the V
// columns of the brick and its halo (x and y -1..+1, z +1) through LDS in chunks of R
// rows; each thread accumulates its 13 (3D) or 4 (2D) dot products in binary64.
// V is row-block-major (block rb of column s at (rb * ldv + s) * 16) with 16 * ceil(m / 16)
// written rows; within a 16-row block the rows may sit in the MFMA's output order, which no
// dot product of two columns depends on.
constexpr int CBX = 8, CBY = 8, CBZ = 4;
constexpr int CHX = CBX + 2, CHY = CBY + 2, CHZ = CBZ + 1;

template <class T, int R>
__global__ void __launch_bounds__(256) k_cross(KParams kp, GridP g, int64_t ldv, int mrows,
                                               const int32_t* __restrict__ slot, const T* __restrict__ V,
                                               double* __restrict__ cross)
{
    __shared__ T sv[CHX * CHY * CHZ][R + 1];
    __shared__ int32_t hs[CHX * CHY * CHZ];
    __shared__ int any;
    const int D = g.dim;
    const int ndir = D == 3 ? 13 : 4;
    const int tid = threadIdx.x;
    const int64_t nbx = (g.n[0] + CBX - 1) / CBX, nby = (g.n[1] + CBY - 1) / CBY;
    const int64_t nbz = D == 3 ? (g.n[2] + CBZ - 1) / CBZ : 1;
    const int hz_n = D == 3 ? CHZ : 1;
    const int nh = CHX * CHY * hz_n;
    for (int64_t brick = blockIdx.x; brick < nbx * nby * nbz; brick += gridDim.x) {
        const int64_t bx = brick % nbx, by = (brick / nbx) % nby, bz = brick / (nbx * nby);
        const int64_t x0 = bx * CBX, y0 = by * CBY, z0 = bz * (D == 3 ? CBZ : 1);
        __syncthreads();
        if (tid == 0) any = 0;
        __syncthreads();
        // slots of the halo vertices
        for (int h = tid; h < nh; h += blockDim.x) {
            const int hx = h % CHX, hy = (h / CHX) % CHY, hz = h / (CHX * CHY);
            const int64_t x = x0 - 1 + hx, y = y0 - 1 + hy, z = z0 + hz;
            int32_t sl = -1;
            if (x >= 0 && x < g.n[0] && y >= 0 && y < g.n[1] && z < g.n[2]) {
                const int64_t vid = x + g.n[0] * (y + g.n[1] * z);
                sl = slot ? slot[vid] : (int32_t)vid;
            }
            hs[h] = sl;
        }
        __syncthreads();
        // owner of this thread
        const int ox = tid % CBX, oy = (tid / CBX) % CBY, oz = D == 3 ? tid / (CBX * CBY) : 0;
        const bool owner_thread = D == 3 || tid < CBX * CBY;
        const int oh = (ox + 1) + CHX * ((oy + 1) + CHY * oz);
        const int32_t my = owner_thread ? hs[oh] : -1;
        if (my >= 0) any = 1;
        __syncthreads();
        if (!any) continue;
        int nbh[13];
        for (int dir = 0; dir < ndir; ++dir) {
            int dx, dy, dz;
            dir_offset(D, dir, dx, dy, dz);
            nbh[dir] = (ox + 1 + dx) + CHX * ((oy + 1 + dy) + CHY * (oz + dz));
        }
        double acc[13];
#pragma unroll
        for (int dir = 0; dir < 13; ++dir) acc[dir] = 0.0;
        // staging: 16-byte loads, all of a thread's loads issued before any LDS store
        constexpr int PV = 16 / sizeof(T);                 // elements per 16-byte load
        constexpr int NV = CHX * CHY * CHZ * R / PV;       // 16-byte pieces per chunk (3D)
        constexpr int PER = (NV + 255) / 256;
        using V4 = T __attribute__((ext_vector_type(16 / sizeof(T))));
        for (int r0 = 0; r0 < mrows; r0 += R) {
            V4 buf[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int e = tid + 256 * k;
                const int h = e / (R / PV), r = (e % (R / PV)) * PV;
                V4 v = V4{};
                if (h < nh) {
                    const int32_t sl = hs[h];
                    const int row = r0 + r;
                    if (sl >= 0 && row < mrows) v = *(const V4*)(V + ((size_t)(row >> 4) * ldv + sl) * 16 + (row & 15));
                }
                buf[k] = v;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int e = tid + 256 * k;
                const int h = e / (R / PV), r = (e % (R / PV)) * PV;
                if (h < nh)
#pragma unroll
                    for (int i = 0; i < PV; ++i) sv[h][r + i] = buf[k][i];
            }
            __syncthreads();
            if (my >= 0) {
#pragma unroll 4
                for (int r = 0; r < R; ++r) {
                    const double vp = (double)sv[oh][r];
#pragma unroll
                    for (int dir = 0; dir < 13; ++dir)
                        if (dir < ndir) acc[dir] = fma(vp, (double)sv[nbh[dir]][r], acc[dir]);
                }
            }
        }
        if (my >= 0) {
            const int64_t px = x0 + ox, py = y0 + oy, pz = z0 + oz;
            const double xp[3] = {vertex_coord(g, 0, px), vertex_coord(g, 1, py), D == 3 ? vertex_coord(g, 2, pz) : 0.0};
            for (int dir = 0; dir < ndir; ++dir) {
                int dx, dy, dz;
                dir_offset(D, dir, dx, dy, dz);
                double out = __builtin_nan("");
                if (hs[nbh[dir]] >= 0) {
                    const double xq[3] = {vertex_coord(g, 0, px + dx), vertex_coord(g, 1, py + dy),
                                          D == 3 ? vertex_coord(g, 2, pz + dz) : 0.0};
                    out = kernel_val(kp, kernel_r2(kp, xp, xq)) - acc[dir];
                }
                cross[(size_t)my * ndir + dir] = out;
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

template <int D, class TM>
__global__ void __launch_bounds__(256) k_cells(CellTask t, int64_t ncells_cap)
{
    constexpr int N = 1 << D;
    constexpr int NDIR = D == 3 ? 13 : 4;
    const GridP& g = t.grid;
    int64_t total;
    int64_t nleaf = 0;
    int64_t cpl = 1;
    if (t.leaves) {
        nleaf = *t.n_leaves;
        if (nleaf > t.leaf_cap) return;          // overflow: reconstruction skipped
        for (int d = 0; d < D; ++d) cpl *= t.leaf_edge;
        total = nleaf * cpl;
    } else {
        total = g.nc[0] * g.nc[1] * g.nc[2];
    }
    if (total > ncells_cap) total = ncells_cap;
    const TM* zb = std::is_same<TM, double>::value ? (const TM*)t.zb64 : (const TM*)t.zb32;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        int64_t cell[3] = {0, 0, 0};
        if (t.leaves) {
            const int64_t lf = it / cpl;
            int64_t loc = it % cpl;
            const uint64_t key = t.leaves[lf];
            const int level = (int)(key >> 58);
            const uint64_t mc = key & ((1ull << 58) - 1);
            int64_t nc[3] = {0, 0, 0};
            for (int b = 0; b < level; ++b)
                for (int d = 0; d < D; ++d) nc[d] |= (int64_t)((mc >> (b * D + d)) & 1) << b;
            const int64_t s = t.S0 >> level;
            bool in = true;
            for (int d = 0; d < D; ++d) {
                cell[d] = nc[d] * s + loc % t.leaf_edge;
                loc /= t.leaf_edge;
                in = in && cell[d] < g.nc[d];
            }
            if (!in) continue;
        } else {
            int64_t r = it;
            cell[0] = r % g.nc[0];
            r /= g.nc[0];
            cell[1] = r % g.nc[1];
            cell[2] = r / g.nc[1];
        }
        // gather corner data
        int64_t sl[N];
        double mu[N];
        double S[N][N];
        bool have = true;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const int64_t vx = cell[0] + (q & 1), vy = cell[1] + ((q >> 1) & 1), vz = cell[2] + ((q >> 2) & 1);
            const int64_t vid = vx + g.n[0] * (vy + g.n[1] * (D == 3 ? vz : 0));
            sl[q] = t.slot ? (int64_t)t.slot[vid] : vid;
            have = have && sl[q] >= 0;
        }
        const int64_t lin = cell[0] + g.nc[0] * (cell[1] + g.nc[1] * cell[2]);
        if (!have) {                      // a corner without posterior data: no estimate
            t.lcp[lin] = __builtin_nanf("");
            continue;
        }
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
        double Cd[N][N];
        chol_sd<N>(S, Cd);
        TM C[N][N], m[N];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            m[q] = (TM)mu[q];
#pragma unroll
            for (int r = 0; r < N; ++r) C[q][r] = (TM)Cd[q][r];
        }
        int cnt = 0;
        for (int s = 0; s < t.ns; ++s) {
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
        t.lcp[lin] = (float)cnt / (float)t.ns;
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

inline unsigned grid_for(int64_t n, int per)
{
    int64_t b = (n + per - 1) / per;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_cross(const Model& M, int prec, const GridP& g, const int32_t* vlist, const int64_t* nv_dev,
                        int64_t nv_cap, const int32_t* slot, const void* V, double* cross, hipStream_t s)
{
    (void)vlist;
    (void)nv_dev;
    if (nv_cap <= 0) return hipSuccess;
    StageScope sc(s, ST_CROSS);
    const int64_t nb = ceil_div(g.n[0], CBX) * ceil_div(g.n[1], CBY) * (g.dim == 3 ? ceil_div(g.n[2], CBZ) : 1);
    const unsigned grid = (unsigned)(nb < 65536 ? nb : 65536);
    if (prec == LCP_FP64)
        hipLaunchKernelGGL((k_cross<double, 16>), dim3(grid), dim3(256), 0, s, M.kp, g, nv_cap, 16 * M.nrb, slot,
                           (const double*)V, cross);
    else
        hipLaunchKernelGGL((k_cross<float, 32>), dim3(grid), dim3(256), 0, s, M.kp, g, nv_cap, 16 * M.nrb, slot,
                           (const float*)V, cross);
    return hipGetLastError();
}

hipError_t launch_cells(const CellTask& t, int64_t ncells_cap, hipStream_t s)
{
    if (ncells_cap <= 0) return hipSuccess;
    StageScope sc(s, ST_CELLS);
    unsigned grid = grid_for(ncells_cap, 256);
    const bool f64 = t.prec == LCP_FP64;
    if (t.grid.dim == 3) {
        if (f64) hipLaunchKernelGGL((k_cells<3, double>), dim3(grid), dim3(256), 0, s, t, ncells_cap);
        else hipLaunchKernelGGL((k_cells<3, float>), dim3(grid), dim3(256), 0, s, t, ncells_cap);
    } else {
        if (f64) hipLaunchKernelGGL((k_cells<2, double>), dim3(grid), dim3(256), 0, s, t, ncells_cap);
        else hipLaunchKernelGGL((k_cells<2, float>), dim3(grid), dim3(256), 0, s, t, ncells_cap);
    }
    return hipGetLastError();
}

hipError_t launch_zbank32(const double* zb, float* zb32, int64_t n, hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, zb, zb32, n);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s)
{
    StageScope sc(s, ST_MISC);
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace lcp
