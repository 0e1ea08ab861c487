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

// One wave per vertex slot: cross[slot][dir] = k(x_p, x_q) - v_p . v_q for q = p + dir.
// Each V column holds 16 * ceil(m / 16) written rows; within a 16-row block the rows
// may sit in the MFMA's output order, which no dot product of two columns depends on.
// Rows beyond the last block are padding and are not read.
template <class T>
__global__ void __launch_bounds__(256) k_cross(KParams kp, GridP g, int mp, int mrows, const int32_t* __restrict__ vlist,
                                               const int64_t* __restrict__ nv_dev, int64_t nv_cap,
                                               const int32_t* __restrict__ slot, const T* __restrict__ V,
                                               double* __restrict__ cross)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int64_t nv = nv_dev ? *nv_dev : nv_cap;
    if (nv > nv_cap) nv = nv_cap;
    const int D = g.dim;
    const int ndir = D == 3 ? 13 : 4;
    constexpr int PER = kMaxM / 64;
    for (int64_t p = wid; p < nv; p += nw) {
        const int64_t vid = vlist ? (int64_t)vlist[p] : p;
        int64_t c[3];
        c[0] = vid % g.n[0];
        c[1] = (vid / g.n[0]) % g.n[1];
        c[2] = vid / (g.n[0] * g.n[1]);
        double xp[3] = {vertex_coord(g, 0, c[0]), vertex_coord(g, 1, c[1]), D == 3 ? vertex_coord(g, 2, c[2]) : 0.0};
        double vp[PER];
        const T* Vp = V + (size_t)p * mp;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            int j = lane + 64 * k;
            vp[k] = j < mrows ? (double)Vp[j] : 0.0;
        }
        for (int dir = 0; dir < ndir; ++dir) {
            int dx, dy, dz;
            dir_offset(D, dir, dx, dy, dz);
            int64_t q[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
            bool in = q[0] >= 0 && q[0] < g.n[0] && q[1] >= 0 && q[1] < g.n[1] && q[2] >= 0 && q[2] < g.n[2];
            int64_t sq = -1;
            if (in) {
                int64_t vq = q[0] + g.n[0] * (q[1] + g.n[1] * q[2]);
                sq = slot ? (int64_t)slot[vq] : vq;
            }
            double out = __builtin_nan("");
            if (sq >= 0) {
                const T* Vq = V + (size_t)sq * mp;
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    int j = lane + 64 * k;
                    if (j < mrows) s = fma(vp[k], (double)Vq[j], s);
                }
                for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
                double xq[3] = {vertex_coord(g, 0, q[0]), vertex_coord(g, 1, q[1]),
                                D == 3 ? vertex_coord(g, 2, q[2]) : 0.0};
                out = kernel_val(kp, kernel_r2(kp, xp, xq)) - s;
            }
            if (lane == 0) cross[(size_t)p * ndir + dir] = out;
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
    if (nv_cap <= 0) return hipSuccess;
    StageScope sc(s, ST_CROSS);
    unsigned grid = grid_for(nv_cap * 64, 256);
    if (prec == LCP_FP64)
        hipLaunchKernelGGL(k_cross<double>, dim3(grid), dim3(256), 0, s, M.kp, g, M.m_pad, 16 * M.nrb, vlist, nv_dev, nv_cap,
                           slot, (const double*)V, cross);
    else
        hipLaunchKernelGGL(k_cross<float>, dim3(grid), dim3(256), 0, s, M.kp, g, M.m_pad, 16 * M.nrb, vlist, nv_dev, nv_cap,
                           slot, (const float*)V, cross);
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
