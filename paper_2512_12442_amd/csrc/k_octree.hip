// Octree adaptive query (Alg. 1) run level-synchronously on the GPU, followed by the
// reconstruction of the emitted nodes only (Sec. 5.3, last paragraph).
//
// Per level: a wave per frontier node tests the observations inside the closed node box
// (p1, p2 of Alg. 1); nodes that need the region bound are compacted by a prefix sum and
// searched in batches (3^D lattice, then projected-gradient steps) through the binary64
// posterior kernel; UB = 1 - B^d decides; a second prefix sum writes the children in
// Morton order, so the frontier -- and the leaf list -- stay sorted by key without a sort.
// All counts stay in device memory: grids are sized by per-level capacities and kernels
// loop over the device count, so the whole query is enqueued without host round trips.
#include "lcp_internal.h"

namespace lcp {

namespace {

struct Oct {
    GridP g;
    int D;
    int64_t S0;              // root edge in cells, a power of two
    int lgS0;                // log2 S0
    int Lmax;
    double theta;
    double alpha;
    int bound_at_max;
    int steps;
    int kd;                  // 1: K-D tree (one axis halved per level), depths 0 .. D Lmax
    int Ldepth;              // deepest level: Lmax (octree) or D Lmax (K-D tree)
    int64_t nodes[72];       // node lattice extent per level and axis: nodes[l*3 + d]
    int64_t statoff[24];     // offset of each level's status grid
};

// K-D tree (Sec. 9: split the axes in turn): the split at depth L halves axis
// D - 1 - (L mod D), so every D-th depth is an octree level with the same Morton code; the
// code of a node lists its split bits in split order, the first split most significant.
__device__ __forceinline__ int kd_axis(int D, int L) { return D - 1 - L % D; }

// Halvings of axis d at this level.
__device__ __forceinline__ int node_shift(const Oct& o, int level, int d)
{
    return o.kd ? level / o.D + (d >= o.D - level % o.D ? 1 : 0) : level;
}

__device__ __forceinline__ void key_coords_oct(int D, uint64_t key, int& level, int64_t* c)
{
    level = (int)(key >> 58);
    uint64_t mc = key & ((1ull << 58) - 1);
    c[0] = c[1] = c[2] = 0;
    for (int b = 0; b < level; ++b)
#pragma unroll
        for (int d = 0; d < 3; ++d)                        // fixed bounds: c stays in registers
            if (d < D) c[d] |= (int64_t)((mc >> (b * D + d)) & 1) << b;
}

__device__ __forceinline__ void key_coords(const Oct& o, uint64_t key, int& level, int64_t* c)
{
    if (!o.kd) {
        key_coords_oct(o.D, key, level, c);
        return;
    }
    level = (int)(key >> 58);
    const uint64_t code = key & ((1ull << 58) - 1);
    // selects rather than c[a] with a run-time a, which would put c in scratch memory
    int64_t c0 = 0, c1 = 0, c2 = 0;
    for (int j = 0; j < level; ++j) {
        const int a = kd_axis(o.D, j);
        const int64_t bit = (int64_t)((code >> (level - 1 - j)) & 1);
        c0 = a == 0 ? 2 * c0 + bit : c0;
        c1 = a == 1 ? 2 * c1 + bit : c1;
        c2 = a == 2 ? 2 * c2 + bit : c2;
    }
    c[0] = c0;
    c[1] = c1;
    c[2] = c2;
}

__device__ __forceinline__ int64_t pick3(const int64_t* c, int a) { return a == 0 ? c[0] : (a == 1 ? c[1] : c[2]); }

__device__ __forceinline__ uint64_t make_key(const Oct& o, int level, const int64_t* c)
{
    const int D = o.D;
    uint64_t k = 0;
    if (o.kd) {
        for (int j = 0; j < level; ++j) {
            const int a = kd_axis(D, j);
            k = (k << 1) | (uint64_t)((pick3(c, a) >> (node_shift(o, level, a) - 1 - j / D)) & 1);
        }
    } else {
        for (int b = 0; b < level; ++b)
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (d < D) k |= (uint64_t)((c[d] >> b) & 1) << (b * D + d);
    }
    return ((uint64_t)level << 58) | k;
}

// Cell range [clo, chi) of a node, its physical box and vertex count d.
__device__ __forceinline__ void node_box(const Oct& o, int level, const int64_t* c, int64_t* clo, int64_t* chi,
                                         double* blo, double* bhi, int64_t* dpts)
{
    int64_t d = 1;
    for (int k = 0; k < 3; ++k) {
        if (k < o.D) {
            const int64_t s = o.S0 >> node_shift(o, level, k);
            clo[k] = c[k] * s;
            chi[k] = (c[k] + 1) * s;
            if (chi[k] > o.g.nc[k]) chi[k] = o.g.nc[k];
            blo[k] = vertex_coord(o.g, k, clo[k]);
            bhi[k] = vertex_coord(o.g, k, chi[k]);
            d *= chi[k] - clo[k] + 1;
        } else {
            clo[k] = 0;
            chi[k] = 1;
            blo[k] = bhi[k] = 0.0;
        }
    }
    *dpts = d;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_isum(int v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Slots in a list shared by the whole launch: every thread of the block passes its item
// count n and gets the first of n consecutive slots of *counter; the block takes its range
// with one atomic.  The order of the blocks' ranges is not fixed, so a list built this way
// only routes per-item work whose results do not depend on the position.  Every thread of
// the block must call it (it holds barriers).
__device__ int block_claim(int n, int64_t* counter)
{
    __shared__ int sh[65];
    int tot;
    const int ex = block_excl_scan(n, sh, &tot);
    __shared__ int base;
    if (threadIdx.x == 0) base = tot > 0 ? (int)atomicAdd((unsigned long long*)counter, (unsigned long long)tot) : 0;
    __syncthreads();
    const int r = base + ex;
    __syncthreads();
    return r;
}

// P(Y_i < theta), P(Y_i > theta) for each observation from its latent posterior.
__global__ void k_obs_q(const double* __restrict__ mu, const double* __restrict__ var, int m, double theta,
                        double* __restrict__ qlo, double* __restrict__ qhi)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (var[i] > 0.0) {
        double z = (theta - mu[i]) / sqrt(var[i]);
        qlo[i] = 0.5 * erfc(-z / 1.41421356237309504880168872421);
        qhi[i] = 0.5 * erfc(z / 1.41421356237309504880168872421);
    } else {
        qlo[i] = mu[i] < theta ? 1.0 : 0.0;
        qhi[i] = mu[i] > theta ? 1.0 : 0.0;
    }
}

__global__ void k_root(uint64_t* keys, int64_t* cnt, int32_t* sp_cnt, uint8_t* hob)
{
    if (threadIdx.x == 0) {
        keys[0] = 0;
        *cnt = 1;
        hob[0] = 1;   // the root may hold observations
    }
    for (int i = threadIdx.x; i < kSplitGrid; i += blockDim.x) sp_cnt[i] = 0;   // shared-tile counters
}

// Preliminary decision of Alg. 1 for every frontier node (one wave per node).
// Work lists and values of the region bound (Sec. 5.1), per level.
struct BoundBufs {
    int32_t* bnode;     // stage-1 node -> frontier index
    double* side;
    double* gmin;
    double* cpts;       // stage-1 centres, 3 per node
    double* cmean;
    double* cvar;
    int32_t* lnode;     // stage-2 node -> stage-1 node
    int32_t* ngrid;     // node lattice of this level -> stage-2 node (-1: not in stage 2)
    int32_t* lmask;     // per stage-2 node: lattice points it evaluates (owns), bit i = point i
    int32_t* loff;      // per stage-2 node: first slot of its owned points
    int32_t* lown;      // per stage-2 node and lattice point i (32 per node): owner's stage-2 index * 32 + its point index
    int32_t* lnode2;    // corners first: the nodes the corners left open -> stage-1 node
    int32_t* bidx;      // corners first: per stage-1 node, the lattice index of its best corner
    double* dpts;       // certificate between the lattice passes: per node the corners left open, its
    double* dbox;       //   centre (3) and box (lo[D], hi[D]),
    double* dcert;      //   mu(c), mu_lo, mu_hi, var_hi,
    int32_t* lnode3;    //   and the nodes it leaves open -> stage-1 node
    double* lat_pts;    // unique lattice points, 3 doubles each
    double* lat_mean;
    double* lat_var;
    int32_t* dnode;     // stage-3 node -> stage-1 node
    double* dbx;        // per stage-3 node: box lo[3], hi[3], side, g_min so far (64 B)
    int64_t* ddp;       //   and its grid points
    int32_t* fcand;     // search: per frontier node, its stage-3 index or -1 (the emit count decides it)
    int32_t* done;
    double* gp_mean;    // posterior (and gradient) at the stage-3 points
    double* gp_var;
    double* gp_dmean;
    double* gp_dvar;
    int64_t* cnt;       // [0] stage-1 nodes, [1] stage-2 nodes, [2] unique lattice points, [3] stage-3 nodes,
                        // [4] nodes the corners left open, [5] of those, the nodes the certificate left open
    double* box;        // certified bound: node box lo[D], hi[D] per stage-1 node (null: search)
    double* cert;       //   mu(c), mu_lo, mu_hi, var_hi per stage-1 node
};

// path: 0 subdivide (both sides above alpha), 1 bound below, 2 bound above,
//       3 finest level emitted without a test, 4 bound with side from the centre mean.
// With direct set (the search bound), the search's stage-1 list is the frontier itself:
// every node's centre is written, the nodes that need no bound are skipped at the stage-1
// decision, the later stage lists start empty and the level's node lattice is cleared.
__global__ void __launch_bounds__(256) k_prelim(Oct o, int level, const uint64_t* __restrict__ keys,
                                                const int64_t* __restrict__ nf_dev, int64_t cap,
                                                const double* __restrict__ X, int m, const double* __restrict__ qlo,
                                                const double* __restrict__ qhi, int32_t* __restrict__ path,
                                                int32_t* __restrict__ need, int32_t* __restrict__ sub, BoundBufs B,
                                                int direct, const uint8_t* __restrict__ hob)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int64_t nf = *nf_dev;
    if (nf > cap) nf = cap;
    if (direct) {
        const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (gt == 0) {
            B.cnt[0] = nf;
            B.cnt[1] = 0;
            B.cnt[2] = 0;
            B.cnt[3] = 0;
            B.cnt[4] = 0;
            B.cnt[5] = 0;
        }
        for (int64_t i = gt; i < cap; i += (int64_t)gridDim.x * blockDim.x) B.ngrid[i] = -1;
    }
    for (int64_t f = wid; f < nf; f += nw) {
        int lv;
        int64_t c[3], clo[3], chi[3], dp;
        double blo[3], bhi[3];
        key_coords(o, keys[f], lv, c);
        node_box(o, level, c, clo, chi, blo, bhi, &dp);
        int pth;
        if (level == o.Ldepth && !o.bound_at_max) {
            pth = 3;
        } else {
            // Observation rows are zero padded beyond the dimension and so is the node box, so
            // the three closed-interval tests hold for every axis; no branch per observation,
            // and each lane's loads are independent of the previous iteration.
            int nin = 0;
            double p1 = -1.0, p2 = -1.0;
            // a node's closed box lies in its parent's, so a parent without observations has
            // children without them (hob: the parent held some)
            const int mm = hob[f] ? m : 0;
#pragma unroll 4
            for (int i = lane; i < mm; i += 64) {
                const double2 x01 = *(const double2*)(X + (int64_t)i * 4);
                const double x2 = X[(int64_t)i * 4 + 2];
                const double ql = qlo[i], qh = qhi[i];
                const bool in = (x01.x >= blo[0]) & (x01.x <= bhi[0]) & (x01.y >= blo[1]) & (x01.y <= bhi[1]) &
                                (x2 >= blo[2]) & (x2 <= bhi[2]);
                nin += in ? 1 : 0;
                p1 = in ? fmax(p1, ql) : p1;
                p2 = in ? fmax(p2, qh) : p2;
            }
            nin = wave_isum(nin);
            p1 = wave_max(p1);
            p2 = wave_max(p2);
            if (nin > 0 && p1 > o.alpha && p2 > o.alpha) pth = 0;
            else if (nin > 0) pth = (p2 <= o.alpha) ? 1 : 2;
            else pth = 4;
        }
        if (lane == 0) {
            path[f] = pth;
            need[f] = (pth == 1 || pth == 2 || pth == 4) ? 1 : 0;
            sub[f] = (pth == 0 || pth == 3) ? 1 : 0;
            if (direct) {
                B.bnode[f] = (int32_t)f;
                B.fcand[f] = -1;
                for (int d = 0; d < 3; ++d) B.cpts[f * 3 + d] = d < o.D ? 0.5 * (blo[d] + bhi[d]) : 0.0;
            }
        }
    }
}

// Region bound of Sec. 5.1 in three stages with the decision of the full search:
// UB = 1 - B^d is non-increasing in g_min and every evaluated point can only lower g_min,
// so a node is subdivided as soon as one evaluated point gives UB > alpha.
//   stage 1: the box centre (also the side for nodes without observations);
//   stage 2: the {lo, mid, hi}^D lattice for nodes stage 1 left open;
//   stage 3: projected-gradient steps for nodes the lattice left open.
// The search's stage-1 list is the frontier; each stage's decision kernel appends the nodes
// it leaves open to the next stage's list (block_claim), so the lists are built without
// scans.  Every value a stage computes depends on its node alone, never on a list position.
// Large levels take the lattice's corners first, and at the largest octree levels the
// certified box bound (k_lattice_cert) settles nodes between the two lattice passes.  The
// descent steps run in the epilogue of their binary64 probes, and the emit count takes the
// decision of the nodes that reached the descent.
__global__ void k_bound_setup(Oct o, int level, const uint64_t* __restrict__ keys, const int64_t* __restrict__ nf_dev,
                              int64_t cap, const int32_t* __restrict__ need, const int32_t* __restrict__ nidx,
                              BoundBufs B)
{
    int64_t nf = *nf_dev;
    if (nf > cap) nf = cap;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += (int64_t)gridDim.x * blockDim.x) {
        if (!need[f]) continue;
        const int64_t b = nidx[f];
        B.bnode[b] = (int32_t)f;
        int lv;
        int64_t c[3], clo[3], chi[3], dp;
        double blo[3], bhi[3];
        key_coords(o, keys[f], lv, c);
        node_box(o, level, c, clo, chi, blo, bhi, &dp);
        for (int d = 0; d < 3; ++d) B.cpts[b * 3 + d] = d < o.D ? 0.5 * (blo[d] + bhi[d]) : 0.0;
        if (B.box) {
            for (int d = 0; d < o.D; ++d) {
                B.box[b * 2 * o.D + d] = blo[d];
                B.box[b * 2 * o.D + o.D + d] = bhi[d];
            }
        }
    }
}

// Certified bound: the side (nodes without observations: from the centre mean), the lower
// bound of the margin over the box -- (theta - mu_hi) / sigma_hi below, (mu_lo - theta) /
// sigma_hi above, -infinity when theta lies within the mean's bounds -- and UB = 1 - B^d.
__global__ void k_cert_decide(Oct o, int level, const uint64_t* __restrict__ keys, const int32_t* __restrict__ path,
                              BoundBufs B, int32_t* __restrict__ sub)
{
    const int64_t nb = B.cnt[0];
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t f = B.bnode[b];
        const int p = path[f];
        const double* cb = B.cert + b * 4;
        const double side = p == 1 ? 1.0 : (p == 2 ? -1.0 : (cb[0] < o.theta ? 1.0 : -1.0));
        const double mu = side > 0 ? cb[2] : cb[1];
        const double g = side * (o.theta - mu) < 0.0 ? -__builtin_inf() : margin(side, o.theta, mu, cb[3]);
        int lv;
        int64_t c[3], clo[3], chi[3], dp;
        double blo[3], bhi[3];
        key_coords(o, keys[f], lv, c);
        node_box(o, level, c, clo, chi, blo, bhi, &dp);
        B.side[b] = side;
        B.gmin[b] = g;
        sub[f] = upper_bound(g, dp) > o.alpha ? 1 : 0;
    }
}

// Linear index of a node in the node lattice of its level.
__device__ __forceinline__ int64_t node_lin(const Oct& o, int level, const int64_t* c)
{
    return c[0] + o.nodes[level * 3 + 0] * (c[1] + o.nodes[level * 3 + 1] * c[2]);
}

// Stage 1: side choice and the centre's bound, for the stage-1 nodes that need a bound.
// The nodes it leaves open join stage 2: a slot in its list and their place in the node
// lattice of this level.  Without centre values (centre = 0) every such node joins stage 2
// and a node without observations takes its side from the lattice's centre point there:
// the centre is a lattice point and the bound only grows with more points, so the decisions
// are those of the staged search.
__global__ void __launch_bounds__(256) k_bound_centre(Oct o, int level, const uint64_t* __restrict__ keys,
                                                      const int32_t* __restrict__ path,
                                                      const int32_t* __restrict__ need, BoundBufs B,
                                                      int32_t* __restrict__ sub, int centre)
{
    const int64_t nb = B.cnt[0];
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nb; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = base + threadIdx.x;
        bool open = false;
        int64_t c[3] = {0, 0, 0};
        if (b < nb) {
            const int32_t f = B.bnode[b];
            if (need[f]) {
                const int p = path[f];
                int lv;
                int64_t clo[3], chi[3], dp;
                double blo[3], bhi[3];
                key_coords(o, keys[f], lv, c);
                if (centre) {
                    const double side = p == 1 ? 1.0 : (p == 2 ? -1.0 : (B.cmean[b] < o.theta ? 1.0 : -1.0));
                    const double g = margin(side, o.theta, B.cmean[b], B.cvar[b]);
                    node_box(o, level, c, clo, chi, blo, bhi, &dp);
                    B.side[b] = side;
                    B.gmin[b] = g;
                    open = !(upper_bound(g, dp) > o.alpha);
                    if (!open) sub[f] = 1;
                } else {
                    B.side[b] = p == 1 ? 1.0 : (p == 2 ? -1.0 : 0.0);   // 0: from the lattice's centre
                    open = true;
                }
            }
        }
        const int l = block_claim(open ? 1 : 0, B.cnt + 1);          // every thread of the block
        if (open) {
            B.lnode[l] = (int32_t)b;
            B.ngrid[node_lin(o, level, c)] = l;
        }
    }
}

// Stage 2 shares lattice points between neighbouring open nodes.  A lattice point with
// digit (0 lo, 1 mid, 2 hi) per axis lies in the nodes offset by 0 or -1 (lo) / +1 (hi)
// along the axes where it sits on the box boundary; those nodes compute bitwise the same
// coordinates for it (the shared face has the same vertex, the mid of a shared edge the
// same two vertices).  It is evaluated once, by the open node with the lowest linear index
// in the node lattice, and every node reads it from there.

// Owner of point i (digits base 3, x fastest) of the node at c: its node lattice coords
// and the point's index in the owner's lattice.  The node itself is always a candidate.
__device__ __forceinline__ void lattice_owner(const Oct& o, int level, const int32_t* __restrict__ ngrid,
                                              const int64_t* c, int i, int64_t* oc, int* oi)
{
    int dig[3] = {1, 1, 1};
    int r = i;
    for (int d = 0; d < o.D; ++d) {
        dig[d] = r % 3;
        r /= 3;
    }
    int64_t best = node_lin(o, level, c);
    int64_t bc[3] = {c[0], c[1], c[2]};
    int bdig[3] = {dig[0], dig[1], dig[2]};
    const int nalt = 1 << o.D;
    for (int mask = 1; mask < nalt; ++mask) {
        int64_t q[3] = {c[0], c[1], c[2]};
        int qd[3] = {dig[0], dig[1], dig[2]};
        bool ok = true;
        for (int d = 0; d < o.D && ok; ++d) {
            if (!((mask >> d) & 1)) continue;
            if (dig[d] == 0) { q[d] = c[d] - 1; qd[d] = 2; }
            else if (dig[d] == 2) { q[d] = c[d] + 1; qd[d] = 0; }
            else ok = false;
            if (ok && (q[d] < 0 || q[d] >= o.nodes[level * 3 + d])) ok = false;
        }
        if (!ok) continue;
        const int64_t lin = node_lin(o, level, q);
        if (ngrid[lin] >= 0 && lin < best) {
            best = lin;
            for (int d = 0; d < 3; ++d) { bc[d] = q[d]; bdig[d] = qd[d]; }
        }
    }
    for (int d = 0; d < 3; ++d) oc[d] = bc[d];
    *oi = bdig[0] + 3 * bdig[1] + (o.D == 3 ? 9 * bdig[2] : 0);
}

__device__ __forceinline__ void lattice_point(const Oct& o, const double* blo, const double* bhi, int i, double* x)
{
    // Every lane forms lo, mid and hi and selects one: per-digit branches here were lowered
    // with the hi copy in the digit-0 block (hipcc of ROCm 7.2, k_lattice with the box kept
    // live), which left digit-2 coordinates unwritten.
    int r = i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int digit = r % 3;
        r /= 3;
        const double lo = blo[d], hi = bhi[d], mid = 0.5 * (lo + hi);
        const double v = digit == 0 ? lo : (digit == 1 ? mid : hi);
        x[d] = d < o.D ? v : 0.0;
    }
}

// Which of the lattice points in pmask (bit i = point i) each node of a stage-2 list owns (32
// lanes per node, lane i = point i), a range of slots for them in the list of unique lattice
// points (count B.cnt[2]), and their coordinates there.  The owners are found among the nodes
// registered in the node lattice.
__global__ void __launch_bounds__(512) k_lattice_own(Oct o, int level, const uint64_t* __restrict__ keys, BoundBufs B,
                                                     const int32_t* __restrict__ list, const int64_t* __restrict__ n_list,
                                                     uint32_t pmask)
{
    const int64_t nl = *n_list;
    const int npt = o.D == 3 ? 27 : 9;
    const int sub_lane = threadIdx.x & 31;
    const int per = blockDim.x / 32;                                   // nodes per block and pass
    for (int64_t base = (int64_t)blockIdx.x * per; base < nl; base += (int64_t)gridDim.x * per) {
        const int64_t l = base + (threadIdx.x >> 5);
        bool own = false;
        double blo[3], bhi[3];
        if (l < nl && sub_lane < npt && ((pmask >> sub_lane) & 1)) {
            int lv;
            int64_t c[3], oc[3], clo[3], chi[3], dp;
            key_coords(o, keys[B.bnode[list[l]]], lv, c);
            node_box(o, level, c, clo, chi, blo, bhi, &dp);
            int oi;
            lattice_owner(o, level, B.ngrid, c, sub_lane, oc, &oi);
            own = node_lin(o, level, oc) == node_lin(o, level, c);
            B.lown[l * 32 + sub_lane] = B.ngrid[node_lin(o, level, oc)] * 32 + oi;
        }
        const uint64_t bal = __ballot(own);
        const uint32_t mask = (uint32_t)(bal >> (threadIdx.x & 32));
        const int first = block_claim((l < nl && sub_lane == 0) ? __builtin_popcount(mask) : 0, B.cnt + 2);
        const int slot0 = __shfl(first, threadIdx.x & 32, 64);            // the node's first slot
        if (own) {
            double x[3];
            lattice_point(o, blo, bhi, sub_lane, x);
            const int64_t slot = slot0 + __builtin_popcount(mask & ((1u << sub_lane) - 1));
            for (int d = 0; d < 3; ++d) B.lat_pts[slot * 3 + d] = x[d];
        }
        if (l < nl && sub_lane == 0) {
            B.lmask[l] = (int32_t)mask;
            B.loff[l] = slot0;
        }
    }
}

// Stage 2: lattice minimum (lowest index wins ties), start point, bound; nodes left open
// join the descent -- a slot in the stage-3 list, their start point in gx -- or are skipped
// when the search has no steps.  32 lanes per node, lane i reads point i (of pmask) from
// its owner's slot (owner as found by k_lattice_own).  Large levels take the corners first:
//   mode 0: every lattice point, the decision above;
//   mode 1: the 2^D corners.  A node whose best corner already gives UB > alpha is
//           subdivided; the others keep their best corner (value and index) and join a
//           second list, which replaces the node lattice's entries (decided nodes: -1);
//   mode 2: the other points of the second list's nodes, then the decision on the minimum
//           of both passes (lowest index on ties), which is the minimum over the lattice.
// A best corner with UB > alpha means a lattice minimum with UB > alpha (UB falls as g_min
// grows, and the minimum is at most the corner's value); otherwise the minimum of both passes
// is the lattice minimum and its point.  The decisions, minima and start points are those of
// mode 0.  The corner passes run only after a centre stage, so every node's side is known.
__global__ void __launch_bounds__(512) k_lattice(Oct o, int level, const uint64_t* __restrict__ keys, BoundBufs B,
                                                  int32_t* __restrict__ sub, double* __restrict__ gx,
                                                  const int32_t* __restrict__ list, const int64_t* __restrict__ n_list,
                                                  uint32_t pmask, int mode, int csave, int cvals)
{
    const int64_t nl = *n_list;
    if (mode == 1 && blockIdx.x == 0 && threadIdx.x == 0) B.cnt[2] = 0;   // the second pass's point slots
    const int npt = o.D == 3 ? 27 : 9;
    const int sub_lane = threadIdx.x & 31;
    const int per = blockDim.x / 32;                                   // nodes per block and pass
    for (int64_t base = (int64_t)blockIdx.x * per; base < nl; base += (int64_t)gridDim.x * per) {
        const int64_t l = base + (threadIdx.x >> 5);
        const bool live = l < nl;
        int32_t b = 0, f = 0;
        int64_t c[3] = {0, 0, 0};
        double gv = __builtin_inf(), side = 1.0, mu = 0.0, var = 0.0;
        const bool in_mask = sub_lane < npt && ((pmask >> sub_lane) & 1);
        // cvals: the centre (point (npt - 1) / 2) is not in pmask; its value is stage 1's
        const bool from_centre = cvals && sub_lane == (npt - 1) / 2;
        if (live) {
            b = list[l];
            f = B.bnode[b];
            side = B.side[b];
            int lv;
            key_coords(o, keys[f], lv, c);
            if (in_mask) {
                const int32_t own = B.lown[l * 32 + sub_lane];
                const int32_t ol = own >> 5, oi = own & 31;
                const int64_t slot = B.loff[ol] + __builtin_popcount(B.lmask[ol] & ((1 << oi) - 1));
                mu = B.lat_mean[slot];
                var = B.lat_var[slot];
            } else if (from_centre) {
                mu = B.cmean[b];
                var = B.cvar[b];
            }
        }
        // stage 1 skipped: a node without observations takes its side from the centre point
        // (digits 1 on every axis: point (npt - 1) / 2), as stage 1 would
        const double mc = __shfl(mu, (threadIdx.x & 32) + (npt - 1) / 2, 64);
        if (mode == 0 && side == 0.0) side = mc < o.theta ? 1.0 : -1.0;
        if (live && (in_mask || from_centre)) gv = margin(side, o.theta, mu, var);
        // minimum over the 32 lanes of the node, lowest point index on ties
        double best = gv;
        int ib = sub_lane;
        for (int off = 16; off >= 1; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oib = __shfl_xor(ib, off, 64);
            if (ob < best || (ob == best && oib < ib)) {
                best = ob;
                ib = oib;
            }
        }
        bool enter = false, cont = false;
        double x[3] = {0.0, 0.0, 0.0};
        double blo[3] = {0.0, 0.0, 0.0}, bhi[3] = {0.0, 0.0, 0.0};
        int64_t dp = 0;
        if (live && sub_lane == 0) {
            int64_t clo[3], chi[3];
            node_box(o, level, c, clo, chi, blo, bhi, &dp);
            if (mode == 2) {
                // the best corner of the first pass against the best of the other points
                const double bc = B.gmin[b];
                const int ic = B.bidx[b];
                if (!(best < bc || (best == bc && ib < ic))) {
                    best = bc;
                    ib = ic;
                }
            }
            if (mode == 1) {
                if (upper_bound(best, dp) > o.alpha) {
                    sub[f] = 1;
                    B.ngrid[node_lin(o, level, c)] = -1;
                } else {
                    cont = true;
                    B.gmin[b] = best;
                    B.bidx[b] = ib;
                }
            } else {
                B.side[b] = side;
                B.gmin[b] = best;
                const bool open = !(upper_bound(best, dp) > o.alpha);
                if (!open) sub[f] = 1;
                enter = open && o.steps > 0;
                lattice_point(o, blo, bhi, best == __builtin_inf() ? 0 : ib, x);
            }
        }
        if (mode == 1) {
            const int l2 = block_claim(cont ? 1 : 0, B.cnt + 4);       // every thread of the block
            if (cont) {
                B.lnode2[l2] = b;
                B.ngrid[node_lin(o, level, c)] = l2;
                if (csave) {
                    for (int k = 0; k < 3; ++k) B.dpts[(int64_t)l2 * 3 + k] = k < o.D ? 0.5 * (blo[k] + bhi[k]) : 0.0;
                    for (int k = 0; k < o.D; ++k) {
                        B.dbox[(int64_t)l2 * 2 * o.D + k] = blo[k];
                        B.dbox[(int64_t)l2 * 2 * o.D + o.D + k] = bhi[k];
                    }
                }
            }
        } else {
            const int d = block_claim(enter ? 1 : 0, B.cnt + 3);       // every thread of the block
            if (enter) {
                B.dnode[d] = b;
                B.done[d] = 0;
                B.ddp[d] = dp;
                B.fcand[f] = d;
                for (int k = 0; k < 3; ++k) {
                    gx[(int64_t)d * 3 + k] = x[k];
                    B.dbx[(int64_t)d * 8 + k] = blo[k];
                    B.dbx[(int64_t)d * 8 + 3 + k] = bhi[k];
                }
                B.dbx[(int64_t)d * 8 + 6] = side;
                B.dbx[(int64_t)d * 8 + 7] = best;
            }
        }
    }
}

// Certificate between the lattice passes (large levels): the certified box bounds of the
// posterior (k_bound.hip, the guaranteed bound Sec. 9 leaves open) for each node the corners
// left open, with the search's own side.  The certified margin is a lower bound of g over
// the whole box, so of every point the rest of the lattice and the descent could visit; when
// it already gives UB <= alpha (eq. (upper_bound)), the search's minimum gives UB <= alpha too
// and the node is not subdivided, as the search would conclude.  Such nodes leave the node
// lattice; the others form the list of the second pass (count B.cnt[5]) and re-register
// there under their new index.
__global__ void __launch_bounds__(256) k_lattice_cert(Oct o, int level, const uint64_t* __restrict__ keys, BoundBufs B)
{
    const int64_t n2 = B.cnt[4];
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n2; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = base + threadIdx.x;
        bool keep = false;
        int32_t b = 0;
        int64_t lin = 0;
        if (j < n2) {
            b = B.lnode2[j];
            const double side = B.side[b];
            const double* cb = B.dcert + j * 4;
            const double mu = side > 0 ? cb[2] : cb[1];
            const double g = side * (o.theta - mu) < 0.0 ? -__builtin_inf() : margin(side, o.theta, mu, cb[3]);
            int lv;
            int64_t c[3], clo[3], chi[3], dp;
            double blo[3], bhi[3];
            key_coords(o, keys[B.bnode[b]], lv, c);
            node_box(o, level, c, clo, chi, blo, bhi, &dp);
            keep = upper_bound(g, dp) > o.alpha;
            lin = node_lin(o, level, c);
            if (!keep) B.ngrid[lin] = -1;
        }
        const int j3 = block_claim(keep ? 1 : 0, B.cnt + 5);           // every thread of the block
        if (keep) {
            B.lnode3[j3] = b;
            B.ngrid[lin] = j3;
        }
    }
}

// Number of keys a node emits: its in-domain children, or itself as a leaf (0 unless sb).
__device__ __forceinline__ int emit_count(const Oct& o, int level, uint64_t key, int sb)
{
    if (!sb) return 0;
    if (level == o.Ldepth) return 1;
    int lv;
    int64_t c[3];
    key_coords(o, key, lv, c);
    if (o.kd) {
        const int a = kd_axis(o.D, level);
        const int64_t hs = o.S0 >> node_shift(o, level + 1, a);
        return 1 + ((2 * pick3(c, a) + 1) * hs < pick3(o.g.nc, a) ? 1 : 0);
    }
    const int64_t hs = (o.S0 >> level) >> 1;
    int n = 0;
    for (int i = 0; i < (1 << o.D); ++i) {
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d)                    // fixed bounds: c stays in registers
            if (d < o.D) ok = ok && (2 * c[d] + ((i >> d) & 1)) * hs < o.g.nc[d];
        n += ok ? 1 : 0;
    }
    return n;
}

// Emit counts of the frontier.
// Emit counts of the frontier.  With the search's descent (fin set), a node that has a
// descent candidate is decided here first: the value at the last point enters g_min, and
// the node is subdivided when the bound 1 - B^d = -expm1(d log1p(-t)) of eq. (upper_bound)
// exceeds alpha.
__global__ void k_emit_count(Oct o, int level, const uint64_t* __restrict__ keys, const int64_t* __restrict__ nf_dev,
                             int64_t cap, int32_t* __restrict__ sub, int32_t* __restrict__ cnt, BoundBufs B, int fin)
{
    int64_t nf = *nf_dev;
    if (nf > cap) nf = cap;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += (int64_t)gridDim.x * blockDim.x) {
        int32_t sb = sub[f];
        const int32_t d = fin ? B.fcand[f] : -1;
        if (d >= 0) {
            const double* rec = B.dbx + (int64_t)d * 8;
            double gmin = rec[7];
            if (!B.done[d]) {
                const double g = margin(rec[6], o.theta, B.gp_mean[d], B.gp_var[d]);
                if (g < gmin) gmin = g;
            }
            sb = upper_bound(gmin, B.ddp[d]) > o.alpha ? 1 : 0;
            sub[f] = sb;
        }
        cnt[f] = emit_count(o, level, keys[f], sb);
    }
}

__global__ void k_emit(Oct o, int level, const uint64_t* __restrict__ keys, const int64_t* __restrict__ nf_dev,
                       int64_t cap, const int32_t* __restrict__ sub, const int32_t* __restrict__ off,
                       uint64_t* __restrict__ out, int64_t out_cap, uint8_t* __restrict__ stat,
                       const int32_t* __restrict__ path, uint8_t* __restrict__ hob_out)
{
    int64_t nf = *nf_dev;
    if (nf > cap) nf = cap;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += (int64_t)gridDim.x * blockDim.x) {
        int lv;
        int64_t c[3];
        key_coords(o, keys[f], lv, c);
        const int64_t* nl = o.nodes + level * 3;
        stat[c[0] + nl[0] * (c[1] + nl[1] * c[2])] = sub[f] ? 2 : 1;
        if (!sub[f]) continue;
        int64_t pos = off[f];
        const uint8_t obs = path[f] != 4 ? 1 : 0;     // path 4: no observation in the node
        if (level == o.Ldepth) {
            // leaves keep the octree key of the finest level (the K-D code at depth D Lmax is
            // the same Morton code)
            if (pos < out_cap) out[pos] = ((uint64_t)o.Lmax << 58) | (keys[f] & ((1ull << 58) - 1));
            continue;
        }
        if (o.kd) {
            const int a = kd_axis(o.D, level);
            const int64_t hs = o.S0 >> node_shift(o, level + 1, a);
            for (int i = 0; i < 2; ++i) {
                const int64_t ca = 2 * pick3(c, a) + i;
                const int64_t cc[3] = {a == 0 ? ca : c[0], a == 1 ? ca : c[1], a == 2 ? ca : c[2]};
                if (ca * hs >= pick3(o.g.nc, a)) continue;
                if (pos < out_cap) {
                    out[pos] = make_key(o, level + 1, cc);
                    hob_out[pos] = obs;
                }
                ++pos;
            }
            continue;
        }
        const int64_t hs = (o.S0 >> level) >> 1;
        for (int i = 0; i < (1 << o.D); ++i) {
            int64_t cc[3] = {0, 0, 0};
            bool ok = true;
#pragma unroll
            for (int d = 0; d < 3; ++d) {                  // fixed bounds: cc stays in registers
                if (d < o.D) {
                    cc[d] = 2 * c[d] + ((i >> d) & 1);
                    ok = ok && cc[d] * hs < o.g.nc[d];
                }
            }
            if (!ok) continue;
            if (pos < out_cap) {
                out[pos] = make_key(o, level + 1, cc);
                hob_out[pos] = obs;
            }
            ++pos;
        }
    }
}

__global__ void k_set_count(int64_t* dst, const int64_t* src, int64_t mul)
{
    *dst = *src * mul;
}

// Mark the vertices of every leaf's cells.
__global__ void k_mark(Oct o, int leaf_edge, const uint64_t* __restrict__ leaves, const int64_t* __restrict__ nl_dev,
                       int64_t leaf_cap, int32_t* __restrict__ vmask)
{
    const int64_t nl = *nl_dev;
    if (nl > leaf_cap) return;
    const int e1 = leaf_edge + 1;
    int per = 1;
    for (int d = 0; d < o.D; ++d) per *= e1;
    const int64_t total = nl * per;
    const bool idx32 = total <= 0x7fffffffll;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        int64_t lf;
        int loc;
        if (idx32) {
            const uint32_t u = (uint32_t)it;
            lf = u / (uint32_t)per;
            loc = (int)(u - (uint32_t)lf * (uint32_t)per);
        } else {
            lf = it / per;
            loc = (int)(it - lf * per);
        }
        int lv;
        int64_t c[3];
        key_coords_oct(o.D, leaves[lf], lv, c);
        const int64_t s = o.S0 >> lv;
        int64_t v[3] = {0, 0, 0};
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (d < o.D) {
                int64_t cmin = c[d] * s;
                int64_t cmax = (c[d] + 1) * s;
                if (cmax > o.g.nc[d]) cmax = o.g.nc[d];
                const int q = loc / e1;
                v[d] = cmin + (loc - q * e1);
                loc = q;
                ok = ok && v[d] <= cmax;
            }
        }
        if (!ok) continue;
        vmask[v[0] + o.g.n[0] * (v[1] + o.g.n[1] * v[2])] = 1;
    }
}

__global__ void k_slots(const int32_t* __restrict__ vmask, const int32_t* __restrict__ off, int64_t nv,
                        int32_t* __restrict__ slot, int32_t* __restrict__ vlist)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        if (vmask[i]) {
            slot[i] = off[i];
            vlist[off[i]] = (int32_t)i;
        } else {
            slot[i] = -1;
        }
    }
}

// ------------------------------------------------------------ edge-crossing bound (Sec. 9)
//
// Sec. 9 proposes a tighter region bound from the crossing probabilities of grid edges.  A
// node has a crossed cell exactly when its vertex values are not all on one side of theta,
// that is when some edge of a spanning tree of its vertices is crossed; so
// P(some cell crossed) <= sum over the tree of P(edge crossed), and each cell's LCP is at
// most that.  The tree: every x-edge, the y-edges of the first x column of each z-plane,
// the z-edges of the first (x, y) column.  The edge terms come from the posterior and
// neighbour cross-covariances the reconstruction has just computed for the node's
// vertices.

// P(edge crossed) for end values X, Y ~ N((mua, mub), [[va, c], [c, vb]]): not both below
// and not both above theta (a value equal to theta counts as crossed).  With standardised
// thresholds h, k and correlation rho >= 0 (a negative one is reflected: Zb -> -Zb, k -> -k
// exchanges crossed and not crossed), write Za = a U + b V, Zb = a U - b V with
// a = sqrt((1 + rho) / 2), b = sqrt((1 - rho) / 2) and U, V independent N(0, 1).  For fixed
// V = v both ends are increasing in U with the same slope a, so the edge is crossed exactly
// when U lies between (h - b v) / a and (k + b v) / a:
//   P = int phi(v) |Phi((h - b v) / a) - Phi((k + b v) / a)| dv.
// The integrand is analytic on either side of its kink v* = (h - k) / (2 b); the integral
// runs over [-9, 9] (phi(9) ~ 1e-18) in six panels with 12-point Gauss-Legendre rules, the
// panel holding v* split there.
__device__ __forceinline__ double phi_cdf(double x) { return 0.5 * erfc(-0.70710678118654752440 * x); }

__device__ double edge_cross_prob(double mua, double mub, double va, double vb, double c, double theta)
{
    const double sa = sqrt(fmax(va, 0.0)), sb = sqrt(fmax(vb, 0.0));
    if (sa == 0.0 && sb == 0.0) {
        const bool below = mua < theta && mub < theta, above = mua > theta && mub > theta;
        return (below || above) ? 0.0 : 1.0;
    }
    if (sa == 0.0 || sb == 0.0) {
        const double mc = sa == 0.0 ? mua : mub, mr = sa == 0.0 ? mub : mua, sr = sa == 0.0 ? sb : sa;
        if (mc == theta) return 1.0;
        const double hr = (theta - mr) / sr;
        return mc < theta ? phi_cdf(-hr) : phi_cdf(hr);
    }
    const double h = (theta - mua) / sa;
    double k = (theta - mub) / sb;
    double rho = c / (sa * sb);
    if (rho >= 1.0) return fabs(phi_cdf(h) - phi_cdf(k));
    if (rho <= -1.0) return 1.0 - fabs(phi_cdf(h) - phi_cdf(-k));
    const bool reflect = rho < 0.0;
    if (reflect) {
        rho = -rho;
        k = -k;
    }
    const double a = sqrt(0.5 * (1.0 + rho)), b = sqrt(0.5 * (1.0 - rho));
    const double ia = 1.0 / a;
    const double vs = (h - k) / (2.0 * b);
    constexpr double gx[6] = {0.1252334085114689, 0.3678314989981802, 0.5873179542866175,
                              0.7699026741943047, 0.9041172563704748, 0.9815606342467192};
    constexpr double gw[6] = {0.2491470458134027, 0.23349253653835464, 0.20316742672306565,
                              0.1600783285433461, 0.10693932599531888, 0.04717533638651202};
    auto f = [&](double v) {
        return exp(-0.5 * v * v) * fabs(phi_cdf((h - b * v) * ia) - phi_cdf((k + b * v) * ia));
    };
    auto panel = [&](double lo, double hi) {
        const double m = 0.5 * (hi + lo), r = 0.5 * (hi - lo);
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) acc += gw[i] * (f(m - r * gx[i]) + f(m + r * gx[i]));
        return r * acc;
    };
    double p = 0.0;
    for (int q = 0; q < 6; ++q) {
        const double lo = -9.0 + 3.0 * q, hi = lo + 3.0;
        if (vs > lo && vs < hi) p += panel(lo, vs) + panel(vs, hi);
        else p += panel(lo, hi);
    }
    p *= 0.39894228040143267794;          // 1 / sqrt(2 pi)
    if (reflect) p = 1.0 - p;
    return fmin(fmax(p, 0.0), 1.0);
}

// One wave per emitted node: flag[i] = (edge-crossing bound of leaf i) > alpha.  Lanes take
// the tree's edges in turn; the partial sums meet in a fixed butterfly (deterministic).
__global__ void __launch_bounds__(256) k_edge_bound(Oct o, int leaf_edge, const uint64_t* __restrict__ leaves,
                                                    const int64_t* __restrict__ nl_dev, int64_t leaf_cap,
                                                    const int32_t* __restrict__ slot, const double* __restrict__ vmean,
                                                    const double* __restrict__ vvar,
                                                    const double* __restrict__ cross, int32_t* __restrict__ flag,
                                                    double* __restrict__ eb_out)
{
    const int64_t nl = *nl_dev;
    if (nl > leaf_cap) return;
    const int lane = threadIdx.x & 63;
    const int D = o.D, NDIR = D == 3 ? 13 : 4;
    for (int64_t lf = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; lf < nl;
         lf += ((int64_t)gridDim.x * blockDim.x) >> 6) {
        int lv;
        int64_t c[3];
        key_coords_oct(D, leaves[lf], lv, c);
        const int64_t sz = o.S0 >> lv;
        int64_t lo[3] = {0, 0, 0}, nv[3] = {1, 1, 1};
        for (int d = 0; d < D; ++d) {
            lo[d] = c[d] * sz;
            int64_t hi = (c[d] + 1) * sz;
            if (hi > o.g.nc[d]) hi = o.g.nc[d];
            nv[d] = hi - lo[d] + 1;
        }
        const int64_t ex = (nv[0] - 1) * nv[1] * nv[2], ey = (nv[1] - 1) * nv[2], ez = D == 3 ? nv[2] - 1 : 0;
        // rounds of 64 edges; the node is kept as soon as the running sum exceeds alpha
        double total = 0.0;
        for (int64_t e0 = 0; e0 < ex + ey + ez && !(total > o.alpha); e0 += 64) {
            const int64_t e = e0 + lane;
            double part = 0.0;
            if (e < ex + ey + ez) {
                int64_t i = 0, j = 0, k = 0;
                int ax;
                if (e < ex) {
                    ax = 0;
                    i = e % (nv[0] - 1);
                    j = (e / (nv[0] - 1)) % nv[1];
                    k = e / ((nv[0] - 1) * nv[1]);
                } else if (e < ex + ey) {
                    ax = 1;
                    j = (e - ex) % (nv[1] - 1);
                    k = (e - ex) / (nv[1] - 1);
                } else {
                    ax = 2;
                    k = e - ex - ey;
                }
                const int64_t va = (lo[0] + i) + o.g.n[0] * ((lo[1] + j) + o.g.n[1] * (lo[2] + k));
                const int64_t step = ax == 0 ? 1 : (ax == 1 ? o.g.n[0] : o.g.n[0] * o.g.n[1]);
                const int64_t sa = slot[va], sb = slot[va + step];
                if (sa < 0 || sb < 0) {           // not reconstructed (never for a leaf's own vertices)
                    part = 1.0;
                } else {
                    // neighbour direction index of +x, +y, +z in the cross-covariance layout
                    const int dir = D == 3 ? (ax == 0 ? 0 : (ax == 1 ? 2 : 8)) : (ax == 0 ? 0 : 2);
                    const double cab = cross[(size_t)sa * NDIR + dir];
                    part = edge_cross_prob(vmean[sa], vmean[sb], vvar[sa], vvar[sb], cab, o.theta);
                }
            }
            for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
            total += part;
        }
        if (lane == 0) {
            flag[lf] = total > o.alpha ? 1 : 0;
            if (eb_out) eb_out[lf] = total;
        }
    }
}

// Keep the flagged leaves (order preserved): out[off[i]] = leaves[i].
__global__ void k_keep_leaves(const uint64_t* __restrict__ leaves, const int64_t* __restrict__ nl_dev, int64_t leaf_cap,
                              const int32_t* __restrict__ flag, const int32_t* __restrict__ off,
                              uint64_t* __restrict__ out)
{
    const int64_t nl = *nl_dev;
    if (nl > leaf_cap) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += (int64_t)gridDim.x * blockDim.x)
        if (flag[i]) out[off[i]] = leaves[i];
}

// Copy the kept leaves back (unless the leaf list overflowed); the count follows in a
// launch of its own, after every block here has read the old count.
__global__ void k_store_kept(const uint64_t* __restrict__ kept, const int64_t* __restrict__ kept_n,
                             uint64_t* __restrict__ leaves, const int64_t* __restrict__ nl_dev, int64_t leaf_cap)
{
    const int64_t nl = *nl_dev, nk = *kept_n;
    if (nl > leaf_cap) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (int64_t)gridDim.x * blockDim.x)
        leaves[i] = kept[i];
}

__global__ void k_set_leaf_count(int64_t* __restrict__ nl_dev, const int64_t* __restrict__ kept_n, int64_t leaf_cap)
{
    if (*nl_dev <= leaf_cap) *nl_dev = *kept_n;
}

// Octree level at which each cell's node stopped.
__global__ void k_level_field(Oct o, const uint8_t* __restrict__ stat, uint8_t* __restrict__ field)
{
    const int64_t nc = o.g.nc[0] * o.g.nc[1] * o.g.nc[2];
    const bool idx32 = nc <= 0xffffffffll;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < nc; it += (int64_t)gridDim.x * blockDim.x) {
        int64_t cell[3];
        if (idx32) {
            const uint32_t u = (uint32_t)it, n0 = (uint32_t)o.g.nc[0], n1 = (uint32_t)o.g.nc[1];
            const uint32_t r = u / n0;
            cell[0] = u - r * n0;
            cell[2] = r / n1;
            cell[1] = r - (uint32_t)cell[2] * n1;
        } else {
            cell[0] = it % o.g.nc[0];
            cell[1] = (it / o.g.nc[0]) % o.g.nc[1];
            cell[2] = it / (o.g.nc[0] * o.g.nc[1]);
        }
        uint8_t out = 255;
        for (int l = 0; l <= o.Ldepth; ++l) {
            const int64_t* nl = o.nodes + l * 3;
            int64_t q[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) q[d] = d < o.D ? cell[d] >> (o.lgS0 - node_shift(o, l, d)) : 0;   // node edge 2^(lgS0 - shift)
            const int64_t lin = q[0] + nl[0] * (q[1] + nl[1] * q[2]);
            uint8_t st = stat[o.statoff[l] + lin];
            if (st == 1 || (st == 2 && l == o.Ldepth)) {
                out = (uint8_t)l;
                break;
            }
            if (st != 2) break;
        }
        field[it] = out;
    }
}

inline unsigned gsz(int64_t n, int per)
{
    int64_t b = (n + per - 1) / per;
    if (b > 16384) b = 16384;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// ------------------------------------------------------- local model bound (Sec. 5.2)
//
// Region test on the local model M': the observations inside the node box enlarged by
// beta lengthscales per axis (the root keeps all of them), conditioned on alone.  One
// work-group per bound node (persistent: a work-group takes the next node from a counter
// when it finishes one, since \|M'\| and the search's length vary by node) gathers M' in its
// order in M, builds K' + noise I in its own slot, factors it (blocked Cholesky, 32-wide
// panels), and runs the search of the full-model path: the {lo, mid, hi}^D lattice (lowest
// index wins ties), then the projected steps.  Every value comes from forward solves only:
// with w = L'^-1 y', v = L'^-1 k(x) and u_d = L'^-1 dk(x)/dx_d,
//   mu = v.w,  var = s2 - |v|^2,  dmu_d = u_d.w,  dvar_d = -2 v.u_d.
// A sparse model (eq. (sgp)) restricts mu_M and A_M to M': with W = L'^-T [v, u_d] the
// variance gains w.A'w and its derivative 2 w.A'(K'^-1 dk/dx_d).
// A factorisation that fails (pivot at or below m' eps (s2 + noise)) gives no bound: the
// node is refined.
constexpr int kLocB = 32;        // panel width; also the most right-hand sides per solve
constexpr int kLocSlots = 1024;  // most work-groups of k_local_bound (four per CU), one slot each;
                                 // the workspace holds as many slots as are resident together

struct LocalBufs {
    KParams kp;
    const double* X;     // m_pad x 4
    const double* y;     // m fitted values: y of an exact GP, mu_M of a sparse model
    int m;
    int ld;              // slot matrix leading dimension (m_pad of the model)
    double noise;
    double piv_scale;    // eps (s2 + noise); the pivot floor is m' piv_scale
    double rad[3];       // beta ell_d
    const double* AM;    // sparse model: A_M (ld x ld); null for an exact GP
    int32_t* next;       // work counter: nodes handed out beyond the first gridDim.x (zeroed per launch)
    double* slots;       // one per resident work-group: ld ld + 4 ld kLocB doubles (L, V, inverted diagonal blocks, W, T)
};

__host__ __device__ __forceinline__ size_t local_slot_doubles(int ld) { return (size_t)ld * ld + 4 * (size_t)ld * kLocB; }

// Forward solve L V = V for columns [0, R) of V (rows [0, n)), right-looking by 32-row
// blocks: y_b = D_b V_b with D_b the inverted diagonal block (Dv), then every row below
// takes V_i -= L_ib y_b.  L lower row-major in Lm.
__device__ void local_fsolve(const double* __restrict__ Lm, const double* __restrict__ Dv, double* __restrict__ V,
                             int ld, int n, int R, double (*ta)[kLocB + 1], double (*tb)[kLocB + 1])
{
    const int tid = threadIdx.x;
    const int r = tid >> 3, c4 = (tid & 7) * 4;
    for (int r0 = 0; r0 < n; r0 += kLocB) {
        const int nb = min(kLocB, n - r0);
        for (int t = tid; t < kLocB * kLocB; t += 256) {
            const int a = t >> 5, b = t & 31;
            ta[a][b] = Dv[(size_t)(r0 + a) * kLocB + b];
            tb[a][b] = (a < nb && b < R) ? V[(size_t)(r0 + a) * kLocB + b] : 0.0;
        }
        __syncthreads();
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
        for (int l = 0; l < kLocB; ++l) {
            const double x = ta[r][l];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = fma(x, tb[l][c4 + q], acc[q]);
        }
        __syncthreads();   // every thread has read tb; it now holds the block's solution
#pragma unroll
        for (int q = 0; q < 4; ++q) tb[r][c4 + q] = r < nb ? acc[q] : 0.0;
        if (r < nb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (c4 + q < R) V[(size_t)(r0 + r) * kLocB + c4 + q] = acc[q];
        __syncthreads();
        for (int i = r0 + nb + r; i < n; i += 32) {
            const double* Li = Lm + (size_t)i * ld + r0;
            double u[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
            for (int l = 0; l < kLocB; ++l) {
                const double x = Li[l];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = fma(x, tb[l][c4 + q], u[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (c4 + q < R) V[(size_t)i * kLocB + c4 + q] -= u[q];
        }
        __syncthreads();
    }
}

// Column sums over rows [0, n): out[c] = sum_i V[i][c] * (w ? w[i] : V[i][c0]) for c < R.
__device__ void local_colsum(const double* __restrict__ V, const double* __restrict__ w, int c0, int n, int R,
                             double (*red)[kLocB + 1], double* __restrict__ out)
{
    const int tid = threadIdx.x, c = tid & 31, g = tid >> 5;
    double s = 0.0;
    if (c < R)
        for (int i = g; i < n; i += 8) {
            const double v = V[(size_t)i * kLocB + c];
            s = fma(v, w ? w[i] : V[(size_t)i * kLocB + c0], s);
        }
    red[g][c] = s;
    __syncthreads();
    if (tid < R) {
        double t = 0.0;
        for (int k = 0; k < 8; ++k) t += red[k][tid];
        out[tid] = t;
    }
    __syncthreads();
}

// Backward solve L^T W = W for columns [0, R) (rows [0, n)), right-looking from the last
// block: x_b = D_b^T W_b, then every row above takes W_i -= sum_l L[b + l][i] x_b[l].
__device__ void local_bsolve(const double* __restrict__ Lm, const double* __restrict__ Dv, double* __restrict__ W,
                             int ld, int n, int R, double (*ta)[kLocB + 1], double (*tb)[kLocB + 1])
{
    const int tid = threadIdx.x;
    const int r = tid >> 3, c4 = (tid & 7) * 4;
    for (int r0 = (n - 1) / kLocB * kLocB; r0 >= 0 && n > 0; r0 -= kLocB) {
        const int nb = min(kLocB, n - r0);
        for (int t = tid; t < kLocB * kLocB; t += 256) {
            const int a = t >> 5, b = t & 31;
            ta[a][b] = Dv[(size_t)(r0 + b) * kLocB + a];
            tb[a][b] = (a < nb && b < R) ? W[(size_t)(r0 + a) * kLocB + b] : 0.0;
        }
        __syncthreads();
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
        for (int l = 0; l < kLocB; ++l) {
            const double x = ta[r][l];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = fma(x, tb[l][c4 + q], acc[q]);
        }
        __syncthreads();   // every thread has read tb; it now holds the block's solution
#pragma unroll
        for (int q = 0; q < 4; ++q) tb[r][c4 + q] = r < nb ? acc[q] : 0.0;
        if (r < nb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (c4 + q < R) W[(size_t)(r0 + r) * kLocB + c4 + q] = acc[q];
        __syncthreads();
        for (int i = r; i < r0; i += 32) {
            double u[4] = {0.0, 0.0, 0.0, 0.0};
            for (int l = 0; l < nb; ++l) {
                const double x = Lm[(size_t)(r0 + l) * ld + i];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = fma(x, tb[l][c4 + q], u[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (c4 + q < R) W[(size_t)i * kLocB + c4 + q] -= u[q];
        }
        __syncthreads();
    }
}

// T = A' W for columns [0, R): A'[i][j] = A_M[idx_i][idx_j], read through the index list.
__device__ void local_aprod(const double* __restrict__ AM, int lda, const int* __restrict__ idx,
                            const double* __restrict__ W, double* __restrict__ T, int n, int R)
{
    const int tid = threadIdx.x;
    const int r = tid >> 3, c4 = (tid & 7) * 4;
    for (int i = r; i < n; i += 32) {
        const double* Ai = AM + (size_t)idx[i] * lda;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int j = 0; j < n; ++j) {
            const double a = Ai[idx[j]];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = fma(a, W[(size_t)j * kLocB + c4 + q], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (c4 + q < R) T[(size_t)i * kLocB + c4 + q] = acc[q];
    }
    __syncthreads();
}

// out[c] = sum_i X[i][c] Y[i][same ? c : 0] for c < R.
__device__ void local_coldot(const double* __restrict__ X, const double* __restrict__ Y, bool same, int n, int R,
                             double (*red)[kLocB + 1], double* __restrict__ out)
{
    const int tid = threadIdx.x, c = tid & 31, g = tid >> 5;
    double s = 0.0;
    if (c < R)
        for (int i = g; i < n; i += 8) s = fma(X[(size_t)i * kLocB + c], Y[(size_t)i * kLocB + (same ? c : 0)], s);
    red[g][c] = s;
    __syncthreads();
    if (tid < R) {
        double t = 0.0;
        for (int k = 0; k < 8; ++k) t += red[k][tid];
        out[tid] = t;
    }
    __syncthreads();
}

template <int D>
__global__ void __launch_bounds__(256, 4) k_local_bound(Oct o, int level, const uint64_t* __restrict__ keys,
                                                     const int32_t* __restrict__ path, BoundBufs B, LocalBufs Lb,
                                                     int32_t* __restrict__ sub)
{
    // sized by the model: M' coordinates (ld x D), w (ld), the indices of M' in M (ld)
    extern __shared__ double lsm[];
    double* xs = lsm;
    double* wv = lsm + (size_t)Lb.ld * D;
    int* sidx = (int*)(wv + Lb.ld);
    __shared__ double ta[kLocB][kLocB + 1], tb[kLocB][kLocB + 1];
    __shared__ double ldg[kLocB];
    __shared__ double red[8][kLocB + 1];
    __shared__ double sums[4][kLocB];
    __shared__ double xcur[3];
    __shared__ int wcnt[4];
    __shared__ int state;            // 0 searching, 1 decided
    __shared__ int fail;
    __shared__ int64_t cur;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ld = Lb.ld;
    double* Lm = Lb.slots + (size_t)blockIdx.x * local_slot_doubles(ld);
    double* V = Lm + (size_t)ld * ld;
    double* Dv = V + (size_t)ld * kLocB;
    double* Wm = Dv + (size_t)ld * kLocB;
    double* Tm = Wm + (size_t)ld * kLocB;
    const bool sparse = Lb.AM != nullptr;
    const int64_t nb_nodes = B.cnt[0];
    const int npt = D == 3 ? 27 : 9;
    const double s2 = Lb.kp.s2;
    if (tid == 0) cur = blockIdx.x;
    __syncthreads();
    for (;;) {
        const int64_t b = cur;
        if (b >= nb_nodes) break;
        const int32_t f = B.bnode[b];
        int lv;
        int64_t c[3], clo[3], chi[3], dp;
        double blo[3], bhi[3];
        key_coords(o, keys[f], lv, c);
        node_box(o, level, c, clo, chi, blo, bhi, &dp);
        // M': order-preserving selection, coordinates to LDS, values to column 0 of V
        int n = 0;
        for (int i0 = 0; i0 < Lb.m; i0 += 256) {
            const int i = i0 + tid;
            bool in = i < Lb.m;
            double xi[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                xi[d] = in ? Lb.X[(size_t)i * 4 + d] : 0.0;
                if (level > 0) in = in && xi[d] >= blo[d] - Lb.rad[d] && xi[d] <= bhi[d] + Lb.rad[d];
            }
            const unsigned long long bal = __ballot(in);
            if (lane == 0) wcnt[wave] = __popcll(bal);
            __syncthreads();
            int off = n;
            for (int w = 0; w < wave; ++w) off += wcnt[w];
            const int tot = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
            if (in) {
                const int pos = off + __popcll(bal & ((1ull << lane) - 1ull));
#pragma unroll
                for (int d = 0; d < D; ++d) xs[pos * D + d] = xi[d];
                V[(size_t)pos * kLocB] = Lb.y[i];
                sidx[pos] = i;
            }
            __syncthreads();
            n += tot;
        }
        // K' + noise I, lower triangle
        for (int64_t t = tid; t < (int64_t)n * n; t += 256) {
            const int i = (int)(t / n), j = (int)(t % n);
            if (j > i) continue;
            double r2 = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const double u = (xs[i * D + d] - xs[j * D + d]) * Lb.kp.inv_ell[d];
                r2 = fma(u, u, r2);
            }
            Lm[(size_t)i * ld + j] = kernel_val(Lb.kp, r2) + (i == j ? Lb.noise : 0.0);
        }
        if (tid == 0) {
            fail = 0;
            state = 0;
        }
        __syncthreads();
        // blocked Cholesky, lower, in place; the inverted diagonal blocks go to Dv
        const double piv_min = (double)n * Lb.piv_scale;
        for (int k0 = 0; k0 < n && !fail; k0 += kLocB) {
            const int nb = min(kLocB, n - k0);
            for (int t = tid; t < kLocB * kLocB; t += 256) {
                const int a = t >> 5, bb = t & 31;
                ta[a][bb] = (a < nb && bb <= a) ? Lm[(size_t)(k0 + a) * ld + k0 + bb] : (a == bb ? 1.0 : 0.0);
            }
            __syncthreads();
            // diagonal block: column j scaled by its pivot's root (kept in ldg), then the
            // rank-1 update of the rows below; ta[j][j] is not rewritten until the end
            for (int j = 0; j < nb; ++j) {
                const double piv = ta[j][j];
                if (!(piv > piv_min)) {
                    if (tid == 0) fail = 1;
                    break;
                }
                const double ljj = sqrt(piv);
                if (tid == j) ldg[j] = ljj;
                if (tid > j && tid < nb) ta[tid][j] /= ljj;
                __syncthreads();
                {
                    // rank-1 update of the trailing part of the block: four entries per thread
                    const int rr = tid >> 3, c4 = (tid & 7) * 4;
                    if (rr > j && rr < nb) {
                        const double lr = ta[rr][j];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int cc = c4 + q;
                            if (cc > j && cc <= rr) ta[rr][cc] = fma(-lr, ta[cc][j], ta[rr][cc]);
                        }
                    }
                }
                __syncthreads();
            }
            __syncthreads();
            if (fail) break;
            if (tid < nb) ta[tid][tid] = ldg[tid];
            __syncthreads();
            // D = L_kk^-1 (identity beyond nb) into tb, column c by thread c; then L_kk and D
            // to the slot, and D into ta for the panel
            if (tid < kLocB) {
                const int cc = tid;
                for (int a = 0; a < kLocB; ++a) {
                    double v = 0.0;
                    if (a >= cc) {
                        double sacc = a == cc ? 1.0 : 0.0;
                        for (int q = cc; q < a; ++q) sacc = fma(-ta[a][q], tb[q][cc], sacc);
                        v = sacc / ta[a][a];
                    }
                    tb[a][cc] = v;
                }
            }
            __syncthreads();
            for (int t = tid; t < kLocB * kLocB; t += 256) {
                const int a = t >> 5, bb = t & 31;
                Dv[(size_t)(k0 + a) * kLocB + bb] = tb[a][bb];
                if (a < nb && bb <= a) Lm[(size_t)(k0 + a) * ld + k0 + bb] = ta[a][bb];
            }
            __syncthreads();
            for (int t = tid; t < kLocB * kLocB; t += 256) {
                const int a = t >> 5, bb = t & 31;
                ta[a][bb] = tb[a][bb];
            }
            __syncthreads();
            // panel: X = A D^T, 32 rows at a time
            {
                const int r = tid >> 3, c4 = (tid & 7) * 4;
                for (int i0 = k0 + nb; i0 < n; i0 += kLocB) {
                    for (int t = tid; t < kLocB * kLocB; t += 256) {
                        const int a = t >> 5, bb = t & 31;
                        tb[a][bb] = (i0 + a < n && bb < nb) ? Lm[(size_t)(i0 + a) * ld + k0 + bb] : 0.0;
                    }
                    __syncthreads();
                    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
                    for (int l = 0; l < kLocB; ++l) {
                        const double x = tb[r][l];
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc[q] = fma(x, ta[c4 + q][l], acc[q]);
                    }
                    if (i0 + r < n)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (c4 + q < nb) Lm[(size_t)(i0 + r) * ld + k0 + c4 + q] = acc[q];
                    __syncthreads();
                }
            }
            // trailing update of the lower triangle, A_ij -= L_ik L_jk^T: for each 32-row chunk
            // of the panel (columns j of A), every row i at or below it updates its entries there
            {
                const int t0 = k0 + nb;
                const int r = tid >> 3, c4 = (tid & 7) * 4;
                for (int j0 = t0; j0 < n; j0 += kLocB) {
                    for (int t = tid; t < kLocB * kLocB; t += 256) {
                        const int a = t >> 5, bb = t & 31;
                        tb[a][bb] = j0 + a < n ? Lm[(size_t)(j0 + a) * ld + k0 + bb] : 0.0;
                    }
                    __syncthreads();
                    for (int i = j0 + r; i < n; i += kLocB) {
                        const double* Pi = Lm + (size_t)i * ld + k0;
                        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
                        for (int l = 0; l < kLocB; ++l) {
                            const double x = Pi[l];
#pragma unroll
                            for (int q = 0; q < 4; ++q) acc[q] = fma(x, tb[c4 + q][l], acc[q]);
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int col = j0 + c4 + q;
                            if (col < n && col <= i) Lm[(size_t)i * ld + col] -= acc[q];
                        }
                    }
                    __syncthreads();
                }
            }
        }
        const int p = path[f];
        double side = p == 1 ? 1.0 : -1.0;
        double gmin = -__builtin_inf();
        if (!fail) {
            // lattice: column 0 = y', columns 1 .. npt = k(lattice point)
            for (int t = tid; t < n * npt; t += 256) {
                const int i = t / npt, q = t % npt;
                double x[3];
                lattice_point(o, blo, bhi, q, x);
                double r2 = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const double u = (x[d] - xs[i * D + d]) * Lb.kp.inv_ell[d];
                    r2 = fma(u, u, r2);
                }
                V[(size_t)i * kLocB + 1 + q] = kernel_val(Lb.kp, r2);
            }
            __syncthreads();
            local_fsolve(Lm, Dv, V, ld, n, 1 + npt, ta, tb);
            for (int i = tid; i < n; i += 256) wv[i] = V[(size_t)i * kLocB];
            __syncthreads();
            local_colsum(V, wv, 0, n, 1 + npt, red, sums[0]);      // means
            // |v|^2 per column
            {
                const int cc = tid & 31, g = tid >> 5;
                double sacc = 0.0;
                if (cc < 1 + npt)
                    for (int i = g; i < n; i += 8) {
                        const double v = V[(size_t)i * kLocB + cc];
                        sacc = fma(v, v, sacc);
                    }
                red[g][cc] = sacc;
                __syncthreads();
                if (tid < 1 + npt) {
                    double t = 0.0;
                    for (int k = 0; k < 8; ++k) t += red[k][tid];
                    sums[1][tid] = t;
                }
                __syncthreads();
            }
            if (sparse) {
                // W = L'^-T V, T = A' W; sums[2][c] = w_c . A' w_c
                for (int t = tid; t < n * kLocB; t += 256) Wm[t] = V[t];
                __syncthreads();
                local_bsolve(Lm, Dv, Wm, ld, n, 1 + npt, ta, tb);
                local_aprod(Lb.AM, ld, sidx, Wm, Tm, n, 1 + npt);
                local_coldot(Wm, Tm, true, n, 1 + npt, red, sums[2]);
            }
            if (tid == 0) {
                const int ic = (npt - 1) / 2;
                if (p != 1 && p != 2) {
                    const double mc = sums[0][1 + ic];
                    side = mc < o.theta ? 1.0 : -1.0;
                }
                double best = __builtin_inf();
                int ib = 0;
                for (int q = 0; q < npt; ++q) {
                    const double var = s2 - sums[1][1 + q] + (sparse ? sums[2][1 + q] : 0.0);
                    const double g = margin(side, o.theta, sums[0][1 + q], var > 0.0 ? var : 0.0);
                    if (g < best) {
                        best = g;
                        ib = q;
                    }
                }
                gmin = best;
                double x[3];
                lattice_point(o, blo, bhi, ib, x);
                for (int d = 0; d < 3; ++d) xcur[d] = x[d];
                red[0][0] = side;
                red[0][1] = gmin;
                state = (upper_bound(gmin, dp) > o.alpha || o.steps == 0) ? 1 : 0;
            }
            __syncthreads();
            side = red[0][0];
            gmin = red[0][1];
            __syncthreads();
            // projected steps: value and gradient at x_k, then the step; x_k (k >= 1) enters the minimum
            double eta = 0.5;
            for (int k = 0; k <= o.steps && !state; ++k) {
                const bool last = k == o.steps;
                const int R = last ? 1 : 1 + D;
                for (int i = tid; i < n; i += 256) {
                    double z[D], r2 = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        z[d] = xcur[d] - xs[i * D + d];
                        const double u = z[d] * Lb.kp.inv_ell[d];
                        r2 = fma(u, u, r2);
                    }
                    double kv, fv;
                    kernel_val_dfac(Lb.kp, r2, &kv, &fv);
                    V[(size_t)i * kLocB] = kv;
                    if (!last)
#pragma unroll
                        for (int d = 0; d < D; ++d)
                            V[(size_t)i * kLocB + 1 + d] = fv * z[d] * Lb.kp.inv_ell[d] * Lb.kp.inv_ell[d];
                }
                __syncthreads();
                local_fsolve(Lm, Dv, V, ld, n, R, ta, tb);
                local_colsum(V, wv, 0, n, R, red, sums[0]);       // mu, dmu_d
                local_colsum(V, nullptr, 0, n, R, red, sums[1]);  // |v|^2, v.u_d
                if (sparse) {
                    // sums[2][0] = w.A'w, sums[2][1 + d] = (K'^-1 dk_d).A'w
                    for (int t = tid; t < n * kLocB; t += 256) Wm[t] = V[t];
                    __syncthreads();
                    local_bsolve(Lm, Dv, Wm, ld, n, R, ta, tb);
                    local_aprod(Lb.AM, ld, sidx, Wm, Tm, n, R);
                    local_coldot(Wm, Tm, false, n, R, red, sums[2]);
                }
                if (tid == 0) {
                    const double mu = sums[0][0];
                    const double vr = s2 - sums[1][0] + (sparse ? sums[2][0] : 0.0);
                    const double var = vr > 0.0 ? vr : 0.0;
                    const double g = margin(side, o.theta, mu, var);
                    if (k >= 1 && g < gmin) gmin = g;
                    int stop = last || !(var > 0.0);
                    if (!stop) {
                        const double sd = sqrt(var);
                        double u[3], nrm = 0.0;
                        for (int a = 0; a < D; ++a) {
                            const double dvar = -2.0 * sums[1][1 + a] + (sparse ? 2.0 * sums[2][1 + a] : 0.0);
                            const double dsd = dvar / (2.0 * sd);
                            const double gr = side * (-sums[0][1 + a] * sd - (o.theta - mu) * dsd) / var;
                            u[a] = (bhi[a] - blo[a]) * gr;
                            nrm += u[a] * u[a];
                        }
                        nrm = sqrt(nrm);
                        if (!(nrm > 0.0) || !isfinite(nrm)) {
                            stop = 1;
                        } else {
                            for (int a = 0; a < D; ++a) {
                                const double w = bhi[a] - blo[a];
                                const double xn = xcur[a] - eta * w * u[a] / nrm;
                                xcur[a] = xn < blo[a] ? blo[a] : (xn > bhi[a] ? bhi[a] : xn);
                            }
                        }
                    }
                    red[0][1] = gmin;
                    state = (stop || upper_bound(gmin, dp) > o.alpha) ? 1 : 0;
                }
                __syncthreads();
                gmin = red[0][1];
                eta *= 0.5;
                __syncthreads();
            }
        }
        if (tid == 0) {
            B.side[b] = side;
            B.gmin[b] = gmin;
            sub[f] = upper_bound(gmin, dp) > o.alpha ? 1 : 0;
            cur = (int64_t)gridDim.x + atomicAdd(Lb.next, 1);
        }
        __syncthreads();
    }
}

}  // namespace

// Workspace layout of lcp_adaptive.
// Levels of the search with at most this many nodes skip the centre stage; levels of at least
// kCornersFirst nodes evaluate the lattice's corners before its other points.
constexpr int64_t kLatticeOnly = 512;
constexpr int64_t kCornersFirst = 32768;
// Octree levels of at least this many nodes (which take the corners first) run the certified
// bound on the nodes the corners leave open (k_lattice_cert).  It costs about one probe of
// those nodes and pays where many of them are far from the level (the octree's 8-way splits
// leave such nodes at the deepest levels); the K-D tree refines one axis at a time, so its
// deep candidates sit near the crossing and the certificate settles few.
constexpr int64_t kLatticeCert = 32768;

struct AdaptLayout {
    size_t total;
    size_t o_q, o_cnt, o_keys0, o_keys1, o_hob0, o_hob1, o_path, o_need, o_nidx, o_sub, o_ecnt, o_eoff, o_ub;
    size_t o_bnode, o_side, o_gmin, o_done, o_latp, o_latm, o_latv, o_gm, o_gv, o_gdm, o_gdv;
    size_t o_cpts, o_cmean, o_cvar, o_lnode, o_dnode, o_dbx, o_ddp, o_fcand, o_spp, o_spc, o_gx, o_ngrid, o_lmask, o_loff, o_lown, o_lnode2, o_bidx;
    size_t o_stat, o_statoff, o_scan, o_vmask, o_voff, o_slot, o_vlist, o_vmean, o_vvar, o_V, o_cross, o_zb, o_cellws;
    size_t o_cw, o_box, o_cert;          // certified bound (o_cw also for the certificate between the lattice passes)
    size_t o_dpts, o_dbox, o_dcert, o_lnode3;   // search: certificate between the lattice passes
    int lcert;                           // 1: the search has a level that runs it
    size_t o_loc, o_lnext;               // local-model bound only: per-work-group slots, work counter
    int nloc;                            // local-model bound only: slots (resident work-groups)
    int64_t capF, nv;
};

// Halvings of axis d at a level of the octree or of the K-D tree (node_shift on the host).
static int level_shift(int kd, int D, int level, int d)
{
    return kd ? level / D + (d >= D - level % D ? 1 : 0) : level;
}

// Work-groups of k_local_bound that are resident together on this device (its persistent
// grid, one workspace slot each): the occupancy for the model's LDS use times the CU count,
// at most kLocSlots.
static hipError_t local_slot_count(const Model& M, int D, int* slots)
{
    const size_t shm = (size_t)M.m_pad * (D + 1) * sizeof(double) + (size_t)M.m_pad * sizeof(int);
    int per_cu = 0, dev = 0, ncu = 0;
    hipError_t e = D == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_local_bound<3>, 256, shm)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_local_bound<2>, 256, shm);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    *slots = e == hipSuccess ? std::max(1, std::min(kLocSlots, per_cu * ncu)) : kLocSlots;
    return e;
}

static AdaptLayout adapt_layout(const Model& M, const GridP& g, int64_t S0, int Lmax, int prec, int ns, int bound_kind,
                                int kd, int64_t* caps, int64_t* nodes)
{
    AdaptLayout L{};
    const int D = g.dim;
    const int Ldepth = kd ? D * Lmax : Lmax;
    int64_t capF = 1, stat_total = 0;
    for (int l = 0; l <= Ldepth; ++l) {
        int64_t c = 1;
        for (int d = 0; d < 3; ++d) {
            const int64_t s = S0 >> level_shift(kd, D, l, d);
            int64_t nd = d < D ? ceil_div(g.nc[d], s) : 1;
            nodes[l * 3 + d] = nd;
            c *= nd;
        }
        caps[l] = c;
        stat_total += c;
        if (c > capF) capF = c;
    }
    const int64_t nv = g.n[0] * g.n[1] * g.n[2];
    const int npt = D == 3 ? 27 : 9;
    const int ndir = D == 3 ? 13 : 4;
    const size_t vb = prec == LCP_FP64 ? 8 : 4;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
    L.o_q = take(sizeof(double) * 2 * M.m_pad);
    L.o_cnt = take(sizeof(int64_t) * 64);
    L.o_keys0 = take(8 * capF);
    L.o_keys1 = take(8 * capF);
    L.o_hob0 = take((size_t)capF);
    L.o_hob1 = take((size_t)capF);
    L.o_path = take(4 * capF);
    L.o_need = take(4 * capF);
    L.o_nidx = take(4 * capF);
    L.o_sub = take(4 * capF);
    L.o_ecnt = take(4 * capF);
    L.o_eoff = take(4 * capF);
    L.o_ub = take(8 * capF);
    L.o_bnode = take(4 * capF);
    L.o_cpts = take(24 * capF);
    L.o_cmean = take(8 * capF);
    L.o_cvar = take(8 * capF);
    L.o_lnode = take(4 * capF);
    L.o_dnode = take(4 * capF);
    L.o_dbx = take(64 * capF);
    L.o_ddp = take(8 * capF);
    L.o_fcand = take(4 * capF);
    L.o_spp = take(8 * (size_t)kSplitGrid * 64);
    L.o_spc = take(4 * (size_t)kSplitGrid);
    L.o_gx = take(24 * capF);
    L.o_side = take(8 * capF);
    L.o_gmin = take(8 * capF);
    L.o_done = take(4 * capF);
    L.o_ngrid = take(4 * capF);
    L.o_lmask = take(4 * capF);
    L.o_loff = take(4 * capF);
    L.o_lown = take(4 * 32 * capF);
    L.o_lnode2 = take(4 * capF);
    L.o_bidx = take(4 * capF);
    L.o_latp = take(24 * capF * npt);
    L.o_latm = take(8 * capF * npt);
    L.o_latv = take(8 * capF * npt);
    L.o_gm = take(8 * capF);
    L.o_gv = take(8 * capF);
    L.o_gdm = take(24 * capF);
    L.o_gdv = take(24 * capF);
    L.o_stat = take(stat_total);
    L.o_statoff = take(8 * (Ldepth + 1));
    L.o_scan = take(scan_workspace(nv > capF ? nv : capF));
    L.o_vmask = take(4 * nv);
    L.o_voff = take(4 * nv);
    L.o_slot = take(4 * nv);
    L.o_vlist = take(4 * nv);
    L.o_vmean = take(8 * nv);
    L.o_vvar = take(8 * nv);
    L.o_V = take(vb * (size_t)nv * M.m_pad);
    L.o_cross = take(8 * (size_t)nv * ndir);
    L.o_zb = take(zbank32_bytes(ns, D));
    {
        int64_t cpl = 1;
        for (int d = 0; d < D; ++d) cpl *= S0 >> Lmax;
        L.o_cellws = take(cells_scratch_bytes(caps[Ldepth] * cpl));
    }
    if (bound_kind == LCP_BOUND_SEARCH && !kd && capF >= kLatticeCert) {
        L.lcert = 1;
        L.o_cw = take(8 * (size_t)M.m_pad * capF);
        L.o_dpts = take(24 * (size_t)capF);
        L.o_dbox = take(8 * 2 * (size_t)D * capF);
        L.o_dcert = take(32 * (size_t)capF);
        L.o_lnode3 = take(4 * (size_t)capF);
    }
    if (bound_kind == LCP_BOUND_CERTIFIED) {
        L.o_cw = take(8 * (size_t)M.m_pad * capF);
        L.o_box = take(8 * 2 * (size_t)D * capF);
        L.o_cert = take(32 * (size_t)capF);
    }
    if (bound_kind == LCP_BOUND_LOCAL) {
        int slots = kLocSlots;
        (void)local_slot_count(M, D, &slots);        // kLocSlots if the query fails
        L.nloc = slots;
        L.o_lnext = take(256);
        L.o_loc = take(8 * local_slot_doubles(M.m_pad) * (size_t)slots);
    }
    L.total = o;
    L.capF = capF;
    L.nv = nv;
    return L;
}

size_t adaptive_workspace(const Model& M, const GridP& g, int64_t S0, int Lmax, int prec, int ns,
                          const lcp_adapt& A)
{
    int64_t caps[24], nodes[72];
    return adapt_layout(M, g, S0, Lmax, prec, ns, A.bound_kind, A.split == LCP_SPLIT_KD, caps, nodes).total;
}

hipError_t run_adaptive(const Model& M, const GridP& g, double theta, const lcp_adapt& A, int64_t S0, int Lmax,
                        int prec, int ns, const double* zb, float* lcp, uint64_t* leaves, int64_t leaf_cap,
                        int64_t* n_leaves, uint8_t* level_field, char* ws, hipStream_t s)
{
    int64_t caps[24], nodes[72];
    const bool cert = A.bound_kind == LCP_BOUND_CERTIFIED;
    const bool local = A.bound_kind == LCP_BOUND_LOCAL;
    const bool search = !cert && !local;
    const int kd = A.split == LCP_SPLIT_KD;
    const int Ldepth = kd ? g.dim * Lmax : Lmax;
    AdaptLayout L = adapt_layout(M, g, S0, Lmax, prec, ns, A.bound_kind, kd, caps, nodes);
    const int D = g.dim;
    const int npt = D == 3 ? 27 : 9;
    Oct o{};
    o.g = g;
    o.D = D;
    o.S0 = S0;
    o.lgS0 = 0;
    while ((int64_t(1) << o.lgS0) < S0) ++o.lgS0;
    o.Lmax = Lmax;
    o.kd = kd;
    o.Ldepth = Ldepth;
    o.theta = theta;
    o.alpha = A.alpha;
    o.bound_at_max = A.bound_at_max_depth;
    o.steps = A.descent_steps;
    for (int i = 0; i < 72; ++i) o.nodes[i] = i < (Ldepth + 1) * 3 ? nodes[i] : 1;

    auto P = [&](size_t off) { return (void*)(ws + off); };
    double* qlo = (double*)P(L.o_q);
    double* qhi = qlo + M.m_pad;
    int64_t* cnt = (int64_t*)P(L.o_cnt);   // [0..22] frontier counts, [32..35] bound stages, [40] vertices
    uint64_t* keys[2] = {(uint64_t*)P(L.o_keys0), (uint64_t*)P(L.o_keys1)};
    uint8_t* hob[2] = {(uint8_t*)P(L.o_hob0), (uint8_t*)P(L.o_hob1)};   // per frontier node: parent held observations
    int32_t* path = (int32_t*)P(L.o_path);
    int32_t* need = (int32_t*)P(L.o_need);
    int32_t* nidx = (int32_t*)P(L.o_nidx);
    int32_t* sub = (int32_t*)P(L.o_sub);
    int32_t* ecnt = (int32_t*)P(L.o_ecnt);
    int32_t* eoff = (int32_t*)P(L.o_eoff);
    uint8_t* stat = (uint8_t*)P(L.o_stat);
    char* scanws = (char*)P(L.o_scan);
    BoundBufs B;
    B.bnode = (int32_t*)P(L.o_bnode);
    B.cpts = (double*)P(L.o_cpts);
    B.cmean = (double*)P(L.o_cmean);
    B.cvar = (double*)P(L.o_cvar);
    B.lnode = (int32_t*)P(L.o_lnode);
    B.ngrid = (int32_t*)P(L.o_ngrid);
    B.lmask = (int32_t*)P(L.o_lmask);
    B.loff = (int32_t*)P(L.o_loff);
    B.lown = (int32_t*)P(L.o_lown);
    B.lnode2 = (int32_t*)P(L.o_lnode2);
    B.bidx = (int32_t*)P(L.o_bidx);
    B.dnode = (int32_t*)P(L.o_dnode);
    B.dbx = (double*)P(L.o_dbx);
    B.ddp = (int64_t*)P(L.o_ddp);
    B.fcand = (int32_t*)P(L.o_fcand);
    double* spp = (double*)P(L.o_spp);
    int32_t* spc = (int32_t*)P(L.o_spc);
    double* gx = (double*)P(L.o_gx);
    B.side = (double*)P(L.o_side);
    B.gmin = (double*)P(L.o_gmin);
    B.done = (int32_t*)P(L.o_done);
    B.lat_pts = (double*)P(L.o_latp);
    B.lat_mean = (double*)P(L.o_latm);
    B.lat_var = (double*)P(L.o_latv);
    B.gp_mean = (double*)P(L.o_gm);
    B.gp_var = (double*)P(L.o_gv);
    B.gp_dmean = (double*)P(L.o_gdm);
    B.gp_dvar = (double*)P(L.o_gdv);
    B.cnt = cnt + 32;
    B.box = cert ? (double*)P(L.o_box) : nullptr;
    B.cert = cert ? (double*)P(L.o_cert) : nullptr;
    double* certW = (cert || L.lcert) ? (double*)P(L.o_cw) : nullptr;
    B.dpts = L.lcert ? (double*)P(L.o_dpts) : nullptr;
    B.dbox = L.lcert ? (double*)P(L.o_dbox) : nullptr;
    B.dcert = L.lcert ? (double*)P(L.o_dcert) : nullptr;
    B.lnode3 = L.lcert ? (int32_t*)P(L.o_lnode3) : nullptr;

    hipError_t e;
    const double* certF64 = M.Q64;   // the certified bound's operand Q, formed by the fit
    {
        int64_t acc = 0;
        for (int l = 0; l < 24; ++l) {
            o.statoff[l] = acc;
            if (l <= Ldepth) acc += caps[l];
        }
        e = launch_fill_u8(stat, 0, acc, s);
        if (e != hipSuccess) return e;
    }
    {
        StageScope sc(s, ST_OCTREE);
        hipLaunchKernelGGL(k_obs_q, dim3((unsigned)ceil_div(M.m, 256)), dim3(256), 0, s, M.obs_mu, M.obs_var, M.m,
                           theta, qlo, qhi);
        hipLaunchKernelGGL(k_root, dim3(1), dim3(256), 0, s, keys[0], cnt + 0, spc, hob[0]);
    }
    e = launch_fill_f32(lcp, 0.0f, g.nc[0] * g.nc[1] * g.nc[2], s);
    if (e != hipSuccess) return e;

    for (int l = 0; l <= Ldepth; ++l) {
        uint64_t* kin = keys[l & 1];
        uint64_t* kout = keys[(l + 1) & 1];
        const int64_t cap = caps[l];
        const int64_t* nf = cnt + l;
        // the finest level without a test emits every node (path 3): no bound to evaluate
        const bool bounded = !(l == Ldepth && !A.bound_at_max_depth);
        {
        StageScope sc(s, ST_OCTREE);
        hipLaunchKernelGGL(k_prelim, dim3(gsz(cap * 64, 256)), dim3(256), 0, s, o, l, kin, nf, cap, M.X, M.m, qlo, qhi,
                           path, need, sub, B, (int)search, hob[l & 1]);
        if (!search) {
            // the local and certified bounds take the nodes that need a bound, compacted
            e = launch_scan(need, nidx, cap, nf, B.cnt + 0, scanws, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_bound_setup, dim3(gsz(cap, 256)), dim3(256), 0, s, o, l, kin, nf, cap, need, nidx, B);
        }
        }
        auto post = [&](int64_t* count, int64_t cap_pts, const double* pts, double* mean, double* var, double* dmean,
                        double* dvar, int group) {
            PostTask t{};
            t.mode = COL_POINTS;
            t.group = group;
            t.count = count;
            t.n_points = cap_pts;
            t.pts = pts;
            t.pstride = 3;
            t.mean = mean;
            t.var = var;
            t.dmean = dmean;
            t.dvar = dvar;
            t.stage = ST_BOUND;
            t.sp_part = spp;
            t.sp_cnt = spc;
            return launch_posterior(M, LCP_FP64, t, s);
        };
        if (!bounded) {
        } else if (local) {
            // the search on each node's local model, one work-group per node
            LocalBufs lb{};
            lb.kp = M.kp;
            lb.X = M.X;
            lb.y = model_values(M);
            lb.m = M.m;
            lb.ld = M.m_pad;
            lb.noise = M.k.noise_var;
            lb.piv_scale = 2.220446049250313e-16 * (M.k.signal_var + M.k.noise_var);
            for (int d = 0; d < 3; ++d) lb.rad[d] = d < D ? A.beta * M.k.lengthscale[d] : 0.0;
            lb.AM = M.sparse ? M.AM : nullptr;
            lb.slots = (double*)P(L.o_loc);
            lb.next = (int32_t*)P(L.o_lnext);
            if ((e = launch_fill_i32(lb.next, 0, 1, s)) != hipSuccess) return e;
            StageScope sc(s, ST_BOUND);
            // a persistent grid of the work-groups that are resident together: one per slot
            const size_t shm = (size_t)M.m_pad * (D + 1) * sizeof(double) + (size_t)M.m_pad * sizeof(int);
            const int grid = L.nloc;
            if (D == 3)
                hipLaunchKernelGGL(k_local_bound<3>, dim3(grid), dim3(256), shm, s, o, l, kin, path, B, lb, sub);
            else
                hipLaunchKernelGGL(k_local_bound<2>, dim3(grid), dim3(256), shm, s, o, l, kin, path, B, lb, sub);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        } else if (cert) {
            // certified box bounds: w = Q k(c) on MFMA, moments per node, decision
            e = launch_cert_w(M, certF64, B.cpts, B.cnt + 0, cap, certW, B.cmean, B.cvar, s);
            if (e != hipSuccess) return e;
            e = launch_cert(M, B.box, B.cnt + 0, cap, certW, B.cert, s);
            if (e != hipSuccess) return e;
            StageScope sc(s, ST_OCTREE);
            hipLaunchKernelGGL(k_cert_decide, dim3(gsz(cap, 256)), dim3(256), 0, s, o, l, kin, path, B, sub);
        } else {
            // stage 1: centres of the frontier; the decision builds the stage-2 list and the
            // node lattice.  Levels of at most kLatticeOnly nodes go to the lattice at once:
            // their probe launches are bound by one tile's latency, so the centre launch
            // would cost as much as the lattice's.
            const bool centre = cap > kLatticeOnly;
            if (centre) {
                e = post(B.cnt + 0, cap, B.cpts, B.cmean, B.cvar, nullptr, nullptr, 1);
                if (e != hipSuccess) return e;
            }
            {
                StageScope sc(s, ST_OCTREE);
                hipLaunchKernelGGL(k_bound_centre, dim3(gsz(cap, 256)), dim3(256), 0, s, o, l, kin, path, need, B, sub,
                                   (int)centre);
            }
            // stage 2: lattice; the decision builds the stage-3 list and its start points.  Levels
            // of at least kCornersFirst nodes (after a centre stage) evaluate the corners first.
            const uint32_t all = (1u << npt) - 1;
            uint32_t corners = 0;
            for (int i = 0; i < npt; ++i) {
                bool c = true;
                for (int d = 0, r = i; d < D; ++d, r /= 3) c = c && (r % 3 != 1);
                if (c) corners |= 1u << i;
            }
            const bool cfirst = centre && cap >= kCornersFirst;
            // the certified bound between the passes (octree levels of at least kLatticeCert nodes)
            const bool ccert = cfirst && L.lcert && cap >= kLatticeCert;
            // after a centre stage the lattice reuses the centres' values (stage 1) instead of
            // evaluating that point again
            const uint32_t ctr = centre ? 1u << ((npt - 1) / 2) : 0u;
            auto lattice_pass = [&](const int32_t* list, int64_t* n_list, uint32_t pmask, int mode) {
                {
                    StageScope sc(s, ST_OCTREE);
                    hipLaunchKernelGGL(k_lattice_own, dim3(gsz(cap * 32, 512)), dim3(512), 0, s, o, l, kin, B, list,
                                       n_list, pmask);
                }
                hipError_t r = post(B.cnt + 2, cap * npt, B.lat_pts, B.lat_mean, B.lat_var, nullptr, nullptr, 1);
                if (r != hipSuccess) return r;
                StageScope sc(s, ST_OCTREE);
                hipLaunchKernelGGL(k_lattice, dim3(gsz(cap * 32, 512)), dim3(512), 0, s, o, l, kin, B, sub, gx, list,
                                   n_list, pmask, mode, (int)(ccert && mode == 1), (int)(centre && mode != 1));
                return hipGetLastError();
            };
            if (cfirst) {
                if ((e = lattice_pass(B.lnode, B.cnt + 1, corners, 1)) != hipSuccess) return e;
                const int32_t* list2 = B.lnode2;
                int64_t* n2 = B.cnt + 4;
                if (ccert) {
                    // w = Q k(c), box moments, decision: settled nodes skip the rest of the lattice
                    // and the descent
                    if ((e = launch_cert_w(M, certF64, B.dpts, B.cnt + 4, cap, certW, B.gp_mean, B.gp_var, s)) != hipSuccess)
                        return e;
                    if ((e = launch_cert(M, B.dbox, B.cnt + 4, cap, certW, B.dcert, s)) != hipSuccess) return e;
                    {
                        StageScope sc(s, ST_OCTREE);
                        hipLaunchKernelGGL(k_lattice_cert, dim3(gsz(cap, 256)), dim3(256), 0, s, o, l, kin, B);
                    }
                    list2 = B.lnode3;
                    n2 = B.cnt + 5;
                }
                if ((e = lattice_pass(list2, n2, all & ~corners & ~ctr, 2)) != hipSuccess) return e;
            } else {
                if ((e = lattice_pass(B.lnode, B.cnt + 1, all & ~ctr, 0)) != hipSuccess) return e;
            }
            // stage 3: projected-gradient steps, each in the epilogue of its probe (value and
            // gradient columns), then the value at the last point and the decision
            for (int k = 0; k < A.descent_steps; ++k) {
                PostTask t{};
                t.mode = COL_POINTS;
                t.group = 4;
                t.count = B.cnt + 3;
                t.n_points = cap;
                t.pts = gx;
                t.pstride = 3;
                t.mean = B.gp_mean;
                t.var = B.gp_var;
                t.dmean = B.gp_dmean;
                t.dvar = B.gp_dvar;
                t.stage = ST_BOUND;
                t.epi = EPI_STEP;
                t.epi_step = k;
                t.theta = theta;
                t.cand_done = B.done;
                t.cand_rec = B.dbx;
                t.sp_part = spp;
                t.sp_cnt = spc;
                if ((e = launch_posterior(M, LCP_FP64, t, s)) != hipSuccess) return e;
            }
            // the value at the last point; the emit count takes the decision
            if (A.descent_steps > 0 && (e = post(B.cnt + 3, cap, gx, B.gp_mean, B.gp_var, nullptr, nullptr, 1)) != hipSuccess)
                return e;
        }
        StageScope sc(s, ST_OCTREE);
        int64_t* nout = (l == Ldepth) ? n_leaves : cnt + l + 1;
        const int fin = search && bounded && A.descent_steps > 0;   // candidates' decisions pending
        hipLaunchKernelGGL(k_emit_count, dim3(gsz(cap, 256)), dim3(256), 0, s, o, l, kin, nf, cap, sub, ecnt, B, fin);
        e = launch_scan(ecnt, eoff, cap, nf, nout, scanws, s);
        if (e != hipSuccess) return e;
        uint64_t* dst = (l == Ldepth) ? leaves : kout;
        const int64_t dcap = (l == Ldepth) ? leaf_cap : caps[l + 1];
        hipLaunchKernelGGL(k_emit, dim3(gsz(cap, 256)), dim3(256), 0, s, o, l, kin, nf, cap, sub, eoff, dst, dcap,
                           stat + o.statoff[l], path, hob[(l + 1) & 1]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (level_field) {
        StageScope sc(s, ST_OCTREE);
        hipLaunchKernelGGL(k_level_field, dim3(gsz(g.nc[0] * g.nc[1] * g.nc[2], 256)), dim3(256), 0, s, o, stat,
                           level_field);
    }

    // ---- reconstruction of the emitted nodes (Sec. 5.3, last paragraph)
    const int leaf_edge = (int)(S0 >> Lmax);
    int32_t* vmask = (int32_t*)P(L.o_vmask);
    int32_t* voff = (int32_t*)P(L.o_voff);
    int32_t* slot = (int32_t*)P(L.o_slot);
    int32_t* vlist = (int32_t*)P(L.o_vlist);
    int64_t* nvd = cnt + 40;
    e = launch_fill_i32(vmask, 0, L.nv, s);
    if (e != hipSuccess) return e;
    int64_t per = 1;
    for (int d = 0; d < D; ++d) per *= leaf_edge + 1;
    {
    StageScope sc(s, ST_OCTREE);
    hipLaunchKernelGGL(k_mark, dim3(gsz(leaf_cap * per, 256)), dim3(256), 0, s, o, leaf_edge, leaves, n_leaves,
                       leaf_cap, vmask);
    e = launch_scan(vmask, voff, L.nv, nullptr, nvd, scanws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_slots, dim3(gsz(L.nv, 256)), dim3(256), 0, s, vmask, voff, L.nv, slot, vlist);
    }
    double* vmean = (double*)P(L.o_vmean);
    double* vvar = (double*)P(L.o_vvar);
    void* V = P(L.o_V);
    double* cross = (double*)P(L.o_cross);
    PostTask tp{};
    tp.mode = COL_GRID;
    tp.group = 1;
    tp.count = nvd;
    tp.n_points = L.nv;
    tp.grid = g;
    tp.vlist = vlist;
    tp.mean = vmean;
    tp.var = vvar;
    tp.V = V;
    tp.stage = ST_POSTERIOR;
    e = launch_posterior(M, prec, tp, s);
    if (e != hipSuccess) return e;
    e = launch_cross(M, prec, g, vlist, nvd, L.nv, slot, V, cross, s);
    if (e != hipSuccess) return e;
    if (A.edge_bound) {
        // keep the emitted nodes whose edge-crossing bound exceeds alpha (octree buffers reused)
        StageScope sc(s, ST_OCTREE);
        int32_t* eflag = need;
        int32_t* eoff2 = nidx;
        uint64_t* kept = (uint64_t*)P(L.o_keys0);
        int64_t* kept_n = cnt + 41;
        hipLaunchKernelGGL(k_edge_bound, dim3(gsz(leaf_cap * 64, 256)), dim3(256), 0, s, o, leaf_edge, leaves,
                           n_leaves, leaf_cap, slot, vmean, vvar, cross, eflag, (double*)nullptr);
        const int64_t ncap = leaf_cap < caps[Ldepth] ? leaf_cap : caps[Ldepth];   // the octree buffers' size
        e = launch_scan(eflag, eoff2, ncap, n_leaves, kept_n, scanws, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_keep_leaves, dim3(gsz(leaf_cap, 256)), dim3(256), 0, s, leaves, n_leaves, leaf_cap,
                           eflag, eoff2, kept);
        hipLaunchKernelGGL(k_store_kept, dim3(gsz(leaf_cap, 256)), dim3(256), 0, s, kept, kept_n, leaves, n_leaves,
                           leaf_cap);
        hipLaunchKernelGGL(k_set_leaf_count, dim3(1), dim3(1), 0, s, n_leaves, kept_n, leaf_cap);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    float* zb32 = (float*)P(L.o_zb);
    if (prec != LCP_FP64) {
        e = launch_zbank32(zb, zb32, ns, D, s);
        if (e != hipSuccess) return e;
    }
    CellTask ct{};
    ct.grid = g;
    ct.prec = prec;
    ct.theta = theta;
    ct.ns = ns;
    ct.zb64 = zb;
    ct.zb32 = zb32;
    ct.mean = vmean;
    ct.var = vvar;
    ct.cross = cross;
    ct.slot = slot;
    ct.leaves = leaves;
    ct.n_leaves = n_leaves;
    ct.leaf_cap = leaf_cap;
    ct.S0 = S0;
    ct.Lmax = Lmax;
    ct.leaf_edge = leaf_edge;
    ct.lcp = lcp;
    {
        int64_t cpl_all = 1;
        for (int d = 0; d < D; ++d) cpl_all *= leaf_edge;
        char* cw = (char*)P(L.o_cellws);
        ct.work = (int32_t*)cw;
        ct.wcount = (int64_t*)(cw + align256(4 * (size_t)(caps[Ldepth] * cpl_all)));
        ct.zmax = (double*)((char*)ct.wcount + 64);
    }
    int64_t cpl = 1;
    for (int d = 0; d < D; ++d) cpl *= leaf_edge;
    return launch_cells(ct, leaf_cap * cpl, s);
}

}  // namespace lcp
