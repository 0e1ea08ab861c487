// Deterministic exclusive prefix sum of int32 flags/counts, built from wavefront scans:
// each 1024-thread block scans 4096 entries (64-lane shuffle scans + a scan of the 16
// wave totals), a single block scans the block totals, and a last pass adds the carries.
// Inputs of at most 16 chunks are scanned by one work-group in a single launch.
#include "lcp_internal.h"

namespace lcp {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kPerThread = 4;
constexpr int kChunk = kScanThreads * kPerThread;

__device__ __forceinline__ int64_t scan_n(const int64_t* n_dev, int64_t n)
{
    if (n_dev) {
        int64_t d = *n_dev;
        return d < n ? d : n;
    }
    return n;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_blocks(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                              int64_t n, const int64_t* n_dev, int32_t* __restrict__ sums)
{
    __shared__ int sh[65];
    const int64_t nn = scan_n(n_dev, n);
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    if (base >= nn) {
        if (threadIdx.x == 0) sums[blockIdx.x] = 0;
        return;
    }
    int v[kPerThread];
    int loc = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kPerThread + k;
        v[k] = i < nn ? in[i] : 0;
        loc += v[k];
    }
    int tot;
    int ex = block_excl_scan(loc, sh, &tot);
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kPerThread + k;
        if (i < nn) out[i] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(int32_t* __restrict__ sums, int nb, int64_t* total)
{
    __shared__ int sh[65];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += kScanThreads) {
        int i = base + threadIdx.x;
        int v = i < nb ? sums[i] : 0;
        int tot;
        int ex = block_excl_scan(v, sh, &tot);
        int c = carry;
        if (i < nb) sums[i] = ex + c;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(int32_t* __restrict__ out, int64_t n, const int64_t* n_dev,
                                                           const int32_t* __restrict__ sums)
{
    const int64_t nn = scan_n(n_dev, n);
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    if (base >= nn) return;
    const int c = sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kPerThread + k;
        if (i < nn) out[i] += c;
    }
}

// Whole scan in one work-group for short inputs: chunks of 4096 in order, with a carry.
__global__ void __launch_bounds__(kScanThreads) k_scan_single(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                              int64_t n, const int64_t* n_dev, int64_t* total)
{
    __shared__ int sh[65];
    const int64_t nn = scan_n(n_dev, n);
    int carry = 0;
    for (int64_t base = 0; base < nn; base += kChunk) {
        int v[kPerThread];
        int loc = 0;
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int64_t i = base + (int64_t)threadIdx.x * kPerThread + k;
            v[k] = i < nn ? in[i] : 0;
            loc += v[k];
        }
        int tot;
        int ex = block_excl_scan(loc, sh, &tot) + carry;
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int64_t i = base + (int64_t)threadIdx.x * kPerThread + k;
            if (i < nn) out[i] = ex;
            ex += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

}  // namespace

size_t scan_workspace(int64_t n)
{
    return align256(sizeof(int32_t) * (size_t)(ceil_div(n, kChunk) + 1));
}

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, const int64_t* n_dev, int64_t* total, char* ws,
                       hipStream_t s)
{
    int64_t nb = ceil_div(n, kChunk);
    if (nb < 1) nb = 1;
    if (nb <= 16) {                 // short inputs: one launch instead of three
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScanThreads), 0, s, in, out, n, n_dev, total);
        return hipGetLastError();
    }
    int32_t* sums = (int32_t*)ws;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, n_dev, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, sums, (int)nb, total);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, out, n, n_dev, sums);
    return hipGetLastError();
}

}  // namespace lcp
