// Exclusive prefix sum of uint32 counts (ray -> first live sample, brick ->
// first bucket slot).  Three launches: per-block scan with block totals,
// scan of the totals in one block, add-back.  out has n+1 entries; out[n] is
// the grand total.
#include "kernels.h"

namespace cic {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanBlock = kScanThreads * kScanPer;   // 2048 elements per block

size_t scan_tmp_elems(int64_t n)
{
    int64_t blocks = (n + kScanBlock - 1) / kScanBlock;
    return (size_t)blocks + 1;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t &total)
{
    __shared__ uint32_t wsum[kScanThreads / kWave];
    const int l = lane_id(), w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t u = __shfl_up(x, off, kWave);
        if (l >= off) x += u;
    }
    if (l == kWave - 1) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        if (i < w) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    total = all;
    return before + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(const uint32_t *in, uint32_t *out, uint32_t *tmp,
                                                              int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t pre = block_exclusive_scan(s, total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < n) out[base + i] = pre;
        pre += v[i];
    }
    if (threadIdx.x == 0) tmp[blockIdx.x] = total;
}

// One block scans up to kScanBlock block totals in place; tmp[nb] = total.
__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint32_t *tmp, int64_t nb)
{
    const int64_t base = (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        v[i] = (base + i < nb) ? tmp[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t pre = block_exclusive_scan(s, total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < nb) tmp[base + i] = pre;
        pre += v[i];
    }
    if (threadIdx.x == 0) tmp[nb] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(uint32_t *out, const uint32_t *tmp, int64_t n, int64_t nb)
{
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    const uint32_t add = tmp[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < n) out[base + i] += add;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tmp[nb];
}

void launch_exclusive_scan(const uint32_t *in, uint32_t *out, uint32_t *tmp, int64_t n, hipStream_t s)
{
    // n <= kScanBlock * kScanBlock (4M) is guaranteed by the callers.
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, tmp, (int64_t)0);
        hipLaunchKernelGGL(k_scan_add, dim3(1), dim3(kScanThreads), 0, s, out, tmp, (int64_t)0, (int64_t)0);
        return;
    }
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, tmp, n);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, out, tmp, n, nb);
}

}  // namespace cic
