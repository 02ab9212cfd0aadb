// vdi_scan.hip -- exclusive prefix sum of per-list supersegment counts into
// the offsets of the compact layout (Sec. 4, Fig. 2b).  The paper computes
// this on the host; here it stays on the device between the threshold
// search and the write pass.
//
// Two levels: each 1024-thread block scans 4096 counts (4 per thread, wave
// prefix via DPP-friendly shuffles, then across the 16 waves in LDS) and
// writes its total; one block scans the block totals; a final pass adds each
// block's base.  Handles up to 4096*4096 counts.
#include "vdi_internal.h"
#include "vdi_kernels.h"

namespace vdi {

namespace {

constexpr int kThreads = 1024;
constexpr int kItems = 4;
constexpr int kTile = kThreads * kItems;

__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Exclusive scan of the block's kTile values in place (in registers); returns the block total.
__device__ inline uint32_t block_scan(uint32_t (&v)[kItems], uint32_t* wave_sums)
{
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        uint32_t x = v[i];
        v[i] = s;
        s += x;
    }
    uint32_t incl = wave_incl_scan(s);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 63) wave_sums[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        uint32_t ws = lane < kThreads / 64 ? wave_sums[lane] : 0u;
        uint32_t wi = wave_incl_scan(ws);
        if (lane < kThreads / 64) wave_sums[lane] = wi - ws;
        if (lane == kThreads / 64 - 1) wave_sums[kThreads / 64] = wi;
    }
    __syncthreads();
    uint32_t base = wave_sums[wave] + incl - s;
#pragma unroll
    for (int i = 0; i < kItems; ++i) v[i] += base;
    uint32_t total = wave_sums[kThreads / 64];
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(kThreads) void scan_tiles(const int* __restrict__ counts, uint32_t* __restrict__ out,
                                                       uint32_t* __restrict__ tile_sums, size_t n)
{
    __shared__ uint32_t wave_sums[kThreads / 64 + 1];
    size_t base = (size_t)blockIdx.x * kTile + (size_t)threadIdx.x * kItems;
    uint32_t v[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        int c = base + i < n ? counts[base + i] : 0;
        v[i] = c > 0 ? (uint32_t)c : 0u;
    }
    uint32_t total = block_scan(v, wave_sums);
#pragma unroll
    for (int i = 0; i < kItems; ++i)
        if (base + i < n) out[base + i] = v[i];
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void scan_sums(uint32_t* __restrict__ tile_sums, size_t ntiles,
                                                      uint32_t* __restrict__ grand_total)
{
    __shared__ uint32_t wave_sums[kThreads / 64 + 1];
    size_t base = (size_t)threadIdx.x * kItems;
    uint32_t v[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) v[i] = base + i < ntiles ? tile_sums[base + i] : 0u;
    uint32_t total = block_scan(v, wave_sums);
#pragma unroll
    for (int i = 0; i < kItems; ++i)
        if (base + i < ntiles) tile_sums[base + i] = v[i];
    if (threadIdx.x == 0) *grand_total = total;
}

__global__ __launch_bounds__(256) void scan_add(uint32_t* __restrict__ out, const uint32_t* __restrict__ tile_sums,
                                                size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_sums[i / kTile];
}

}  // namespace

size_t scan_scratch_bytes(size_t n)
{
    size_t tiles = (n + kTile - 1) / kTile;
    return (tiles + 1) * sizeof(uint32_t);
}

void launch_scan(const int* counts, uint32_t* offsets, size_t n, void* scratch, hipStream_t s)
{
    size_t tiles = (n + kTile - 1) / kTile;
    if (tiles == 0) tiles = 1;
    uint32_t* sums = (uint32_t*)scratch;
    hipLaunchKernelGGL(scan_tiles, dim3(tiles), dim3(kThreads), 0, s, counts, offsets, sums, n);
    // the grand total lands in offsets[n]
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kThreads), 0, s, sums, tiles, offsets + n);
    if (n > 0) hipLaunchKernelGGL(scan_add, dim3((n + 255) / 256), dim3(256), 0, s, offsets, sums, n);
}

}  // namespace vdi
