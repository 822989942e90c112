// Device-wide exclusive prefix sum of u32 (reduce, scan the block sums, scan
// again with the block offsets).  out has n + 1 entries; out[n] is the total.
#include "tc_internal.h"

namespace tc {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

__device__ inline uint32_t wave_inclusive_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over the block; returns the block
// total through *total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* total)
{
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / 64; ++i) {
        if (i < w) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const uint32_t* __restrict__ in, int64_t n,
                                                            uint32_t* __restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t v = 0;
    for (int j = threadIdx.x; j < kScanTile; j += kScanThreads) {
        int64_t i = base + j;
        if (i < n) v += in[i];
    }
    uint32_t tot;
    block_exclusive_scan(v, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One block scans the tile sums in place (exclusive) and writes the total.
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(uint32_t* __restrict__ sums, int64_t nt,
                                                            uint32_t* __restrict__ total_out)
{
    uint32_t carry = 0;
    for (int64_t b = 0; b < nt; b += kScanThreads) {
        int64_t i = b + threadIdx.x;
        uint32_t v = i < nt ? sums[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, &tot);
        if (i < nt) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const uint32_t* __restrict__ in, int64_t n,
                                                             const uint32_t* __restrict__ sums,
                                                             uint32_t* __restrict__ out)
{
    __shared__ uint32_t buf[kScanTile];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int j = threadIdx.x; j < kScanTile; j += kScanThreads) {
        int64_t i = base + j;
        buf[j] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t loc[kScanItems];
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        loc[k] = buf[threadIdx.x * kScanItems + k];
        v += loc[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(v, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        buf[threadIdx.x * kScanItems + k] = ex;
        ex += loc[k];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kScanTile; j += kScanThreads) {
        int64_t i = base + j;
        if (i < n) out[i] = buf[j];
    }
}

}  // namespace

size_t scan_temp_bytes(int64_t n)
{
    int64_t nt = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nt + 1) * sizeof(uint32_t);
}

void launch_exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t s)
{
    int64_t nt = (n + kScanTile - 1) / kScanTile;
    uint32_t* sums = (uint32_t*)temp;
    if (nt > 0) k_tile_sums<<<(unsigned)nt, kScanThreads, 0, s>>>(in, n, sums);
    k_scan_sums<<<1, kScanThreads, 0, s>>>(sums, nt, out + n);
    if (nt > 0) k_scan_tiles<<<(unsigned)nt, kScanThreads, 0, s>>>(in, n, sums, out);
}

}  // namespace tc
