// Stable LSD radix sort of (u64 key, u32 value) pairs, 8-bit digits.
//
// Each pass is reduce-then-scan: per-tile digit counts (digit-major table),
// one exclusive scan of that table, then a stable scatter.  Within a tile the
// rank of an element among equal digits comes from 64-lane ballots (the peer
// mask of lanes holding the same digit), accumulated wave by wave in LDS, so
// element order inside every digit run is the input order: the sort is
// stable, which makes ties fall back to the original particle index.
// The scatter goes through LDS so that every digit run is written to HBM as
// contiguous, coalesced stores.
#include "tc_internal.h"

namespace tc {
namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortThreads = 256;          // 4 waves
constexpr int kSortWaves = kSortThreads / 64;
// 15 keys per lane: the scatter kernel's 52 240 bytes of LDS fit 3 blocks per CU
// (16 keys, 55 312 bytes, fit only 2 in 512-byte allocation granules)
constexpr int kSortItems = 15;             // per lane
constexpr int kWaveTile = 64 * kSortItems; // 960 per wave
constexpr int kSortTile = kSortThreads * kSortItems;  // 3840 per block

__device__ inline uint32_t lane_id() { return threadIdx.x & 63; }

// Count of set bits of m strictly below this lane.
__device__ inline uint32_t popc_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Mask of the lanes of this wave whose (valid) digit equals ours.
__device__ inline uint64_t peer_mask(uint32_t d, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        uint64_t bal = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

__global__ __launch_bounds__(kSortThreads) void k_upsweep(const uint64_t* __restrict__ keys, int64_t n,
                                                          int shift, uint32_t* __restrict__ counts,
                                                          int64_t ntiles)
{
    __shared__ uint32_t hist[kSortWaves][kRadix];
    for (int j = threadIdx.x; j < kSortWaves * kRadix; j += kSortThreads) (&hist[0][0])[j] = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const uint32_t lane = lane_id();
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)w * kWaveTile;
#pragma unroll 4
    for (int k = 0; k < kSortItems; ++k) {
        int64_t i = base + k * 64 + lane;
        bool valid = i < n;
        uint32_t d = valid ? (uint32_t)(keys[i] >> shift) & (kRadix - 1) : 0u;
        uint64_t peers = peer_mask(d, valid);
        if (valid && popc_below(peers) == 0) hist[w][d] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kSortThreads) {
        uint32_t t = 0;
        for (int ww = 0; ww < kSortWaves; ++ww) t += hist[ww][d];
        counts[(int64_t)d * ntiles + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_downsweep(const uint64_t* __restrict__ kin,
                                                            const uint32_t* __restrict__ vin,
                                                            uint64_t* __restrict__ kout,
                                                            uint32_t* __restrict__ vout, int64_t n,
                                                            int shift,
                                                            const uint32_t* __restrict__ offsets,
                                                            int64_t ntiles)
{
    __shared__ uint32_t wcnt[kSortWaves][kRadix];
    __shared__ uint32_t tstart[kRadix];
    __shared__ uint32_t gbase[kRadix];
    __shared__ uint32_t dsum[kSortWaves];
    __shared__ uint64_t sk[kSortTile];
    __shared__ uint32_t sv[kSortTile];

    for (int j = threadIdx.x; j < kSortWaves * kRadix; j += kSortThreads) (&wcnt[0][0])[j] = 0;
    for (int d = threadIdx.x; d < kRadix; d += kSortThreads)
        gbase[d] = offsets[(int64_t)d * ntiles + blockIdx.x];
    __syncthreads();

    const int w = threadIdx.x >> 6;
    const uint32_t lane = lane_id();
    const int64_t tbase = (int64_t)blockIdx.x * kSortTile;
    const int64_t base = tbase + (int64_t)w * kWaveTile;

    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rank[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int64_t i = base + k * 64 + lane;
        bool valid = i < n;
        key[k] = valid ? kin[i] : 0ull;
        val[k] = valid ? vin[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int64_t i = base + k * 64 + lane;
        bool valid = i < n;
        uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
        uint64_t peers = peer_mask(d, valid);
        uint32_t below = popc_below(peers);
        uint32_t old = valid ? wcnt[w][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) wcnt[w][d] = old + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        rank[k] = old + below;
    }
    __syncthreads();
    // wave-exclusive prefix per digit, tile total per digit
    uint32_t tot = 0;
    const int d0 = threadIdx.x;  // kSortThreads == kRadix
    for (int ww = 0; ww < kSortWaves; ++ww) {
        uint32_t c = wcnt[ww][d0];
        wcnt[ww][d0] = tot;
        tot += c;
    }
    // exclusive scan of tot over the 256 digits (one per thread)
    {
        uint32_t v = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t t = __shfl_up(v, o, 64);
            if ((int)lane >= o) v += t;
        }
        if (lane == 63) dsum[w] = v;
        __syncthreads();
        uint32_t off = 0;
        for (int ww = 0; ww < w; ++ww) off += dsum[ww];
        tstart[d0] = off + v - tot;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int64_t i = base + k * 64 + lane;
        if (i < n) {
            uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
            uint32_t p = tstart[d] + wcnt[w][d] + rank[k];
            sk[p] = key[k];
            sv[p] = val[k];
        }
    }
    __syncthreads();
    const int64_t rem = n - tbase;
    const int tn = rem < kSortTile ? (int)rem : kSortTile;
    for (int j = threadIdx.x; j < tn; j += kSortThreads) {
        uint64_t k = sk[j];
        uint32_t d = (uint32_t)(k >> shift) & (kRadix - 1);
        int64_t g = (int64_t)gbase[d] + (j - (int64_t)tstart[d]);
        if (g >= 0 && g < n) {  // always true for consistent counts; guards the store
            kout[g] = k;
            vout[g] = sv[j];
        }
    }
}

}  // namespace

size_t radix_temp_bytes(int64_t n)
{
    int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    int64_t m = ntiles * kRadix;
    size_t b = (size_t)m * 4 * 2 + 8 + scan_temp_bytes(m);
    return (b + 255) & ~(size_t)255;
}

void radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                      int bits, void* temp, hipStream_t s, uint64_t** keys_out, uint32_t** vals_out)
{
    *keys_out = keys;
    *vals_out = vals;
    if (n <= 1) return;
    int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    int64_t m = ntiles * kRadix;
    uint32_t* counts = (uint32_t*)temp;
    uint32_t* offsets = counts + m;                 // m + 1 entries
    void* stemp = (void*)(offsets + m + 2);
    uint64_t* kin = keys;
    uint32_t* vin = vals;
    uint64_t* ko = keys_alt;
    uint32_t* vo = vals_alt;
    for (int shift = 0; shift < bits; shift += kRadixBits) {
        k_upsweep<<<(unsigned)ntiles, kSortThreads, 0, s>>>(kin, n, shift, counts, ntiles);
        launch_exclusive_scan_u32(counts, offsets, m, stemp, s);
        k_downsweep<<<(unsigned)ntiles, kSortThreads, 0, s>>>(kin, vin, ko, vo, n, shift, offsets, ntiles);
        uint64_t* tk = kin; kin = ko; ko = tk;
        uint32_t* tv = vin; vin = vo; vo = tv;
    }
    *keys_out = kin;
    *vals_out = vin;
}

}  // namespace tc
