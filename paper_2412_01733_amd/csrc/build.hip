// Bottom-up octree construction from sorted Morton keys.
//
// The tree is the canonical octree of the TreeCode description (section 2):
// a level-l cell (particles sharing the top 3l key bits) is a node iff it is
// the root or its parent cell holds >= 2 particles; cells of one particle and
// level-21 cells are leaves; a cell whose particles all fall in one octant
// keeps its single child (chain node).
//
// With c_s = the deepest level at which keys s and s+1 share a cell
// (c_s = min(21, floor((clz64(k_s ^ k_{s+1}) - 1) / 3)), c_{-1} = c_{n-1} = -1),
// the nodes whose first particle is s are exactly the levels
//   c_{s-1} + 1 ... min(21, max(c_{s-1}, c_s) + 1),
// so the node count per particle is local and the pre-order index of every
// node is an exclusive scan over s (pre-order = order by (first, level)).
// A node's end is found by galloping search on the keys, and its skip link
// ("next") is the pre-order index of the first node starting at its end.
//
// The walk wants siblings contiguous and the upward pass wants each level
// contiguous, so the walk's node array is in breadth-first order: sorted by
// (level, first), obtained by one stable 8-bit radix pass on the level of
// the pre-order nodes.  The children of pre-order node p then start at the
// breadth-first index of p + 1 and are consecutive.
#include "tc_internal.h"

namespace tc {
namespace {

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

__global__ __launch_bounds__(256) void k_adjacent(const uint64_t* __restrict__ k, int64_t n,
                                                  int8_t* __restrict__ c)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    if (s == n - 1) {
        c[s] = -1;
        return;
    }
    uint64_t x = k[s] ^ k[s + 1];
    int lv = 21;
    if (x != 0) {
        int z = __clzll((long long)x);
        lv = (z - 1) / 3;
        if (lv > 21) lv = 21;
    }
    c[s] = (int8_t)lv;
}

__device__ inline void node_range(const int8_t* c, int64_t s, int& lo, int& hi)
{
    int cp = s > 0 ? (int)c[s - 1] : -1;
    int cs = (int)c[s];
    lo = cp + 1;
    int m = cp > cs ? cp : cs;
    hi = m + 1 < kMaxLevel ? m + 1 : kMaxLevel;
}

// Node count per first particle, plus a histogram of node levels and the
// leaf counts (counted per wave with ballots, then one atomic per entry and
// block).  hist[0..21]: nodes per level; hist[22]: leaves; hist[23]:
// multi-particle leaves.  The deepest node starting at s is always a leaf,
// and it holds several particles iff it sits at level 21 and s + 1 shares it.
__global__ __launch_bounds__(256) void k_node_counts(const int8_t* __restrict__ c, int64_t n,
                                                     uint32_t* __restrict__ cnt,
                                                     uint32_t* __restrict__ level_hist)
{
    constexpr int kH = kLevels + 2;
    __shared__ uint32_t h[256 / 64][kH];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t acc = 0;  // lane l < kH of each wave accumulates entry l
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t s0 = start - threadIdx.x; s0 < n; s0 += stride) {
        const int64_t s = s0 + threadIdx.x;
        int lo = 1, hi = 0, cs = -1;
        if (s < n) {
            node_range(c, s, lo, hi);
            cs = (int)c[s];
            int k = hi - lo + 1;
            cnt[s] = (uint32_t)(k > 0 ? k : 0);
        }
        for (int l = 0; l < kLevels; ++l) {
            const uint32_t b = (uint32_t)__popcll(__ballot(lo <= l && l <= hi));
            if (lane == l) acc += b;
        }
        const uint32_t bl = (uint32_t)__popcll(__ballot(lo <= hi));
        const uint32_t bm = (uint32_t)__popcll(__ballot(lo <= hi && hi == kMaxLevel && cs == kMaxLevel));
        if (lane == kLevels) acc += bl;
        if (lane == kLevels + 1) acc += bm;
    }
    if (lane < kH) h[w][lane] = acc;
    __syncthreads();
    if (threadIdx.x < kH) {
        uint32_t t = 0;
        for (int ww = 0; ww < 256 / 64; ++ww) t += h[ww][threadIdx.x];
        if (t) atomicAdd(&level_hist[threadIdx.x], t);
    }
}

// First index j > s whose level-l prefix differs from that of key (or n).
// The caller guarantees that s + 1 < n shares the prefix.
__device__ inline int64_t cell_end(const uint64_t* __restrict__ k, int64_t n, int64_t s, uint64_t key, int l)
{
    const int sh = 3 * (kMaxLevel - l);
    const uint64_t P = key >> sh;
    int64_t in = s + 1;  // known inside
    int64_t step = 1;
    int64_t probe = in + step;
    while (probe < n && (k[probe] >> sh) == P) {
        in = probe;
        step <<= 1;
        probe = in + step;
    }
    int64_t lo = in + 1, hi = probe < n ? probe : n;
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if ((k[mid] >> sh) == P) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_emit(const uint64_t* __restrict__ k, const int8_t* __restrict__ c,
                                              const uint32_t* __restrict__ pre, int64_t n,
                                              uint8_t* __restrict__ level, uint32_t* __restrict__ first,
                                              uint32_t* __restrict__ count, uint32_t* __restrict__ next,
                                              uint8_t* __restrict__ octant)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int lo, hi;
    node_range(c, s, lo, hi);
    const int cs = (int)c[s];
    const uint64_t key = k[s];
    uint32_t p = pre[s];
    for (int l = lo; l <= hi; ++l, ++p) {
        int64_t end = (l > cs) ? s + 1 : cell_end(k, n, s, key, l);
        level[p] = (uint8_t)l;
        octant[p] = l > 0 ? (uint8_t)((key >> (3 * (kMaxLevel - l))) & 7u) : (uint8_t)0;  // key digit at level l
        first[p] = (uint32_t)s;
        count[p] = (uint32_t)(end - s);
        next[p] = pre[end];
    }
}

__device__ inline bool is_internal(uint8_t level, uint32_t count) { return count >= 2 && level < kMaxLevel; }

// Children per node, walked through the skip links.
__global__ __launch_bounds__(256) void k_count_children(const uint8_t* __restrict__ level,
                                                        const uint32_t* __restrict__ count,
                                                        const uint32_t* __restrict__ next, int64_t nn,
                                                        uint32_t* __restrict__ nchild)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nn) return;
    if (!is_internal(level[p], count[p])) {
        nchild[p] = 0;
        return;
    }
    uint32_t e = next[p], ch = (uint32_t)p + 1, k = 0;
    while (ch < e) {
        ++k;
        ch = next[ch];
    }
    nchild[p] = k;
}

// Sort input for the breadth-first permutation: key = level, value = p.
__global__ __launch_bounds__(256) void k_level_keys(const uint8_t* __restrict__ level, int64_t nn,
                                                    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nn) return;
    keys[p] = level[p];
    vals[p] = (uint32_t)p;
}

__global__ __launch_bounds__(256) void k_bfs_scatter(const uint32_t* __restrict__ bfs_to_pre, int64_t nn,
                                                     uint32_t* __restrict__ bfs)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nn) return;
    bfs[bfs_to_pre[b]] = (uint32_t)b;
}

}  // namespace

void launch_adjacent_levels(const uint64_t* skeys, int64_t n, int8_t* c, hipStream_t s)
{
    if (n == 0) return;
    k_adjacent<<<grid_for(n, 256), 256, 0, s>>>(skeys, n, c);
}

void launch_node_counts(const int8_t* c, int64_t n, uint32_t* cnt, uint32_t* level_hist, hipStream_t s)
{
    if (n == 0) return;
    unsigned b = grid_for(n, 256);
    if (b > 1024) b = 1024;
    k_node_counts<<<b, 256, 0, s>>>(c, n, cnt, level_hist);
}

void launch_emit_nodes(const uint64_t* skeys, const int8_t* c, const uint32_t* pre, int64_t n,
                       uint8_t* level, uint32_t* first, uint32_t* count, uint32_t* next, uint8_t* octant,
                       hipStream_t s)
{
    if (n == 0) return;
    k_emit<<<grid_for(n, 256), 256, 0, s>>>(skeys, c, pre, n, level, first, count, next, octant);
}

void launch_count_children(const uint8_t* level, const uint32_t* count, const uint32_t* next, int64_t nn,
                           uint32_t* nchild, hipStream_t s)
{
    if (nn == 0) return;
    k_count_children<<<grid_for(nn, 256), 256, 0, s>>>(level, count, next, nn, nchild);
}

void launch_bfs_order(const uint8_t* level, int64_t nn, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                      void* sort_temp, uint32_t* bfs, uint32_t** bfs_to_pre, hipStream_t s)
{
    if (nn == 0) return;
    k_level_keys<<<grid_for(nn, 256), 256, 0, s>>>(level, nn, k0, v0);
    uint64_t* ko;
    radix_sort_pairs(k0, v0, k1, v1, nn, 8, sort_temp, s, &ko, bfs_to_pre);
    k_bfs_scatter<<<grid_for(nn, 256), 256, 0, s>>>(*bfs_to_pre, nn, bfs);
}

}  // namespace tc
