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
// The walk wants siblings contiguous, so a second numbering ("group order")
// places the root at 0 and the children of internal node p at
// 1 + (number of children of all internal nodes before p in pre-order).
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

// Node count per first particle, plus a histogram of node levels.
__global__ __launch_bounds__(256) void k_node_counts(const int8_t* __restrict__ c, int64_t n,
                                                     uint32_t* __restrict__ cnt,
                                                     uint32_t* __restrict__ level_hist)
{
    __shared__ uint32_t h[kLevels];
    if (threadIdx.x < kLevels) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) {
        int lo, hi;
        node_range(c, s, lo, hi);
        int k = hi - lo + 1;
        if (k < 0) k = 0;
        cnt[s] = (uint32_t)k;
        for (int l = lo; l <= hi; ++l) atomicAdd(&h[l], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kLevels && h[threadIdx.x]) atomicAdd(&level_hist[threadIdx.x], h[threadIdx.x]);
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
                                              uint32_t* __restrict__ count, uint32_t* __restrict__ next)
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
        first[p] = (uint32_t)s;
        count[p] = (uint32_t)(end - s);
        next[p] = pre[end];
    }
}

__device__ inline bool is_internal(uint8_t level, uint32_t count) { return count >= 2 && level < kMaxLevel; }

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

__global__ __launch_bounds__(256) void k_assign_groups(const uint32_t* __restrict__ next,
                                                       const uint32_t* __restrict__ nchild,
                                                       const uint32_t* __restrict__ cs, int64_t nn,
                                                       uint32_t* __restrict__ gidx,
                                                       uint32_t* __restrict__ parent)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nn) return;
    if (p == 0) {
        gidx[0] = 0;
        parent[0] = 0xFFFFFFFFu;
    }
    const uint32_t nc = nchild[p];
    uint32_t ch = (uint32_t)p + 1;
    const uint32_t base = 1 + cs[p];
    for (uint32_t k = 0; k < nc; ++k) {
        gidx[ch] = base + k;
        parent[ch] = (uint32_t)p;
        ch = next[ch];
    }
}

// Per-level node lists (order inside a level is irrelevant to the results).
__global__ __launch_bounds__(256) void k_level_lists(const uint8_t* __restrict__ level, int64_t nn,
                                                     const uint32_t* __restrict__ off,
                                                     uint32_t* __restrict__ cursor,
                                                     uint32_t* __restrict__ list)
{
    __shared__ uint32_t h[kLevels];
    __shared__ uint32_t hb[kLevels];
    if (threadIdx.x < kLevels) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int l = -1;
    uint32_t r = 0;
    if (p < nn) {
        l = level[p];
        r = atomicAdd(&h[l], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kLevels) hb[threadIdx.x] = h[threadIdx.x] ? atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]) : 0u;
    __syncthreads();
    if (p < nn) list[off[l] + hb[l] + r] = (uint32_t)p;
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
    k_node_counts<<<grid_for(n, 256), 256, 0, s>>>(c, n, cnt, level_hist);
}

void launch_emit_nodes(const uint64_t* skeys, const int8_t* c, const uint32_t* pre, int64_t n,
                       uint8_t* level, uint32_t* first, uint32_t* count, uint32_t* next, hipStream_t s)
{
    if (n == 0) return;
    k_emit<<<grid_for(n, 256), 256, 0, s>>>(skeys, c, pre, n, level, first, count, next);
}

void launch_count_children(const uint8_t* level, const uint32_t* count, const uint32_t* next, int64_t nn,
                           uint32_t* nchild, hipStream_t s)
{
    if (nn == 0) return;
    k_count_children<<<grid_for(nn, 256), 256, 0, s>>>(level, count, next, nn, nchild);
}

void launch_assign_groups(const uint32_t* next, const uint32_t* nchild, const uint32_t* cs, int64_t nn,
                          uint32_t* gidx, uint32_t* parent, hipStream_t s)
{
    if (nn == 0) return;
    k_assign_groups<<<grid_for(nn, 256), 256, 0, s>>>(next, nchild, cs, nn, gidx, parent);
}

void launch_level_lists(const uint8_t* level, int64_t nn, const uint32_t* level_off, uint32_t* cursor,
                        uint32_t* list, hipStream_t s)
{
    if (nn == 0) return;
    k_level_lists<<<grid_for(nn, 256), 256, 0, s>>>(level, nn, level_off, cursor, list);
}

}  // namespace tc
