// The walk's target order: the particles along the Hilbert curve.
//
// The walk gives each wavefront 64 consecutive targets of this order.  The
// tree, its keys and its node table stay in Morton (key) order; only the
// grouping of targets into wavefronts changes.  A Hilbert segment of 64
// particles is spatially more compact than a Morton segment, which jumps
// between distant cells at the Z-curve's seams, so the 64 lanes open fewer
// nodes between them.  No result depends on the order: every target's
// interaction set and terms are its own.
//
// Every octree cell is a contiguous range of the Hilbert order, just as it is
// of the key order, so the order follows from the tree top-down (reading the
// dense breadth-first topology records {first, count, child, meta}): a node's
// particles start at its offset; its children follow each other in the order
// of their Hilbert digits at their level (siblings share all higher digits);
// a leaf lays out its particles in key order.  Level by level, root first
// (one launch per populous level, one single-workgroup launch per run of
// small levels).
//
// Hilbert digits.  The index is that of the transposition algorithm of
// J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707, 381
// (2004), read out with the first transposed coordinate highest in each
// triple.  That algorithm visits the bit levels top down; at each level it
// reflects or exchanges the lower bits of the coordinates according to the
// current level's bits, and its Gray-code step makes each output digit depend
// on the current level and on the parity of the higher levels only.  The
// reflections and exchanges accumulated above a level therefore form a signed
// permutation of the three axes, which together with that parity is the state
// a cell hands to its children:
//   X_a   = raw bit of axis perm[a], xor flip[a]          (a = 0, 1, 2)
//   digit = (X_0, X_0^X_1, X_0^X_1^X_2), each xor parity  (first bit highest)
//   then, for i = 0, 1, 2 in turn: if X_i, flip[0] ^= 1, else exchange
//   (perm, flip) entries 0 and i; parity ^= X_0^X_1^X_2.
// State word: perm[a] in bits 2a..2a+1, flip[a] in bit 6 + a, parity in bit 9.
#include "tc_internal.h"

namespace tc {
namespace {

constexpr uint32_t kRootState = 0u | (1u << 2) | (2u << 4);  // identity permutation, no flips, even parity

// Hilbert digit of octant d (key digit: x bit 2, y bit 1, z bit 0) under
// state st, and the state the child in that octant inherits.
__device__ inline uint32_t hilbert_step(uint32_t st, uint32_t d, uint32_t* child_state)
{
    uint32_t perm[3], flip[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        perm[a] = (st >> (2 * a)) & 3u;
        flip[a] = (st >> (6 + a)) & 1u;
    }
    const uint32_t par = (st >> 9) & 1u;
    uint32_t X[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) X[a] = ((d >> (2 - perm[a])) & 1u) ^ flip[a];
    const uint32_t g0 = X[0], g1 = X[0] ^ X[1], g2 = g1 ^ X[2];
    const uint32_t digit = ((g0 ^ par) << 2) | ((g1 ^ par) << 1) | (g2 ^ par);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (X[i]) {
            flip[0] ^= 1u;
        } else if (i > 0) {
            const uint32_t tp = perm[0], tf = flip[0];
            perm[0] = perm[i];
            flip[0] = flip[i];
            perm[i] = tp;
            flip[i] = tf;
        }
    }
    uint32_t ns = (par ^ g2) << 9;
#pragma unroll
    for (int a = 0; a < 3; ++a) ns |= (perm[a] << (2 * a)) | (flip[a] << (6 + a));
    *child_state = ns;
    return digit;
}

// Node b (breadth-first index): a leaf writes its particles' places in the
// order; an internal node gives each child its offset and Hilbert state.
// nord[b] = {offset, state} was written by the parent (the root starts at
// offset 0 in the root state).
__device__ inline void order_node(int64_t b, const uint4* __restrict__ topo, uint2* __restrict__ nord,
                                  uint32_t* __restrict__ order)
{
    const uint4 rec = topo[b];  // first, count, child, meta
    const uint2 me = b == 0 ? make_uint2(0u, kRootState) : nord[b];
    if (meta_leaf(rec.w)) {
        for (uint32_t j = 0; j < rec.y; ++j) order[me.x + j] = rec.x + j;
        return;
    }
    const uint32_t nc = meta_nchild(rec.w) < 8u ? meta_nchild(rec.w) : 8u;
    // fixed-size, fully unrolled, so that the arrays stay in registers; an
    // absent child counts 0 and sorts last (digit 8)
    uint32_t cnt[8], dig[8], cst[8];
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
        cnt[k] = 0u;
        dig[k] = 8u;
        cst[k] = 0u;
        if (k < nc) {
            const uint4 c = topo[rec.z + k];
            cnt[k] = c.y;
            dig[k] = hilbert_step(me.y, meta_octant(c.w), &cst[k]);
        }
    }
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
        if (k < nc) {
            uint32_t o = me.x;
#pragma unroll
            for (uint32_t j = 0; j < 8; ++j)
                if (dig[j] < dig[k]) o += cnt[j];
            nord[rec.z + k] = make_uint2(o, cst[k]);
        }
    }
}

__global__ __launch_bounds__(256) void k_order_level(uint32_t b0, uint32_t b1, const uint4* __restrict__ topo,
                                                     uint2* __restrict__ nord, uint32_t* __restrict__ order)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)b0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < (int64_t)b1; b += stride)
        order_node(b, topo, nord, order);
}

// A run of consecutive small levels [llo, lhi], root side first, in one
// workgroup; a barrier separates the levels.
__global__ __launch_bounds__(kSmallLevelThreads) void k_order_small(int llo, int lhi, LevelOffsets off,
                                                                   const uint4* __restrict__ topo,
                                                                   uint2* __restrict__ nord,
                                                                   uint32_t* __restrict__ order)
{
    for (int l = llo; l <= lhi; ++l) {
        for (int64_t b = (int64_t)off.off[l] + threadIdx.x; b < (int64_t)off.off[l + 1]; b += blockDim.x)
            order_node(b, topo, nord, order);
        __syncthreads();
    }
}

}  // namespace

void launch_target_order(const uint32_t* level_off_host, const uint4* topo, uint2* nord, uint32_t* order,
                         hipStream_t s)
{
    LevelOffsets off;
    for (int l = 0; l <= kLevels; ++l) off.off[l] = level_off_host[l];
    int l = 0;
    while (l <= kMaxLevel) {
        if (off.size(l) <= kSmallLevel) {
            int hi = l;
            while (hi < kMaxLevel && off.size(hi + 1) <= kSmallLevel) ++hi;
            if (off.off[hi + 1] > off.off[l]) k_order_small<<<1, kSmallLevelThreads, 0, s>>>(l, hi, off, topo, nord, order);
            l = hi + 1;
            continue;
        }
        int64_t blocks = ((int64_t)off.size(l) + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        k_order_level<<<(unsigned)blocks, 256, 0, s>>>(off.off[l], off.off[l + 1], topo, nord, order);
        ++l;
    }
}

}  // namespace tc
