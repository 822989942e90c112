// Upward pass: monopole moments of every node (TreeCode description of
// section 2: a distant cell acts as its total mass at its centre of mass).
//
// Level by level, deepest first, over that level's contiguous range of the
// breadth-first node array, so a parent reads finished children, which are
// consecutive records: one launch per populous level, one single-workgroup
// launch per run of small levels.
// Everything is FP64 with no FMA contraction, summed in a fixed order
// (particles in key order inside a leaf, children in octant order), so the
// result does not depend on scheduling:
//   leaf of one particle:  M = m_j, X = x_j exactly;
//   otherwise:             M = sum M_c, X = (sum M_c X_c) / M,
//                          X = the cell centre when M = 0.
// The same pass writes the node's whole walk record.
#include "tc_internal.h"

namespace tc {
namespace {

__device__ inline uint32_t compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v | (v >> 2)) & 0x10C30C30C30C30C3ull;
    v = (v | (v >> 4)) & 0x100F00F00F00F00Full;
    v = (v | (v >> 8)) & 0x001F0000FF0000FFull;
    v = (v | (v >> 16)) & 0x001F00000000FFFFull;
    v = (v | (v >> 32)) & 0x00000000001FFFFFull;
    return (uint32_t)v;
}

__device__ inline void cell_centre(uint64_t key, int level, const Geom* g, double X[3])
{
    uint32_t q[3] = {compact3(key >> 2), compact3(key >> 1), compact3(key)};
    const uint32_t span = 1u << (kMaxLevel - level);
    for (int k = 0; k < 3; ++k) {
        uint32_t corner = q[k] & ~(span - 1u);
        X[k] = g->lo[k] + ((double)corner + 0.5 * (double)span) * g->h;
    }
}

// One node, at breadth-first position b (pre-order index p).
__device__ inline void moments_node(int64_t b, int l, const uint32_t* __restrict__ bfs_to_pre,
                                    const uint32_t* __restrict__ bfs, const uint32_t* __restrict__ first,
                                    const uint32_t* __restrict__ count, const uint32_t* __restrict__ nchild,
                                    const uint64_t* __restrict__ skeys, const uint8_t* __restrict__ octant,
                                    const Particle* __restrict__ sp,
                                    const Geom* __restrict__ g, WalkNode* __restrict__ wn,
                                    uint32_t* __restrict__ parent, uint4* __restrict__ topo)
{
    const uint32_t p = bfs_to_pre[b];
    const uint32_t f = first[p], c = count[p], nc = nchild[p];
    double M = 0.0, X[3];
    bool centre = false;
    uint32_t child = 0;
    if (nc == 0) {
        if (c == 1) {
            const Particle q = sp[f];
            M = q.m;
            X[0] = q.x;
            X[1] = q.y;
            X[2] = q.z;
        } else {
            double S0 = 0.0, S1 = 0.0, S2 = 0.0;
            for (uint32_t j = f; j < f + c; ++j) {
                const Particle q = sp[j];
                M += q.m;
                S0 += q.m * q.x;
                S1 += q.m * q.y;
                S2 += q.m * q.z;
            }
            if (M == 0.0) centre = true;
            else {
                X[0] = S0 / M;
                X[1] = S1 / M;
                X[2] = S2 / M;
            }
        }
    } else {
        child = bfs[p + 1];  // the first child follows its parent in pre-order
        double S0 = 0.0, S1 = 0.0, S2 = 0.0;
        for (uint32_t k = 0; k < nc; ++k) {
            parent[child + k] = (uint32_t)b;
            const double2 xy = *reinterpret_cast<const double2*>(&wn[child + k].x);
            const double2 zm = *reinterpret_cast<const double2*>(&wn[child + k].z);
            const double mc = zm.y;
            M += mc;
            S0 += mc * xy.x;
            S1 += mc * xy.y;
            S2 += mc * zm.x;
        }
        if (M == 0.0) centre = true;
        else {
            X[0] = S0 / M;
            X[1] = S1 / M;
            X[2] = S2 / M;
        }
    }
    if (centre) cell_centre(skeys[f], l, g, X);
    const bool single = nc == 0 && c == 1;
    const uint32_t oc = octant[p];
    const uint32_t meta = nc | ((uint32_t)l << 8) | (single ? (1u << 13) : 0u) | (nc == 0 ? (1u << 16) : 0u) |
                          (single ? (1u << 17) : 0u) | (oc << 18);
    uint4* o = reinterpret_cast<uint4*>(wn + b);
    o[0] = make_uint4(__double2loint(X[0]), __double2hiint(X[0]), __double2loint(X[1]), __double2hiint(X[1]));
    o[1] = make_uint4(__double2loint(X[2]), __double2hiint(X[2]), __double2loint(M), __double2hiint(M));
    o[2] = make_uint4(f, c, child, meta);
    topo[b] = make_uint4(f, c, child, meta);  // the same topology half, densely, for the target-order pass
}

#define MOM_ARGS                                                                                                  \
    const uint32_t *__restrict__ bfs_to_pre, const uint32_t *__restrict__ bfs, const uint32_t *__restrict__ first, \
        const uint32_t *__restrict__ count, const uint32_t *__restrict__ nchild, const uint64_t *__restrict__ skeys, \
        const uint8_t *__restrict__ octant, const Particle *__restrict__ sp, const Geom *__restrict__ g, WalkNode *__restrict__ wn,                  \
        uint32_t *__restrict__ parent, uint4 *__restrict__ topo
#define MOM_PASS bfs_to_pre, bfs, first, count, nchild, skeys, octant, sp, g, wn, parent, topo

// One level with many nodes: one thread per node.
__global__ __launch_bounds__(256) void k_moments_level(int l, uint32_t b0, uint32_t b1, MOM_ARGS)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)b0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < (int64_t)b1; b += stride)
        moments_node(b, l, MOM_PASS);
}

// A run of consecutive small levels [llo, lhi], deepest first, in one
// workgroup: a barrier separates the levels (the waves of one workgroup share
// a CU and its L1, so the barrier's workgroup-scope fence makes the finished
// level visible).
__global__ __launch_bounds__(kSmallLevelThreads) void k_moments_small(int lhi, int llo, LevelOffsets off, MOM_ARGS)
{
    for (int l = lhi; l >= llo; --l) {
        for (int64_t b = (int64_t)off.off[l] + threadIdx.x; b < (int64_t)off.off[l + 1]; b += blockDim.x)
            moments_node(b, l, MOM_PASS);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_export_moments(const WalkNode* __restrict__ wn,
                                                        const uint32_t* __restrict__ bfs, int64_t nn,
                                                        double* __restrict__ com, double* __restrict__ mass)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nn) return;
    const WalkNode r = wn[bfs[p]];
    if (com) {
        com[3 * p + 0] = r.x;
        com[3 * p + 1] = r.y;
        com[3 * p + 2] = r.z;
    }
    if (mass) mass[p] = r.m;
}

}  // namespace

void launch_moments(const uint32_t* level_off_host, const uint32_t* bfs_to_pre, const uint32_t* bfs,
                    const uint32_t* first, const uint32_t* count, const uint32_t* nchild, const uint64_t* skeys,
                    const uint8_t* octant, const Particle* sp, const Geom* g, WalkNode* wn, uint32_t* parent,
                    uint4* topo, hipStream_t s)
{
    LevelOffsets off;
    for (int l = 0; l <= kLevels; ++l) off.off[l] = level_off_host[l];
    int l = kMaxLevel;
    while (l >= 0) {
        if (off.size(l) <= kSmallLevel) {
            int lo = l;
            while (lo > 0 && off.size(lo - 1) <= kSmallLevel) --lo;
            if (off.off[l + 1] > off.off[lo]) k_moments_small<<<1, kSmallLevelThreads, 0, s>>>(l, lo, off, MOM_PASS);
            l = lo - 1;
            continue;
        }
        int64_t blocks = ((int64_t)off.size(l) + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        k_moments_level<<<(unsigned)blocks, 256, 0, s>>>(l, off.off[l], off.off[l + 1], MOM_PASS);
        --l;
    }
}

void launch_export_moments(const WalkNode* wn, const uint32_t* bfs, int64_t nn, double* com, double* mass,
                           hipStream_t s)
{
    if (nn == 0) return;
    k_export_moments<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(wn, bfs, nn, com, mass);
}

}  // namespace tc
