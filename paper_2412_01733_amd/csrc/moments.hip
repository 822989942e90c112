// Upward pass: monopole moments of every node (TreeCode description of
// section 2: a distant cell acts as its total mass at its centre of mass).
//
// One launch per level, deepest first, so a parent reads finished children.
// Everything is FP64 with no FMA contraction, summed in a fixed order
// (particles in key order inside a leaf, children in octant order), so the
// result does not depend on scheduling:
//   leaf of one particle:  M = m_j, X = x_j exactly;
//   otherwise:             M = sum M_c, X = (sum M_c X_c) / M,
//                          X = the cell centre when M = 0.
// The same launch writes the node's walk record in group order.
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

__global__ __launch_bounds__(256) void k_moments_level(
    int l, uint32_t cnt, const uint32_t* __restrict__ list, const uint32_t* __restrict__ first,
    const uint32_t* __restrict__ count, const uint32_t* __restrict__ next,
    const uint32_t* __restrict__ nchild, const uint32_t* __restrict__ cs,
    const uint32_t* __restrict__ gidx, const uint64_t* __restrict__ skeys,
    const double* __restrict__ sx, const double* __restrict__ sy, const double* __restrict__ sz,
    const double* __restrict__ sm, const Geom* __restrict__ g, double* __restrict__ nm,
    double* __restrict__ nx, WalkNode* __restrict__ wn)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += stride) {
        const uint32_t p = list[t];
        const uint32_t b = first[p], c = count[p], nc = nchild[p];
        double M = 0.0, X[3];
        bool centre = false;
        if (nc == 0) {
            if (c == 1) {
                M = sm[b];
                X[0] = sx[b];
                X[1] = sy[b];
                X[2] = sz[b];
            } else {
                double S0 = 0.0, S1 = 0.0, S2 = 0.0;
                for (uint32_t j = b; j < b + c; ++j) {
                    const double mj = sm[j];
                    M += mj;
                    S0 += mj * sx[j];
                    S1 += mj * sy[j];
                    S2 += mj * sz[j];
                }
                if (M == 0.0) centre = true;
                else {
                    X[0] = S0 / M;
                    X[1] = S1 / M;
                    X[2] = S2 / M;
                }
            }
        } else {
            double S0 = 0.0, S1 = 0.0, S2 = 0.0;
            uint32_t ch = p + 1;
            for (uint32_t k = 0; k < nc; ++k) {
                const double mc = nm[ch];
                M += mc;
                S0 += mc * nx[3 * (int64_t)ch + 0];
                S1 += mc * nx[3 * (int64_t)ch + 1];
                S2 += mc * nx[3 * (int64_t)ch + 2];
                ch = next[ch];
            }
            if (M == 0.0) centre = true;
            else {
                X[0] = S0 / M;
                X[1] = S1 / M;
                X[2] = S2 / M;
            }
        }
        if (centre) cell_centre(skeys[b], l, g, X);
        nm[p] = M;
        nx[3 * (int64_t)p + 0] = X[0];
        nx[3 * (int64_t)p + 1] = X[1];
        nx[3 * (int64_t)p + 2] = X[2];
        WalkNode r;
        r.x = X[0];
        r.y = X[1];
        r.z = X[2];
        r.m = M;
        r.first = b;
        r.count = c;
        r.child = nc ? 1u + cs[p] : 0u;
        r.meta = nc | ((uint32_t)l << 8) | (nc == 0 ? (1u << 16) : 0u);
        wn[gidx[p]] = r;
    }
}

}  // namespace

void launch_moments(const uint32_t* first, const uint32_t* count, const uint32_t* next,
                    const uint32_t* nchild, const uint32_t* cs, const uint32_t* gidx,
                    const uint32_t* level_off_host, const uint32_t* list, const uint64_t* skeys,
                    const double* sx, const double* sy, const double* sz, const double* sm,
                    const Geom* geom, double* nm, double* nx, WalkNode* wn, hipStream_t s)
{
    for (int l = kMaxLevel; l >= 0; --l) {
        uint32_t cnt = level_off_host[l + 1] - level_off_host[l];
        if (cnt == 0) continue;
        unsigned blocks = (cnt + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        k_moments_level<<<blocks, 256, 0, s>>>(l, cnt, list + level_off_host[l], first, count, next, nchild,
                                               cs, gidx, skeys, sx, sy, sz, sm, geom, nm, nx, wn);
    }
}

}  // namespace tc
