// Top-down half of the adjoint: node gradients to particle gradients.
//
// The walk's source-side gradients per node, dL/dX_n and dL/dM_n, reach the
// particles through the monopole moments M_n = sum_j m_j and
// X_n = sum_j m_j x_j / M_n (tree membership held fixed):
//   dL/dm_j += dL/dM_n + (dL/dX_n) . (x_j - X_n) / M_n,   dL/dx_j += (m_j / M_n) dL/dX_n.
// With u_n = (dL/dX_n) / M_n and c_n = dL/dM_n - u_n . X_n this is
//   dL/dm_j += c_n + u_n . x_j,   dL/dx_j += m_j u_n,
// summed over every node holding j, i.e. along the root-to-leaf path: level
// by level, root first, carrying the running sums (U, C) down (one launch
// per populous level, one single-workgroup launch per run of small levels).  A
// node of zero mass sits at its fixed cell centre, so u_n = 0 for it.  At a
// leaf, every particle adds its target-side gradient and any direct-term
// gradient and is written in the caller's order.  All FP64.
#include "tc_internal.h"

namespace tc {
namespace {

#define ADJ_ARGS                                                                                            \
    const WalkNode *__restrict__ wn, const uint32_t *__restrict__ parent, const double *__restrict__ node_grad, \
        double *__restrict__ uc, const Particle *__restrict__ sp, const uint32_t *__restrict__ perm,          \
        const double *__restrict__ target_grad, const double *__restrict__ part_grad, void *__restrict__ g_pos, \
        void *__restrict__ g_mass
#define ADJ_PASS wn, parent, node_grad, uc, sp, perm, target_grad, part_grad, g_pos, g_mass

template <bool OUT64>
__device__ inline void adjoint_node(int64_t b, bool root, ADJ_ARGS)
{
    const WalkNode nd = wn[b];
    const double* gn = node_grad + 4 * b;
    double u0 = 0.0, u1 = 0.0, u2 = 0.0;
    if (nd.m != 0.0) {
        u0 = gn[0] / nd.m;
        u1 = gn[1] / nd.m;
        u2 = gn[2] / nd.m;
    }
    double c = gn[3] - (u0 * nd.x + u1 * nd.y + u2 * nd.z);
    if (!root) {
        const double* up = uc + 4 * (int64_t)parent[b];
        u0 += up[0];
        u1 += up[1];
        u2 += up[2];
        c += up[3];
    }
    double* mine = uc + 4 * b;
    mine[0] = u0;
    mine[1] = u1;
    mine[2] = u2;
    mine[3] = c;
    if (meta_leaf(nd.meta)) {
        for (uint32_t j = nd.first; j < nd.first + nd.count; ++j) {
            const Particle q = sp[j];
            const double mj = q.m;
            const double* tg = target_grad + 3 * (int64_t)j;
            const double* pg = part_grad + 4 * (int64_t)j;
            const double gx = tg[0] + pg[0] + mj * u0;
            const double gy = tg[1] + pg[1] + mj * u1;
            const double gz = tg[2] + pg[2] + mj * u2;
            const double gm = pg[3] + c + (u0 * q.x + u1 * q.y + u2 * q.z);
            const int64_t i = perm[j];
            if constexpr (OUT64) {
                if (g_pos) {
                    double* o = (double*)g_pos + 3 * i;
                    o[0] = gx; o[1] = gy; o[2] = gz;
                }
                if (g_mass) ((double*)g_mass)[i] = gm;
            } else {
                if (g_pos) {
                    float* o = (float*)g_pos + 3 * i;
                    o[0] = (float)gx; o[1] = (float)gy; o[2] = (float)gz;
                }
                if (g_mass) ((float*)g_mass)[i] = (float)gm;
            }
        }
    }
}

// One level with many nodes: one thread per node.
template <bool OUT64>
__global__ __launch_bounds__(256) void k_adjoint_down(uint32_t b0, uint32_t b1, bool root, ADJ_ARGS)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)b0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < (int64_t)b1; b += stride)
        adjoint_node<OUT64>(b, root, ADJ_PASS);
}

// A run of consecutive small levels [llo, lhi], root side first, in one
// workgroup; a barrier separates the levels.
template <bool OUT64>
__global__ __launch_bounds__(kSmallLevelThreads) void k_adjoint_small(int llo, int lhi, LevelOffsets off, ADJ_ARGS)
{
    for (int l = llo; l <= lhi; ++l) {
        for (int64_t b = (int64_t)off.off[l] + threadIdx.x; b < (int64_t)off.off[l + 1]; b += blockDim.x)
            adjoint_node<OUT64>(b, l == 0, ADJ_PASS);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_zero_f64(double* __restrict__ p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

}  // namespace

void launch_fill_f64_zero(double* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    k_zero_f64<<<(unsigned)b, 256, 0, s>>>(p, n);
}

void launch_adjoint_down(const uint32_t* level_off_host, const WalkNode* wn, const uint32_t* parent,
                         const double* node_grad, double* uc, const Particle* sp, const uint32_t* perm,
                         const double* target_grad, const double* part_grad,
                         void* g_pos, void* g_mass, bool out_f64, hipStream_t s)
{
    LevelOffsets off;
    for (int l = 0; l <= kLevels; ++l) off.off[l] = level_off_host[l];
    int l = 0;
    while (l <= kMaxLevel) {
        if (off.size(l) <= kSmallLevel) {
            int hi = l;
            while (hi < kMaxLevel && off.size(hi + 1) <= kSmallLevel) ++hi;
            if (off.off[hi + 1] > off.off[l]) {
                if (out_f64) k_adjoint_small<true><<<1, kSmallLevelThreads, 0, s>>>(l, hi, off, ADJ_PASS);
                else k_adjoint_small<false><<<1, kSmallLevelThreads, 0, s>>>(l, hi, off, ADJ_PASS);
            }
            l = hi + 1;
            continue;
        }
        int64_t blocks = ((int64_t)off.size(l) + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        if (out_f64)
            k_adjoint_down<true><<<(unsigned)blocks, 256, 0, s>>>(off.off[l], off.off[l + 1], l == 0, ADJ_PASS);
        else
            k_adjoint_down<false><<<(unsigned)blocks, 256, 0, s>>>(off.off[l], off.off[l + 1], l == 0, ADJ_PASS);
        ++l;
    }
}

}  // namespace tc
