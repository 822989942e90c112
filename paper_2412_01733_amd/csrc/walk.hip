// The Barnes-Hut walk: accelerations and potentials of Eq.(1) with the
// opening rule of the TreeCode description (section 2).
//
// Layout of the work.  One wavefront serves 64 consecutive targets of the
// target order, the particles along the Hilbert curve (spatially compact; see
// order.hip).  It walks the union of the 64 lanes' open sets
// depth first: a stack in LDS holds groups of sibling nodes together with the
// 64-bit mask of lanes that opened their parent.  Popping a group stages its
// <= 8 children into LDS (one lane per child); every active lane then applies
// the exact per-particle rule to each child:
//   - the node contains the target           -> open (never accepted);
//   - |X - x|^2 > (s_l / theta)^2            -> accept: one monopole term;
//   - otherwise                              -> open.
// A ballot of the opening lanes decides whether the child's own group is
// pushed.  A one-particle leaf gives the same term whether accepted or
// opened, so it is taken directly (self excluded); a multi-particle leaf
// (several particles sharing a level-21 cell) that is opened contributes its
// particles one by one.  The interaction sets are therefore exactly those of
// the per-particle algorithm; only the summation order differs.
//
// Precision.  F32C: node and target coordinates enter as FP32 offsets from a
// per-wave FP64 anchor (the first target of the wave), formed in FP64 once
// per staged node, so differences stay small and accurate; interactions are
// FP32 (hardware reciprocal square root); each group's partial sums are added
// into per-lane Kahan-compensated totals.  F64: absolute FP64 coordinates,
// FP64 reciprocal square root refined by one third-order correction, plain FP64
// sums.  Both walks also reduce sum_i m_i a_i and sum_i m_i |a_i| in FP64,
// one partial per wave, for the momentum diagnostic.
//
// The adjoint walk (tc_forces_backward) is the same kernel with ADJ = true:
// it re-walks the tree with the same decisions and differentiates every
// term, the tree membership and the interaction sets held fixed.
#include <type_traits>

#include "tc_internal.h"

namespace tc {
namespace {

constexpr int kWalkWaves = 4;
constexpr int kWalkThreads = 64 * kWalkWaves;
constexpr uint32_t kXcdRun = 64;  // consecutive blocks one XCD takes at a time
// A step of the walk takes up to kBatchGroups sibling groups off the stack and
// stages all their children at once, 8 lanes per group.
constexpr int kBatchGroups = 6;
constexpr int kBatchGroupsF64 = 4;  // the FP64 walk's 64-byte staged records (7 waves per SIMD)
// Stack bound.  Taking one group and pushing the groups of its opened
// children (at most 8) grows the stack by at most 7 per level below the
// group, so a depth-first run that starts at height S never exceeds
// S + 7 * 20 + 1 (groups lie at levels 1..21).  A step takes ng > 1 groups
// only while sp + 7 ng <= kStackBatch, which leaves it at height
// <= kStackBatch; single-group steps from there stay below
// kStackBatch + 141 <= kStack.  A push beyond the stack therefore cannot
// happen; it would be refused and flagged (status bit 0).
constexpr int kStackDfs = 7 * 20 + 1;
// 248 entries: the F32C walk's 4-wave block (stack, 48 staged children) takes
// 20 192 bytes and fits 8 to a CU's LDS (allocated in 512-byte granules).
constexpr int kStackMulti = 248;
// The FP64 walk's 64-byte staged records leave less room: with 256 entries its
// 4-wave block (22 272 bytes) fits 7 to a CU, with 272 only 6.
constexpr int kStackMultiF64 = 256;
// The adjoint walk keeps its gradients in LDS as well; it takes one group per
// step and a depth-first stack (<= 141 groups), which keeps 7 waves per SIMD.
constexpr int kStackSingle = 160;
static_assert(kStackSingle >= kStackDfs, "depth-first stack bound");
// Stored-list records are staged in LDS and written out this many at a time.
constexpr uint32_t kListBuf = 32;
// The adjoint replays stored records this many at a time.
constexpr uint32_t kReplayChunk = 32;


// What a child needs on the hot path, staged once per group in LDS.
struct __align__(16) Hot32 {
    float x, y, z, m;              // FP32 offsets from the wave anchor, mass
    uint32_t first, count, child;
    float tau;                     // opening threshold (s_l/theta)^2; -1 for a one-particle leaf
};

// A replayed record with its node's data staged as for the walk.
template <typename R>
struct RecHot {
    R x, y, z, m;
    uint32_t node, kind, mlo, mhi;
};

struct __align__(16) Hot64 {
    double x, y, z, m;
    double tau;
    uint32_t first, count, child, pad;
};

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float uni_r(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ inline double uni_r(double v)
{
    const long long b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b), hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// 1/sqrt(x) in FP64: with the hardware estimate y (relative error below
// 2^-24, measured) and r = 1 - x y^2, the exact value is y (1 - r)^(-1/2);
// its series truncated after the quadratic term, y (1 + r/2 + 3 r^2/8), leaves
// an error of order r^3 ~ 2^-72, below FP64 rounding (measured maximum 1.25
// ulp, the same as two Newton-Raphson steps, with 5 operations instead of 8).
__device__ inline double rsqrt64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double r = fma(-x * y, y, 1.0);
    return fma(y * r, fma(0.375, r, 0.5), y);
}

__device__ inline float rsqrt_any(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsqrt_any(double x) { return rsqrt64(x); }

__device__ inline void kahan_add(float& s, float& c, float v)
{
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

template <typename R>
__device__ inline R wave_sum(R v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Adjoint of one term (mass mu at offset (dx,dy,dz) from the target,
// q = d^2 + eps^2) for dL/da = (gx,gy,gz), dL/dphi = h.  With
// T = q^-3/2 I - 3 q^-5/2 Delta Delta^T the source receives
//   dL/dy  = G mu (T g + q^-3/2 Delta h)   (the target receives the negative),
//   dL/dmu = G (Delta.g q^-3/2 - h q^-1/2).
// Both are linear in (g, h): the caller passes G g and G h.
template <typename R>
__device__ inline void adj_term(R dx, R dy, R dz, R q, R mu, R gx, R gy, R gz, R h, R& sx, R& sy, R& sz, R& sm)
{
    const R ri = rsqrt_any(q);
    const R ri2 = ri * ri;
    const R ri3 = ri2 * ri;
    const R dg = fma(dx, gx, fma(dy, gy, dz * gz));
    const R c1 = mu * ri3;
    const R c2 = c1 * fma((R)-3 * ri2, dg, h);
    sx = fma(c1, gx, c2 * dx);
    sy = fma(c1, gy, c2 * dy);
    sz = fma(c1, gz, c2 * dz);
    sm = fma(dg, ri3, -h * ri);
}

// Sum over the wave of four values; the result is uniform.
template <typename R>
__device__ inline void wave_sum4(R& a0, R& a1, R& a2, R& a3)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o, 64);
        a1 += __shfl_xor(a1, o, 64);
        a2 += __shfl_xor(a2, o, 64);
        a3 += __shfl_xor(a3, o, 64);
    }
}

// Sum over each 16-lane row of the wave (DPP: xor 1, xor 2, half-row
// mirror, row mirror); afterwards every lane holds its row's sum.
__device__ inline float dpp_f(float v, int ctrl)
{
    switch (ctrl) {  // the control word must be a constant
    case 0: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
    case 1: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
    case 2: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
    default: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, false));
    }
}

__device__ inline double dpp_d(double v, int ctrl)
{
    const long long b = __double_as_longlong(v);
    int lo = (int)(b & 0xFFFFFFFF), hi = (int)(b >> 32);
    switch (ctrl) {
    case 0: lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false); hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false); break;
    case 1: lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false); hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false); break;
    case 2: lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false); hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false); break;
    default: lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false); hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false); break;
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename R>
__device__ inline R row_sum(R v)
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if constexpr (sizeof(R) == 8) v += dpp_d(v, c);
        else v += dpp_f(v, c);
    }
    return v;
}

__device__ inline void add4(double* dst, double v0, double v1, double v2, double v3)
{
    unsafeAtomicAdd(dst + 0, v0);
    unsafeAtomicAdd(dst + 1, v1);
    unsafeAtomicAdd(dst + 2, v2);
    unsafeAtomicAdd(dst + 3, v3);
}

// ADJ = false: accelerations and potentials; with STORE it also records, per
// wave and in visit order, every (node, accepting lanes) pair and every
// multi-particle leaf opened with its lanes.  ADJ = true: the adjoint walk
// with identical decisions and arithmetic, which writes the target-side
// gradient per particle and accumulates the source-side gradients per node
// (and per particle for opened multi-particle leaves) with FP64 atomics after
// a wave reduction.  It replays the wave's stored records when there are
// valid ones and re-walks the tree otherwise.
// The walk is bound by latency at full occupancy, so the timed forward walks
// are held to 64 VGPRs (8 waves per SIMD); both need the request.
template <bool F64, bool COUNT, bool ADJ, bool STORE>
__global__ __launch_bounds__(kWalkThreads) __attribute__((amdgpu_waves_per_eu((!COUNT && !ADJ && !STORE) ? 8 : 1)))
void k_walk(WalkArgs a)
{
    static_assert(!(ADJ && (COUNT || STORE)), "the adjoint walk neither counts nor stores");
    // the straight run over decided accepts: the forward walks (the adjoint and
    // the storing walk act per node with wave-wide steps, and take every child
    // through the general path)
    constexpr bool FAST = !ADJ && !STORE;
    using R = typename std::conditional<F64, double, float>::type;
    using Hot = typename std::conditional<F64, Hot64, Hot32>::type;
    // groups per step and the stack they need
    constexpr int kGroups = ADJ ? 1 : (F64 ? kBatchGroupsF64 : kBatchGroups);
    constexpr int kStack = kGroups == 1 ? kStackSingle : (F64 ? kStackMultiF64 : kStackMulti);
    constexpr int kStackBatch = kStack - kStackDfs - 7;
    // the stack of pending sibling groups: first node, child count, lanes that opened the parent
    // (several groups per step: three arrays, 13 bytes an entry, so that the deeper stack
    // fits beside the staging slots; one group per step: one 16-byte record an entry)
    constexpr int kStackSoa = kGroups > 1 ? kStack : 1;
    __shared__ uint32_t stk_gs[kWalkWaves][kStackSoa];
    __shared__ uint8_t stk_nc[kWalkWaves][kStackSoa];
    __shared__ uint64_t stk_m[kWalkWaves][kStackSoa];
    __shared__ uint4 stk1[kWalkWaves][kGroups == 1 ? kStack : 1];
    // staged children of the groups of one step: slot 8 j + k holds child k of group j
    __shared__ Hot stg[kWalkWaves][8 * kGroups];
    __shared__ uint32_t stg_meta[kWalkWaves][8 * kGroups];
    __shared__ uint4 popped[kWalkWaves][kGroups];  // the step's groups: first node, count, mask
    // single-group walks: opening thresholds by meta_tau_index (tau0 4^-l at level l, -1 for a
    // one-particle leaf), one table per wave filled with exact power-of-two scalings
    __shared__ R taut[kGroups == 1 ? kWalkWaves : 1][64];
    // adjoint, source side: FP64 walk - per pending node, the 4 row partials of
    // (dL/dX, dL/dM); FP32 walk - per pending node, every lane's 4 values
    constexpr int kSrcBatch = F64 ? 8 : 2;
    __shared__ R rowp[(ADJ && F64) ? kWalkWaves : 1][8][4][4];
    __shared__ float sval[(ADJ && !F64) ? kWalkWaves : 1][2][4][64];
    __shared__ uint32_t rnode[ADJ ? kWalkWaves : 1][8];          // node of each pending slot
    __shared__ uint4 lbuf[STORE ? kWalkWaves : 1][kListBuf];
    R tau0;
    if constexpr (F64) tau0 = a.tau0_64;
    else tau0 = a.tau0_32;

    // FP64 walk: the wave index made uniform keeps the per-wave LDS slices in
    // scalar registers, so the kernel fits 64 VGPRs (8 waves per SIMD) unspilled
    const int w = F64 ? uni((int)(threadIdx.x >> 6)) : (int)(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    // Workgroups are dealt to the 8 XCDs round-robin.  Dealing runs of
    // kXcdRun consecutive blocks instead (a bijection on whole rounds of 8
    // runs, the identity on the tail) keeps each XCD's L2 on compact regions
    // of space: the walk's HBM traffic falls ~2.3x at the same speed.
    const uint32_t nb = gridDim.x, b = blockIdx.x, full = nb / (8 * kXcdRun) * (8 * kXcdRun);
    const uint32_t i8 = b >> 3;
    const uint32_t lb = b < full ? ((i8 / kXcdRun) * 8 + (b & 7u)) * kXcdRun + i8 % kXcdRun : b;
    const int64_t wave_id = (int64_t)lb * kWalkWaves + w;
    const int64_t base = wave_id * 64;
    if (base >= a.n) return;  // whole wave; no block barrier follows
    if constexpr (kGroups == 1) taut[w][lane] = lane < 32 ? (R)ldexp(tau0, -2 * (int)lane) : (R)-1;
    // this lane's target (sorted position) and the range of sorted positions the
    // wavefront's targets span (a superset of them: only a node overlapping it
    // can hold one of the targets)
    const bool valid = base + lane < a.n;
    const uint32_t first_t = uni(a.order[base]);
    const uint32_t su = valid ? a.order[base + lane] : first_t;
    uint32_t smin = valid ? su : 0xFFFFFFFFu, smax = valid ? su : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        smin = min(smin, (uint32_t)__shfl_xor((int)smin, o, 64));
        smax = max(smax, (uint32_t)__shfl_xor((int)smax, o, 64));
    }
    const uint32_t wave_lo = uni(smin), wave_end = uni(smax) + 1u;

    const Particle anchor = a.sp[first_t];
    const double Ax = anchor.x, Ay = anchor.y, Az = anchor.z;
    const Particle self = a.sp[su];
    const double xs = self.x, ys = self.y, zs = self.z;
    R px, py, pz;
    if constexpr (F64) {
        px = xs; py = ys; pz = zs;
    } else {
        px = (float)(xs - Ax); py = (float)(ys - Ay); pz = (float)(zs - Az);
    }
    const R eps2 = (R)a.eps2;
    const R Gc = (R)a.G;
    R gxl = 0, gyl = 0, gzl = 0, hl = 0;  // adjoint: G dL/da and G dL/dphi of this lane's target
    if constexpr (ADJ) {
        if (valid) {
            const uint32_t i = a.perm[su];
            const R* ga = (const R*)a.g_acc;
            gxl = Gc * ga[3 * (int64_t)i + 0];
            gyl = Gc * ga[3 * (int64_t)i + 1];
            gzl = Gc * ga[3 * (int64_t)i + 2];
            if (a.g_pot) hl = Gc * ((const R*)a.g_pot)[i];
        }
    }

    // running totals: F32C keeps (sum, compensation) pairs fed by plain partial sums
    R tx = 0, ty = 0, tz = 0, tp = 0;
    float cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;
    R bx = 0, by = 0, bz = 0, bp = 0;
    uint32_t nint = 0;
    // counting walk: wave-level node evaluations and how they were decided
    uint64_t vis_nodes = 0, vis_lanes = 0, vis_groups = 0, vis_noacc = 0, vis_allacc = 0, vis_boxopen = 0,
             vis_boxacc = 0, vis_steps = 0, vis_single = 0, vis_ovl = 0, vis_slow_acc_ovl = 0;
    int max_sp = 0;
    // The bounding box [bn, bx] of the wavefront's targets (the same offsets the
    // lanes use).  Rounding is monotone, so for a node at X every lane's
    // |fl(X - p)| lies between the box's fl-gap and its fl-far side per axis, and
    // the lane's d^2 (the same fused operations) between the box's two d^2:
    // a node whose near d^2 exceeds the threshold is far from every lane, one
    // whose far d^2 does not is near to every lane, with no margin needed.
    R bnx = valid ? px : (R)INFINITY, bny = valid ? py : (R)INFINITY, bnz = valid ? pz : (R)INFINITY;
    R bxx = valid ? px : (R)-INFINITY, bxy = valid ? py : (R)-INFINITY, bxz = valid ? pz : (R)-INFINITY;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        bnx = fmin(bnx, __shfl_xor(bnx, o, 64)); bny = fmin(bny, __shfl_xor(bny, o, 64));
        bnz = fmin(bnz, __shfl_xor(bnz, o, 64)); bxx = fmax(bxx, __shfl_xor(bxx, o, 64));
        bxy = fmax(bxy, __shfl_xor(bxy, o, 64)); bxz = fmax(bxz, __shfl_xor(bxz, o, 64));
    }
    bnx = uni_r(bnx); bny = uni_r(bny); bnz = uni_r(bnz);
    bxx = uni_r(bxx); bxy = uni_r(bxy); bxz = uni_r(bxz);

    int sp = 0, since_fold = 0;
    bool stack_over = false, corrupt = false;

    // The terms of an opened leaf's particles f .. f+cnt-1 for the lanes in om,
    // the target itself excluded.
    // Particles that share a level-21 cell can sit far closer together than
    // FP32 offsets from the wave's anchor resolve, so their separation is
    // formed in FP64 from this lane's own position (read again here: the leaf
    // is rare, and keeping it in registers would cost the walk occupancy).
    auto leaf_terms = [&](const uint32_t f, const uint32_t cnt, const uint64_t om) {
        const bool lane_open = (om >> lane) & 1ull;
        double mx = xs, my = ys, mz = zs;
        if constexpr (!F64) {
            // a volatile read stays here, on this rare path: hoisted out of the
            // walk loop, the position would occupy registers the whole walk
            const volatile double* me = &a.sp[su].x;
            mx = me[0]; my = me[1]; mz = me[2];
        }
        for (uint32_t j = f; j < f + cnt; ++j) {
            const Particle pj = a.sp[j];
            const double xj = pj.x, yj = pj.y, zj = pj.z;
            const R mj = (R)pj.m;
            R sx0 = 0, sy0 = 0, sz0 = 0, sm0 = 0;
            if (lane_open && j != su) {
                const R ex = (R)(xj - mx), ey = (R)(yj - my), ez = (R)(zj - mz);
                const R q = fma(ex, ex, fma(ey, ey, ez * ez)) + eps2;
                if constexpr (!ADJ) {
                    const R ri = rsqrt_any(q);
                    const R mr = mj * ri;
                    const R mr3 = mr * (ri * ri);
                    bx = fma(mr3, ex, bx);
                    by = fma(mr3, ey, by);
                    bz = fma(mr3, ez, bz);
                    bp -= mr;
                } else {
                    adj_term(ex, ey, ez, q, mj, gxl, gyl, gzl, hl, sx0, sy0, sz0, sm0);
                    bx -= sx0;
                    by -= sy0;
                    bz -= sz0;
                }
                if constexpr (COUNT) ++nint;
            }
            if constexpr (ADJ) {
                wave_sum4(sx0, sy0, sz0, sm0);
                if (lane == 0) add4(a.part_grad + 4 * (int64_t)j, sx0, sy0, sz0, sm0);
            }
        }
    };

    // Adjoint, source side.  The per-lane values of up to kSrcBatch accepted
    // nodes wait in LDS; a flush reduces each (node, component) over the wave
    // in a fixed order and adds it to node_grad with one FP64 atomic.
    int nsrc = 0;
    auto src_flush = [&]() {
        if (nsrc == 0) return;
        wave_sync();
        if constexpr (F64) {
            // lane = 4 k + component; the four 16-lane row partials added in FP64
            const uint32_t k = lane >> 2, c = lane & 3;
            if (k < (uint32_t)nsrc) {
                const double v = (double)rowp[w][k][0][c] + (double)rowp[w][k][1][c] +
                                 (double)rowp[w][k][2][c] + (double)rowp[w][k][3][c];
                unsafeAtomicAdd(a.node_grad + 4 * (int64_t)rnode[w][k] + c, v);
            }
        } else {
            // lane = 32 k + 8 component + eighth: 8 values each, then the eighths
            // (quad swaps and the half-row mirror sum each aligned group of 8 lanes)
            const uint32_t k = lane >> 5, c = (lane >> 3) & 3, e8 = lane & 7;
            const float4* v4 = reinterpret_cast<const float4*>(&sval[w][k][c][8 * e8]);
            const float4 v0 = v4[0], v1 = v4[1];
            float t = ((v0.x + v0.y) + (v0.z + v0.w)) + ((v1.x + v1.y) + (v1.z + v1.w));
            t += dpp_f(t, 0);
            t += dpp_f(t, 1);
            t += dpp_f(t, 2);
            if (e8 == 0 && k < (uint32_t)nsrc) unsafeAtomicAdd(a.node_grad + 4 * (int64_t)rnode[w][k] + c, (double)t);
        }
        wave_sync();
        nsrc = 0;
    };
    auto src_put = [&](const uint32_t node, R sx0, R sy0, R sz0, R sm0) {
        if constexpr (F64) {
            sx0 = row_sum(sx0);
            sy0 = row_sum(sy0);
            sz0 = row_sum(sz0);
            sm0 = row_sum(sm0);
            if ((lane & 15) == 0) {
                R* rp = &rowp[w][nsrc][lane >> 4][0];
                rp[0] = sx0; rp[1] = sy0; rp[2] = sz0; rp[3] = sm0;
            }
        } else {
            sval[w][nsrc][0][lane] = sx0;
            sval[w][nsrc][1][lane] = sy0;
            sval[w][nsrc][2][lane] = sz0;
            sval[w][nsrc][3][lane] = sm0;
        }
        if (lane == 0) rnode[w][nsrc] = node;
        if (++nsrc == kSrcBatch) src_flush();
    };

    auto fold = [&]() {
        if constexpr (F64) {
            tx += bx; ty += by; tz += bz; tp += bp;
        } else {
            kahan_add(tx, cx, bx);
            kahan_add(ty, cy, by);
            kahan_add(tz, cz, bz);
            kahan_add(tp, cp, bp);
        }
        bx = 0; by = 0; bz = 0; bp = 0;
    };

    // Storing walk: records go through a small LDS buffer to the wave's slice.
    uint32_t nl = 0, lw = 0;
    bool list_over = false;
    auto list_flush = [&]() {
        wave_sync();
        if (lw + nl <= a.list_cap) {
            if (lane < nl) a.lists[wave_id * (int64_t)a.list_cap + lw + lane] = lbuf[w][lane];
        } else {
            list_over = true;
        }
        lw += nl;
        nl = 0;
        wave_sync();
    };
    auto list_put = [&](const uint32_t node, const uint32_t kind, const uint64_t m) {
        if (lane == 0) lbuf[w][nl] = make_uint4(node, kind, (uint32_t)m, (uint32_t)(m >> 32));
        nl = uni(nl + 1);
        if (nl == kListBuf) list_flush();
    };

    bool replayed = false;
    if constexpr (ADJ) {
        // a wave that replays its records never walks, so the replay chunk lives in
        // the wave's (then unused) stack slice
        static_assert(kGroups == 1 && sizeof(RecHot<R>) * kReplayChunk <= sizeof(uint4) * kStack,
                      "replay chunk within the stack slice");
        RecHot<R>* const rb = reinterpret_cast<RecHot<R>*>(&stk1[w][0]);
        if (a.lists) {
            const uint32_t len = uni(a.list_len[wave_id]);
            if (len != kListInvalid && len <= a.list_cap) {
                replayed = true;
                const uint4* L = a.lists + wave_id * (int64_t)a.list_cap;
                for (uint32_t c0 = 0; c0 < len; c0 += kReplayChunk) {
                    // one lane per record: fetch it and stage its node as the walk does
                    const uint32_t cn = uni(len - c0 < kReplayChunk ? len - c0 : kReplayChunk);
                    if (lane < cn) {
                        const uint4 rec = L[c0 + lane];
                        const WalkNode& nd = a.nodes[rec.x];
                        RecHot<R> e;
                        if constexpr (F64) {
                            e.x = nd.x; e.y = nd.y; e.z = nd.z; e.m = nd.m;
                        } else {
                            e.x = (float)(nd.x - Ax); e.y = (float)(nd.y - Ay); e.z = (float)(nd.z - Az);
                            e.m = (float)nd.m;
                        }
                        e.node = rec.x; e.kind = rec.y; e.mlo = rec.z; e.mhi = rec.w;
                        rb[lane] = e;
                    }
                    wave_sync();
                    for (uint32_t r = 0; r < cn; ++r) {
                        const RecHot<R> e = rb[r];  // one broadcast read
                        const uint32_t node = uni(e.node), kind = uni(e.kind);
                        const uint64_t m = ((uint64_t)uni(e.mhi) << 32) | uni(e.mlo);
                        if (kind == 0) {
                            const R dx = e.x - px, dy = e.y - py, dz = e.z - pz;
                            const R d2 = fma(dx, dx, fma(dy, dy, dz * dz));
                            R sx0 = 0, sy0 = 0, sz0 = 0, sm0 = 0;
                            if (__builtin_amdgcn_inverse_ballot_w64(m)) {
                                adj_term(dx, dy, dz, d2 + eps2, e.m, gxl, gyl, gzl, hl, sx0, sy0, sz0, sm0);
                                bx -= sx0;
                                by -= sy0;
                                bz -= sz0;
                            }
                            src_put(node, sx0, sy0, sz0, sm0);
                        } else {
                            leaf_terms(uni(a.nodes[node].first), uni(a.nodes[node].count), m);
                        }
                    }
                    wave_sync();  // the next chunk overwrites the buffer
                    fold();
                }
                src_flush();
            }
        }
    }

    const uint64_t vmask = __ballot(valid);
    if (!replayed) {
        const uint32_t rmeta = uni(a.nodes[0].meta);
        const uint32_t rchild = uni(a.nodes[0].child);
        if (!meta_leaf(rmeta)) {
            if (lane == 0) {
                if constexpr (kGroups == 1) {
                    stk1[w][0] = make_uint4(rchild, meta_nchild(rmeta), (uint32_t)vmask, (uint32_t)(vmask >> 32));
                } else {
                    stk_gs[w][0] = rchild;
                    stk_nc[w][0] = (uint8_t)meta_nchild(rmeta);
                    stk_m[w][0] = vmask;
                }
            }
            sp = 1;
        }
    }
    wave_sync();

    while (sp > 0) {
        // take ng groups off the top; lanes 8 j .. 8 j + 7 stage the children of group j
        // as many groups as the stack bound allows: after the step sp <= kStackBatch
        const int ng = kGroups > 1 ? max(1, min(min(sp, kGroups), (kStackBatch - sp) / 7)) : 1;
        if constexpr (COUNT) {
            vis_steps += 1;
            vis_single += ng == 1;
        }
        const int gj = (int)(lane >> 3), gk = (int)(lane & 7);
        uint32_t e_gs = 0, e_nc = 0;
        uint4 e1 = make_uint4(0, 0, 0, 0);  // single-group walks: the popped record (uniform)
        if constexpr (kGroups == 1) {
            e1 = stk1[w][sp - 1];
            e_gs = e1.x;
            e_nc = e1.y;
        } else if (gj < ng) {
            const int slot = sp - 1 - gj;
            e_gs = stk_gs[w][slot];
            e_nc = stk_nc[w][slot];
            if (gk == 0) {
                const uint64_t e_m = stk_m[w][slot];
                popped[w][gj] = make_uint4(e_gs, e_nc, (uint32_t)e_m, (uint32_t)(e_m >> 32));
            }
        }
        sp = uni(sp - ng);
        bool ovl = false;  // may the child contain one of this wave's targets?
        bool bad = false, all_far = false, all_near = false;
        if (gj < ng && gk < (int)e_nc) {
            bad = e_nc > 8u;
            const WalkNode nd = a.nodes[e_gs + (uint32_t)gk];
            ovl = nd.first < wave_end && nd.first + nd.count > wave_lo;
            Hot h;
            if constexpr (F64) {
                h.x = nd.x; h.y = nd.y; h.z = nd.z; h.m = nd.m;
            } else {
                h.x = (float)(nd.x - Ax); h.y = (float)(nd.y - Ay); h.z = (float)(nd.z - Az);
                h.m = (float)nd.m;
            }
            // opening threshold tau0 4^-l (an exact power-of-two scaling); a
            // one-particle leaf is always taken (-1)
            if constexpr (kGroups == 1) h.tau = taut[w][meta_tau_index(nd.meta)];
            else h.tau = meta_single(nd.meta) ? (R)-1 : (R)ldexp(tau0, -2 * (int)meta_level(nd.meta));
            h.first = nd.first;
            h.count = nd.count;
            h.child = nd.child;
            stg[w][lane] = h;
            stg_meta[w][lane] = nd.meta;
            // the box test (see bn, bx): decided for every target of the wavefront;
            // paid once per step, it pays off when a step stages several groups
            if constexpr (kGroups > 1) {
                const R gx = fmax(fmax(bnx - h.x, h.x - bxx), (R)0), fx = fmax(fabs(h.x - bnx), fabs(h.x - bxx));
                const R gy = fmax(fmax(bny - h.y, h.y - bxy), (R)0), fy = fmax(fabs(h.y - bny), fabs(h.y - bxy));
                const R gz = fmax(fmax(bnz - h.z, h.z - bxz), (R)0), fz = fmax(fabs(h.z - bnz), fabs(h.z - bxz));
                all_far = !ovl && fma(gx, gx, fma(gy, gy, gz * gz)) > h.tau;
                all_near = !(fma(fx, fx, fma(fy, fy, fz * fz)) > h.tau);
            }
        }
        const uint64_t ovl_m = __ballot(ovl);
        const uint64_t far_all = __ballot(all_far), near_all = __ballot(all_near);
        if (__ballot(bad)) corrupt = true;
        wave_sync();

        for (int j = 0; j < ng; ++j) {
            uint32_t gs, nc;
            uint64_t mask;
            if constexpr (kGroups == 1) {
                gs = uni(e1.x);
                nc = min(uni(e1.y), 8u);
                mask = ((uint64_t)uni(e1.w) << 32) | uni(e1.z);
            } else {
                const uint4 e = popped[w][j];
                gs = uni(e.x);
                nc = min(uni(e.y), 8u);
                mask = ((uint64_t)uni(e.w) << 32) | uni(e.z);
            }
            if constexpr (COUNT) {
                vis_nodes += nc;
                vis_lanes += (uint64_t)nc * (uint64_t)__popcll(mask);
                vis_groups += 1;
                vis_ovl += __popc((uint32_t)(ovl_m >> (8 * j)) & ((1u << nc) - 1u));
            }
            const uint32_t all = (1u << nc) - 1u;
            // decided accepted by every target, and not holding any (the forward
            // walks take these in one straight run with the active lanes enabled;
            // the others take them through the general path without the tests)
            const uint32_t far_bits = (uint32_t)(far_all >> (8 * j)) & all;
            uint32_t fast = FAST ? far_bits : 0u;
            // decided opened by every active target
            uint32_t opened = (uint32_t)(near_all >> (8 * j)) & all & ~fast;
            const uint32_t slow = all & ~fast & ~opened;
            if constexpr (COUNT) {
                vis_allacc += __popc(fast);
                vis_boxacc += __popc(fast);
                vis_noacc += __popc(opened);
                vis_boxopen += __popc(opened);
            }
            const Hot* g8 = &stg[w][8 * j];
            if (fast && __builtin_amdgcn_inverse_ballot_w64(mask)) {
                // no opening test here, so the softening enters the distance chain
                if constexpr (!F64) {
                    // each slot's position and mass are read while the slot before it is
                    // evaluated, so the LDS latency is not paid child by child (the FP64
                    // walk's 32-byte reads gain nothing from it)
                    float4 hc = *reinterpret_cast<const float4*>(&g8[0]);
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const float4 hn = k < 7 ? *reinterpret_cast<const float4*>(&g8[k + 1]) : hc;
                        if ((fast >> k) & 1u) {
                            const R dx = hc.x - px, dy = hc.y - py, dz = hc.z - pz;
                            const R ri = rsqrt_any(fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2))));
                            const R mr = hc.w * ri;
                            const R mr3 = mr * (ri * ri);
                            bx = fma(mr3, dx, bx);
                            by = fma(mr3, dy, by);
                            bz = fma(mr3, dz, bz);
                            bp -= mr;
                            if constexpr (COUNT) ++nint;
                        }
                        hc = hn;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        if ((fast >> k) & 1u) {
                            const Hot h = g8[k];
                            const R dx = h.x - px, dy = h.y - py, dz = h.z - pz;
                            const R ri = rsqrt_any(fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2))));
                            const R mr = h.m * ri;
                            const R mr3 = mr * (ri * ri);
                            bx = fma(mr3, dx, bx);
                            by = fma(mr3, dy, by);
                            bz = fma(mr3, dz, bz);
                            bp -= mr;
                            if constexpr (COUNT) ++nint;
                        }
                    }
                }
            }
            // an opened child: its own group is pushed, or an opened leaf's particles
            // are taken one by one, the target itself excluded (for a one-particle
            // leaf only the lane holding that particle gets here, and it contributes nothing)
            auto open_child = [&](const uint32_t slot, const uint32_t k, const uint64_t om, const uint32_t child_v,
                                  const uint32_t first_v, const uint32_t count_v) {
                const uint32_t meta = uni(stg_meta[w][slot]);
                if (!meta_leaf(meta)) {
                    const uint32_t child = uni(child_v);
                    if (sp < kStack) {
                        if (lane == 0) {
                            if constexpr (kGroups == 1) {
                                stk1[w][sp] = make_uint4(child, meta_nchild(meta), (uint32_t)om, (uint32_t)(om >> 32));
                            } else {
                                stk_gs[w][sp] = child;
                                stk_nc[w][sp] = (uint8_t)meta_nchild(meta);
                                stk_m[w][sp] = om;
                            }
                        }
                        sp = uni(sp + 1);
                        if constexpr (COUNT) max_sp = max(max_sp, sp);
                    } else {
                        stack_over = true;
                    }
                } else {
                    const uint32_t f = uni(first_v), cnt = uni(count_v);
                    if (cnt > 1) {
                        leaf_terms(f, cnt, om);
                        if constexpr (STORE) list_put(gs + k, 1u, om);
                    }
                }
            };
            while (opened) {
                const uint32_t k = __builtin_ctz(opened);
                opened &= opened - 1u;
                const uint32_t slot = 8u * (uint32_t)j + k;
                open_child(slot, k, mask, stg[w][slot].child, stg[w][slot].first, stg[w][slot].count);
            }
            // the general path: per-lane opening test, containment where the child may hold a target
            auto general = [&](const uint32_t k) {
                const uint32_t slot = 8u * (uint32_t)j + k;
                const Hot h = g8[k];  // one broadcast read of the whole record
                const R dx = h.x - px, dy = h.y - py, dz = h.z - pz;
                const R d2 = fma(dx, dx, fma(dy, dy, dz * dz));
                // lane masks combined on the scalar unit: accepted = active, not containing, far enough
                uint64_t am = mask;
                if (FAST || !((far_bits >> k) & 1u)) {
                    uint64_t in_m = 0;
                    if ((ovl_m >> slot) & 1ull) in_m = __ballot((su - h.first) < h.count);
                    am &= __ballot(d2 > h.tau) & ~in_m;
                }
                if constexpr (COUNT) {
                    vis_noacc += am == 0;
                    vis_allacc += am == mask;
                    vis_slow_acc_ovl += am == mask && ((ovl_m >> slot) & 1ull);
                }
                if constexpr (!ADJ) {
                    if (__builtin_amdgcn_inverse_ballot_w64(am)) {
                        const R ri = rsqrt_any(d2 + eps2);
                        const R mr = h.m * ri;
                        const R mr3 = mr * (ri * ri);
                        bx = fma(mr3, dx, bx);
                        by = fma(mr3, dy, by);
                        bz = fma(mr3, dz, bz);
                        bp -= mr;
                        if constexpr (COUNT) ++nint;
                    }
                    if constexpr (STORE) {
                        if (am) list_put(gs + k, 0u, am);
                    }
                } else {
                    if (am) {
                        R sx0 = 0, sy0 = 0, sz0 = 0, sm0 = 0;
                        if (__builtin_amdgcn_inverse_ballot_w64(am)) {
                            adj_term(dx, dy, dz, d2 + eps2, h.m, gxl, gyl, gzl, hl, sx0, sy0, sz0, sm0);
                            bx -= sx0;
                            by -= sy0;
                            bz -= sz0;
                        }
                        src_put(gs + k, sx0, sy0, sz0, sm0);
                    }
                }
                const uint64_t om = mask & ~am;
                if (om) open_child(slot, k, om, h.child, h.first, h.count);
            };
            if constexpr (kGroups == 1) {
                // one group per step (the adjoint): unrolled over the children,
                // records read at fixed offsets
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if ((uint32_t)k >= nc) break;
                    if ((slow >> k) & 1u) general((uint32_t)k);
                }
            } else {
                for (uint32_t rest = slow; rest;) {
                    const uint32_t k = __builtin_ctz(rest);
                    rest &= rest - 1u;
                    general(k);
                }
            }
        }
        wave_sync();  // the next step restages the slots and rereads the stack
        // a step adds up to ~30 terms per lane to the plain partial sums; they go
        // into the compensated totals every second step (every fourth for
        // single-group steps)
        if (++since_fold == (kGroups == 1 ? 4 : 2) || sp == 0) {
            since_fold = 0;
            fold();
        }
    }
    if (lane == 0 && (stack_over || corrupt)) atomicOr(a.status, (stack_over ? 1u : 0u) | (corrupt ? 2u : 0u));
    if constexpr (ADJ) src_flush();
    if constexpr (STORE) {
        list_flush();
        if (lane == 0) a.list_len[wave_id] = list_over ? kListInvalid : lw;
    }

    if constexpr (ADJ) {
        if (valid) {
            double* tg = a.target_grad + 3 * (int64_t)su;
            if constexpr (F64) {
                tg[0] = tx; tg[1] = ty; tg[2] = tz;
            } else {
                tg[0] = (double)(tx - cx); tg[1] = (double)(ty - cy); tg[2] = (double)(tz - cz);
            }
        }
        return;
    }
    R ox, oy, oz, op;
    if constexpr (F64) {
        ox = tx; oy = ty; oz = tz; op = tp;
    } else {
        ox = tx - cx; oy = ty - cy; oz = tz - cz; op = tp - cp;
    }
    ox *= Gc; oy *= Gc; oz *= Gc; op *= Gc;

    double dm[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
        const uint32_t i = a.perm[su];
        R* acc = (R*)a.acc;
        acc[3 * (int64_t)i + 0] = ox;
        acc[3 * (int64_t)i + 1] = oy;
        acc[3 * (int64_t)i + 2] = oz;
        if (a.pot) ((R*)a.pot)[i] = op;
        if constexpr (COUNT) a.counts[su] = nint;
        const double m = self.m;
        const double ex = (double)ox, ey = (double)oy, ez = (double)oz;
        dm[0] = m * ex;
        dm[1] = m * ey;
        dm[2] = m * ez;
        dm[3] = m * sqrt(ex * ex + ey * ey + ez * ez);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) dm[k] = wave_sum(dm[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.diag[4 * wave_id + k] = dm[k];
        if constexpr (COUNT) {
            atomicAdd(&a.visits[0], (unsigned long long)vis_nodes);
            atomicAdd(&a.visits[1], (unsigned long long)vis_lanes);
            atomicAdd(&a.visits[2], (unsigned long long)vis_groups);
            atomicAdd(&a.visits[3], (unsigned long long)vis_noacc);
            atomicAdd(&a.visits[4], (unsigned long long)vis_allacc);
            atomicAdd(&a.visits[5], (unsigned long long)vis_boxopen);
            atomicAdd(&a.visits[6], (unsigned long long)vis_boxacc);
            atomicMax(&a.visits[7], (unsigned long long)max_sp);
            atomicAdd(&a.visits[8], (unsigned long long)vis_steps);
            atomicAdd(&a.visits[9], (unsigned long long)vis_single);
            atomicAdd(&a.visits[10], (unsigned long long)vis_ovl);
            atomicAdd(&a.visits[11], (unsigned long long)vis_slow_acc_ovl);
        }
    }
}

}  // namespace

int64_t walk_waves(int64_t n) { return (n + 63) / 64; }

template <bool F64>
void launch_walk_t(const WalkArgs& a, unsigned blocks, bool count, bool store, hipStream_t s)
{
    if (count) {
        if (store) k_walk<F64, true, false, true><<<blocks, kWalkThreads, 0, s>>>(a);
        else k_walk<F64, true, false, false><<<blocks, kWalkThreads, 0, s>>>(a);
    } else {
        if (store) k_walk<F64, false, false, true><<<blocks, kWalkThreads, 0, s>>>(a);
        else k_walk<F64, false, false, false><<<blocks, kWalkThreads, 0, s>>>(a);
    }
}

void launch_walk(const WalkArgs& a, tc_walk mode, bool count, bool store, hipStream_t s)
{
    if (a.n == 0) return;
    const int64_t waves = walk_waves(a.n);
    const unsigned blocks = (unsigned)((waves + kWalkWaves - 1) / kWalkWaves);
    if (mode == TC_WALK_F64) launch_walk_t<true>(a, blocks, count, store, s);
    else launch_walk_t<false>(a, blocks, count, store, s);
}

void launch_walk_adjoint(const WalkArgs& a, tc_walk mode, hipStream_t s)
{
    if (a.n == 0) return;
    const int64_t waves = walk_waves(a.n);
    const unsigned blocks = (unsigned)((waves + kWalkWaves - 1) / kWalkWaves);
    if (mode == TC_WALK_F64) k_walk<true, false, true, false><<<blocks, kWalkThreads, 0, s>>>(a);
    else k_walk<false, false, true, false><<<blocks, kWalkThreads, 0, s>>>(a);
}

}  // namespace tc
