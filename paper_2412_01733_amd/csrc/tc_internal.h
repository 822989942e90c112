// Internal definitions shared by the HIP translation units of libtreecode.
// Nothing here is part of the C ABI (include/treecode.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/treecode.h"

namespace tc {

constexpr int kMaxLevel = 21;          // 21 bits per axis, 63-bit keys
constexpr int kLevels = kMaxLevel + 1;  // levels 0..21
constexpr uint32_t kQMax = (1u << 21) - 1;

// Root cube and input checks produced on the device by the bounds pass.
struct Geom {
    double lo[3];
    double L;        // root side, a power of two
    double scale;    // 2^21 / L (exact)
    double h;        // L 2^-21, the finest cell side
    int32_t log2L;
    uint32_t bad;    // bit 0: non-finite position, bit 1: negative / non-finite mass
    uint32_t nnodes; // filled by the build (node count read back to the host)
    uint32_t pad;
};

// One node as the walk reads it.  Nodes are stored in breadth-first order:
// sorted by (level, first), so the root is at 0, every level is contiguous
// and the children of every internal node are consecutive in octant order.
struct __align__(16) WalkNode {
    double x, y, z;   // centre of mass
    double m;         // total mass
    uint32_t first;   // sorted index of the first particle
    uint32_t count;   // particles in the node
    uint32_t child;   // group index of the first child (internal nodes)
    uint32_t meta;    // bits 0-3 nchild, bits 8-12 level, bit 16 leaf, bit 17 one-particle leaf,
                      // bits 18-20 the node's octant in its parent (key digit at its level)
};
static_assert(sizeof(WalkNode) == 48, "WalkNode layout");

// A particle in key order: position and mass, FP64 (one 32-byte record, so
// that a leaf or a target reads one aligned line).
struct __align__(32) Particle {
    double x, y, z, m;
};

// Breadth-first offsets of the levels (level l occupies [off[l], off[l+1])),
// passed by value to the level-batched kernels.  Levels with at most
// kSmallLevel nodes are processed in runs by a single workgroup.
struct LevelOffsets {
    uint32_t off[kLevels + 1];
    __host__ __device__ uint32_t size(int l) const { return off[l + 1] - off[l]; }
};
constexpr uint32_t kSmallLevel = 4096;
constexpr int kSmallLevelThreads = 1024;

__host__ __device__ inline uint32_t meta_nchild(uint32_t m) { return m & 0xFu; }
__host__ __device__ inline uint32_t meta_level(uint32_t m) { return (m >> 8) & 0x1Fu; }
__host__ __device__ inline bool meta_leaf(uint32_t m) { return (m >> 16) & 1u; }
__host__ __device__ inline bool meta_single(uint32_t m) { return (m >> 17) & 1u; }
__host__ __device__ inline uint32_t meta_octant(uint32_t m) { return (m >> 18) & 7u; }
// level + 32 * single (bit 13 repeats the single flag): the walk's threshold table index
__host__ __device__ inline uint32_t meta_tau_index(uint32_t m) { return (m >> 8) & 0x3Fu; }

// ---------------------------------------------------------------------------
// launch wrappers (each defined next to its kernels)
// ---------------------------------------------------------------------------

// keys.hip
void launch_bounds(const void* pos, const void* mass, int64_t n, tc_dtype dt, double* partials,
                   int nblocks, Geom* geom, hipStream_t s);
int bounds_blocks(int64_t n);
// keys also writes the packed {x, y, z, m} record (record_bytes) that the gather reads
size_t record_bytes(int64_t n, tc_dtype dt);
void launch_keys(const void* pos, const void* mass, int64_t n, tc_dtype dt, const Geom* geom, uint64_t* keys,
                 uint32_t* idx, void* rec, hipStream_t s);
void launch_gather(const void* rec, int64_t n, tc_dtype dt, const uint32_t* perm, Particle* sp, hipStream_t s);

// scan.hip: exclusive scan, out[n] = total (out has n+1 entries)
size_t scan_temp_bytes(int64_t n);
void launch_exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* temp,
                               hipStream_t s);

// sort.hip: stable LSD radix sort of (u64 key, u32 value) pairs over the
// low `bits` key bits.  Result ends in (keys_out, vals_out); the *_alt
// buffers are scratch.
size_t radix_temp_bytes(int64_t n);
void radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                      int64_t n, int bits, void* temp, hipStream_t s, uint64_t** keys_out,
                      uint32_t** vals_out);

// build.hip
void launch_adjacent_levels(const uint64_t* skeys, int64_t n, int8_t* c, hipStream_t s);
// level_hist: [kLevels + 2] = nodes per level, leaves, multi-particle leaves
void launch_node_counts(const int8_t* c, int64_t n, uint32_t* cnt, uint32_t* level_hist, hipStream_t s);
void launch_emit_nodes(const uint64_t* skeys, const int8_t* c, const uint32_t* pre, int64_t n,
                       uint8_t* level, uint32_t* first, uint32_t* count, uint32_t* next, uint8_t* octant,
                       hipStream_t s);
void launch_count_children(const uint8_t* level, const uint32_t* count, const uint32_t* next,
                           int64_t nn, uint32_t* nchild, hipStream_t s);
// Breadth-first order of the pre-order nodes (stable sort by level): writes
// bfs[p] and points *bfs_to_pre at the inverse (inside v0 or v1).
void launch_bfs_order(const uint8_t* level, int64_t nn, uint64_t* k0, uint32_t* v0, uint64_t* k1,
                      uint32_t* v1, void* sort_temp, uint32_t* bfs, uint32_t** bfs_to_pre,
                      hipStream_t s);

// moments.hip: one launch per level over the breadth-first ranges
// [level_off_host[l], level_off_host[l+1]), deepest level first.
void launch_moments(const uint32_t* level_off_host, const uint32_t* bfs_to_pre, const uint32_t* bfs,
                    const uint32_t* first, const uint32_t* count, const uint32_t* nchild, const uint64_t* skeys,
                    const uint8_t* octant, const Particle* sp, const Geom* geom, WalkNode* wn, uint32_t* parent,
                    uint4* topo, hipStream_t s);
// Canonical export: com/mass of pre-order node p from wn[bfs[p]].
void launch_export_moments(const WalkNode* wn, const uint32_t* bfs, int64_t nn, double* com, double* mass,
                           hipStream_t s);

// walk.hip
struct WalkArgs {
    const WalkNode* nodes;
    const Particle* sp;     // particles in key order
    const uint32_t* order;  // [n] targets by wavefront: wavefront w takes order[64 w .. 64 w + 63]
    const uint32_t* perm;
    int64_t n;
    double eps2;
    double G;
    double tau0_64;         // (L / theta)^2, +inf for theta == 0; level l uses tau0 4^-l
    float tau0_32;          // the same rounded to FP32 (scaling by 4^-l stays exact)
    void* acc;              // caller order, FP32 (F32C) or FP64 (F64)
    void* pot;              // may be NULL
    uint32_t* counts;       // sorted order (counting walk only)
    double* diag;           // [waves, 4] partials of sum m a, sum m |a|
    uint32_t* status;       // bit 0: stack overflow (never expected)
    unsigned long long* visits;  // counting walk: [kNumVisitCounters], see tc_stats (node_visits ... max_stack)
    // adjoint walk only
    const void* g_acc;      // dL/da [n,3], caller order, walk precision
    const void* g_pot;      // dL/dphi [n] or NULL
    double* node_grad;      // [nodes, 4] breadth-first: dL/dX (3), dL/dM, accumulated
    double* part_grad;      // [n, 4] sorted order: dL/dx_j (3), dL/dm_j from opened multi-particle leaves
    double* target_grad;    // [n, 3] sorted order: dL/dx_i from the target side
    // stored interaction lists: per wave, in visit order, records {node, kind, lane mask lo, hi};
    // kind 0: the node was accepted by the mask's lanes; kind 1: the multi-particle leaf was
    // opened by them.  Written by a storing forward walk, replayed by the adjoint walk.
    uint4* lists;           // [waves, list_cap], or NULL (adjoint: re-walk)
    uint32_t* list_len;     // [waves]: records of the wave, or kListInvalid if they did not fit
    uint32_t list_cap;      // records per wave
};
// counting walk: node evaluations, active lanes, group pops, evaluations with no
// accepting lane, with every active lane accepting, decided "all open" and "all
// accept" by the per-wave box test, deepest stack (atomic max), steps, steps
// that took a single group, evaluations of nodes whose particle range overlaps
// the wavefront's targets, of those taken by the general path with every
// active lane accepting
constexpr int kNumVisitCounters = 12;
constexpr uint32_t kListCap = 8192;                     // records per wave (128 KiB)
constexpr uint32_t kListInvalid = 0xFFFFFFFFu;
constexpr uint64_t kListMaxBytes = 4ull << 30;          // lists are stored only up to this size
int64_t walk_waves(int64_t n);
void launch_walk(const WalkArgs& a, tc_walk mode, bool count, bool store, hipStream_t s);
void launch_walk_adjoint(const WalkArgs& a, tc_walk mode, hipStream_t s);

// order.hip: the walk's target order (Hilbert order of the particles), from
// the breadth-first topology records {first, count, child, meta} (written
// densely by the upward pass) top-down; nord is node-sized scratch.
void launch_target_order(const uint32_t* level_off_host, const uint4* topo, uint2* nord, uint32_t* order,
                         hipStream_t s);

// adjoint.hip: top-down pass from node gradients to particle gradients.
void launch_adjoint_down(const uint32_t* level_off_host, const WalkNode* wn, const uint32_t* parent,
                         const double* node_grad, double* uc, const Particle* sp, const uint32_t* perm,
                         const double* target_grad,
                         const double* part_grad, void* g_pos, void* g_mass, bool out_f64, hipStream_t s);
void launch_fill_f64_zero(double* p, int64_t n, hipStream_t s);

// integrate.hip: leapfrog pieces and FP64 step diagnostics
void launch_kick_drift(void* pos, void* vel, const void* acc, int64_t n, tc_dtype dt, bool acc64, double tau,
                       hipStream_t s);
void launch_kick(void* vel, const void* acc, int64_t n, tc_dtype dt, bool acc64, double tau, hipStream_t s);
size_t step_diag_temp_bytes();
// out10: kinetic, potential energy, momentum (3), angular momentum (3), total mass, 0
void launch_step_diag(const void* pos, const void* vel, const void* mass, const void* pot, int64_t n, tc_dtype dt,
                      bool pot64, void* temp, double* out10, hipStream_t s);

// diag.hip
size_t diag_temp_bytes(int64_t nwaves);
void launch_diag_final(const double* part, int64_t nwaves, void* temp, double* out4, hipStream_t s);
void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
void launch_sum_counts(const uint32_t* counts, int64_t n, unsigned long long* out, hipStream_t s);
void launch_scatter_counts(const uint32_t* sorted_counts, const uint32_t* perm, int64_t n,
                           uint32_t* out, hipStream_t s);

}  // namespace tc
