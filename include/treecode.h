/*
 * treecode.h — C ABI of the MI355X (gfx950) TreeCode gravity library.
 *
 * The library evaluates Plummer-softened Newtonian accelerations and
 * potentials of N particles with the Barnes-Hut TreeCode method, following
 * Kuzmin, Sirotin & Khoperskov (2024):
 *   - Eq.(1): a_i = sum_{j != i} G m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^{3/2};
 *     the matching potential phi_i = -G sum_{j != i} m_j (|r_j - r_i|^2 + eps^2)^{-1/2}.
 *   - Section 2, TreeCode description: octree split into eight octants until a
 *     cell holds at most one particle; a distant cell acts as its total mass at
 *     its centre of mass; theta sets "distant"; theta = 0 is the direct sum.
 *   - Eqs.(2)-(5): kick-drift-kick leapfrog with the forces of Eq.(4) taken
 *     from a tree rebuilt at the drifted positions.
 *
 * Conventions shared by every entry point:
 *   - Every data pointer is DEVICE memory on the current HIP device and is
 *     owned by the caller; the library never frees or keeps caller pointers
 *     beyond the call (the tree handle keeps its own copies).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  All work
 *     is enqueued on it; no hidden streams.  Results are valid once the
 *     stream has been synchronised, except where an entry point says it
 *     blocks.
 *   - Arguments are validated before any launch; on an error nothing is
 *     written to the caller's outputs and a status other than TC_OK is
 *     returned.  tc_last_error() gives a thread-local message.
 *   - Positions are [n,3] row-major (x0 y0 z0 x1 ...), masses [n]; both FP32
 *     or both FP64 (tc_dtype).  0 <= n < 2^31.
 */
#ifndef TREECODE_H
#define TREECODE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TC_OK = 0,
    TC_ERR_INVALID = 1,   /* bad argument (null pointer, n out of range, theta < 0, ...) */
    TC_ERR_NOMEM = 2,     /* the allocator returned NULL */
    TC_ERR_DEVICE = 3,    /* no usable HIP device, or a HIP call failed */
    TC_ERR_STATE = 4,     /* call out of order (e.g. tc_forces before tc_moments) */
    TC_ERR_OVERFLOW = 5,  /* a size limit was exceeded (node count >= 2^32, list budget) */
    TC_ERR_INPUT = 6      /* non-finite position or negative / non-finite mass found on device */
} tc_status;

typedef enum { TC_F32 = 0, TC_F64 = 1 } tc_dtype;

/* Walk precision.  F32C: FP32 interactions on anchor-relative coordinates with
 * Kahan-compensated FP32 accumulation, FP32 outputs.  F64: FP64 throughout,
 * FP64 outputs. */
typedef enum { TC_WALK_F32C = 0, TC_WALK_F64 = 1 } tc_walk;

/* tc_forces flags */
#define TC_COUNT 1u        /* record the interaction count of every target */
/* TC_STORE_LISTS: record, per wavefront of 64 consecutive targets of the
 * target order (tc_tree_target_order), every (node, accepting lanes) pair and every opened multi-particle
 * leaf of the walk, 16 bytes each, for tc_forces_backward to replay instead of
 * re-walking the tree.  At most 8192 records per wavefront; a wavefront whose
 * records do not fit is re-walked by the backward pass.  The lists are kept
 * only while they fit 4 GiB (n up to 2^21); beyond that the flag is accepted
 * and the backward pass re-walks (same result to rounding). */
#define TC_STORE_LISTS 2u

typedef struct tc_tree tc_tree;

/* Device allocator used for every buffer the library owns.  alloc returns
 * NULL on failure; both receive the stream of the call that allocates. */
typedef void* (*tc_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*tc_free_fn)(void* ptr, void* stream, void* ctx);

/* Install the allocator used by handles created afterwards (process-wide).
 * Passing NULL for both restores the default (hipMallocAsync / hipFreeAsync on
 * the call's stream, from the device's default memory pool).  A handle
 * frees a buffer it grows past on the stream of the growing call, and frees
 * everything in tc_tree_free after its enqueued work is done; a stream-ordered
 * allocator (the Python binding installs torch's caching allocator) needs no
 * device synchronisation for either.
 * Errors: TC_ERR_INVALID if exactly one of alloc/free is NULL. */
tc_status tc_set_allocator(tc_alloc_fn alloc, tc_free_fn free_fn, void* ctx);

/* Keys, sort and octree of a particle set (TreeCode description, section 2).
 *   pos  [n,3], mass [n]: device arrays of `dtype`.
 *   *tree: NULL to create a handle, or an existing handle to rebuild in place
 *          (its buffers grow as needed; earlier results are invalidated).
 * The root cube is lo_k = min_i x_ik with side L = the smallest power of two
 * >= the largest extent (1 if all points coincide); 21-bit grid coordinates,
 * 63-bit Morton keys (x highest), stable sort, canonical octree with chain
 * nodes kept and leaves of one particle (several only at level 21).
 * BLOCKS once: the node count is read back to size the node arrays.
 * Errors: TC_ERR_INVALID (null pointers with n > 0, n out of range, bad
 * dtype), TC_ERR_INPUT (non-finite position, negative or non-finite mass),
 * TC_ERR_NOMEM, TC_ERR_OVERFLOW (>= 2^32 nodes), TC_ERR_DEVICE.  At its
 * synchronisation a rebuild also reports the status of the previous walk on
 * the handle (see tc_tree_stats): TC_ERR_OVERFLOW or TC_ERR_DEVICE if that walk
 * was incomplete, in which case the rebuild has not run. */
tc_status tc_build(const void* pos, const void* mass, int64_t n, tc_dtype dtype,
                   void* stream, tc_tree** tree);

/* Upward pass: total mass M and centre of mass X of every node (monopole,
 * TreeCode description of section 2).  One-particle leaf: M = m, X = x
 * verbatim; otherwise M = sum M_c, X = sum(M_c X_c) / M in FP64 with the
 * children in octant order; M = 0 gives X = the cell centre.  Also lays out
 * the walk's target order (see tc_tree_target_order).
 * Errors: TC_ERR_INVALID (null tree), TC_ERR_STATE (no successful tc_build),
 * TC_ERR_NOMEM. */
tc_status tc_moments(tc_tree* tree, void* stream);

/* Accelerations and potentials, Eq.(1), by the Barnes-Hut walk.  For target
 * i, node n (side s = L 2^-level) is accepted as a monopole iff it does not
 * contain i and s < theta |X_n - x_i| (tested as |X_n - x_i|^2 > (s/theta)^2);
 * a rejected leaf contributes its particles j != i directly; theta = 0 never
 * accepts, giving the direct sum.
 *   acc [n,3] (required), pot [n] (may be NULL): device, in the caller's
 *   particle order, FP32 for TC_WALK_F32C and FP64 for TC_WALK_F64.
 *   flags: TC_COUNT, TC_STORE_LISTS.
 * Errors: TC_ERR_INVALID (theta < 0 or not finite, eps < 0 or not finite, G
 * not finite, acc NULL with n > 0, bad mode or flags, theta > 0 with
 * (L/theta)^2 beyond the walk's float range), TC_ERR_STATE (no
 * tc_moments since the last tc_build), TC_ERR_NOMEM, TC_ERR_DEVICE. */
tc_status tc_forces(tc_tree* tree, double theta, double eps, double G, tc_walk mode,
                    uint32_t flags, void* acc, void* pot, void* stream);

/* Adjoint of the last tc_forces with the tree and every interaction set held
 * fixed (node membership frozen, moments still functions of x and m).
 * Given L(acc, pot): g_acc = dL/dacc [n,3], g_pot = dL/dpot [n] (may be NULL),
 * writes g_pos = dL/dx [n,3] and g_mass = dL/dm [n] (either may be NULL), all
 * in the caller's order and in the dtype of the last walk's outputs.
 * Each wavefront of 64 targets replays the records the last tc_forces stored
 * (TC_STORE_LISTS) or, without them, re-walks the tree with the same
 * decisions and arithmetic; the two agree to rounding (summation order).
 * Errors: TC_ERR_INVALID, TC_ERR_STATE (no tc_forces since the last build),
 * TC_ERR_NOMEM, TC_ERR_DEVICE. */
tc_status tc_forces_backward(tc_tree* tree, const void* g_acc, const void* g_pot,
                             void* g_pos, void* g_mass, void* stream);

/* One kick-drift-kick step, Eqs.(2)-(5): v += tau/2 a; x += tau v; rebuild
 * the tree at x and evaluate a (and pot); v += tau/2 a.  pos, vel updated in
 * place; acc holds a^n on entry and a^{n+1} on exit; pot (may be NULL)
 * receives phi^{n+1}.  pos/vel/mass are of `dtype`; acc/pot are of the walk
 * precision (FP32 for F32C, FP64 for F64).  *tree as for tc_build.
 * Blocks once (inside the rebuild).  Errors: as tc_build and tc_forces;
 * arguments are checked before anything is written, but an error raised by
 * the rebuild (TC_ERR_INPUT, TC_ERR_NOMEM, ...) leaves pos and vel at the
 * drifted state of Eqs.(2)-(3). */
tc_status tc_leapfrog_step(tc_tree** tree, void* pos, void* vel, const void* mass,
                           void* acc, void* pot, int64_t n, tc_dtype dtype, double tau,
                           double theta, double eps, double G, tc_walk mode, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * sequence tc_build + tc_moments + tc_forces (flags 0) in one call that
 * allocates nothing.  No handle: every buffer of the build, the moments and
 * the walk comes from one static device array of 128 MiB per GPU (held until
 * the process ends, addressed through hipGetSymbolAddress), and the host side
 * uses static storage.  Results are bitwise those of the three calls above
 * (the same kernels in the same order).
 *   pos [n,3], mass [n] of `dtype`; acc [n,3] (required) and pot [n] (may be
 *   NULL) of the walk precision, caller order.  0 <= n <= 2^18.
 * Blocks once (node count read back), as tc_build.  Every call on a GPU
 * shares that GPU's array, which keeps the last call's contents; calls that
 * overlap on one GPU (from several host threads or on several streams) race
 * and must be serialised by the caller.
 * Errors: as tc_build and tc_forces; TC_ERR_INVALID for n > 2^18, before any
 * launch; TC_ERR_OVERFLOW when the particles' octree needs more than the
 * static array (too many nodes), reported before any node kernel runs and
 * before anything is written to acc or pot. */
tc_status tc_forces_noalloc(const void* pos, const void* mass, int64_t n, tc_dtype dtype, double theta,
                            double eps, double G, tc_walk mode, void* acc, void* pot, void* stream);

/* Sizes, geometry, diagnostics and per-stage timings of a handle. */
typedef struct {
    int64_t n;               /* particles */
    int64_t n_nodes;         /* octree nodes (chain nodes included) */
    int64_t n_leaves;
    int64_t n_multi_leaves;  /* level-21 leaves holding >= 2 particles */
    double lo[3];            /* root cube corner */
    double L;                /* root cube side (a power of two) */
    int32_t log2L;
    int32_t max_level;
    uint32_t state;          /* bit 0 built, bit 1 moments, bit 2 forces */
    uint32_t last_mode;      /* tc_walk of the last tc_forces */
    uint64_t interactions;   /* sum over targets of the interaction count (TC_COUNT), else 0 */
    uint64_t node_visits;    /* TC_COUNT: node evaluations summed over wavefronts (64 targets each) */
    uint64_t lane_visits;    /* TC_COUNT: the same weighted by the lanes active at each evaluation */
    double momentum[3];      /* sum_i m_i a_i of the last tc_forces (FP64) */
    double sum_m_abs_a;      /* sum_i m_i |a_i| (FP64) */
    double kinetic;          /* after the last tc_leapfrog_step (FP64): sum m v^2 / 2 */
    double potential;        /*   sum m phi / 2 (0 if pot was NULL) */
    double lin_momentum[3];  /*   sum m v */
    double ang_momentum[3];  /*   sum m x cross v */
    float stage_ms[8];       /* last timed durations: 0 keys, 1 sort, 2 tree, 3 moments (with the
                                walk's target order),
                                4 walk, 5 diagnostics, 6 backward walk, 7 backward down-pass
                                (-1 if not recorded) */
    uint32_t lists_stored;   /* 1 if the last tc_forces stored interaction lists (TC_STORE_LISTS
                                within the list budget), else 0 */
    uint32_t max_stack;      /* TC_COUNT: deepest traversal stack of any wavefront (groups) */
    uint64_t group_pops;     /* TC_COUNT: sibling groups taken from the stacks, summed over wavefronts */
    uint64_t visits_no_accept;   /* TC_COUNT: node evaluations at which no active lane accepts */
    uint64_t visits_all_accept;  /* TC_COUNT: node evaluations at which every active lane accepts */
    uint64_t visits_box_open;    /* TC_COUNT: evaluations the per-wavefront box test shows every
                                    target must open (the node is nearer than s/theta to the box) */
    uint64_t visits_box_accept;  /* TC_COUNT: evaluations the box test shows every target accepts */
    uint64_t walk_steps;         /* TC_COUNT: traversal steps (each stages one or more sibling groups) */
    uint64_t walk_single_steps;  /* TC_COUNT: steps that staged a single group */
    uint64_t visits_overlap;     /* TC_COUNT: evaluations of nodes whose particle range overlaps the
                                    range of the wavefront's targets (they may hold a target) */
    uint64_t visits_overlap_all_accept;  /* TC_COUNT: of those, evaluations every active lane accepts */
    uint64_t list_bytes;     /* device bytes holding the stored interaction lists of the last
                                tc_forces (16 bytes a record, 8192 records a wavefront), 0 if none */
} tc_stats;

/* Fill *out.  Synchronises `stream` when diagnostics, timings or a walk's
 * status are pending.
 * Errors: TC_ERR_INVALID (null pointer); after filling *out, the status of
 * the walks since the last build: TC_ERR_OVERFLOW if a traversal stack would
 * have overflowed (terms dropped), TC_ERR_DEVICE if a walk met a node with
 * more than 8 children.  Neither can happen for a tree built by tc_build: the
 * traversal stack is sized from the depth bound of the octree. */
tc_status tc_tree_stats(tc_tree* tree, tc_stats* out, void* stream);

/* Testing hook for the error path above: sets the handle's walk status word
 * on the device to `bits` (bit 0: a refused stack push, bit 1: a node with more
 * than 8 children), on `stream`, as a walk that met either would leave it, so
 * that callers and tests can see how tc_tree_stats and the next tc_build report
 * it.  No kernel is made to misbehave.  The next tc_build clears the word.
 * Errors: TC_ERR_INVALID (null tree, bits outside 0..3), TC_ERR_STATE (no
 * tc_build on the handle). */
tc_status tc_tree_set_walk_status(tc_tree* tree, uint32_t bits, void* stream);

/* Record per-stage durations with HIP events on the call's stream (off by
 * default).  Errors: TC_ERR_INVALID (null tree). */
tc_status tc_tree_set_timing(tc_tree* tree, int on);

/* Copy the canonical tree to caller device buffers (any may be NULL):
 * keys u64[n] (sorted), perm u32[n] (sorted position -> caller index),
 * and, in pre-order (= sorted by (first, level)), level u8[n_nodes],
 * first u32[n_nodes], count u32[n_nodes], com f64[n_nodes,3], mass f64[n_nodes]
 * (com and mass need tc_moments).
 * Errors: TC_ERR_INVALID, TC_ERR_STATE. */
tc_status tc_tree_export(const tc_tree* tree, uint64_t* keys, uint32_t* perm, uint8_t* level,
                         uint32_t* first, uint32_t* count, double* com, double* mass,
                         void* stream);

/* The walk's target order, set by tc_moments: order u32[n] (device), the
 * sorted positions of the particles along the Hilbert curve; wavefront w of
 * every walk serves the targets order[64 w .. 64 w + 63].  It fixes only how
 * targets are grouped, never a result (each target's interaction set is its
 * own, section 2).  Provided for tests and diagnostics.
 * Errors: TC_ERR_INVALID, TC_ERR_STATE (no tc_moments since the last build). */
tc_status tc_tree_target_order(const tc_tree* tree, uint32_t* order, void* stream);

/* Per-target interaction counts of the last tc_forces run with TC_COUNT, in
 * the caller's order: counts u32[n] (device).
 * Errors: TC_ERR_INVALID, TC_ERR_STATE (no counted walk). */
tc_status tc_interaction_counts(const tc_tree* tree, uint32_t* counts, void* stream);

/* Release a handle and everything it owns (NULL is a no-op).  Waits for the
 * work the handle's calls enqueued (an event recorded by each call), not for
 * the whole device, then frees. */
void tc_tree_free(tc_tree* tree);

/* Message of the last error on this thread ("" if none). */
const char* tc_last_error(void);

/* Library version string. */
const char* tc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TREECODE_H */
