// Host side of the C ABI declared in include/treecode.h: argument checks,
// handle lifetime, buffer growth, stream plumbing and the order of launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "tc_internal.h"

using namespace tc;

namespace {

thread_local std::string g_err;
std::mutex g_alloc_mu;
tc_alloc_fn g_alloc = nullptr;
tc_free_fn g_free = nullptr;
void* g_actx = nullptr;

tc_status fail(tc_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

// Default allocator: stream-ordered (the device's default memory pool), so that
// growing a buffer or freeing a handle never synchronises the device.
void* default_alloc(size_t bytes, void* stream, void*)
{
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void default_free(void* p, void* stream, void*) { (void)hipFreeAsync(p, (hipStream_t)stream); }

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

enum Stage { kStKeys = 0, kStSort, kStTree, kStMoments, kStWalk, kStDiag, kStBwdWalk, kStBwdDown, kNumStages };

struct HostMirror {
    Geom geom;
    uint32_t level_hist[kLevels + 2];
    uint32_t total;
    uint32_t level_off[kLevels + 1];
    double diag[4];
    unsigned long long inter;
    unsigned long long visits[kNumVisitCounters];
    double step[10];
    uint32_t status;
};

}  // namespace

struct tc_tree {
    int device = -1;
    tc_alloc_fn alloc = nullptr;
    tc_free_fn freef = nullptr;
    void* actx = nullptr;

    int64_t n = 0;
    int64_t nn = 0;
    tc_dtype dtype = TC_F32;

    // particle-sized
    Buf keys0, keys1, vals0, vals1, rec, sp, c, cnt, pre, sorted_counts, diag_part;
    uint64_t* skeys = nullptr;
    uint32_t* perm = nullptr;
    Buf sort_temp, scan_temp, bounds_part;
    // node-sized
    Buf level, first, count, next, nchild, bfs, nk0, nk1, nv0, nv1, node_sort_temp, wn, diag_temp, parent, octant;
    Buf topo, nord, order;     // the walk's target order (particle-sized); dense topology and scratch (node-sized)
    // adjoint and leapfrog
    Buf node_grad, uc, part_grad, target_grad, step_temp;
    Buf lists, list_len;       // stored interaction lists of the last tc_forces (TC_STORE_LISTS)
    uint32_t* bfs_to_pre = nullptr;  // inside nv0 or nv1
    // small device block
    Buf small;
    Geom* geom = nullptr;
    uint32_t* level_hist = nullptr;
    double* diag_out = nullptr;
    double* step_out = nullptr;  // [10]
    unsigned long long* inter_total = nullptr;
    unsigned long long* visits = nullptr;      // [kNumVisitCounters]
    uint32_t* status = nullptr;

    HostMirror* host = nullptr;
    uint32_t state = 0;  // bit 0 built, bit 1 moments, bit 2 forces
    tc_walk last_mode = TC_WALK_F32C;
    bool counted = false;
    bool lists_stored = false;  // the last tc_forces stored lists that tc_forces_backward may replay
    bool diag_pending = false;
    bool build_pending = false;
    bool step_pending = false;
    bool step_valid = false;
    double f_theta = 0.0, f_eps = 0.0, f_G = 1.0;  // parameters of the last tc_forces
    Geom geom_host{};

    bool exact = false;  // size buffers exactly (the fixed scratch of tc_forces_noalloc), no growth slack
    bool timing = false;
    hipEvent_t ev[2 * kNumStages] = {};
    bool ev_used[kNumStages] = {};
    hipEvent_t done = nullptr;  // recorded after the last work each call enqueues (tc_tree_free waits on it)
    bool walk_status_pending = false;  // a walk's status word is on its way to host->status
};

namespace {

tc_status ensure(tc_tree* t, Buf& b, size_t bytes, hipStream_t s)
{
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return TC_OK;
    if (b.p) t->freef(b.p, s, t->actx);
    b.p = nullptr;
    b.bytes = 0;
    size_t want = t->exact ? bytes : bytes + bytes / 4;
    want = (want + 255) & ~(size_t)255;
    void* p = t->alloc(want, s, t->actx);
    if (!p) return fail(TC_ERR_NOMEM, "allocation of %zu bytes failed", want);
    b.p = p;
    b.bytes = want;
    return TC_OK;
}

void release(tc_tree* t, Buf& b)
{
    if (b.p) t->freef(b.p, nullptr, t->actx);
    b.p = nullptr;
    b.bytes = 0;
}

template <typename T>
T* P(const Buf& b) { return (T*)b.p; }

#define TC_TRY(expr)                          \
    do {                                      \
        tc_status _st = (expr);               \
        if (_st != TC_OK) return _st;         \
    } while (0)

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess) return fail(TC_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

tc_status check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TC_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return TC_OK;
}

void stage_begin(tc_tree* t, int st, hipStream_t s)
{
    if (!t->timing) return;
    if (!t->ev[2 * st]) {
        (void)hipEventCreate(&t->ev[2 * st]);
        (void)hipEventCreate(&t->ev[2 * st + 1]);
    }
    (void)hipEventRecord(t->ev[2 * st], s);
}

void stage_end(tc_tree* t, int st, hipStream_t s)
{
    if (!t->timing) return;
    (void)hipEventRecord(t->ev[2 * st + 1], s);
    t->ev_used[st] = true;
}

tc_status current_device(int* dev)
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(TC_ERR_DEVICE, "no HIP device available");
    }
    HIP_TRY(hipGetDevice(dev));
    return TC_OK;
}

// The handle's small device block: root cube, diagnostics, counters, status.
tc_status carve_small(tc_tree* t, hipStream_t s)
{
    TC_TRY(ensure(t, t->small, 1024, s));
    char* p = (char*)t->small.p;
    t->geom = (Geom*)p;
    p += (sizeof(Geom) + 15) & ~(size_t)15;
    t->diag_out = (double*)p;
    p += 4 * sizeof(double);
    t->step_out = (double*)p;
    p += 10 * sizeof(double);
    t->inter_total = (unsigned long long*)p;
    p += 8;
    t->visits = (unsigned long long*)p;
    p += 8 * kNumVisitCounters;
    t->level_hist = (uint32_t*)p;
    p += 4 * (kLevels + 2);
    t->status = (uint32_t*)p;
    return TC_OK;
}

tc_status create_tree(tc_tree** out, hipStream_t s)
{
    int dev;
    TC_TRY(current_device(&dev));
    tc_tree* t = new tc_tree();
    t->device = dev;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        t->alloc = g_alloc ? g_alloc : default_alloc;
        t->freef = g_free ? g_free : default_free;
        t->actx = g_alloc ? g_actx : nullptr;
    }
    tc_status st = carve_small(t, s);
    if (st != TC_OK) {
        delete t;
        return st;
    }
    if (hipHostMalloc((void**)&t->host, sizeof(HostMirror), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        release(t, t->small);
        delete t;
        return fail(TC_ERR_NOMEM, "pinned host allocation failed");
    }
    memset(t->host, 0, sizeof(HostMirror));
    if (hipEventCreateWithFlags(&t->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(t->host);
        release(t, t->small);
        delete t;
        return fail(TC_ERR_DEVICE, "event creation failed");
    }
    *out = t;
    return TC_OK;
}

// Record the handle's completion event after the work a call enqueued on s.
tc_status mark_done(tc_tree* t, hipStream_t s, tc_status st)
{
    if (t && t->done && hipEventRecord(t->done, s) != hipSuccess) (void)hipGetLastError();
    return st;
}

// Status word of the walks, cleared by each build and kept until the next
// (bit 0: a traversal stack would have overflowed, so terms were dropped;
// bit 1: a node with more than 8 children, i.e. a corrupt tree).  Neither can
// happen for a tree built by tc_build (the stack bound is proven in
// walk.hip); both are checked wherever the host synchronises anyway.
tc_status walk_status_error(tc_tree* t)
{
    if (!t->walk_status_pending) return TC_OK;
    t->walk_status_pending = false;
    const uint32_t st = t->host->status;
    t->host->status = 0;
    if (st & 1u) return fail(TC_ERR_OVERFLOW, "a walk on this handle overflowed its traversal stack; its outputs are incomplete");
    if (st & 2u) return fail(TC_ERR_DEVICE, "a walk on this handle met a node with more than 8 children (corrupt tree)");
    return TC_OK;
}

tc_status check_device(const tc_tree* t)
{
    int dev;
    TC_TRY(current_device(&dev));
    if (dev != t->device) return fail(TC_ERR_INVALID, "tree was created on device %d, current is %d", t->device, dev);
    return TC_OK;
}

tc_status build_impl(tc_tree* t, const void* pos, const void* mass, int64_t n, tc_dtype dt, hipStream_t s)
{
    t->state = 0;
    t->n = n;
    t->nn = 0;
    t->dtype = dt;
    t->diag_pending = false;
    t->build_pending = false;
    t->counted = false;
    t->lists_stored = false;
    for (int l = 0; l < kLevels + 2; ++l) t->host->level_hist[l] = 0;
    if (n == 0) {
        Geom g{};
        g.L = 1.0;
        g.scale = std::ldexp(1.0, 21);
        g.h = std::ldexp(1.0, -21);
        t->geom_host = g;
        t->state = 1;
        return TC_OK;
    }
    const size_t n8 = (size_t)n * 8, n4 = (size_t)n * 4;
    TC_TRY(ensure(t, t->keys0, n8, s));
    TC_TRY(ensure(t, t->keys1, n8, s));
    TC_TRY(ensure(t, t->vals0, n4, s));
    TC_TRY(ensure(t, t->vals1, n4, s));
    TC_TRY(ensure(t, t->rec, record_bytes(n, dt), s));
    TC_TRY(ensure(t, t->sp, (size_t)n * sizeof(Particle), s));
    TC_TRY(ensure(t, t->c, (size_t)n, s));
    TC_TRY(ensure(t, t->cnt, n4, s));
    TC_TRY(ensure(t, t->pre, n4 + 8, s));
    TC_TRY(ensure(t, t->sort_temp, radix_temp_bytes(n), s));
    TC_TRY(ensure(t, t->scan_temp, scan_temp_bytes(n), s));
    const int nb = bounds_blocks(n);
    TC_TRY(ensure(t, t->bounds_part, (size_t)nb * 8 * sizeof(double), s));

    stage_begin(t, kStKeys, s);
    launch_bounds(pos, mass, n, dt, P<double>(t->bounds_part), nb, t->geom, s);
    launch_keys(pos, mass, n, dt, t->geom, P<uint64_t>(t->keys0), P<uint32_t>(t->vals0), t->rec.p, s);
    stage_end(t, kStKeys, s);
    TC_TRY(check_launch("keys"));

    stage_begin(t, kStSort, s);
    radix_sort_pairs(P<uint64_t>(t->keys0), P<uint32_t>(t->vals0), P<uint64_t>(t->keys1), P<uint32_t>(t->vals1),
                     n, 63, t->sort_temp.p, s, &t->skeys, &t->perm);
    launch_gather(t->rec.p, n, dt, t->perm, P<Particle>(t->sp), s);
    stage_end(t, kStSort, s);
    TC_TRY(check_launch("sort"));

    stage_begin(t, kStTree, s);
    launch_adjacent_levels(t->skeys, n, P<int8_t>(t->c), s);
    launch_fill_u32(t->level_hist, kLevels + 2, 0u, s);
    launch_node_counts(P<int8_t>(t->c), n, P<uint32_t>(t->cnt), t->level_hist, s);
    launch_exclusive_scan_u32(P<uint32_t>(t->cnt), P<uint32_t>(t->pre), n, t->scan_temp.p, s);
    HIP_TRY(hipMemcpyAsync(&t->host->geom, t->geom, sizeof(Geom), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(t->host->level_hist, t->level_hist, 4 * (kLevels + 2), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&t->host->total, P<uint32_t>(t->pre) + n, 4, hipMemcpyDeviceToHost, s));
    TC_TRY(check_launch("tree counts"));
    HIP_TRY(hipStreamSynchronize(s));
    // the previous walk on this handle, enqueued before this build on the same stream, is complete
    TC_TRY(walk_status_error(t));
    t->geom_host = t->host->geom;
    if (t->geom_host.bad & 1u) return fail(TC_ERR_INPUT, "non-finite particle position");
    if (t->geom_host.bad & 2u) return fail(TC_ERR_INPUT, "negative or non-finite particle mass");
    uint64_t total = 0;
    for (int l = 0; l < kLevels; ++l) {
        t->host->level_off[l] = (uint32_t)total;
        total += t->host->level_hist[l];
    }
    if (total >= 0xFFFFFFFFull) return fail(TC_ERR_OVERFLOW, "octree needs %llu nodes (limit 2^32 - 1)",
                                           (unsigned long long)total);
    t->host->level_off[kLevels] = (uint32_t)total;
    if (total != t->host->total) return fail(TC_ERR_DEVICE, "node count mismatch (%llu vs %u)",
                                             (unsigned long long)total, t->host->total);
    const int64_t nn = (int64_t)total;
    t->nn = nn;
    const size_t m4 = (size_t)nn * 4;
    TC_TRY(ensure(t, t->level, (size_t)nn, s));
    TC_TRY(ensure(t, t->octant, (size_t)nn, s));
    TC_TRY(ensure(t, t->first, m4, s));
    TC_TRY(ensure(t, t->count, m4, s));
    TC_TRY(ensure(t, t->next, m4, s));
    TC_TRY(ensure(t, t->nchild, m4, s));
    TC_TRY(ensure(t, t->bfs, m4, s));
    TC_TRY(ensure(t, t->nk0, (size_t)nn * 8, s));
    TC_TRY(ensure(t, t->nk1, (size_t)nn * 8, s));
    TC_TRY(ensure(t, t->nv0, m4, s));
    TC_TRY(ensure(t, t->nv1, m4, s));
    TC_TRY(ensure(t, t->node_sort_temp, radix_temp_bytes(nn), s));
    TC_TRY(ensure(t, t->wn, (size_t)nn * sizeof(WalkNode), s));
    TC_TRY(ensure(t, t->parent, m4, s));
    TC_TRY(ensure(t, t->topo, (size_t)nn * 16, s));

    launch_fill_u32(t->status, 1, 0u, s);  // status bits stay set until the next build
    launch_emit_nodes(t->skeys, P<int8_t>(t->c), P<uint32_t>(t->pre), n, P<uint8_t>(t->level), P<uint32_t>(t->first),
                      P<uint32_t>(t->count), P<uint32_t>(t->next), P<uint8_t>(t->octant), s);
    launch_count_children(P<uint8_t>(t->level), P<uint32_t>(t->count), P<uint32_t>(t->next), nn,
                          P<uint32_t>(t->nchild), s);
    launch_bfs_order(P<uint8_t>(t->level), nn, P<uint64_t>(t->nk0), P<uint32_t>(t->nv0), P<uint64_t>(t->nk1),
                     P<uint32_t>(t->nv1), t->node_sort_temp.p, P<uint32_t>(t->bfs), &t->bfs_to_pre, s);
    stage_end(t, kStTree, s);
    TC_TRY(check_launch("tree"));
    t->state = 1;
    return TC_OK;
}

tc_status moments_impl(tc_tree* t, hipStream_t s)
{
    if (t->n > 0) {
        stage_begin(t, kStMoments, s);
        launch_moments(t->host->level_off, t->bfs_to_pre, P<uint32_t>(t->bfs), P<uint32_t>(t->first),
                       P<uint32_t>(t->count), P<uint32_t>(t->nchild), t->skeys, P<uint8_t>(t->octant), P<Particle>(t->sp), t->geom,
                       P<WalkNode>(t->wn), P<uint32_t>(t->parent), P<uint4>(t->topo), s);
        TC_TRY(ensure(t, t->nord, (size_t)t->nn * sizeof(uint2), s));
        TC_TRY(ensure(t, t->order, (size_t)t->n * 4, s));
        launch_target_order(t->host->level_off, P<uint4>(t->topo), P<uint2>(t->nord), P<uint32_t>(t->order), s);
        stage_end(t, kStMoments, s);
        TC_TRY(check_launch("moments"));
    }
    t->state |= 2u;
    return TC_OK;
}

// The walk's common arguments: tree arrays, softening, G and the opening
// threshold tau_l = (L 2^-l / theta)^2 = tau_0 4^-l.
tc_status walk_args(tc_tree* t, double theta, double eps, double G, tc_walk mode, WalkArgs& a)
{
    a.nodes = P<WalkNode>(t->wn);
    a.sp = P<Particle>(t->sp);
    a.order = P<uint32_t>(t->order);
    a.perm = t->perm;
    a.n = t->n;
    a.eps2 = eps * eps;
    a.G = G;
    const double side = t->geom_host.L;
    const double tv = theta > 0.0 ? (side / theta) * (side / theta) : INFINITY;
    a.tau0_64 = tv;
    a.tau0_32 = (float)tv;
    if (theta > 0.0 && (!std::isfinite(tv) || (mode == TC_WALK_F32C && !std::isfinite(a.tau0_32))))
        return fail(TC_ERR_INVALID, "tc_forces: (L/theta)^2 = (%g/%g)^2 overflows the walk precision", side, theta);
    a.status = t->status;
    return TC_OK;
}

tc_status forces_impl(tc_tree* t, double theta, double eps, double G, tc_walk mode, uint32_t flags, void* acc,
                      void* pot, hipStream_t s)
{
    const int64_t n = t->n;
    t->last_mode = mode;
    t->counted = (flags & TC_COUNT) != 0;
    t->lists_stored = false;
    t->f_theta = theta;
    t->f_eps = eps;
    t->f_G = G;
    if (n == 0) {
        t->state |= 4u;
        t->host->diag[0] = t->host->diag[1] = t->host->diag[2] = t->host->diag[3] = 0.0;
        t->host->inter = 0;
        t->diag_pending = false;
        return TC_OK;
    }
    const int64_t waves = walk_waves(n);
    TC_TRY(ensure(t, t->diag_part, (size_t)waves * 4 * sizeof(double), s));
    TC_TRY(ensure(t, t->diag_temp, diag_temp_bytes(waves), s));
    if (t->counted) TC_TRY(ensure(t, t->sorted_counts, (size_t)n * 4, s));

    WalkArgs a{};
    TC_TRY(walk_args(t, theta, eps, G, mode, a));
    a.acc = acc;
    a.pot = pot;
    a.counts = t->counted ? P<uint32_t>(t->sorted_counts) : nullptr;
    a.diag = P<double>(t->diag_part);
    a.status = t->status;
    a.visits = t->visits;
    // Lists are kept only while they fit the budget; otherwise the adjoint re-walks.
    const bool store = (flags & TC_STORE_LISTS) != 0 &&
                       (uint64_t)waves * kListCap * sizeof(uint4) <= kListMaxBytes;
    if (store) {
        TC_TRY(ensure(t, t->lists, (size_t)waves * kListCap * sizeof(uint4), s));
        TC_TRY(ensure(t, t->list_len, (size_t)waves * sizeof(uint32_t), s));
        a.lists = P<uint4>(t->lists);
        a.list_len = P<uint32_t>(t->list_len);
        a.list_cap = kListCap;
    }

    if (t->counted) launch_fill_u32((uint32_t*)t->visits, 2 * kNumVisitCounters, 0u, s);
    stage_begin(t, kStWalk, s);
    launch_walk(a, mode, t->counted, store, s);
    stage_end(t, kStWalk, s);
    TC_TRY(check_launch("walk"));
    stage_begin(t, kStDiag, s);
    launch_diag_final(P<double>(t->diag_part), waves, t->diag_temp.p, t->diag_out, s);
    if (t->counted) launch_sum_counts(P<uint32_t>(t->sorted_counts), n, t->inter_total, s);
    stage_end(t, kStDiag, s);
    TC_TRY(check_launch("diagnostics"));
    HIP_TRY(hipMemcpyAsync(t->host->diag, t->diag_out, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&t->host->status, t->status, 4, hipMemcpyDeviceToHost, s));
    t->walk_status_pending = true;
    if (t->counted) {
        HIP_TRY(hipMemcpyAsync(&t->host->inter, t->inter_total, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(t->host->visits, t->visits, 8 * kNumVisitCounters, hipMemcpyDeviceToHost, s));
    }
    t->diag_pending = true;
    t->state |= 4u;
    t->lists_stored = store;
    return TC_OK;
}

bool is_finite(double v) { return std::isfinite(v); }

tc_status backward_impl(tc_tree* t, const void* g_acc, const void* g_pot, void* g_pos, void* g_mass, hipStream_t s)
{
    const int64_t n = t->n, nn = t->nn;
    if (n == 0) return TC_OK;
    TC_TRY(ensure(t, t->node_grad, (size_t)nn * 4 * sizeof(double), s));
    TC_TRY(ensure(t, t->uc, (size_t)nn * 4 * sizeof(double), s));
    TC_TRY(ensure(t, t->part_grad, (size_t)n * 4 * sizeof(double), s));
    TC_TRY(ensure(t, t->target_grad, (size_t)n * 3 * sizeof(double), s));
    WalkArgs a{};
    TC_TRY(walk_args(t, t->f_theta, t->f_eps, t->f_G, t->last_mode, a));
    a.g_acc = g_acc;
    a.g_pot = g_pot;
    a.node_grad = P<double>(t->node_grad);
    a.part_grad = P<double>(t->part_grad);
    a.target_grad = P<double>(t->target_grad);
    if (t->lists_stored) {
        a.lists = P<uint4>(t->lists);
        a.list_len = P<uint32_t>(t->list_len);
        a.list_cap = kListCap;
    }
    stage_begin(t, kStBwdWalk, s);
    launch_fill_f64_zero(a.node_grad, nn * 4, s);
    launch_fill_f64_zero(a.part_grad, n * 4, s);
    launch_walk_adjoint(a, t->last_mode, s);
    stage_end(t, kStBwdWalk, s);
    TC_TRY(check_launch("adjoint walk"));
    HIP_TRY(hipMemcpyAsync(&t->host->status, t->status, 4, hipMemcpyDeviceToHost, s));
    t->walk_status_pending = true;
    stage_begin(t, kStBwdDown, s);
    launch_adjoint_down(t->host->level_off, P<WalkNode>(t->wn), P<uint32_t>(t->parent), a.node_grad, P<double>(t->uc),
                        a.sp, t->perm, a.target_grad, a.part_grad, g_pos, g_mass,
                        t->last_mode == TC_WALK_F64, s);
    stage_end(t, kStBwdDown, s);
    TC_TRY(check_launch("adjoint down-pass"));
    return TC_OK;
}

tc_status leapfrog_impl(tc_tree* t, void* pos, void* vel, const void* mass, void* acc, void* pot, int64_t n,
                        tc_dtype dtype, double tau, double theta, double eps, double G, tc_walk mode, hipStream_t s)
{
    const bool acc64 = mode == TC_WALK_F64;
    launch_kick_drift(pos, vel, acc, n, dtype, acc64, tau, s);            // Eqs.(2), (3)
    TC_TRY(check_launch("kick-drift"));
    TC_TRY(build_impl(t, pos, mass, n, dtype, s));                       // Eq.(4): rebuild ...
    TC_TRY(moments_impl(t, s));
    TC_TRY(forces_impl(t, theta, eps, G, mode, 0u, acc, pot, s));        // ... and evaluate
    launch_kick(vel, acc, n, dtype, acc64, tau, s);                      // Eq.(5)
    TC_TRY(check_launch("kick"));
    if (n > 0) {
        TC_TRY(ensure(t, t->step_temp, step_diag_temp_bytes(), s));
        launch_step_diag(pos, vel, mass, pot, n, dtype, acc64, t->step_temp.p, t->step_out, s);
        TC_TRY(check_launch("step diagnostics"));
        HIP_TRY(hipMemcpyAsync(t->host->step, t->step_out, 10 * sizeof(double), hipMemcpyDeviceToHost, s));
        t->step_pending = true;
    } else {
        for (int k = 0; k < 10; ++k) t->host->step[k] = 0.0;
    }
    t->step_valid = true;
    return TC_OK;
}


// ---------------------------------------------------------------------------
// tc_forces_noalloc: every buffer of the build, the moments and the walk comes
// from one fixed device array per GPU, handed out by a bump allocator; the
// host side uses a per-device handle and host mirror held in static storage.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = 128ull << 20;  // 128 MiB per GPU
constexpr int64_t kNoAllocMaxN = 1 << 18;
constexpr int kNoAllocMaxDevices = 64;

}  // namespace

// The scratch array.  In host code its name is only a stand-in: the device
// address comes from hipGetSymbolAddress, once per device (each GPU holds its
// own copy of the array, at its own address, until the process ends).
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

struct Bump {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
};

void* bump_alloc(size_t bytes, void*, void* ctx)
{
    Bump* b = (Bump*)ctx;
    const size_t off = (b->used + 255) & ~(size_t)255;
    if (off > b->cap || bytes > b->cap - off) return nullptr;
    b->used = off + bytes;
    return b->base + off;
}

void bump_free(void*, void*, void*) {}

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocMaxDevices] = {};  // device address of `scratch` on each device
tc_tree g_noalloc_tree[kNoAllocMaxDevices];
HostMirror g_noalloc_host[kNoAllocMaxDevices];
Bump g_noalloc_bump[kNoAllocMaxDevices];

tc_status noalloc_scratch(int dev, char** base)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(TC_ERR_DEVICE, "tc_forces_noalloc: hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        }
        g_noalloc_ptr[dev] = ptr;
    }
    *base = (char*)g_noalloc_ptr[dev];
    return TC_OK;
}

}  // namespace

extern "C" {

tc_status tc_set_allocator(tc_alloc_fn alloc, tc_free_fn free_fn, void* ctx)
{
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(TC_ERR_INVALID, "tc_set_allocator: give both alloc and free, or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = alloc;
    g_free = free_fn;
    g_actx = alloc ? ctx : nullptr;
    return TC_OK;
}

tc_status tc_build(const void* pos, const void* mass, int64_t n, tc_dtype dtype, void* stream, tc_tree** tree)
{
    g_err.clear();
    if (!tree) return fail(TC_ERR_INVALID, "tc_build: tree is NULL");
    if (n < 0 || n >= (int64_t)1 << 31) return fail(TC_ERR_INVALID, "tc_build: n = %lld out of range [0, 2^31)", (long long)n);
    if (dtype != TC_F32 && dtype != TC_F64) return fail(TC_ERR_INVALID, "tc_build: bad dtype %d", (int)dtype);
    if (n > 0 && (!pos || !mass)) return fail(TC_ERR_INVALID, "tc_build: pos and mass must be non-NULL");
    hipStream_t s = (hipStream_t)stream;
    if (!*tree) {
        TC_TRY(create_tree(tree, s));
    } else {
        TC_TRY(check_device(*tree));
    }
    return mark_done(*tree, s, build_impl(*tree, pos, mass, n, dtype, s));
}

tc_status tc_moments(tc_tree* t, void* stream)
{
    g_err.clear();
    if (!t) return fail(TC_ERR_INVALID, "tc_moments: tree is NULL");
    if (!(t->state & 1u)) return fail(TC_ERR_STATE, "tc_moments: no successful tc_build on this handle");
    TC_TRY(check_device(t));
    return mark_done(t, (hipStream_t)stream, moments_impl(t, (hipStream_t)stream));
}

tc_status tc_forces(tc_tree* t, double theta, double eps, double G, tc_walk mode, uint32_t flags, void* acc,
                    void* pot, void* stream)
{
    g_err.clear();
    if (!t) return fail(TC_ERR_INVALID, "tc_forces: tree is NULL");
    if (!is_finite(theta) || theta < 0.0) return fail(TC_ERR_INVALID, "tc_forces: theta must be finite and >= 0");
    if (!is_finite(eps) || eps < 0.0) return fail(TC_ERR_INVALID, "tc_forces: eps must be finite and >= 0");
    if (!is_finite(G)) return fail(TC_ERR_INVALID, "tc_forces: G must be finite");
    if (mode != TC_WALK_F32C && mode != TC_WALK_F64) return fail(TC_ERR_INVALID, "tc_forces: bad walk mode %d", (int)mode);
    if (flags & ~(TC_COUNT | TC_STORE_LISTS)) return fail(TC_ERR_INVALID, "tc_forces: unknown flags 0x%x", flags);
    if (t->n > 0 && !acc) return fail(TC_ERR_INVALID, "tc_forces: acc must be non-NULL");
    if ((t->state & 3u) != 3u) return fail(TC_ERR_STATE, "tc_forces: call tc_build and tc_moments first");
    TC_TRY(check_device(t));
    return mark_done(t, (hipStream_t)stream, forces_impl(t, theta, eps, G, mode, flags, acc, pot, (hipStream_t)stream));
}

tc_status tc_forces_backward(tc_tree* t, const void* g_acc, const void* g_pot, void* g_pos, void* g_mass,
                             void* stream)
{
    g_err.clear();
    if (!t) return fail(TC_ERR_INVALID, "tc_forces_backward: tree is NULL");
    if (!(t->state & 4u)) return fail(TC_ERR_STATE, "tc_forces_backward: no tc_forces since the last tc_build");
    if (t->n > 0 && !g_acc) return fail(TC_ERR_INVALID, "tc_forces_backward: g_acc must be non-NULL");
    TC_TRY(check_device(t));
    return mark_done(t, (hipStream_t)stream, backward_impl(t, g_acc, g_pot, g_pos, g_mass, (hipStream_t)stream));
}

tc_status tc_forces_noalloc(const void* pos, const void* mass, int64_t n, tc_dtype dtype, double theta, double eps,
                            double G, tc_walk mode, void* acc, void* pot, void* stream)
{
    g_err.clear();
    if (n < 0 || n > kNoAllocMaxN)
        return fail(TC_ERR_INVALID, "tc_forces_noalloc: n = %lld outside [0, %lld], the size its static scratch serves",
                    (long long)n, (long long)kNoAllocMaxN);
    if (dtype != TC_F32 && dtype != TC_F64) return fail(TC_ERR_INVALID, "tc_forces_noalloc: bad dtype %d", (int)dtype);
    if (n > 0 && (!pos || !mass || !acc))
        return fail(TC_ERR_INVALID, "tc_forces_noalloc: pos, mass and acc must be non-NULL");
    if (!is_finite(theta) || theta < 0.0) return fail(TC_ERR_INVALID, "tc_forces_noalloc: theta must be finite and >= 0");
    if (!is_finite(eps) || eps < 0.0) return fail(TC_ERR_INVALID, "tc_forces_noalloc: eps must be finite and >= 0");
    if (!is_finite(G)) return fail(TC_ERR_INVALID, "tc_forces_noalloc: G must be finite");
    if (mode != TC_WALK_F32C && mode != TC_WALK_F64) return fail(TC_ERR_INVALID, "tc_forces_noalloc: bad walk mode");
    int dev;
    TC_TRY(current_device(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(TC_ERR_DEVICE, "tc_forces_noalloc: device %d not served", dev);
    char* base = nullptr;
    TC_TRY(noalloc_scratch(dev, &base));
    hipStream_t s = (hipStream_t)stream;
    // a fresh handle over the scratch; the status of the previous call's walk is
    // still reported at this call's synchronisation
    tc_tree* t = &g_noalloc_tree[dev];
    const bool status_pending = t->walk_status_pending;
    *t = tc_tree{};
    Bump* b = &g_noalloc_bump[dev];
    *b = Bump{base, kNoAllocScratchBytes, 0};
    t->device = dev;
    t->alloc = bump_alloc;
    t->freef = bump_free;
    t->actx = b;
    t->exact = true;
    t->host = &g_noalloc_host[dev];
    t->walk_status_pending = status_pending;
    tc_status st = carve_small(t, s);
    if (st == TC_OK) st = build_impl(t, pos, mass, n, dtype, s);
    if (st == TC_OK) st = moments_impl(t, s);
    if (st == TC_OK) st = forces_impl(t, theta, eps, G, mode, 0u, acc, pot, s);
    if (st == TC_ERR_NOMEM)
        return fail(TC_ERR_OVERFLOW, "tc_forces_noalloc: n = %lld particles with %lld octree nodes need more than the "
                    "%zu-byte static scratch", (long long)n, (long long)t->nn, kNoAllocScratchBytes);
    return st;
}

tc_status tc_leapfrog_step(tc_tree** tree, void* pos, void* vel, const void* mass, void* acc, void* pot,
                           int64_t n, tc_dtype dtype, double tau, double theta, double eps, double G, tc_walk mode,
                           void* stream)
{
    g_err.clear();
    if (!tree) return fail(TC_ERR_INVALID, "tc_leapfrog_step: tree is NULL");
    if (n < 0 || n >= (int64_t)1 << 31) return fail(TC_ERR_INVALID, "tc_leapfrog_step: n out of range");
    if (dtype != TC_F32 && dtype != TC_F64) return fail(TC_ERR_INVALID, "tc_leapfrog_step: bad dtype");
    if (n > 0 && (!pos || !vel || !mass || !acc))
        return fail(TC_ERR_INVALID, "tc_leapfrog_step: pos, vel, mass and acc must be non-NULL");
    if (!is_finite(tau)) return fail(TC_ERR_INVALID, "tc_leapfrog_step: tau must be finite");
    if (!is_finite(theta) || theta < 0.0) return fail(TC_ERR_INVALID, "tc_leapfrog_step: theta must be finite and >= 0");
    if (!is_finite(eps) || eps < 0.0) return fail(TC_ERR_INVALID, "tc_leapfrog_step: eps must be finite and >= 0");
    if (!is_finite(G)) return fail(TC_ERR_INVALID, "tc_leapfrog_step: G must be finite");
    if (mode != TC_WALK_F32C && mode != TC_WALK_F64) return fail(TC_ERR_INVALID, "tc_leapfrog_step: bad walk mode");
    hipStream_t s = (hipStream_t)stream;
    if (!*tree) {
        TC_TRY(create_tree(tree, s));
    } else {
        TC_TRY(check_device(*tree));
    }
    return mark_done(*tree, s, leapfrog_impl(*tree, pos, vel, mass, acc, pot, n, dtype, tau, theta, eps, G, mode, s));
}


tc_status tc_tree_set_walk_status(tc_tree* t, uint32_t bits, void* stream)
{
    g_err.clear();
    if (!t) return fail(TC_ERR_INVALID, "tc_tree_set_walk_status: NULL tree");
    if (bits > 3u) return fail(TC_ERR_INVALID, "tc_tree_set_walk_status: bits must be within 0..3");
    if (!(t->state & 1u)) return fail(TC_ERR_STATE, "tc_tree_set_walk_status: no successful tc_build on this handle");
    TC_TRY(check_device(t));
    hipStream_t s = (hipStream_t)stream;
    launch_fill_u32(t->status, 1, bits, s);
    TC_TRY(check_launch("status"));
    HIP_TRY(hipMemcpyAsync(&t->host->status, t->status, 4, hipMemcpyDeviceToHost, s));
    t->walk_status_pending = true;
    return mark_done(t, s, TC_OK);
}

tc_status tc_tree_stats(tc_tree* t, tc_stats* out, void* stream)
{
    g_err.clear();
    if (!t || !out) return fail(TC_ERR_INVALID, "tc_tree_stats: NULL argument");
    memset(out, 0, sizeof *out);
    bool any_ev = false;
    for (int i = 0; i < kNumStages; ++i) any_ev |= t->ev_used[i];
    if (t->diag_pending || t->build_pending || t->step_pending || t->walk_status_pending || any_ev) {
        TC_TRY(check_device(t));
        HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
        t->diag_pending = false;
        t->build_pending = false;
        t->step_pending = false;
    }
    out->n = t->n;
    out->n_nodes = t->nn;
    for (int k = 0; k < 3; ++k) out->lo[k] = t->geom_host.lo[k];
    out->L = t->geom_host.L;
    out->log2L = t->geom_host.log2L;
    int maxl = 0;
    for (int l = 0; l < kLevels; ++l)
        if (t->n > 0 && (t->state & 1u) && t->host->level_hist[l]) maxl = l;
    out->max_level = maxl;
    out->state = t->state;
    if (t->state & 1u) {
        out->n_leaves = t->n > 0 ? (int64_t)t->host->level_hist[kLevels] : 0;
        out->n_multi_leaves = t->n > 0 ? (int64_t)t->host->level_hist[kLevels + 1] : 0;
    }
    out->last_mode = (uint32_t)t->last_mode;
    out->lists_stored = t->lists_stored ? 1u : 0u;
    out->list_bytes = t->lists_stored ? (uint64_t)walk_waves(t->n) * kListCap * sizeof(uint4) : 0u;
    if (t->state & 4u) {
        for (int k = 0; k < 3; ++k) out->momentum[k] = t->host->diag[k];
        out->sum_m_abs_a = t->host->diag[3];
        out->interactions = t->counted ? t->host->inter : 0;
        out->node_visits = t->counted ? t->host->visits[0] : 0;
        out->lane_visits = t->counted ? t->host->visits[1] : 0;
        if (t->counted) {
            out->group_pops = t->host->visits[2];
            out->visits_no_accept = t->host->visits[3];
            out->visits_all_accept = t->host->visits[4];
            out->visits_box_open = t->host->visits[5];
            out->visits_box_accept = t->host->visits[6];
            out->max_stack = (uint32_t)t->host->visits[7];
            out->walk_steps = t->host->visits[8];
            out->walk_single_steps = t->host->visits[9];
            out->visits_overlap = t->host->visits[10];
            out->visits_overlap_all_accept = t->host->visits[11];
        }
    }
    if (t->step_valid) {
        out->kinetic = t->host->step[0];
        out->potential = t->host->step[1];
        for (int k = 0; k < 3; ++k) {
            out->lin_momentum[k] = t->host->step[2 + k];
            out->ang_momentum[k] = t->host->step[5 + k];
        }
    }
    for (int i = 0; i < 8; ++i) {
        out->stage_ms[i] = -1.0f;
        if (t->ev_used[i]) {
            float ms = -1.0f;
            if (hipEventElapsedTime(&ms, t->ev[2 * i], t->ev[2 * i + 1]) == hipSuccess) out->stage_ms[i] = ms;
            else (void)hipGetLastError();
        }
    }
    return walk_status_error(t);
}

tc_status tc_tree_set_timing(tc_tree* t, int on)
{
    g_err.clear();
    if (!t) return fail(TC_ERR_INVALID, "tc_tree_set_timing: tree is NULL");
    t->timing = on != 0;
    for (int i = 0; i < kNumStages; ++i) t->ev_used[i] = false;
    return TC_OK;
}

tc_status tc_tree_export(const tc_tree* t, uint64_t* keys, uint32_t* perm, uint8_t* level, uint32_t* first,
                         uint32_t* count, double* com, double* mass, void* stream)
{
    g_err.clear();
    if (!t) return fail(TC_ERR_INVALID, "tc_tree_export: tree is NULL");
    if (!(t->state & 1u)) return fail(TC_ERR_STATE, "tc_tree_export: no successful tc_build");
    if ((com || mass) && !(t->state & 2u)) return fail(TC_ERR_STATE, "tc_tree_export: com/mass need tc_moments");
    TC_TRY(check_device(t));
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)t->n, nn = (size_t)t->nn;
    if (n == 0) return TC_OK;
    auto cp = [&](void* dst, const void* src, size_t bytes) -> tc_status {
        if (!dst) return TC_OK;
        HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
        return TC_OK;
    };
    TC_TRY(cp(keys, t->skeys, n * 8));
    TC_TRY(cp(perm, t->perm, n * 4));
    TC_TRY(cp(level, t->level.p, nn));
    TC_TRY(cp(first, t->first.p, nn * 4));
    TC_TRY(cp(count, t->count.p, nn * 4));
    if (com || mass) {
        launch_export_moments(P<WalkNode>(t->wn), P<uint32_t>(t->bfs), (int64_t)nn, com, mass, s);
        TC_TRY(check_launch("export"));
    }
    return mark_done(const_cast<tc_tree*>(t), s, TC_OK);
}

tc_status tc_tree_target_order(const tc_tree* t, uint32_t* order, void* stream)
{
    g_err.clear();
    if (!t || !order) return fail(TC_ERR_INVALID, "tc_tree_target_order: NULL argument");
    if (!(t->state & 2u)) return fail(TC_ERR_STATE, "tc_tree_target_order: no tc_moments since the last build");
    TC_TRY(check_device(t));
    if (t->n == 0) return TC_OK;
    HIP_TRY(hipMemcpyAsync(order, t->order.p, (size_t)t->n * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return mark_done(const_cast<tc_tree*>(t), (hipStream_t)stream, TC_OK);
}

tc_status tc_interaction_counts(const tc_tree* t, uint32_t* counts, void* stream)
{
    g_err.clear();
    if (!t || !counts) return fail(TC_ERR_INVALID, "tc_interaction_counts: NULL argument");
    if (!(t->state & 4u) || !t->counted) return fail(TC_ERR_STATE, "tc_interaction_counts: no counted tc_forces");
    TC_TRY(check_device(t));
    launch_scatter_counts(P<uint32_t>(t->sorted_counts), t->perm, t->n, counts, (hipStream_t)stream);
    return mark_done(const_cast<tc_tree*>(t), (hipStream_t)stream, check_launch("counts"));
}

void tc_tree_free(tc_tree* t)
{
    if (!t) return;
    // wait for the work the handle's calls enqueued (on whichever stream), not the whole device
    if (t->done && hipEventSynchronize(t->done) != hipSuccess) (void)hipGetLastError();
    Buf* bufs[] = {&t->keys0, &t->keys1, &t->vals0, &t->vals1, &t->rec, &t->sp, &t->c, &t->cnt,
                   &t->pre, &t->sorted_counts, &t->diag_part, &t->sort_temp, &t->scan_temp, &t->bounds_part,
                   &t->level, &t->first, &t->count, &t->next, &t->nchild, &t->bfs, &t->nk0, &t->nk1,
                   &t->nv0, &t->nv1, &t->node_sort_temp, &t->wn, &t->diag_temp, &t->parent, &t->topo, &t->nord, &t->order, &t->octant, &t->node_grad,
                   &t->uc, &t->part_grad, &t->target_grad, &t->step_temp, &t->lists, &t->list_len, &t->small};
    for (Buf* b : bufs) release(t, *b);
    for (auto& e : t->ev)
        if (e) (void)hipEventDestroy(e);
    if (t->done) (void)hipEventDestroy(t->done);
    if (t->host) (void)hipHostFree(t->host);
    delete t;
}

const char* tc_last_error(void) { return g_err.c_str(); }

const char* tc_version(void) { return "treecode-gfx950 0.1"; }

}  // extern "C"
