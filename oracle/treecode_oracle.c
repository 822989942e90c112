/*
 * FP64 CPU oracle for the TreeCode (Barnes-Hut) gravity evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the HIP library; the two agree only through the
 * mathematics written down below.
 *
 * What is computed, and where it comes from (Kuzmin, Sirotin, Khoperskov,
 * "Efficiency of parallel computations of gravitational forces by TreeCode
 * method in N-body models", 2024):
 *   - Softened pairwise gravity, Eq.(1): a_i = sum_{j != i} G m_j (r_j - r_i)
 *     / (|r_j - r_i|^2 + eps^2)^{3/2}.  The potential that goes with it is
 *     phi_i = -G sum_{j != i} m_j (|r_j - r_i|^2 + eps^2)^{-1/2}  (so that
 *     a = -grad phi); the paper does not print phi, this is that reading.
 *   - TreeCode (section 2, description of the method): space is split into
 *     eight octants recursively until every cell holds at most one particle;
 *     a distant cell acts as one particle of the cell's total mass placed at
 *     its centre of mass; theta decides "distant"; theta -> 0 gives the direct
 *     particle-particle sum.
 *   - Kick-drift-kick leapfrog, Eqs.(2)-(5), with the tree rebuilt from the
 *     drifted positions for Eq.(4).
 *
 * Readings where the paper is silent (each one is also listed in the design
 * notes of the repository):
 *   - Root cube: lo_k = min_i x_ik, E = max_k (max_i x_ik - lo_k), L = the
 *     smallest power of two >= E (L = 1 when E = 0).
 *   - Quantisation: q_ik = min(2^21 - 1, floor((x_ik - lo_k) * 2^21 / L)).
 *   - Key: 63-bit interleave, x bit highest within each triple; the child
 *     digit at level l (1..21) is (key >> 3(21 - l)) & 7 = 4x + 2y + z.
 *   - Sort: ascending key, ties by original index (stable).
 *   - Tree: a cell at level l < 21 holding >= 2 particles is split into its
 *     non-empty octants (a cell whose particles all fall in one octant gets
 *     one child; such chain nodes are kept).  Level 21 cells are leaves even
 *     when several particles share the key.
 *   - Moments: monopole only.  Leaf with one particle: M = m_j, X = x_j
 *     verbatim.  Otherwise M = sum of masses, X = (sum M x) / M, summed in
 *     sorted (leaf) or digit (internal) order.  M = 0: X = the cell centre.
 *   - Opening test: a node n that does not contain the target is accepted iff
 *     theta > 0 and s_l < theta * |X_n - x_i|, where s_l = L 2^-l is the side
 *     of the geometric cell.  A node that contains the target is never
 *     accepted.  An opened leaf contributes its particles directly.
 *   - Summation: plain FP64 in visit order (children in digit order).
 *
 * Build flags: -O3 -fno-fast-math -ffp-contract=off (no FMA contraction, the
 * paper's own choice of strict IEEE arithmetic).  Threads (POSIX) split the
 * independent per-target work only; every target is computed by one thread in
 * a fixed order, so results do not depend on the thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXLEVEL 21
#define OR_QMAX ((int64_t)(1 << 21) - 1)

/* ------------------------------------------------------------------------ */
/* Root cube and Morton keys                                                  */
/* ------------------------------------------------------------------------ */

/* Root cube of a particle set.  Returns 0, or -1 when a coordinate is not
 * finite.  *log2L receives the exponent e with L = 2^e. */
int or_root_cube(const double* pos, int64_t n, double lo[3], double* L, int* log2L)
{
    double hi[3];
    for (int k = 0; k < 3; ++k) { lo[k] = 0.0; hi[k] = 0.0; }
    if (n > 0)
        for (int k = 0; k < 3; ++k) { lo[k] = pos[k]; hi[k] = pos[k]; }
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) {
            double x = pos[3 * i + k];
            if (!isfinite(x)) return -1;
            if (x < lo[k]) lo[k] = x;
            if (x > hi[k]) hi[k] = x;
        }
    }
    double E = 0.0;
    for (int k = 0; k < 3; ++k) {
        double ext = hi[k] - lo[k];
        if (ext > E) E = ext;
    }
    if (!isfinite(E)) return -1;
    if (E == 0.0) { *L = 1.0; *log2L = 0; return 0; }
    /* E = f 2^e with f in [0.5, 1): E is a power of two iff f == 0.5. */
    int e;
    double f = frexp(E, &e);
    int eL = (f == 0.5) ? e - 1 : e;
    *L = ldexp(1.0, eL);
    *log2L = eL;
    return 0;
}

/* Quantised grid coordinate of one axis. */
static int64_t quantise(double x, double lo, int log2L)
{
    double scaled = (x - lo) * ldexp(1.0, 21 - log2L);  /* exact power of two */
    double f = floor(scaled);
    if (f < 0.0) f = 0.0;
    if (f > (double)OR_QMAX) return OR_QMAX;
    return (int64_t)f;
}

/* Interleave three 21-bit integers into a 63-bit key, x highest. */
static uint64_t interleave(int64_t qx, int64_t qy, int64_t qz)
{
    uint64_t key = 0;
    for (int b = 0; b < 21; ++b) {
        key |= (uint64_t)((qx >> b) & 1) << (3 * b + 2);
        key |= (uint64_t)((qy >> b) & 1) << (3 * b + 1);
        key |= (uint64_t)((qz >> b) & 1) << (3 * b + 0);
    }
    return key;
}

void or_keys(const double* pos, int64_t n, const double lo[3], int log2L,
             int64_t* q /* [n,3] or NULL */, uint64_t* keys)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t qq[3];
        for (int k = 0; k < 3; ++k) qq[k] = quantise(pos[3 * i + k], lo[k], log2L);
        if (q) for (int k = 0; k < 3; ++k) q[3 * i + k] = qq[k];
        keys[i] = interleave(qq[0], qq[1], qq[2]);
    }
}

/* ------------------------------------------------------------------------ */
/* Stable sort by key (bottom-up merge sort of (key, index) pairs)            */
/* ------------------------------------------------------------------------ */

void or_sort(const uint64_t* keys, int64_t n, int64_t* perm)
{
    int64_t* a = perm;
    int64_t* b = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) a[i] = i;
    int64_t* src = a;
    int64_t* dst = b;
    for (int64_t width = 1; width < n; width *= 2) {
        for (int64_t lo = 0; lo < n; lo += 2 * width) {
            int64_t mid = lo + width < n ? lo + width : n;
            int64_t hi = lo + 2 * width < n ? lo + 2 * width : n;
            int64_t i = lo, j = mid, k = lo;
            while (i < mid && j < hi) {
                /* take from the left run on ties: keeps original order */
                if (keys[src[j]] < keys[src[i]]) dst[k++] = src[j++];
                else dst[k++] = src[i++];
            }
            while (i < mid) dst[k++] = src[i++];
            while (j < hi) dst[k++] = src[j++];
        }
        int64_t* t = src; src = dst; dst = t;
    }
    if (src != a) memcpy(a, src, sizeof(int64_t) * (size_t)n);
    free(b);
}

/* ------------------------------------------------------------------------ */
/* The tree                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct or_tree {
    int64_t n;
    double lo[3];
    double L;
    int log2L;
    /* particles in sorted order */
    uint64_t* skey;
    int64_t* perm;   /* sorted position -> caller index */
    int64_t* spos;   /* caller index -> sorted position */
    double* sx;      /* [n,3] */
    double* sm;      /* [n]   */
    /* nodes in pre-order */
    int64_t nn, cap;
    int* level;
    int64_t* first;
    int64_t* count;
    int* nchild;
    int64_t* child;  /* [cap, 8] */
    int64_t* parent;
    double* com;     /* [cap, 3] */
    double* mass;    /* [cap] */
} or_tree;

static void grow(or_tree* T)
{
    int64_t c = T->cap ? 2 * T->cap : 1024;
    T->level = (int*)realloc(T->level, sizeof(int) * (size_t)c);
    T->first = (int64_t*)realloc(T->first, sizeof(int64_t) * (size_t)c);
    T->count = (int64_t*)realloc(T->count, sizeof(int64_t) * (size_t)c);
    T->nchild = (int*)realloc(T->nchild, sizeof(int) * (size_t)c);
    T->child = (int64_t*)realloc(T->child, sizeof(int64_t) * 8 * (size_t)c);
    T->parent = (int64_t*)realloc(T->parent, sizeof(int64_t) * (size_t)c);
    T->cap = c;
}

static int digit_at(uint64_t key, int level) /* level in 1..21 */
{
    return (int)((key >> (3 * (OR_MAXLEVEL - level))) & 7u);
}

/* Top-down construction: the cell (level, [b, e)) and its descendants,
 * emitted in pre-order. */
static int64_t build_rec(or_tree* T, int level, int64_t b, int64_t e, int64_t parent)
{
    if (T->nn == T->cap) grow(T);
    int64_t id = T->nn++;
    T->level[id] = level;
    T->first[id] = b;
    T->count[id] = e - b;
    T->nchild[id] = 0;
    T->parent[id] = parent;
    if (e - b == 1 || level == OR_MAXLEVEL) return id;
    int64_t i = b;
    while (i < e) {
        int d = digit_at(T->skey[i], level + 1);
        int64_t j = i;
        while (j < e && digit_at(T->skey[j], level + 1) == d) ++j;
        int64_t c = build_rec(T, level + 1, i, j, id);
        T->child[8 * id + T->nchild[id]] = c;
        T->nchild[id] += 1;
        i = j;
    }
    return id;
}

static int is_leaf(const or_tree* T, int64_t id) { return T->nchild[id] == 0; }

/* Centre of the geometric cell of node id (used only when its mass is 0). */
static void cell_centre(const or_tree* T, int64_t id, double c[3])
{
    /* corner = quantised coordinates of the first particle with the bits
     * below the node's level cleared */
    int64_t s = T->first[id];
    int l = T->level[id];
    double h = ldexp(T->L, -21);
    for (int k = 0; k < 3; ++k) {
        int64_t q = quantise(T->sx[3 * s + k], T->lo[k], T->log2L);
        int64_t span = (int64_t)1 << (OR_MAXLEVEL - l);
        int64_t corner = q - (q % span);
        c[k] = T->lo[k] + ((double)corner + 0.5 * (double)span) * h;
    }
}

/* Upward pass: total mass and centre of mass of every node. */
static void moments(or_tree* T)
{
    T->com = (double*)malloc(sizeof(double) * 3 * (size_t)(T->nn > 0 ? T->nn : 1));
    T->mass = (double*)malloc(sizeof(double) * (size_t)(T->nn > 0 ? T->nn : 1));
    /* children always have larger pre-order ids than their parent */
    for (int64_t id = T->nn - 1; id >= 0; --id) {
        double M = 0.0, S[3] = {0.0, 0.0, 0.0};
        if (is_leaf(T, id)) {
            int64_t b = T->first[id], e = b + T->count[id];
            if (e - b == 1) {
                T->mass[id] = T->sm[b];
                for (int k = 0; k < 3; ++k) T->com[3 * id + k] = T->sx[3 * b + k];
                continue;
            }
            for (int64_t j = b; j < e; ++j) {
                M += T->sm[j];
                for (int k = 0; k < 3; ++k) S[k] += T->sm[j] * T->sx[3 * j + k];
            }
        } else {
            for (int c = 0; c < T->nchild[id]; ++c) {
                int64_t ch = T->child[8 * id + c];
                M += T->mass[ch];
                for (int k = 0; k < 3; ++k) S[k] += T->mass[ch] * T->com[3 * ch + k];
            }
        }
        T->mass[id] = M;
        if (M == 0.0) {
            cell_centre(T, id, &T->com[3 * id]);
        } else {
            for (int k = 0; k < 3; ++k) T->com[3 * id + k] = S[k] / M;
        }
    }
}

void or_tree_free(or_tree* T)
{
    if (!T) return;
    free(T->skey); free(T->perm); free(T->spos); free(T->sx); free(T->sm);
    free(T->level); free(T->first); free(T->count); free(T->nchild);
    free(T->child); free(T->parent); free(T->com); free(T->mass);
    free(T);
}

/* Build the whole tree (root cube, keys, sort, topology, moments) for caller
 * positions pos[n,3] and masses m[n].  Returns NULL on non-finite input or a
 * negative mass. */
or_tree* or_tree_new(const double* pos, const double* m, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(m[i]) || m[i] < 0.0) return NULL;
    or_tree* T = (or_tree*)calloc(1, sizeof(or_tree));
    T->n = n;
    if (or_root_cube(pos, n, T->lo, &T->L, &T->log2L) != 0) { free(T); return NULL; }
    size_t nz = (size_t)(n > 0 ? n : 1);
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * nz);
    or_keys(pos, n, T->lo, T->log2L, NULL, keys);
    T->perm = (int64_t*)malloc(sizeof(int64_t) * nz);
    or_sort(keys, n, T->perm);
    T->skey = (uint64_t*)malloc(sizeof(uint64_t) * nz);
    T->spos = (int64_t*)malloc(sizeof(int64_t) * nz);
    T->sx = (double*)malloc(sizeof(double) * 3 * nz);
    T->sm = (double*)malloc(sizeof(double) * nz);
    for (int64_t s = 0; s < n; ++s) {
        int64_t i = T->perm[s];
        T->skey[s] = keys[i];
        T->spos[i] = s;
        for (int k = 0; k < 3; ++k) T->sx[3 * s + k] = pos[3 * i + k];
        T->sm[s] = m[i];
    }
    free(keys);
    if (n > 0) build_rec(T, 0, 0, n, -1);
    moments(T);
    return T;
}

int64_t or_tree_nnodes(const or_tree* T) { return T->nn; }

void or_tree_geometry(const or_tree* T, double lo[3], double* L, int* log2L)
{
    for (int k = 0; k < 3; ++k) lo[k] = T->lo[k];
    *L = T->L;
    *log2L = T->log2L;
}

/* Sorted keys and permutation (sorted position -> caller index). */
void or_tree_sorted(const or_tree* T, uint64_t* keys, int64_t* perm)
{
    for (int64_t s = 0; s < T->n; ++s) { keys[s] = T->skey[s]; perm[s] = T->perm[s]; }
}

/* Canonical node table in pre-order plus moments and links.
 * child: [nn, 8], -1 padded.  parent: -1 for the root. */
void or_tree_nodes(const or_tree* T, int32_t* level, int64_t* first, int64_t* count,
                   int32_t* nchild, int64_t* child, int64_t* parent,
                   double* com, double* mass)
{
    for (int64_t id = 0; id < T->nn; ++id) {
        level[id] = T->level[id];
        first[id] = T->first[id];
        count[id] = T->count[id];
        if (nchild) nchild[id] = T->nchild[id];
        if (child)
            for (int c = 0; c < 8; ++c)
                child[8 * id + c] = c < T->nchild[id] ? T->child[8 * id + c] : -1;
        if (parent) parent[id] = T->parent[id];
        if (com) for (int k = 0; k < 3; ++k) com[3 * id + k] = T->com[3 * id + k];
        if (mass) mass[id] = T->mass[id];
    }
}

/* ------------------------------------------------------------------------ */
/* The walk                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    double a[3];
    double phi;
    int64_t nint;
} acc_t;

/* One softened interaction with a source of mass mu at y, Eq.(1). */
static void term(acc_t* r, const double x[3], const double y[3], double mu, double eps2, double G)
{
    double d[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
    double q = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
    double inv = 1.0 / sqrt(q);
    double inv3 = inv * inv * inv;
    for (int k = 0; k < 3; ++k) r->a[k] += G * mu * d[k] * inv3;
    r->phi -= G * mu * inv;
    r->nint += 1;
}

typedef struct {
    const or_tree* T;
    double theta, eps2, G;
} walk_ctx;

static void walk_rec(const walk_ctx* C, int64_t id, int64_t si, const double x[3], acc_t* r)
{
    const or_tree* T = C->T;
    int64_t b = T->first[id], e = b + T->count[id];
    int contains = (si >= b && si < e);
    if (contains) {
        if (is_leaf(T, id)) {
            for (int64_t j = b; j < e; ++j)
                if (j != si) term(r, x, &T->sx[3 * j], T->sm[j], C->eps2, C->G);
        } else {
            for (int c = 0; c < T->nchild[id]; ++c) walk_rec(C, T->child[8 * id + c], si, x, r);
        }
        return;
    }
    const double* X = &T->com[3 * id];
    double d[3] = {X[0] - x[0], X[1] - x[1], X[2] - x[2]};
    double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double side = ldexp(T->L, -T->level[id]);
    if (C->theta > 0.0 && side < C->theta * dist) {
        term(r, x, X, T->mass[id], C->eps2, C->G);
    } else if (is_leaf(T, id)) {
        for (int64_t j = b; j < e; ++j) term(r, x, &T->sx[3 * j], T->sm[j], C->eps2, C->G);
    } else {
        for (int c = 0; c < T->nchild[id]; ++c) walk_rec(C, T->child[8 * id + c], si, x, r);
    }
}

/* ------------------------------------------------------------------------ */
/* A tiny thread pool over independent targets                                */
/* ------------------------------------------------------------------------ */

typedef void (*task_fn)(void* ctx, int64_t t);
typedef struct {
    task_fn fn;
    void* ctx;
    int64_t ntask;
    int64_t next;
    pthread_mutex_t mu;
} pool_t;

static void* pool_worker(void* arg)
{
    pool_t* P = (pool_t*)arg;
    const int64_t chunk = 16;
    for (;;) {
        pthread_mutex_lock(&P->mu);
        int64_t b = P->next;
        P->next += chunk;
        pthread_mutex_unlock(&P->mu);
        if (b >= P->ntask) break;
        int64_t e = b + chunk < P->ntask ? b + chunk : P->ntask;
        for (int64_t t = b; t < e; ++t) P->fn(P->ctx, t);
    }
    return NULL;
}

static void run_parallel(task_fn fn, void* ctx, int64_t ntask, int nthreads)
{
    pool_t P;
    P.fn = fn; P.ctx = ctx; P.ntask = ntask; P.next = 0;
    pthread_mutex_init(&P.mu, NULL);
    if (nthreads <= 1 || ntask < 64) {
        pool_worker(&P);
    } else {
        if (nthreads > 256) nthreads = 256;
        pthread_t th[256];
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, pool_worker, &P);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    pthread_mutex_destroy(&P.mu);
}

typedef struct {
    walk_ctx C;
    const int64_t* targets;   /* caller indices, or NULL = all */
    double* acc;
    double* pot;
    int64_t* nint;
} forces_job;

static void forces_task(void* p, int64_t t)
{
    forces_job* J = (forces_job*)p;
    const or_tree* T = J->C.T;
    int64_t i = J->targets ? J->targets[t] : t;
    int64_t si = T->spos[i];
    acc_t r;
    memset(&r, 0, sizeof r);
    if (T->nn > 0) walk_rec(&J->C, 0, si, &T->sx[3 * si], &r);
    for (int k = 0; k < 3; ++k) J->acc[3 * t + k] = r.a[k];
    if (J->pot) J->pot[t] = r.phi;
    if (J->nint) J->nint[t] = r.nint;
}

/* Barnes-Hut accelerations and potentials for nt targets (caller indices;
 * targets == NULL means all n in caller order).  Outputs are indexed by t. */
void or_tree_forces(const or_tree* T, double theta, double eps, double G,
                    const int64_t* targets, int64_t nt,
                    double* acc, double* pot, int64_t* nint, int nthreads)
{
    forces_job J;
    J.C.T = T; J.C.theta = theta; J.C.eps2 = eps * eps; J.C.G = G;
    J.targets = targets; J.acc = acc; J.pot = pot; J.nint = nint;
    run_parallel(forces_task, &J, nt, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Direct particle-particle summation, Eq.(1), the textbook O(N^2) sum        */
/* ------------------------------------------------------------------------ */

typedef struct {
    const double* pos;
    const double* m;
    int64_t n;
    double eps2, G;
    const int64_t* targets;
    double* acc;
    double* pot;
} direct_job;

static void direct_task(void* p, int64_t t)
{
    direct_job* J = (direct_job*)p;
    int64_t i = J->targets ? J->targets[t] : t;
    acc_t r;
    memset(&r, 0, sizeof r);
    for (int64_t j = 0; j < J->n; ++j)
        if (j != i) term(&r, &J->pos[3 * i], &J->pos[3 * j], J->m[j], J->eps2, J->G);
    for (int k = 0; k < 3; ++k) J->acc[3 * t + k] = r.a[k];
    if (J->pot) J->pot[t] = r.phi;
}

void or_direct(const double* pos, const double* m, int64_t n, double eps, double G,
               const int64_t* targets, int64_t nt, double* acc, double* pot, int nthreads)
{
    direct_job J;
    J.pos = pos; J.m = m; J.n = n; J.eps2 = eps * eps; J.G = G;
    J.targets = targets; J.acc = acc; J.pot = pot;
    run_parallel(direct_task, &J, nt, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Frozen interaction lists, the frozen-list evaluation and its adjoint      */
/* ------------------------------------------------------------------------ */
/*
 * With the tree's membership (which particles each node holds) and every
 * target's interaction set held fixed, the forces become a smooth function
 * F(x, m; lists): node moments are recomputed from (x, m) by the same
 * recursive definition, and each target sums Eq.(1) terms over its recorded
 * sources.  A source code >= 0 is a pre-order node (its monopole), a code
 * < 0 is the particle with sorted position -(code + 1) (a direct term).
 */

typedef struct {
    const or_tree* T;
    double theta;
    int64_t* cnt;      /* per target: number of sources */
    int64_t** codes;   /* per target: the sources in visit order */
    const int64_t* targets;
} lists_job;

static void push_code(int64_t** buf, int64_t* n, int64_t* cap, int64_t code)
{
    if (*n == *cap) {
        *cap = *cap ? 2 * *cap : 64;
        *buf = (int64_t*)realloc(*buf, sizeof(int64_t) * (size_t)*cap);
    }
    (*buf)[(*n)++] = code;
}

static void lists_rec(const or_tree* T, double theta, int64_t id, int64_t si, const double x[3],
                      int64_t** buf, int64_t* n, int64_t* cap)
{
    int64_t b = T->first[id], e = b + T->count[id];
    if (si >= b && si < e) {
        if (is_leaf(T, id)) {
            for (int64_t j = b; j < e; ++j)
                if (j != si) push_code(buf, n, cap, -(j + 1));
        } else {
            for (int c = 0; c < T->nchild[id]; ++c) lists_rec(T, theta, T->child[8 * id + c], si, x, buf, n, cap);
        }
        return;
    }
    const double* X = &T->com[3 * id];
    double d[3] = {X[0] - x[0], X[1] - x[1], X[2] - x[2]};
    double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double side = ldexp(T->L, -T->level[id]);
    if (theta > 0.0 && side < theta * dist) {
        push_code(buf, n, cap, id);
    } else if (is_leaf(T, id)) {
        for (int64_t j = b; j < e; ++j) push_code(buf, n, cap, -(j + 1));
    } else {
        for (int c = 0; c < T->nchild[id]; ++c) lists_rec(T, theta, T->child[8 * id + c], si, x, buf, n, cap);
    }
}

static void lists_task(void* p, int64_t t)
{
    lists_job* J = (lists_job*)p;
    const or_tree* T = J->T;
    int64_t i = J->targets ? J->targets[t] : t;
    int64_t si = T->spos[i];
    int64_t n = 0, cap = 0;
    int64_t* buf = NULL;
    if (T->nn > 0) lists_rec(T, J->theta, 0, si, &T->sx[3 * si], &buf, &n, &cap);
    J->cnt[t] = n;
    J->codes[t] = buf;
}

/* The interaction list of every particle (caller order) in CSR form:
 * *offsets [n+1] and *codes [offsets[n]], both malloc'd (free with
 * or_free). */
void or_tree_lists(const or_tree* T, double theta, int64_t** offsets, int64_t** codes, int nthreads)
{
    int64_t n = T->n;
    lists_job J;
    J.T = T; J.theta = theta; J.targets = NULL;
    J.cnt = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    J.codes = (int64_t**)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t*));
    run_parallel(lists_task, &J, n, nthreads);
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + J.cnt[i];
    int64_t* all = (int64_t*)malloc(sizeof(int64_t) * (size_t)(off[n] > 0 ? off[n] : 1));
    for (int64_t i = 0; i < n; ++i) {
        if (J.cnt[i]) memcpy(all + off[i], J.codes[i], sizeof(int64_t) * (size_t)J.cnt[i]);
        free(J.codes[i]);
    }
    free(J.cnt);
    free(J.codes);
    *offsets = off;
    *codes = all;
}

void or_free(void* p) { free(p); }

/* Node moments of the frozen tree for new particle data (caller order
 * pos[n,3], m[n]): same recursion as the build (children in octant order). */
static void frozen_moments(const or_tree* T, const double* pos, const double* m, double* sx, double* sm,
                           double* com, double* mass)
{
    for (int64_t s = 0; s < T->n; ++s) {
        int64_t i = T->perm[s];
        for (int k = 0; k < 3; ++k) sx[3 * s + k] = pos[3 * i + k];
        sm[s] = m[i];
    }
    for (int64_t id = T->nn - 1; id >= 0; --id) {
        double M = 0.0, S[3] = {0.0, 0.0, 0.0};
        if (is_leaf(T, id)) {
            int64_t b = T->first[id], e = b + T->count[id];
            if (e - b == 1) {
                mass[id] = sm[b];
                for (int k = 0; k < 3; ++k) com[3 * id + k] = sx[3 * b + k];
                continue;
            }
            for (int64_t j = b; j < e; ++j) {
                M += sm[j];
                for (int k = 0; k < 3; ++k) S[k] += sm[j] * sx[3 * j + k];
            }
        } else {
            for (int c = 0; c < T->nchild[id]; ++c) {
                int64_t ch = T->child[8 * id + c];
                M += mass[ch];
                for (int k = 0; k < 3; ++k) S[k] += mass[ch] * com[3 * ch + k];
            }
        }
        mass[id] = M;
        if (M == 0.0) {
            for (int k = 0; k < 3; ++k) com[3 * id + k] = T->com[3 * id + k];  /* cell centre, fixed */
        } else {
            for (int k = 0; k < 3; ++k) com[3 * id + k] = S[k] / M;
        }
    }
}

typedef struct {
    const or_tree* T;
    const double *sx, *sm, *com, *mass;
    const int64_t *offsets, *codes;
    double eps2, G;
    double* acc;
    double* pot;
} frozen_job;

/* one target's frozen list, summed in list order */
static void frozen_task(void* p, int64_t i)
{
    frozen_job* J = (frozen_job*)p;
    int64_t si = J->T->spos[i];
    acc_t r;
    memset(&r, 0, sizeof r);
    for (int64_t q = J->offsets[i]; q < J->offsets[i + 1]; ++q) {
        int64_t c = J->codes[q];
        if (c >= 0) term(&r, &J->sx[3 * si], &J->com[3 * c], J->mass[c], J->eps2, J->G);
        else term(&r, &J->sx[3 * si], &J->sx[3 * (-c - 1)], J->sm[-c - 1], J->eps2, J->G);
    }
    for (int k = 0; k < 3; ++k) J->acc[3 * i + k] = r.a[k];
    if (J->pot) J->pot[i] = r.phi;
}

/* F(x, m; lists): accelerations and potentials (caller order) with the tree
 * membership and the lists frozen.  Targets are independent: nthreads share
 * them, each target's sum is the same whatever the thread count. */
void or_frozen_forces(const or_tree* T, const double* pos, const double* m, const int64_t* offsets,
                      const int64_t* codes, double eps, double G, double* acc, double* pot, int nthreads)
{
    int64_t n = T->n, nn = T->nn;
    double* sx = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double* sm = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* com = (double*)malloc(sizeof(double) * 3 * (size_t)(nn > 0 ? nn : 1));
    double* mass = (double*)malloc(sizeof(double) * (size_t)(nn > 0 ? nn : 1));
    frozen_moments(T, pos, m, sx, sm, com, mass);
    frozen_job J;
    J.T = T; J.sx = sx; J.sm = sm; J.com = com; J.mass = mass;
    J.offsets = offsets; J.codes = codes; J.eps2 = eps * eps; J.G = G; J.acc = acc; J.pot = pot;
    run_parallel(frozen_task, &J, n, nthreads);
    free(sx); free(sm); free(com); free(mass);
}

/* Adjoint of F(x, m; lists).  Given g_acc = dL/da [n,3] and g_pot = dL/dphi
 * [n] (may be NULL), writes g_pos = dL/dx [n,3] and g_mass = dL/dm [n]
 * (caller order).  For one term with Delta = y - x_i, q = |Delta|^2 + eps^2,
 * T = q^-3/2 I - 3 q^-5/2 Delta Delta^T:
 *   da/dy = G mu T, da/dx_i = -G mu T, da/dmu = G Delta q^-3/2,
 *   dphi/dy = G mu Delta q^-3/2, dphi/dx_i = -G mu Delta q^-3/2, dphi/dmu = -G q^-1/2.
 * A node source carries dL/dX_n and dL/dM_n down to its particles through
 * M_n = sum m_j and X_n = sum m_j x_j / M_n: with u_n = (dL/dX_n) / M_n and
 * c_n = dL/dM_n - u_n . X_n, every particle j gets dL/dm_j += c_n + u_n . x_j
 * and dL/dx_j += m_j u_n, summed over the nodes that hold it (top-down
 * prefix sums).  A node of zero mass sits at its fixed cell centre: it has
 * u_n = 0. */
void or_frozen_adjoint(const or_tree* T, const int64_t* offsets, const int64_t* codes, double eps, double G,
                       const double* g_acc, const double* g_pot, double* g_pos, double* g_mass)
{
    int64_t n = T->n, nn = T->nn;
    double eps2 = eps * eps;
    double* gX = (double*)calloc((size_t)(3 * (nn > 0 ? nn : 1)), sizeof(double));
    double* gM = (double*)calloc((size_t)(nn > 0 ? nn : 1), sizeof(double));
    double* gx = (double*)calloc((size_t)(3 * (n > 0 ? n : 1)), sizeof(double));  /* sorted order */
    double* gm = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        int64_t si = T->spos[i];
        const double* x = &T->sx[3 * si];
        const double* g = &g_acc[3 * i];
        double h = g_pot ? g_pot[i] : 0.0;
        for (int64_t q = offsets[i]; q < offsets[i + 1]; ++q) {
            int64_t c = codes[q];
            const double* y;
            double mu;
            if (c >= 0) { y = &T->com[3 * c]; mu = T->mass[c]; }
            else { y = &T->sx[3 * (-c - 1)]; mu = T->sm[-c - 1]; }
            double d[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
            double qq = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
            double inv = 1.0 / sqrt(qq);
            double inv3 = inv * inv * inv;
            double inv5 = inv3 * inv * inv;
            double dg = d[0] * g[0] + d[1] * g[1] + d[2] * g[2];
            double gy[3], gmu;
            for (int k = 0; k < 3; ++k) gy[k] = G * mu * (inv3 * g[k] - 3.0 * inv5 * d[k] * dg + inv3 * d[k] * h);
            gmu = G * (dg * inv3 - h * inv);
            for (int k = 0; k < 3; ++k) gx[3 * si + k] -= gy[k];
            if (c >= 0) {
                for (int k = 0; k < 3; ++k) gX[3 * c + k] += gy[k];
                gM[c] += gmu;
            } else {
                int64_t j = -c - 1;
                for (int k = 0; k < 3; ++k) gx[3 * j + k] += gy[k];
                gm[j] += gmu;
            }
        }
    }
    /* top-down: prefix sums of u and c along every root-to-leaf path */
    double* U = (double*)calloc((size_t)(3 * (nn > 0 ? nn : 1)), sizeof(double));
    double* C = (double*)calloc((size_t)(nn > 0 ? nn : 1), sizeof(double));
    for (int64_t id = 0; id < nn; ++id) {           /* parents precede children */
        double u[3] = {0.0, 0.0, 0.0}, cc;
        double M = T->mass[id];
        if (M != 0.0)
            for (int k = 0; k < 3; ++k) u[k] = gX[3 * id + k] / M;
        cc = gM[id] - (u[0] * T->com[3 * id] + u[1] * T->com[3 * id + 1] + u[2] * T->com[3 * id + 2]);
        int64_t p = T->parent[id];
        for (int k = 0; k < 3; ++k) U[3 * id + k] = (p >= 0 ? U[3 * p + k] : 0.0) + u[k];
        C[id] = (p >= 0 ? C[p] : 0.0) + cc;
        if (is_leaf(T, id)) {
            for (int64_t j = T->first[id]; j < T->first[id] + T->count[id]; ++j) {
                const double* xj = &T->sx[3 * j];
                gm[j] += C[id] + U[3 * id] * xj[0] + U[3 * id + 1] * xj[1] + U[3 * id + 2] * xj[2];
                for (int k = 0; k < 3; ++k) gx[3 * j + k] += T->sm[j] * U[3 * id + k];
            }
        }
    }
    for (int64_t s = 0; s < n; ++s) {
        int64_t i = T->perm[s];
        for (int k = 0; k < 3; ++k) g_pos[3 * i + k] = gx[3 * s + k];
        g_mass[i] = gm[s];
    }
    free(gX); free(gM); free(gx); free(gm); free(U); free(C);
}

/* ------------------------------------------------------------------------ */
/* Kick-drift-kick leapfrog, Eqs.(2)-(5)                                      */
/* ------------------------------------------------------------------------ */

/* One step on caller-order arrays (updated in place): v += tau/2 a;
 * x += tau v; a = Barnes-Hut forces of a tree rebuilt at the new x;
 * v += tau/2 a.  pot (may be NULL) receives the new potentials.  Returns 0,
 * or -1 if the rebuilt tree is rejected (non-finite position). */
int or_leapfrog_step(double* pos, double* vel, const double* m, double* acc, double* pot, int64_t n,
                     double tau, double theta, double eps, double G, int nthreads)
{
    for (int64_t i = 0; i < 3 * n; ++i) vel[i] += 0.5 * tau * acc[i];
    for (int64_t i = 0; i < 3 * n; ++i) pos[i] += tau * vel[i];
    or_tree* T = or_tree_new(pos, m, n);
    if (!T) return -1;
    or_tree_forces(T, theta, eps, G, NULL, n, acc, pot, NULL, nthreads);
    or_tree_free(T);
    for (int64_t i = 0; i < 3 * n; ++i) vel[i] += 0.5 * tau * acc[i];
    return 0;
}
