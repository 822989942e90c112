// Root cube, 63-bit Morton keys and the gather of particles into key order.
//
// The octree of the TreeCode method (section 2: recursive split into eight
// octants) is built from the particles sorted along a Morton curve.  The
// root cube is lo_k = min_i x_ik with side L = the smallest power of two not
// below the largest extent; every coordinate is quantised to 21 bits with an
// exact power-of-two scale, so the keys are bit-reproducible:
//   q_k = min(2^21 - 1, floor((x_k - lo_k) * 2^21 / L)),
//   key = interleave(q_x, q_y, q_z), x bit highest in every triple.
// All arithmetic here is FP64 (FP32 inputs are widened exactly) with no FMA
// contraction (the library is compiled with -ffp-contract=off).
#include <float.h>
#include <math.h>

#include "tc_internal.h"

namespace tc {
namespace {

constexpr int kBoundsThreads = 256;

template <typename T>
__global__ __launch_bounds__(kBoundsThreads) void k_bounds_partial(const T* __restrict__ pos,
                                                                   const T* __restrict__ mass,
                                                                   int64_t n,
                                                                   double* __restrict__ part)
{
    double mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX};
    double mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    uint32_t bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double x = (double)pos[3 * i + k];
            if (!isfinite(x)) {
                bad |= 1u;
            } else {
                mn[k] = fmin(mn[k], x);
                mx[k] = fmax(mx[k], x);
            }
        }
        double m = (double)mass[i];
        if (!(m >= 0.0) || !isfinite(m)) bad |= 2u;
    }
    __shared__ double red[6][kBoundsThreads];
    __shared__ uint32_t redbad[kBoundsThreads];
    for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = mn[k];
        red[3 + k][threadIdx.x] = mx[k];
    }
    redbad[threadIdx.x] = bad;
    __syncthreads();
    for (int o = kBoundsThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            for (int k = 0; k < 3; ++k) {
                red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + o]);
                red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + o]);
            }
            redbad[threadIdx.x] |= redbad[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < 6; ++k) part[8 * blockIdx.x + k] = red[k][0];
        part[8 * blockIdx.x + 6] = (double)redbad[0];
        part[8 * blockIdx.x + 7] = 0.0;
    }
}

__global__ __launch_bounds__(kBoundsThreads) void k_bounds_final(const double* __restrict__ part,
                                                                 int nblocks, int64_t n,
                                                                 Geom* __restrict__ g)
{
    __shared__ double red[6][kBoundsThreads];
    __shared__ uint32_t redbad[kBoundsThreads];
    double mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX};
    double mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    uint32_t bad = 0;
    for (int b = threadIdx.x; b < nblocks; b += kBoundsThreads) {
        for (int k = 0; k < 3; ++k) {
            mn[k] = fmin(mn[k], part[8 * b + k]);
            mx[k] = fmax(mx[k], part[8 * b + 3 + k]);
        }
        bad |= (uint32_t)part[8 * b + 6];
    }
    for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = mn[k];
        red[3 + k][threadIdx.x] = mx[k];
    }
    redbad[threadIdx.x] = bad;
    __syncthreads();
    for (int o = kBoundsThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            for (int k = 0; k < 3; ++k) {
                red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + o]);
                red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + o]);
            }
            redbad[threadIdx.x] |= redbad[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double E = 0.0;
    for (int k = 0; k < 3; ++k) {
        double lo = n > 0 ? red[k][0] : 0.0;
        double hi = n > 0 ? red[3 + k][0] : 0.0;
        g->lo[k] = lo;
        double ext = hi - lo;
        if (ext > E) E = ext;
    }
    uint32_t b = redbad[0];
    int eL = 0;
    if (!isfinite(E)) {
        b |= 1u;
    } else if (E > 0.0) {
        // E = f 2^e, f in [0.5, 1): a power of two iff f == 0.5
        int e;
        double f = frexp(E, &e);
        eL = (f == 0.5) ? e - 1 : e;
    }
    g->log2L = eL;
    g->L = ldexp(1.0, eL);
    g->scale = ldexp(1.0, 21 - eL);
    g->h = ldexp(1.0, eL - 21);
    g->bad = b;
    g->nnodes = 0;
}

// Spread the low 21 bits of v so that bit b lands on bit 3b.
__device__ inline uint64_t spread3(uint64_t v)
{
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x001F00000000FFFFull;
    v = (v | (v << 16)) & 0x001F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ inline uint64_t quantise(double x, double lo, double scale)
{
    double f = floor((x - lo) * scale);
    if (!(f >= 0.0)) f = 0.0;
    if (f > (double)kQMax) return kQMax;
    return (uint64_t)f;
}

// Packed particle record {x, y, z, m} in caller order, so that the gather
// after the sort reads one aligned record per particle instead of four
// scattered scalars.
template <typename T> struct Rec;
template <> struct Rec<float> {
    __device__ static void put(float* r, int64_t i, float x, float y, float z, float m)
    {
        reinterpret_cast<float4*>(r)[i] = make_float4(x, y, z, m);
    }
    __device__ static void get(const float* r, int64_t i, double& x, double& y, double& z, double& m)
    {
        const float4 v = reinterpret_cast<const float4*>(r)[i];
        x = v.x; y = v.y; z = v.z; m = v.w;
    }
};
template <> struct Rec<double> {
    __device__ static void put(double* r, int64_t i, double x, double y, double z, double m)
    {
        reinterpret_cast<double2*>(r)[2 * i] = make_double2(x, y);
        reinterpret_cast<double2*>(r)[2 * i + 1] = make_double2(z, m);
    }
    __device__ static void get(const double* r, int64_t i, double& x, double& y, double& z, double& m)
    {
        const double2 a = reinterpret_cast<const double2*>(r)[2 * i];
        const double2 b = reinterpret_cast<const double2*>(r)[2 * i + 1];
        x = a.x; y = a.y; z = b.x; m = b.y;
    }
};

template <typename T>
__global__ __launch_bounds__(256) void k_keys(const T* __restrict__ pos, const T* __restrict__ mass, int64_t n,
                                              const Geom* __restrict__ g,
                                              uint64_t* __restrict__ keys,
                                              uint32_t* __restrict__ idx, T* __restrict__ rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double sc = g->scale;
    const T x = pos[3 * i + 0], y = pos[3 * i + 1], z = pos[3 * i + 2];
    uint64_t qx = quantise((double)x, g->lo[0], sc);
    uint64_t qy = quantise((double)y, g->lo[1], sc);
    uint64_t qz = quantise((double)z, g->lo[2], sc);
    keys[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    idx[i] = (uint32_t)i;
    Rec<T>::put(rec, i, x, y, z, mass[i]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather(const T* __restrict__ rec, int64_t n,
                                                const uint32_t* __restrict__ perm, Particle* __restrict__ sp)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    double x, y, z, m;
    Rec<T>::get(rec, perm[s], x, y, z, m);
    double2* o = reinterpret_cast<double2*>(sp + s);
    o[0] = make_double2(x, y);
    o[1] = make_double2(z, m);
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

int bounds_blocks(int64_t n)
{
    int64_t b = (n + kBoundsThreads * 8 - 1) / (kBoundsThreads * 8);
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

void launch_bounds(const void* pos, const void* mass, int64_t n, tc_dtype dt, double* partials,
                   int nblocks, Geom* geom, hipStream_t s)
{
    if (dt == TC_F32)
        k_bounds_partial<float><<<nblocks, kBoundsThreads, 0, s>>>((const float*)pos, (const float*)mass,
                                                                   n, partials);
    else
        k_bounds_partial<double><<<nblocks, kBoundsThreads, 0, s>>>((const double*)pos,
                                                                    (const double*)mass, n, partials);
    k_bounds_final<<<1, kBoundsThreads, 0, s>>>(partials, nblocks, n, geom);
}

size_t record_bytes(int64_t n, tc_dtype dt) { return (size_t)n * 4 * (dt == TC_F32 ? sizeof(float) : sizeof(double)); }

void launch_keys(const void* pos, const void* mass, int64_t n, tc_dtype dt, const Geom* geom, uint64_t* keys,
                 uint32_t* idx, void* rec, hipStream_t s)
{
    if (n == 0) return;
    if (dt == TC_F32)
        k_keys<float><<<grid_for(n, 256), 256, 0, s>>>((const float*)pos, (const float*)mass, n, geom, keys, idx,
                                                       (float*)rec);
    else
        k_keys<double><<<grid_for(n, 256), 256, 0, s>>>((const double*)pos, (const double*)mass, n, geom, keys,
                                                        idx, (double*)rec);
}

void launch_gather(const void* rec, int64_t n, tc_dtype dt, const uint32_t* perm, Particle* sp, hipStream_t s)
{
    if (n == 0) return;
    if (dt == TC_F32)
        k_gather<float><<<grid_for(n, 256), 256, 0, s>>>((const float*)rec, n, perm, sp);
    else
        k_gather<double><<<grid_for(n, 256), 256, 0, s>>>((const double*)rec, n, perm, sp);
}

}  // namespace tc
