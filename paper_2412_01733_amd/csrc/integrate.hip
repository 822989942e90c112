// Kick-drift-kick leapfrog pieces (Eqs.(2)-(5)) and the FP64 step
// diagnostics.  The first kick and the drift are fused:
//   v^{n+1/2} = v^n + tau/2 a^n,   x^{n+1} = x^n + tau v^{n+1/2}   (Eqs.(2), (3));
// the second kick, v^{n+1} = v^{n+1/2} + tau/2 a^{n+1} (Eq.(5)), follows the
// force evaluation of Eq.(4).  Positions and velocities keep the caller's
// precision; accelerations come in the walk's precision.
#include "tc_internal.h"

namespace tc {
namespace {

template <typename T, typename A>
__global__ __launch_bounds__(256) void k_kick_drift(T* __restrict__ pos, T* __restrict__ vel,
                                                    const A* __restrict__ acc, int64_t n3, double tau)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const double v = (double)vel[i] + 0.5 * tau * (double)acc[i];
    const T vt = (T)v;
    vel[i] = vt;
    pos[i] = (T)((double)pos[i] + tau * (double)vt);
}

template <typename T, typename A>
__global__ __launch_bounds__(256) void k_kick(T* __restrict__ vel, const A* __restrict__ acc, int64_t n3, double tau)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    vel[i] = (T)((double)vel[i] + 0.5 * tau * (double)acc[i]);
}

constexpr int kRows = 10;  // KE, PE, P (3), L (3), mass, unused

// Per-block FP64 partial sums, fixed order: KE = sum m v^2 / 2,
// PE = sum m phi / 2, P = sum m v, L = sum m x cross v, M = sum m.
template <typename T, typename A>
__global__ __launch_bounds__(256) void k_step_diag(const T* __restrict__ pos, const T* __restrict__ vel,
                                                   const T* __restrict__ mass, const A* __restrict__ pot, int64_t n,
                                                   double* __restrict__ part)
{
    __shared__ double red[kRows][256];
    double v[kRows] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double m = (double)mass[i];
        const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
        const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
        v[0] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
        if (pot) v[1] += 0.5 * m * (double)pot[i];
        v[2] += m * vx;
        v[3] += m * vy;
        v[4] += m * vz;
        v[5] += m * (y * vz - z * vy);
        v[6] += m * (z * vx - x * vz);
        v[7] += m * (x * vy - y * vx);
        v[8] += m;
    }
    for (int k = 0; k < kRows; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < kRows; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < kRows; ++k) part[kRows * blockIdx.x + k] = red[k][0];
}

__global__ __launch_bounds__(64) void k_rows_final(const double* __restrict__ part, int nb, double* __restrict__ out)
{
    if (threadIdx.x >= kRows) return;
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part[kRows * b + threadIdx.x];
    out[threadIdx.x] = t;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_kick_drift(void* pos, void* vel, const void* acc, int64_t n, tc_dtype dt, bool acc64, double tau,
                       hipStream_t s)
{
    const int64_t n3 = 3 * n;
    if (n3 == 0) return;
    if (dt == TC_F32) {
        if (acc64) k_kick_drift<float, double><<<grid_for(n3), 256, 0, s>>>((float*)pos, (float*)vel, (const double*)acc, n3, tau);
        else k_kick_drift<float, float><<<grid_for(n3), 256, 0, s>>>((float*)pos, (float*)vel, (const float*)acc, n3, tau);
    } else {
        if (acc64) k_kick_drift<double, double><<<grid_for(n3), 256, 0, s>>>((double*)pos, (double*)vel, (const double*)acc, n3, tau);
        else k_kick_drift<double, float><<<grid_for(n3), 256, 0, s>>>((double*)pos, (double*)vel, (const float*)acc, n3, tau);
    }
}

void launch_kick(void* vel, const void* acc, int64_t n, tc_dtype dt, bool acc64, double tau, hipStream_t s)
{
    const int64_t n3 = 3 * n;
    if (n3 == 0) return;
    if (dt == TC_F32) {
        if (acc64) k_kick<float, double><<<grid_for(n3), 256, 0, s>>>((float*)vel, (const double*)acc, n3, tau);
        else k_kick<float, float><<<grid_for(n3), 256, 0, s>>>((float*)vel, (const float*)acc, n3, tau);
    } else {
        if (acc64) k_kick<double, double><<<grid_for(n3), 256, 0, s>>>((double*)vel, (const double*)acc, n3, tau);
        else k_kick<double, float><<<grid_for(n3), 256, 0, s>>>((double*)vel, (const float*)acc, n3, tau);
    }
}

size_t step_diag_temp_bytes() { return (size_t)1024 * kRows * sizeof(double); }

void launch_step_diag(const void* pos, const void* vel, const void* mass, const void* pot, int64_t n, tc_dtype dt,
                      bool pot64, void* temp, double* out10, hipStream_t s)
{
    int64_t nb = (n + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    double* part = (double*)temp;
    if (dt == TC_F32) {
        if (pot64) k_step_diag<float, double><<<(unsigned)nb, 256, 0, s>>>((const float*)pos, (const float*)vel, (const float*)mass, (const double*)pot, n, part);
        else k_step_diag<float, float><<<(unsigned)nb, 256, 0, s>>>((const float*)pos, (const float*)vel, (const float*)mass, (const float*)pot, n, part);
    } else {
        if (pot64) k_step_diag<double, double><<<(unsigned)nb, 256, 0, s>>>((const double*)pos, (const double*)vel, (const double*)mass, (const double*)pot, n, part);
        else k_step_diag<double, float><<<(unsigned)nb, 256, 0, s>>>((const double*)pos, (const double*)vel, (const double*)mass, (const float*)pot, n, part);
    }
    k_rows_final<<<1, 64, 0, s>>>(part, (int)nb, out10);
}

}  // namespace tc
