// Small reductions after the walk: the FP64 momentum diagnostic
// (sum_i m_i a_i and sum_i m_i |a_i|, from one partial per wave, summed in a
// fixed order so the result is reproducible) and interaction-count totals.
#include "tc_internal.h"

namespace tc {
namespace {

constexpr int kDiagThreads = 256;

// Sum of rows [b*chunk, (b+1)*chunk) of a [nw, 4] array into out[b, 4], in a
// fixed order (thread-strided partial sums, then a fixed tree).
__global__ __launch_bounds__(kDiagThreads) void k_diag_reduce(const double* __restrict__ part, int64_t nw,
                                                              int64_t chunk, double* __restrict__ out)
{
    __shared__ double red[4][kDiagThreads];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t b0 = (int64_t)blockIdx.x * chunk;
    const int64_t b1 = b0 + chunk < nw ? b0 + chunk : nw;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kDiagThreads)
        for (int k = 0; k < 4; ++k) v[k] += part[4 * i + k];
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = kDiagThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) out[4 * blockIdx.x + k] = red[k][0];
}

__global__ __launch_bounds__(256) void k_sum_counts(const uint32_t* __restrict__ c, int64_t n,
                                                    unsigned long long* __restrict__ out)
{
    unsigned long long v = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) v += c[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, v);
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_scatter_counts(const uint32_t* __restrict__ sc,
                                                        const uint32_t* __restrict__ perm, int64_t n,
                                                        uint32_t* __restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) out[perm[s]] = sc[s];
}

}  // namespace

constexpr int64_t kDiagChunk = 2048;

size_t diag_temp_bytes(int64_t nwaves)
{
    int64_t nb = (nwaves + kDiagChunk - 1) / kDiagChunk;
    return (size_t)(nb + 1) * 4 * sizeof(double);
}

void launch_diag_final(const double* part, int64_t nwaves, void* temp, double* out4, hipStream_t s)
{
    int64_t nb = (nwaves + kDiagChunk - 1) / kDiagChunk;
    if (nb < 1) nb = 1;
    double* mid = (double*)temp;
    k_diag_reduce<<<(unsigned)nb, kDiagThreads, 0, s>>>(part, nwaves, kDiagChunk, mid);
    k_diag_reduce<<<1, kDiagThreads, 0, s>>>(mid, nb, nb, out4);
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0) return;
    k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
}

void launch_sum_counts(const uint32_t* counts, int64_t n, unsigned long long* out, hipStream_t s)
{
    launch_fill_u32((uint32_t*)out, 2, 0u, s);
    if (n == 0) return;
    int64_t b = (n + 255) / 256;
    if (b > 2048) b = 2048;
    k_sum_counts<<<(unsigned)b, 256, 0, s>>>(counts, n, out);
}

void launch_scatter_counts(const uint32_t* sorted_counts, const uint32_t* perm, int64_t n, uint32_t* out,
                           hipStream_t s)
{
    if (n == 0) return;
    k_scatter_counts<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(sorted_counts, perm, n, out);
}

}  // namespace tc
