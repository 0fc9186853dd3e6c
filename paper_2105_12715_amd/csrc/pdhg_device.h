// Device helpers shared by the HIP translation units of the library.
#pragma once

#include "pdhg_internal.h"

namespace pdhg {

// ---------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sums of K values; result valid in thread 0.
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double *sh) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sh[w * K + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i * K + k];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Sum partials[b*stride + k] over b in [0, nb) in a fixed order; thread 0.
template <int K>
__device__ __forceinline__ void reduce_partials(const double *part, int nb, int stride,
                                                double (&out)[K], double *sh) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = 0.0;
    for (int bb = threadIdx.x; bb < nb; bb += blockDim.x) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] += part[(size_t)bb * stride + k];
    }
    block_sums<K>(out, sh);
}

__host__ __device__ inline int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }

}  // namespace pdhg
