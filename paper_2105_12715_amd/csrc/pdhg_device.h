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

// ---------------------------------------------------------------------
// SpMV core
// ---------------------------------------------------------------------
// LDS of one SpMV block: the staged products and the block's row starts
// relative to its first entry (at most kLdsProducts, so 16 bits suffice).
struct SpmvShared {
    double prod[kLdsProducts];
    unsigned short rows[kUnits + 1];
};
constexpr int kPerThread = kLdsProducts / kWG;

// matrix loads: non-temporal unless built with PDHG_MATRIX_TEMPORAL
template <class T>
__device__ __forceinline__ T ld_matrix(const T *p) {
#ifdef PDHG_MATRIX_TEMPORAL
    return *p;
#else
    return __builtin_nontemporal_load(p);
#endif
}

template <class Epi>
__device__ __forceinline__ void spmv_rows(const int *__restrict__ rp, const int *__restrict__ ci,
                                          const double *__restrict__ v,
                                          const double *__restrict__ xin, int r0, int r1,
                                          const Epi &epi, SpmvShared &sm) {
    const int tid = threadIdx.x;
    const int p0 = rp[r0], p1 = rp[r1];
    const int nb = p1 - p0;
    const int R = r1 - r0;  // <= kUnits: every row start takes one unit of the block
    if (nb <= kLdsProducts) {
        // Every global load of a thread is issued before the first is used:
        // row starts and matrix entries together, then all gathers, so one
        // block waits on three memory round trips instead of one per entry.
        // The matrix is read once per launch: non-temporal loads keep it
        // from evicting the gathered vector from L2 and the MALL.
        for (int i = tid; i <= R; i += kWG) sm.rows[i] = (unsigned short)(rp[r0 + i] - p0);
        int col[kPerThread];
        double val[kPerThread], g[kPerThread];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int e = tid + k * kWG;
            if (e < nb) {
                col[k] = ld_matrix(ci + p0 + e);
                val[k] = ld_matrix(v + p0 + e);
            }
        }
#pragma unroll
        for (int k = 0; k < kPerThread; ++k)
            if (tid + k * kWG < nb) g[k] = xin[col[k]];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int e = tid + k * kWG;
            if (e < nb) sm.prod[e] = val[k] * g[k];
        }
        __syncthreads();
        const int avg = nb / R;
        int L = 1;
        while (L < 64 && 2 * L <= avg) L <<= 1;
        const int G = kWG / L;
        const int lane = tid & (L - 1), grp = tid / L;
        // A group reduces at most kLdsProducts / kWG rows: L = 1 when the
        // mean row length avg = nb / R is below 2 (and R <= kUnits), else
        // L <= avg, so R L <= nb <= kLdsProducts and R / G = R L / kWG.
        constexpr int kRounds = kLdsProducts / kWG;
        double mine[kRounds];
#pragma unroll
        for (int t = 0; t < kRounds; ++t) {
            const int rr = grp + t * G;
            if (rr < R) {
                const int s0 = sm.rows[rr], s1 = sm.rows[rr + 1];
                double s = 0.0;
                for (int e = s0 + lane; e < s1; e += L) s += sm.prod[e];
                for (int off = L >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
                mine[t] = s;
            }
        }
        // row sums back to LDS, then the epilogue on consecutive rows with
        // every lane active, so its loads and stores are coalesced and in
        // flight together
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int t = 0; t < kRounds; ++t)
                if (grp + t * G < R) sm.prod[grp + t * G] = mine[t];
        }
        __syncthreads();
        for (int rr = tid; rr < R; rr += kWG) epi(r0 + rr, sm.prod[rr]);
    } else {
        const int wave = tid >> 6, lane = tid & 63;
        for (int row = r0 + wave; row < r1; row += kWG / 64) {
            double s = 0.0;
            for (int p = rp[row] + lane; p < rp[row + 1]; p += 64)
                s += ld_matrix(v + p) * xin[ld_matrix(ci + p)];
            s = wave_sum(s);
            if (lane == 0) epi(row, s);
        }
    }
}

template <class Epi>
__global__ __launch_bounds__(kWG) void k_spmv(const int *__restrict__ rp,
                                              const int *__restrict__ ci,
                                              const double *__restrict__ v,
                                              const double *__restrict__ xin,
                                              const int *__restrict__ br, Epi epi,
                                              const int *skip) {
    if (skip && *skip) return;
    __shared__ SpmvShared lds;
    const int r0 = br[blockIdx.x], r1 = br[blockIdx.x + 1];
    if (r0 >= r1) return;
    spmv_rows(rp, ci, v, xin, r0, r1, epi, lds);
}

struct EpiStore {
    double *out;
    __device__ __forceinline__ void operator()(int r, double s) const { out[r] = s; }
};

// bit position of the radix digit of level 0..5 (11-bit digits, last 8)
__host__ __device__ constexpr int shift_of(int level) { return level >= 5 ? 0 : 52 - 11 * level; }

__device__ __forceinline__ unsigned long long key_of(double a, double d) {
    return (unsigned long long)__double_as_longlong(d / a);
}

__device__ __forceinline__ bool bad_pair(double a, double d) {
    return a != a || d != d || a < 0.0 || d < 0.0 || a == INFINITY;
}

// deterministic exclusive prefix (from the left) and suffix (from the right)
// of one double per thread
__device__ double block_excl_prefix(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kWG; off <<= 1) {
        double o = t >= off ? sh[t - off] : 0.0;
        __syncthreads();
        sh[t] += o;
        __syncthreads();
    }
    double r = t ? sh[t - 1] : 0.0;
    __syncthreads();
    return r;
}

__device__ double block_excl_suffix(double v, double *sh) {
    const int p = kWG - 1 - threadIdx.x;
    sh[p] = v;
    __syncthreads();
    for (int off = 1; off < kWG; off <<= 1) {
        double o = p >= off ? sh[p - off] : 0.0;
        __syncthreads();
        sh[p] += o;
        __syncthreads();
    }
    double r = p ? sh[p - 1] : 0.0;
    __syncthreads();
    return r;
}

struct ChooseShared {
    double pre[kWG];
    int best;
};

// Move the bracket to the last bucket b (of nbuck at bit position `shift`)
// whose lower end lambda_b keeps
//   f(lambda_b) = F_acc + sum_{b'<b} D[b'] + lambda_b^2 (A_acc + sum_{b'>=b} A[b'])
// at most r^2.  ts lives in LDS; called by the whole workgroup.
__device__ void choose_bucket(TRState &ts, const unsigned int *cnt, const double *D,
                              const double *A, int nbuck, int level, ChooseShared &cs) {
    const int shift = shift_of(level);
    constexpr int per = kBuckets / kWG;
    const int tid = threadIdx.x;
    const int b0 = tid * per;
    double dl[per], al[per];
    unsigned int cl[per];
    double Dt = 0.0, At = 0.0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        const int b = b0 + k;
        if (b < nbuck) {
            dl[k] = D[b];
            al[k] = A[b];
            cl[k] = cnt[b];
        } else {
            dl[k] = 0.0;
            al[k] = 0.0;
            cl[k] = 0u;
        }
        Dt += dl[k];
        At += al[k];
    }
    const double Dpre = block_excl_prefix(Dt, cs.pre);
    const double Asuf = block_excl_suffix(At, cs.pre);
    double asuf_in[per];
    double acc = Asuf;
#pragma unroll
    for (int k = per - 1; k >= 0; --k) {
        acc += al[k];
        asuf_in[k] = acc;
    }
    if (tid == 0) cs.best = -1;
    __syncthreads();
    const double F0 = ts.F_acc, A0 = ts.A_acc, r2 = ts.r2;
    const unsigned long long prefix = ts.prefix;
    double dacc = Dpre;
    int best = -1;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        const int b = b0 + k;
        if (b < nbuck) {
            const double lam =
                __longlong_as_double((long long)(prefix | ((unsigned long long)b << shift)));
            const double f = F0 + dacc + lam * lam * (A0 + asuf_in[k]);
            if (f <= r2) best = b;
        }
        dacc += dl[k];
    }
    if (best >= 0) atomicMax(&cs.best, best);
    __syncthreads();
    int bb = cs.best;
    if (bb < 0) bb = 0;  // the bracket's own lower end (f <= r^2 up to rounding)
    if (bb / per == tid) {
        const int k = bb - b0;
        double dpre = Dpre;
        for (int q = 0; q < k; ++q) dpre += dl[q];
        const double aex = (k + 1 < per) ? asuf_in[k + 1] : Asuf;
        ts.F_acc = F0 + dpre;
        ts.A_acc = A0 + aex;
        ts.klo = prefix | ((unsigned long long)bb << shift);
        ts.prefix = ts.klo;
        ts.count = cl[k];
        if (ts.count == 0u || level == 5) ts.mode = TR_RESOLVED;
        else ts.level = level + 1;
    }
    __syncthreads();
}

}  // namespace pdhg
