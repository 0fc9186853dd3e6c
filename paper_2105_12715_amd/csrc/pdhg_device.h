// Device helpers shared by the HIP translation units of the library.
#pragma once

#include "pdhg_internal.h"

namespace pdhg {

// ---------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------
// a double from another lane of the same row of 16 (DPP lane pattern CTRL);
// a source lane outside the row or switched off gives 0
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over a whole wave (every lane active), the same value in every lane
// and a fixed order: a butterfly inside each row of 16 lanes (DPP quad
// permutations for lane ^ 1 and lane ^ 2; once the lanes of each quad
// agree, the mirrors inside 8 and 16 lanes pair each quad with the other
// of its half and each half with the other), then the four row sums.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Deterministic block sums of K <= 64 values over a workgroup of NW full
// waves (sh holds NW * K doubles): lane k of wave 0 adds the wave sums of
// value k in wave order; result valid in wave 0 (so in thread 0).
template <int K, int NW = kWG / 64>
__device__ __forceinline__ void block_sums(double (&v)[K], double *sh) {
    static_assert(K <= 64, "one lane per value");
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sh[w * K + k] = v[k];
    }
    __syncthreads();
    if (w == 0) {
        double s = 0.0;
        if (lane < K) {
#pragma unroll
            for (int i = 0; i < NW; ++i) s += sh[i * K + lane];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = lane_f64(s, k);
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

// One chunk of a block's staging: row starts [rbase, rbase + KR WG) and
// entries [ebase, ebase + K WG) (clipped to the block), every slot loading
// from a clamped address so that the loads of a thread form one straight
// run: the compiler's wait counts then keep them all in flight (a branch per
// slot made it wait for each load before issuing the next).  Loads are
// issued row starts first, then column indices, then values, then gathers.
template <int WG, int K, int KR, class Idx, bool PK>
__device__ __forceinline__ void spmv_stage(const int *__restrict__ rp, const Idx *__restrict__ ci,
                                           const double *__restrict__ v,
                                           const double *__restrict__ xin, int r0, int R, int p0,
                                           int nb, int rbase, int ebase, SpmvShared &sm) {
    const int tid = threadIdx.x;
    int rw[KR], col[K];
    double val[K], g[K];
#pragma unroll
    for (int k = 0; k < KR; ++k) rw[k] = rp[r0 + min(rbase + tid + k * WG, R)];
#pragma unroll
    for (int k = 0; k < K; ++k) col[k] = (int)ld_matrix(ci + p0 + min(ebase + tid + k * WG, nb - 1));
#pragma unroll
    for (int k = 0; k < K; ++k) val[k] = ld_matrix(v + p0 + min(ebase + tid + k * WG, nb - 1));
#pragma unroll
    for (int k = 0; k < K; ++k) g[k] = xin[PK ? (int)((unsigned)col[k] >> kPkSlotBits) : col[k]];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int i = rbase + tid + k * WG;
        if (i <= R) sm.rows[i] = (unsigned short)(rw[k] - p0);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = ebase + tid + k * WG;
        if (e < nb) sm.prod[PK ? (int)((unsigned)col[k] & kPkSlotMask) : e] = val[k] * g[k];
    }
}

// Idx: int column indices, or unsigned short ones relative to the start of
// xin (a caller that knows a block's columns lie in one 65,536-wide window
// passes xin shifted to that window)
// PK: the block's entries are stored sorted by column, each as one 32-bit
// word col << kPkSlotBits | slot, where slot is the entry's place in the
// block's row order (see k_sort_blocks); values follow the same order.
// The product of an entry goes to LDS at its slot, so the row sums add
// exactly the same terms in exactly the same order as the plain layout.
// WG: threads of the workgroup running the block.
// lbias moves the lanes per row one power of two down (-1) or up (+1) from
// the rule below (a per-matrix choice of the tuner; 0 keeps the rule)
template <class Epi, class Idx = int, bool PK = false, int WG = kWG>
__device__ __forceinline__ void spmv_rows(const int *__restrict__ rp, const Idx *__restrict__ ci,
                                          const double *__restrict__ v,
                                          const double *__restrict__ xin, int r0, int r1,
                                          int p0, int p1, const Epi &epi, SpmvShared &sm,
                                          int lbias = 0) {
    // rows [r0, r1) hold entries [p0, p1) (from the block table, see
    // k_rowsplit)
    const int tid = threadIdx.x;
    const int nb = p1 - p0;
    const int R = r1 - r0;  // <= kUnits: every row start takes one unit of the block
    if (nb <= kLdsProducts) {
        // The block's row starts, entries and gathers in chunks (one chunk
        // for a typical block: about kUnits entries and a few hundred rows).
        // The matrix is read once per launch: non-temporal loads keep it
        // from evicting the gathered vector from L2 and the MALL.
        constexpr int K = 1024 / WG, KR = 512 / WG;
        if (nb == 0) {
            for (int i = tid; i <= R; i += WG) sm.rows[i] = 0;
        } else {
            for (int base = 0, rbase = 0; base < nb || rbase <= R;
                 base += K * WG, rbase += KR * WG) {
                if (base < nb)
                    spmv_stage<WG, K, KR, Idx, PK>(rp, ci, v, xin, r0, R, p0, nb,
                                                   rbase <= R ? rbase : R, base, sm);
                else
                    for (int i = rbase + tid; i <= R && i < rbase + KR * WG; i += WG)
                        sm.rows[i] = (unsigned short)(rp[r0 + i] - p0);
            }
        }
        __syncthreads();
        const int avg = nb / R;
        int L = 1;
        while (L < 64 && 2 * L <= avg) L <<= 1;
        // the bias keeps R L <= kLdsProducts, so the rounds below still
        // cover every row
        if (lbias < 0 && L > 1) L >>= 1;
        else if (lbias > 0 && L < 64 && R * 2 * L <= kLdsProducts) L <<= 1;
        const int G = WG / L;
        const int lane = tid & (L - 1), grp = tid / L;
        // A group reduces at most kLdsProducts / WG rows: L = 1 when the
        // mean row length avg = nb / R is below 2 (and R <= kUnits), else
        // L <= avg, so R L <= nb <= kLdsProducts and R / G = R L / WG.
        constexpr int kRounds = kLdsProducts / WG;
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
        for (int rr = tid; rr < R; rr += WG) epi(r0 + rr, sm.prod[rr]);
    } else {
        const int wave = tid >> 6, lane = tid & 63;
        for (int row = r0 + wave; row < r1; row += WG / 64) {
            double s = 0.0;
            for (int p = rp[row] + lane; p < rp[row + 1]; p += 64) {
                const Idx c = ld_matrix(ci + p);
                s += ld_matrix(v + p) * xin[PK ? (int)((unsigned)c >> kPkSlotBits) : (int)c];
            }
            s = wave_sum(s);
            if (lane == 0) epi(row, s);
        }
    }
}

template <class Epi, class Idx = int, bool PK = false, int WG = kWG>
__global__ __launch_bounds__(WG) void k_spmv(const int *__restrict__ rp,
                                             const Idx *__restrict__ ci,
                                             const double *__restrict__ v,
                                             const double *__restrict__ xin,
                                             const int *__restrict__ br, int nblk, Epi epi,
                                             const int *skip, int lbias = 0) {
    __shared__ SpmvShared lds;
    // the gate and the block table are loaded together (one round trip)
    const int b = blockIdx.x;
    const int r0 = br[b], r1 = br[b + 1], p0 = br[nblk + 1 + b], p1 = br[nblk + 2 + b];
    const int off = skip ? *skip : 0;
    if (off || r0 >= r1) return;
    spmv_rows<Epi, Idx, PK, WG>(rp, ci, v, xin, r0, r1, p0, p1, epi, lds, lbias);
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

// Deterministic exclusive prefix (from the left) and suffix (from the
// right) of one double per thread: a scan inside each wave by shuffles
// (the exclusive value is the neighbour's inclusive one, so no subtraction
// enters), then the totals of the waves before (after) added in wave
// order.  sh holds kWG / 64 doubles; two barriers.
__device__ double block_excl_prefix(double v, double *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    double ex = __shfl_up(x, 1, 64);
    if (lane == 0) ex = 0.0;
    if (lane == 63) sh[w] = x;
    __syncthreads();
    double base = 0.0;
    for (int q = 0; q < w; ++q) base += sh[q];
    __syncthreads();
    return base + ex;
}

__device__ double block_excl_suffix(double v, double *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int NW = kWG / 64;
    double x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_down(x, off, 64);
        if (lane + off < 64) x += y;
    }
    double ex = __shfl_down(x, 1, 64);
    if (lane == 63) ex = 0.0;
    if (lane == 0) sh[w] = x;
    __syncthreads();
    double base = 0.0;
    for (int q = NW - 1; q > w; --q) base += sh[q];
    __syncthreads();
    return base + ex;
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


// ---------------------------------------------------------------------
// PDHG half-step epilogues
// ---------------------------------------------------------------------
// x+ = proj_[l,u](x - tau (c - A'y)); sx += x+   (eq. PDHG-update, primal;
// the running sum of Algorithm 1 in pairs of iterations, see sum_mode)
struct EpiPrimal {
    const double *__restrict__ c, *__restrict__ l, *__restrict__ u;
    double *__restrict__ x, *__restrict__ sx;
    double tau;
    DevState *st;
    const unsigned char *__restrict__ cls;  // bound class of each column, or null
    double blo[kBoundClasses], bhi[kBoundClasses];
    int smode;  // running sum: 0 add x+, 1 nothing yet, 2 add the previous x, then x+
    __device__ __forceinline__ void operator()(int j, double aty) const {
        double g = c[j] - aty;
        const double xo = x[j];
        double xn = xo - tau * g;
        double lo, hi;
        if (cls) {
            const int k = cls[j];
            lo = (k & 2) ? ((k & 1) ? blo[3] : blo[2]) : ((k & 1) ? blo[1] : blo[0]);
            hi = (k & 2) ? ((k & 1) ? bhi[3] : bhi[2]) : ((k & 1) ? bhi[1] : bhi[0]);
        } else {
            lo = l[j];
            hi = u[j];
        }
        if (xn < lo) xn = lo;
        if (xn > hi) xn = hi;
        x[j] = xn;
        if (smode == 0) sx[j] += xn;
        else if (smode == 2) sx[j] = (sx[j] + xo) + xn;
        if (j == 0) {  // iteration counters of Algorithm 1
            st->k += 1;
            st->t += 1;
        }
    }
};

// y+ = proj_Y(y + sigma (b - (2 A x+ - A x))); sy += y+ (in pairs as for
// x); q = A x+
struct EpiDual {
    const double *__restrict__ b;
    const signed char *__restrict__ kind;
    double *__restrict__ y, *__restrict__ sy, *__restrict__ q;
    double sigma;
    int smode;
    __device__ __forceinline__ void operator()(int i, double ax) const {
        const double yo = y[i];
        double yv = yo + sigma * (b[i] - (2.0 * ax - q[i]));
        if (kind && kind[i] && yv < 0.0) yv = 0.0;
        y[i] = yv;
        if (smode == 0) sy[i] += yv;
        else if (smode == 2) sy[i] = (sy[i] + yo) + yv;
        q[i] = ax;
    }
};

// ---------------------------------------------------------------------
// check steps shared by the multi-kernel check and the one-workgroup path
// ---------------------------------------------------------------------
// z-bar = S / t at coordinate i (x first, then y); the empty window
// averages to z itself
__device__ __forceinline__ void average_at(const Dev &d, long long i, long long t) {
    const double tt = (double)t;
    if (i < d.n) d.xbar[i] = t ? d.sx[i] / tt : d.x[i];
    else if (i < (long long)d.n + d.m) {
        const long long r = i - d.n;
        d.ybar[r] = t ? d.sy[r] / tt : d.y[r];
    }
}

// KKT sums of coordinate i (x coordinates first, then y) at the points of
// P2 (slot 0: the current point, slot 1: the average) and the squared
// distances of both to the anchor (eq. define:K-and-h-for-lp rows).
__device__ __forceinline__ void kkt_elem(const Dev &d, const KktPoints &P2, long long i,
                                         double (&v)[kKktSums]) {
    // squared distances to the anchor, added after the branch (one of the
    // pairs is zero) so that the two branches write different slots
    double rxa = 0.0, rxc = 0.0, rya = 0.0, ryc = 0.0;
    if (i < d.n) {
        const int j = (int)i;
        const double cj = d.c[j], lj = d.l[j], uj = d.u[j], x0 = d.x0[j];
        const bool lf = isfinite(lj), uf = isfinite(uj);
        const double xs[2] = {P2.x[0][j], P2.x[1][j]};
        const double ats[2] = {P2.aty[0][j], P2.aty[1][j]};
#pragma unroll
        for (int P = 0; P < 2; ++P) {
            const double xp = xs[P];
            const double rc = cj - ats[P];
            double lam;
            if (lf && uf) lam = rc;
            else if (lf) lam = rc > 0.0 ? rc : 0.0;
            else if (uf) lam = rc < 0.0 ? rc : 0.0;
            else lam = 0.0;
            const double dr = rc - lam;
            v[S_DRES2_C + P] += dr * dr;
            double dob = 0.0;
            if (lam > 0.0) dob += lj * lam;
            if (lam < 0.0) dob += uj * lam;
            v[S_DOBJ_C + P] += dob;
            v[S_POBJ_C + P] += cj * xp;
            double bv = 0.0;
            if (xp < lj) bv = lj - xp;
            if (xp > uj) bv = xp - uj;
            v[S_BV2_C + P] += bv * bv;
        }
        const double da = xs[1] - x0, dc = xs[0] - x0;
        rxa = da * da;
        rxc = dc * dc;
    } else {
        const int r = (int)(i - d.n);
        const double br = d.b[r], y0 = d.y0[r];
        const bool ge = d.kind && d.kind[r];
        const double ys[2] = {P2.y[0][r], P2.y[1][r]};
        const double axs[2] = {P2.ax[0][r], P2.ax[1][r]};
#pragma unroll
        for (int P = 0; P < 2; ++P) {
            double p = br - axs[P];
            if (ge && p < 0.0) p = 0.0;
            v[S_PRES2_C + P] += p * p;
            v[S_DOBJ_C + P] += br * ys[P];
            const double yneg = (ge && ys[P] < 0.0) ? ys[P] : 0.0;
            v[S_BV2_C + P] += yneg * yneg;
        }
        const double da = ys[1] - y0, dc = ys[0] - y0;
        rya = da * da;
        ryc = dc * dc;
    }
    v[S_RX2_A] += rxa;
    v[S_RX2_C] += rxc;
    v[S_RY2_A] += rya;
    v[S_RY2_C] += ryc;
}

// KKT parts at z (avg false) or z-bar (avg true) from the 14 sums S:
// o[1..7] = relative KKT, |primal residual|, |dual residual|, primal and
// dual objective, the paper's absolute form, the max form
__device__ __forceinline__ void kkt_parts(const DevState *st, const double *S, bool avg,
                                          double (&o)[8]) {
    const double pres2 = avg ? S[S_PRES2_A] : S[S_PRES2_C];
    const double dres2 = avg ? S[S_DRES2_A] : S[S_DRES2_C];
    const double pobj = avg ? S[S_POBJ_A] : S[S_POBJ_C];
    const double dobj = avg ? S[S_DOBJ_A] : S[S_DOBJ_C];
    const double bv2 = avg ? S[S_BV2_A] : S[S_BV2_C];
    const double pres = sqrt(pres2), dres = sqrt(dres2);
    const double gap = pobj - dobj;
    const double rel_p = pres / (1.0 + sqrt(st->nb2));
    const double rel_d = dres / (1.0 + sqrt(st->nc2));
    const double rel_g = fabs(gap) / (1.0 + fabs(pobj) + fabs(dobj));
    double rel = rel_p;
    if (rel_d > rel) rel = rel_d;
    if (rel_g > rel) rel = rel_g;
    const double gpos = gap > 0.0 ? gap : 0.0;
    double mx = pres;
    if (dres > mx) mx = dres;
    if (fabs(gap) > mx) mx = fabs(gap);
    o[0] = 0.0;
    o[1] = rel;
    o[2] = pres;
    o[3] = dres;
    o[4] = pobj;
    o[5] = dobj;
    o[6] = sqrt(bv2 + pres2 + dres2 + gpos * gpos);
    o[7] = mx;
}

__device__ __forceinline__ void kkt_point(const Dev &d, const double *S, int P, double *out) {
    double o[8];
    kkt_parts(d.st, S, P != 0, o);
#pragma unroll
    for (int k = 1; k < 8; ++k) out[k] = o[k];
}

// The stopping test of a check from the 14 KKT sums S: KKT at z and z-bar,
// the converged flag (termination first), the radii, and the trust-region
// slots armed for the restart test.  Called by every lane of one whole
// wave with S in each lane: lane 0 takes z and lane 1 z-bar (KKT parts and
// radius side by side), lane 0 writes the state.  Returns the armed slots
// in every lane.
__device__ __forceinline__ int kkt_conclude(const Dev &d, const double *S, double tol, int kkt_kind,
                                            double omega, int gap_slots) {
    DevState *st = d.st;
    const int lane = threadIdx.x & 63;
    const bool odd = (lane & 1) != 0;
    double o[8];
    kkt_parts(st, S, odd, o);
    const double rad = sqrt(odd ? omega * S[S_RX2_A] + S[S_RY2_A] / omega
                                : omega * S[S_RX2_C] + S[S_RY2_C] / omega);
    double cur[8], avg[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        cur[k] = lane_f64(o[k], 0);
        avg[k] = lane_f64(o[k], 1);
    }
    const double r_cur = lane_f64(rad, 0), r_avg = lane_f64(rad, 1);
    const double kc = kkt_kind == 1 ? cur[6] : (kkt_kind == 2 ? cur[7] : cur[1]);
    const double ka = kkt_kind == 1 ? avg[6] : (kkt_kind == 2 ? avg[7] : avg[1]);
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kKktSums; ++k) bad |= !isfinite(S[k]);
    const int conv = (tol > 0.0 && (kc <= tol || ka <= tol)) ? 1 : 0;
    int slots = 0;
    if (!conv && !bad && st->t > 0) slots = gap_slots;
    if (lane == 0) {
        st->in_check = 1;
        st->restarted = 0;
        st->cand = 0;
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            st->kkt_cur[k] = cur[k];
            st->kkt_avg[k] = avg[k];
        }
        st->kkt_cur[0] = kc;
        st->kkt_avg[0] = ka;
        st->numerr = bad ? 1 : 0;
        // a breakdown ends the run like convergence: the blocks replayed
        // after this check do nothing, so the iterates stay at this check
        if (bad) st->done = 1;
        st->conv_which = -1;
        if (conv) {
            st->done = 1;
            st->conv_which = (ka <= kc) ? 1 : 0;
            st->conv_k = st->k;
        }
        st->r_avg = r_avg;
        st->r_cur = r_cur;
        st->gap_slots = slots;
        for (int sidx = 0; sidx < kTrSlots; ++sidx) {
            TRState &ts = st->tr[sidx];
            ts.mode = TR_IDLE;
            ts.rho = 0.0;
            ts.lam = 0.0;
            if (slots & (1 << sidx)) {
                ts.mode = TR_SEARCH;
                ts.r = sidx == 0 ? r_avg : r_cur;
                ts.r2 = ts.r * ts.r;
                ts.F_acc = 0.0;
                ts.A_acc = 0.0;
                ts.prefix = 0ull;
                ts.klo = 0ull;
                ts.level = 0;
                ts.count = 0;
                ts.ncomp = 0;
                ts.nan_seen = 0;
            }
        }
    }
    return slots;
}

// The restart test of a check (eq. adaptive-restart-scheme, Remark
// rem:flexible) from the trust-region results, the restart bookkeeping,
// and the check record.  One thread.
__device__ __forceinline__ void decide_restart(const Dev &d, double beta, int tau0) {
    DevState *st = d.st;
    double rec[kRec];
    rec[0] = (double)st->k;
    rec[1] = (double)st->t;
    rec[2] = (double)st->restarts;
    rec[3] = st->kkt_cur[0];
    rec[4] = st->kkt_avg[0];
    rec[5] = 0.0;
    rec[6] = 0.0;
    rec[7] = 0.0;
    rec[8] = -1.0;
    rec[9] = 0.0;
    rec[10] = 0.0;
    rec[11] = (double)st->conv_which;
    rec[12] = st->rho_prev;
    rec[13] = 0.0;
    const int slots = st->gap_slots;
    if (slots & 1) {
        rec[5] = st->r_avg;
        rec[6] = st->tr[0].rho;
        rec[13] = st->tr[0].lam;
        if (st->tr[0].nan_seen) st->numerr = 1;
    }
    if (slots & 2) {
        rec[7] = st->r_cur;
        rec[8] = st->tr[1].rho;
        if (st->tr[1].nan_seen) st->numerr = 1;
    }
    if ((slots & 1) && !st->done && !st->numerr) {
        const double rho_a = st->tr[0].rho;
        double rho_c = rho_a;
        int cand = 0;
        if ((slots & 2) && st->tr[1].rho < rho_a) {  // strict, as in Remark rem:flexible
            cand = 1;
            rho_c = st->tr[1].rho;
        }
        bool restart;
        if (st->restarts == 0) restart = st->t >= (long long)tau0;
        else restart = rho_c <= beta * st->rho_prev;
        rec[10] = (double)cand;
        if (restart) {
            rec[9] = 1.0;
            st->restarted = 1;
            st->cand = cand;
            st->restarts += 1;
            st->t = 0;
            st->rho_prev = rho_c;
        }
    }
    double *dst = d.log + (size_t)(st->checks % kLogCap) * kRec;
    for (int q = 0; q < kRec; ++q) dst[q] = rec[q];
    st->checks += 1;
    st->in_check = 0;
}

// The restart of Algorithm 1 at coordinate i: the anchor and the current
// point become the candidate (z-bar, or z itself when cand = 1), with
// q = A x kept consistent, and the running sums restart.
__device__ __forceinline__ void apply_restart_at(const Dev &d, long long i, int cand) {
    if (i < d.n) {
        if (cand == 0) {
            const double v = d.xbar[i];
            d.x[i] = v;
            d.x0[i] = v;
        } else {
            d.x0[i] = d.x[i];
        }
        d.sx[i] = 0.0;
    }
    if (i < d.m) {
        if (cand == 0) {
            const double v = d.ybar[i];
            d.y[i] = v;
            d.y0[i] = v;
            d.q[i] = d.axb[i];
        } else {
            d.y0[i] = d.y[i];
        }
        d.sy[i] = 0.0;
    }
}

// coordinates (|g_i|, distance to the bound g_i points at) of the linear
// trust region at a point (x, y) with A x and A'y, in the omega-weighted norm
struct GapElems {
    int n, m;
    const double *c, *b, *l, *u;
    const signed char *kind;
    const double *x, *y, *ax, *aty;
    double sw;  // sqrt(omega): the norm is omega |x|^2 + |y|^2 / omega
    __device__ __forceinline__ long long size() const { return (long long)n + m; }
    __device__ __forceinline__ void get(long long i, double &a, double &d) const {
        if (i < n) {
            const int j = (int)i;
            const double g = c[j] - aty[j];
            double dist = 0.0;
            if (g > 0.0) dist = x[j] - l[j];
            else if (g < 0.0) dist = u[j] - x[j];
            if (dist < 0.0) dist = 0.0;
            a = fabs(g) / sw;
            d = dist * sw;
        } else {
            const int r = (int)(i - n);
            const double g = ax[r] - b[r];
            const double lo = (kind && kind[r]) ? 0.0 : -INFINITY;
            double dist = 0.0;
            if (g > 0.0) dist = y[r] - lo;
            else if (g < 0.0) dist = INFINITY;
            if (dist < 0.0) dist = 0.0;
            a = fabs(g) * sw;
            d = dist / sw;
        }
    }
};

}  // namespace pdhg
