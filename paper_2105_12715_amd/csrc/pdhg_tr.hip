// Normalized duality gap, restart decision and point bookkeeping.
//
// rho_r(w) (eq. rhorz) for the LP saddle function equals
//     max { F(w)'(w - w~) : w~ in Z, ||w~ - w|| <= r } / r
// (eq. bilinear-0), a linear trust region over a box (Section 6.3.1).
// Coordinate i with gradient g_i moves toward the bound that lowers g'w~:
// a_i = |g_i|, d_i = distance to that bound (inf when there is none), and
// w~_i = w_i - sign(g_i) min(lambda a_i, d_i).  lambda* is the largest
// lambda with f(lambda) = sum_i min(lambda a_i, d_i)^2 <= r^2
// (eq. lp-trust-region:summation).
//
// The search is bisection on the multiplier, 2048 candidates at a time:
// the keys are the IEEE bit patterns of the breakpoints d_i / a_i, which
// order like the values for non-negative doubles.  Level 0 histograms the
// 11 exponent bits over all N coordinates; level 1 histograms the next 11
// bits over the coordinates still in the bracket and each block copies
// them into its own region of a compaction buffer; levels 2 and 3 run over
// the compacted regions on all blocks while the bracket holds more than
// 65536 coordinates, and one workgroup finishes the remaining levels.  At each level the
// bracket moves to the last bucket whose lower end keeps f <= r^2.  Once
// the bracket holds no breakpoint (or one repeated value), every
// coordinate is either clamped (key <= klo) or free, and a deterministic
// pass gives F = sum_clamped d^2, A = sum_free a^2, lambda* =
// sqrt((r^2 - F)/A), the closing formula of Algorithm 2.
#include "pdhg_device.h"

#include <math.h>

namespace pdhg {

// ---------------------------------------------------------------------
// coordinate providers
// ---------------------------------------------------------------------
struct RawElems {
    long long N;
    const double *a, *d;
    __device__ __forceinline__ long long size() const { return N; }
    __device__ __forceinline__ void get(long long i, double &aa, double &dd) const {
        aa = a[i];
        dd = d[i];
    }
};

// ---------------------------------------------------------------------
// level 0: exponent histogram over all coordinates + full-box sums
// ---------------------------------------------------------------------
template <class E>
__global__ __launch_bounds__(kWG) void k_tr_hist0(E e, TRState *ts, TRWork w, const int *gate) {
    if (gate && !*gate) return;
    if (ts->mode != TR_SEARCH || ts->level != 0) return;
    __shared__ unsigned int scnt[kBuckets];
    __shared__ double sD[kBuckets], sA[kBuckets];
    __shared__ double sh[4 * 4];
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        scnt[b] = 0u;
        sD[b] = 0.0;
        sA[b] = 0.0;
    }
    __syncthreads();
    double v[4] = {0.0, 0.0, 0.0, 0.0};  // sum d^2 (finite d), #inf d, sum a d, #bad
    const long long N = e.size();
    for (long long base = (long long)blockIdx.x * kWG; base < N; base += (long long)gridDim.x * kWG) {
        const long long i = base + threadIdx.x;
        if (i < N) {
            double a, d;
            e.get(i, a, d);
            if (bad_pair(a, d)) {
                v[3] += 1.0;
            } else if (a > 0.0) {
                const unsigned long long key = key_of(a, d);
                const int b = (int)(key >> 52);
                atomicAdd(&scnt[b], 1u);
                atomicAdd(&sA[b], a * a);
                if (d < INFINITY) {
                    atomicAdd(&sD[b], d * d);
                    v[0] += d * d;
                    v[2] += a * d;
                } else {
                    v[1] += 1.0;
                }
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        if (scnt[b]) {
            atomicAdd(&w.hcnt[b], scnt[b]);
            atomicAdd(&w.hD[b], sD[b]);
            atomicAdd(&w.hA[b], sA[b]);
        }
    }
    block_sums<4>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) w.part[blockIdx.x * 4 + k] = v[k];
    }
}

__device__ void zero_hist(const TRWork &w, int slot) {
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        w.hcnt[slot * kBuckets + b] = 0u;
        w.hD[slot * kBuckets + b] = 0.0;
        w.hA[slot * kBuckets + b] = 0.0;
    }
}

__global__ __launch_bounds__(kWG) void k_tr_decide0(TRState *ts, TRWork w, int nb, const int *gate) {
    if (gate && !*gate) return;
    if (ts->mode != TR_SEARCH || ts->level != 0) return;
    __shared__ TRState sts;
    __shared__ ChooseShared cs;
    __shared__ double sh[4 * 4];
    __shared__ int go;
    if (threadIdx.x == 0) {
        sts = *ts;
        *w.fcount = 0u;  // the gather before the last levels starts empty
    }
    double tot[4];
    reduce_partials<4>(w.part, nb, 4, tot, sh);
    if (threadIdx.x == 0) {
        go = 0;
        if (tot[3] > 0.0) {
            sts.nan_seen = 1;
            sts.mode = TR_ZERO;
            sts.rho = NAN;
            sts.lam = NAN;
            sts.value = NAN;
        } else if (!(sts.r > 0.0)) {
            sts.mode = TR_ZERO;
            sts.rho = 0.0;
            sts.lam = 0.0;
            sts.value = 0.0;
        } else if (tot[1] == 0.0 && tot[0] <= sts.r2) {
            // first line of Algorithm 2: the whole box fits in the ball
            sts.mode = TR_FULLBOX;
            sts.value = tot[2];
            sts.rho = tot[2] / sts.r;
            sts.lam = INFINITY;
        } else {
            go = 1;
        }
    }
    __syncthreads();
    if (go) choose_bucket(sts, w.hcnt, w.hD, w.hA, kBuckets, 0, cs);
    zero_hist(w, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        sts.ncomp = 0u;
        *ts = sts;
    }
}

// Level 1 over all coordinates: histogram of bits 51..41 of the bracket's
// keys, and each block copies its bracket members into its own region of
// the compaction buffer (no global counter).
template <class E>
__global__ __launch_bounds__(kWG) void k_tr_pass1(E e, TRState *ts, TRWork w, const int *gate,
                                                  int cap) {
    if (gate && !*gate) return;
    if (ts->mode != TR_SEARCH || ts->level != 1) return;
    __shared__ unsigned int scnt[kBuckets];
    __shared__ double sD[kBuckets], sA[kBuckets];
    __shared__ unsigned int nloc;
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        scnt[b] = 0u;
        sD[b] = 0.0;
        sA[b] = 0.0;
    }
    if (threadIdx.x == 0) nloc = 0u;
    __syncthreads();
    const unsigned long long top = ts->prefix >> 52;
    const size_t region = (size_t)blockIdx.x * (size_t)cap;
    const long long N = e.size();
    for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < N;
         i += (long long)gridDim.x * kWG) {
        double a, d;
        e.get(i, a, d);
        if (bad_pair(a, d) || !(a > 0.0)) continue;
        const unsigned long long key = key_of(a, d);
        if ((key >> 52) != top) continue;
        const int b = (int)((key >> 41) & (kBuckets - 1));
        atomicAdd(&scnt[b], 1u);
        atomicAdd(&sD[b], d * d);
        atomicAdd(&sA[b], a * a);
        const unsigned int slot = atomicAdd(&nloc, 1u);
        w.ckey[region + slot] = key;
        w.ca[region + slot] = a;
        w.cd[region + slot] = d;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        if (scnt[b]) {
            atomicAdd(&w.hcnt[kBuckets + b], scnt[b]);
            atomicAdd(&w.hD[kBuckets + b], sD[b]);
            atomicAdd(&w.hA[kBuckets + b], sA[b]);
        }
    }
    if (threadIdx.x == 0) w.ccount[blockIdx.x] = nloc;
}

// exclusive prefix of the per-block counts (nb <= kRedBlocks = 4 * kWG)
__device__ void scan_counts(const TRWork &w, int nb, unsigned int *sh) {
    const int t = threadIdx.x;
    unsigned int loc[4];
    unsigned int sum = 0u;
    for (int k = 0; k < 4; ++k) {
        const int b = 4 * t + k;
        loc[k] = b < nb ? w.ccount[b] : 0u;
        sum += loc[k];
    }
    sh[t] = sum;
    __syncthreads();
    for (int off = 1; off < kWG; off <<= 1) {
        unsigned int o = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += o;
        __syncthreads();
    }
    unsigned int run = t ? sh[t - 1] : 0u;
    for (int k = 0; k < 4; ++k) {
        const int b = 4 * t + k;
        if (b < nb) w.coff[b] = run;
        run += loc[k];
    }
    if (t == kWG - 1) w.coff[nb] = sh[kWG - 1];  // the total (nb may equal 4 * kWG)
    __syncthreads();
}

__global__ __launch_bounds__(kWG) void k_tr_decide1(TRState *ts, TRWork w, int nb, const int *gate) {
    if (gate && !*gate) return;
    if (ts->mode != TR_SEARCH || ts->level != 1) return;
    __shared__ TRState sts;
    __shared__ ChooseShared cs;
    __shared__ unsigned int shs[kWG];
    if (threadIdx.x == 0) sts = *ts;
    scan_counts(w, nb, shs);
    if (threadIdx.x == 0) sts.ncomp = shs[kWG - 1];  // total, still in LDS
    __syncthreads();
    choose_bucket(sts, w.hcnt + kBuckets, w.hD + kBuckets, w.hA + kBuckets, kBuckets, 1, cs);
    zero_hist(w, 0);
    __syncthreads();
    if (threadIdx.x == 0) *ts = sts;
}

// Levels 2 and 3 across all blocks while the bracket is still large: block b
// histograms the members of its own compaction region.

__global__ __launch_bounds__(kWG) void k_tr_cpass(TRState *ts, TRWork w, const int *gate, int cap,
                                                  int level) {
    if (gate && !*gate) return;
    if (ts->mode != TR_SEARCH || ts->level != level || ts->count <= kFinishMax) return;
    __shared__ unsigned int scnt[kBuckets];
    __shared__ double sD[kBuckets], sA[kBuckets];
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        scnt[b] = 0u;
        sD[b] = 0.0;
        sA[b] = 0.0;
    }
    __syncthreads();
    const int shift = shift_of(level), above = shift_of(level - 1);
    const unsigned long long want = ts->prefix >> above;
    const size_t region = (size_t)blockIdx.x * (size_t)cap;
    unsigned int cnt = w.ccount[blockIdx.x];
    if (cnt > (unsigned int)cap) cnt = (unsigned int)cap;
    for (unsigned int q = threadIdx.x; q < cnt; q += kWG) {
        const unsigned long long key = w.ckey[region + q];
        if ((key >> above) != want) continue;
        const int b = (int)((key >> shift) & (kBuckets - 1));
        const double a = w.ca[region + q], d = w.cd[region + q];
        atomicAdd(&scnt[b], 1u);
        atomicAdd(&sD[b], d * d);
        atomicAdd(&sA[b], a * a);
    }
    __syncthreads();
    const int hs = level & 1;
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        if (scnt[b]) {
            atomicAdd(&w.hcnt[hs * kBuckets + b], scnt[b]);
            atomicAdd(&w.hD[hs * kBuckets + b], sD[b]);
            atomicAdd(&w.hA[hs * kBuckets + b], sA[b]);
        }
    }
}

__global__ __launch_bounds__(kWG) void k_tr_cdecide(TRState *ts, TRWork w, const int *gate,
                                                    int level) {
    if (gate && !*gate) return;
    if (ts->mode != TR_SEARCH || ts->level != level || ts->count <= kFinishMax) return;
    __shared__ TRState sts;
    __shared__ ChooseShared cs;
    if (threadIdx.x == 0) sts = *ts;
    __syncthreads();
    const int hs = level & 1;
    choose_bucket(sts, w.hcnt + hs * kBuckets, w.hD + hs * kBuckets, w.hA + hs * kBuckets,
                  kBuckets, level, cs);
    zero_hist(w, 1 - hs);
    __syncthreads();
    if (threadIdx.x == 0) *ts = sts;
}

// The bracket's members, copied from the compaction regions into one dense
// list (up to kFinishMax; the count keeps growing past it) for the last levels.
__global__ __launch_bounds__(kWG) void k_tr_gather(TRState *ts, TRWork w, const int *gate,
                                                   int cap) {
    if (gate && !*gate) return;
    if (ts->mode != TR_SEARCH) return;
    __shared__ unsigned int nloc, base, fill;
    const int above = shift_of(ts->level - 1);
    const unsigned long long want = ts->prefix >> above;
    const size_t region = (size_t)blockIdx.x * (size_t)cap;
    unsigned int cnt = w.ccount[blockIdx.x];
    if (cnt > (unsigned int)cap) cnt = (unsigned int)cap;
    if (threadIdx.x == 0) {
        nloc = 0u;
        fill = 0u;
    }
    __syncthreads();
    for (unsigned int q = threadIdx.x; q < cnt; q += kWG)
        if ((w.ckey[region + q] >> above) == want) atomicAdd(&nloc, 1u);
    __syncthreads();
    if (threadIdx.x == 0) base = nloc ? atomicAdd(w.fcount, nloc) : 0u;
    __syncthreads();
    if (nloc == 0u || base >= kFinishMax) return;
    for (unsigned int q = threadIdx.x; q < cnt; q += kWG) {
        const unsigned long long key = w.ckey[region + q];
        if ((key >> above) != want) continue;
        const unsigned int at = base + atomicAdd(&fill, 1u);
        if (at < kFinishMax) {
            w.fkey[at] = key;
            w.fa[at] = w.ca[region + q];
            w.fd[at] = w.cd[region + q];
        }
    }
}

// remaining levels on the gathered list (or, past kFinishMax members, on
// the compaction regions), one workgroup
__global__ __launch_bounds__(kWG) void k_tr_finish(TRState *ts, TRWork w, const int *gate, int cap,
                                                   int nb) {
    if (gate && !*gate) return;
    if (ts->mode != TR_SEARCH) return;
    __shared__ TRState sts;
    __shared__ ChooseShared cs;
    __shared__ unsigned int scnt[kBuckets];
    __shared__ double sD[kBuckets], sA[kBuckets];
    __shared__ unsigned int off[kRedBlocks + 1];
    if (threadIdx.x == 0) sts = *ts;
    for (int b = threadIdx.x; b <= nb; b += kWG) off[b] = w.coff[b];
    __syncthreads();
    const unsigned int nf = *w.fcount;
    const bool dense = nf <= kFinishMax;
    // never walk past the compaction buffer, whatever the counts say
    unsigned int total = dense ? nf : off[nb];
    const unsigned long long room = (unsigned long long)nb * (unsigned long long)cap;
    if (!dense && (unsigned long long)total > room) total = (unsigned int)room;
    while (sts.mode == TR_SEARCH) {
        const int level = sts.level;
        const int shift = shift_of(level);
        const int nbuck = level == 5 ? 256 : kBuckets;
        const int above = shift_of(level - 1);
        const unsigned long long want = sts.prefix >> above;
        for (int b = threadIdx.x; b < kBuckets; b += kWG) {
            scnt[b] = 0u;
            sD[b] = 0.0;
            sA[b] = 0.0;
        }
        __syncthreads();
        for (unsigned int idx = threadIdx.x; idx < total; idx += kWG) {
            unsigned long long key;
            double a, d;
            if (dense) {
                key = w.fkey[idx];
                if ((key >> above) != want) continue;
                a = w.fa[idx];
                d = w.fd[idx];
            } else {
                // region holding the idx-th compacted element: last b with off[b] <= idx
                int lo = 0, hi = nb - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (off[mid] <= idx) lo = mid;
                    else hi = mid - 1;
                }
                const unsigned int within = idx - off[lo];
                if (within >= (unsigned int)cap) continue;
                const size_t at = (size_t)lo * (size_t)cap + within;
                key = w.ckey[at];
                if ((key >> above) != want) continue;
                a = w.ca[at];
                d = w.cd[at];
            }
            const int b = (int)((key >> shift) & (unsigned long long)(nbuck - 1));
            atomicAdd(&scnt[b], 1u);
            atomicAdd(&sD[b], d * d);
            atomicAdd(&sA[b], a * a);
        }
        __syncthreads();
        choose_bucket(sts, scnt, sD, sA, nbuck, level, cs);
    }
    if (threadIdx.x == 0) *ts = sts;
}

// deterministic sums on either side of klo
template <class E>
__global__ __launch_bounds__(kWG) void k_tr_final_partials(E e, TRState *ts, TRWork w,
                                                           const int *gate) {
    if (gate && !*gate) return;
    if (ts->mode != TR_RESOLVED) return;
    __shared__ double sh[4 * 3];
    const unsigned long long klo = ts->klo;
    double v[3] = {0.0, 0.0, 0.0};  // F = sum d^2 (clamped), A = sum a^2 (free), AD = sum a d
    const long long N = e.size();
    for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < N;
         i += (long long)gridDim.x * kWG) {
        double a, d;
        e.get(i, a, d);
        if (bad_pair(a, d) || !(a > 0.0)) continue;
        const unsigned long long key = key_of(a, d);
        if (key <= klo) {
            v[0] += d * d;
            v[2] += a * d;
        } else {
            v[1] += a * a;
        }
    }
    block_sums<3>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) w.part[blockIdx.x * 4 + k] = v[k];
    }
}

__global__ __launch_bounds__(kWG) void k_tr_final(TRState *ts, TRWork w, int nb, const int *gate) {
    if (gate && !*gate) return;
    if (ts->mode != TR_RESOLVED) return;
    __shared__ double sh[4 * 3];
    double tot[3];
    reduce_partials<3>(w.part, nb, 4, tot, sh);
    if (threadIdx.x == 0) {
        const double F = tot[0], A = tot[1], AD = tot[2];
        double lam, val;
        if (A > 0.0) {
            double num = ts->r2 - F;
            if (num < 0.0) num = 0.0;
            lam = sqrt(num / A);
            val = AD + lam * A;
        } else {
            lam = INFINITY;
            val = AD;
        }
        ts->lam = lam;
        ts->value = val;
        ts->rho = val / ts->r;
    }
}

template <class E>
static void run_tr(const E &e, long long N, TRState *ts, const TRWork &w, const int *gate,
                   hipStream_t s) {
    const int g = red_grid(N);
    // longest run of coordinates one block visits in a grid-stride pass
    const long long per = (N + (long long)g * kWG - 1) / ((long long)g * kWG);
    const int cap = (int)(per * kWG);
    hipLaunchKernelGGL(k_tr_hist0<E>, dim3(g), dim3(kWG), 0, s, e, ts, w, gate);
    hipLaunchKernelGGL(k_tr_decide0, dim3(1), dim3(kWG), 0, s, ts, w, g, gate);
    hipLaunchKernelGGL(k_tr_pass1<E>, dim3(g), dim3(kWG), 0, s, e, ts, w, gate, cap);
    hipLaunchKernelGGL(k_tr_decide1, dim3(1), dim3(kWG), 0, s, ts, w, g, gate);
    // The multi-block levels only work while the bracket holds more than
    // kFinishMax members.  Up to 4 kFinishMax coordinates they are not
    // launched at all: the one-workgroup finish then walks the compacted
    // regions itself in the rare case of a bracket that large, instead of
    // every check paying four launches that return at once.
    if (N > 4ll * kFinishMax) {
        for (int level = 2; level <= 3; ++level) {
            hipLaunchKernelGGL(k_tr_cpass, dim3(g), dim3(kWG), 0, s, ts, w, gate, cap, level);
            hipLaunchKernelGGL(k_tr_cdecide, dim3(1), dim3(kWG), 0, s, ts, w, gate, level);
        }
    }
    hipLaunchKernelGGL(k_tr_gather, dim3(g), dim3(kWG), 0, s, ts, w, gate, cap);
    hipLaunchKernelGGL(k_tr_finish, dim3(1), dim3(kWG), 0, s, ts, w, gate, cap, g);
    hipLaunchKernelGGL(k_tr_final_partials<E>, dim3(g), dim3(kWG), 0, s, e, ts, w, gate);
    hipLaunchKernelGGL(k_tr_final, dim3(1), dim3(kWG), 0, s, ts, w, g, gate);
}

static GapElems gap_elems(const Dev &d, const double *x, const double *y, const double *ax,
                          const double *aty) {
    GapElems e;
    e.n = d.n;
    e.m = d.m;
    e.c = d.c;
    e.b = d.b;
    e.l = d.l;
    e.u = d.u;
    e.kind = d.kind;
    e.x = x;
    e.y = y;
    e.ax = ax;
    e.aty = aty;
    e.sw = sqrt(d.omega);
    return e;
}

void launch_gap(const Dev &d, int slot, hipStream_t s) {
    GapElems e = slot == 0 ? gap_elems(d, d.xbar, d.ybar, d.axb, d.atyb)
                           : gap_elems(d, d.x, d.y, d.q, d.aty);
    run_tr(e, (long long)d.n + d.m, &d.st->tr[slot], d.tr[slot], &d.st->in_check, s);
}

// arm a trust-region evaluation with radius r and clear the level-0 histogram
__global__ void k_tr_arm(TRState *ts, TRWork w, double r) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ts->mode = TR_SEARCH;
        ts->r = r;
        ts->r2 = r * r;
        ts->F_acc = 0.0;
        ts->A_acc = 0.0;
        ts->prefix = 0ull;
        ts->klo = 0ull;
        ts->level = 0;
        ts->count = 0u;
        ts->ncomp = 0u;
        ts->nan_seen = 0;
        ts->rho = 0.0;
        ts->lam = 0.0;
        ts->value = 0.0;
    }
    for (int b = threadIdx.x; b < kBuckets; b += blockDim.x) {
        w.hcnt[b] = 0u;
        w.hD[b] = 0.0;
        w.hA[b] = 0.0;
    }
}

void launch_tr_raw(int64_t N, const double *a, const double *dd, double r, const TRWork &w,
                   TRState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_tr_arm, dim3(1), dim3(kWG), 0, s, st, w, r);
    RawElems e{N, a, dd};
    run_tr(e, (long long)N, st, w, nullptr, s);
}

// ---------------------------------------------------------------------
// restart decision (eq. adaptive-restart-scheme, Remark rem:flexible) and
// the restart itself (Algorithm 1: z^{n+1,0} = candidate, window cleared)
// ---------------------------------------------------------------------
__global__ void k_decide(Dev d, int mode, double beta, int tau0) {
    (void)mode;
    if (!d.st->in_check) return;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    decide_restart(d, beta, tau0);
}

void launch_decide(const Dev &d, int mode, double beta, int tau0, hipStream_t s) {
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(64), 0, s, d, mode, beta, tau0);
}

__global__ void k_apply(Dev d, int force) {
    const DevState *st = d.st;
    if (!force && !st->restarted) return;
    const int cand = force ? 0 : st->cand;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    apply_restart_at(d, i, cand);
}

void launch_apply(const Dev &d, hipStream_t s) {
    const long long mx = d.n > d.m ? d.n : d.m;
    hipLaunchKernelGGL(k_apply, dim3(div_up(mx, kWG)), dim3(kWG), 0, s, d, 0);
}

__global__ void k_fixed_bump(DevState *st) {
    st->restarts += 1;
    st->t = 0;
    st->rho_prev = 0.0;
}

// fixed-length restart (eq. define:t-star): restart to the average now
void launch_fixed_restart(const Dev &d, hipStream_t s) {
    launch_average(d, s);
    launch_spmv_A(d, d.xbar, d.axb, s);
    const long long mx = d.n > d.m ? d.n : d.m;
    hipLaunchKernelGGL(k_apply, dim3(div_up(mx, kWG)), dim3(kWG), 0, s, d, 1);
    hipLaunchKernelGGL(k_fixed_bump, dim3(1), dim3(1), 0, s, d.st);
}

// ---------------------------------------------------------------------
// points
// ---------------------------------------------------------------------
__global__ void k_copy_point(Dev d, int which, double *ox, double *oy) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const DevState *st = d.st;
    const long long t = st->t;
    const bool sol_avg = st->conv_which == 1;
    if (i < d.n) {
        double v;
        if (which == 0) v = d.x[i];
        else if (which == 1) v = t ? d.sx[i] / (double)t : d.x[i];
        else if (which == 2) v = d.x0[i];
        else v = sol_avg ? d.xbar[i] : d.x[i];
        ox[i] = v;
    }
    if (i < d.m) {
        double v;
        if (which == 0) v = d.y[i];
        else if (which == 1) v = t ? d.sy[i] / (double)t : d.y[i];
        else if (which == 2) v = d.y0[i];
        else v = sol_avg ? d.ybar[i] : d.y[i];
        oy[i] = v;
    }
}

void launch_copy_point(const Dev &d, int which, double *x, double *y, hipStream_t s) {
    const long long mx = d.n > d.m ? d.n : d.m;
    hipLaunchKernelGGL(k_copy_point, dim3(div_up(mx, kWG)), dim3(kWG), 0, s, d, which, x, y);
}

__global__ void k_set_point(Dev d, const double *ix, const double *iy) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.n) {
        d.x[i] = ix[i];
        d.x0[i] = ix[i];
        d.sx[i] = 0.0;
    }
    if (i < d.m) {
        d.y[i] = iy[i];
        d.y0[i] = iy[i];
        d.sy[i] = 0.0;
    }
    if (i == 0) d.st->t = 0;
}

void launch_set_point(const Dev &d, const double *x, const double *y, hipStream_t s) {
    const long long mx = d.n > d.m ? d.n : d.m;
    hipLaunchKernelGGL(k_set_point, dim3(div_up(mx, kWG)), dim3(kWG), 0, s, d, x, y);
    launch_spmv_A(d, d.x, d.q, s);
}

// distance of (gx, gy) to the anchor in the primal-weight norm
__global__ __launch_bounds__(kWG) void k_dist_partials(Dev d) {
    __shared__ double sh[4 * 2];
    double v[2] = {0.0, 0.0};
    const long long N = (long long)d.n + d.m;
    for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < N;
         i += (long long)gridDim.x * kWG) {
        if (i < d.n) {
            const double dx = d.gx[i] - d.x0[i];
            v[0] += dx * dx;
        } else {
            const double dy = d.gy[i - d.n] - d.y0[i - d.n];
            v[1] += dy * dy;
        }
    }
    block_sums<2>(v, sh);
    if (threadIdx.x == 0) {
        d.part[blockIdx.x * kKktSums + 0] = v[0];
        d.part[blockIdx.x * kKktSums + 1] = v[1];
    }
}

__global__ __launch_bounds__(kWG) void k_dist_arm(Dev d, int nb, double r_given) {
    __shared__ double sh[4 * 2];
    double tot[2];
    reduce_partials<2>(d.part, nb, kKktSums, tot, sh);
    __shared__ double rr;
    if (threadIdx.x == 0) rr = r_given >= 0.0 ? r_given : sqrt(d.omega * tot[0] + tot[1] / d.omega);
    __syncthreads();
    TRState *ts = &d.st->tr[0];
    const TRWork &w = d.tr[0];
    if (threadIdx.x == 0) {
        ts->mode = TR_SEARCH;
        ts->r = rr;
        ts->r2 = rr * rr;
        ts->F_acc = 0.0;
        ts->A_acc = 0.0;
        ts->prefix = 0ull;
        ts->klo = 0ull;
        ts->level = 0;
        ts->count = 0u;
        ts->ncomp = 0u;
        ts->nan_seen = 0;
        ts->rho = 0.0;
        ts->lam = 0.0;
        ts->value = 0.0;
    }
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        w.hcnt[b] = 0u;
        w.hD[b] = 0.0;
        w.hA[b] = 0.0;
    }
}

void launch_gap_point(const Dev &d, int which, double r, hipStream_t s) {
    launch_copy_point(d, which, d.gx, d.gy, s);
    launch_spmv_A(d, d.gx, d.gax, s);
    launch_spmv_T(d, d.gy, d.gaty, s);
    const int g = red_grid((long long)d.n + d.m);
    hipLaunchKernelGGL(k_dist_partials, dim3(g), dim3(kWG), 0, s, d);
    hipLaunchKernelGGL(k_dist_arm, dim3(1), dim3(kWG), 0, s, d, g, r);
    GapElems e = gap_elems(d, d.gx, d.gy, d.gax, d.gaty);
    run_tr(e, (long long)d.n + d.m, &d.st->tr[0], d.tr[0], nullptr, s);
}

}  // namespace pdhg
