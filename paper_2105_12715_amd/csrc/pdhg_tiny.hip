// Restarted PDHG in one workgroup, for LPs whose iteration vectors fit one
// CU's LDS.
//
// A tiny LP leaves the chip idle: every half-step of the multi-kernel path
// is a launch of a few blocks, and the check of Section 7 is a dozen more.
// Here one workgroup of kTinyWG threads runs whole blocks of the check
// period: the iterations of eq. (PDHG-update), then the check (averages,
// KKT, radii, the restart test of eq. adaptive-restart-scheme and the
// restart of Algorithm 1), with barriers between the phases.  The host
// launches a batch of blocks and polls the state between launches.  When
// every row fits half the workgroup, the check of a block runs on one half
// beside the next block's iterations on the other (see tiny_body): the
// block is dropped and run again when the check restarts or stops.
//
// Rows of A' (primal half-step) and of A (dual half-step) go to aligned
// groups of L lanes.  When every row has at most kTinyK L entries for one
// L in {1, 2, 4, 8} (a compile-time constant of the kernel) and each group
// holds one row, every lane keeps its entries (value, column) in registers
// and the row's owner keeps its coordinate of the iterate, its running sum
// and its LP data there too: a half-step is one gather from LDS, a tree
// of products, a butterfly and a barrier.  Otherwise the matrix sits in
// LDS in CSR with 16-bit column indices.
//
// The trust region of the normalized duality gap (Section 6.3.1) has the
// same answer as in the multi-kernel path: with breakpoints
// lambda_i = d_i / a_i (compared as IEEE key bits),
//     f(lambda_p) = sum_{key_i <= key_p} d_i^2 + lambda_p^2 sum_{key_i > key_p} a_i^2
// is nondecreasing in the key.  The breakpoints with a finite key (at most
// n + m <= 1024, compacted in coordinate order) are evaluated directly:
// first 64 of them spread over the coordinates, which bracket the answer,
// then every one strictly inside the bracket (one pass over the keys per
// breakpoint by a group of lanes, LDS broadcast reads).  The clamped set is
// every key up to the largest breakpoint with f <= r^2, and the closing
// formula of Algorithm 2 takes the sums in a fixed order.
#include "pdhg_device.h"

#include <math.h>
#include <stdlib.h>

#include <vector>

namespace pdhg {

namespace {

constexpr int WG = kTinyWG;
constexpr int kWaves = WG / 64;
constexpr int K = kTinyK;
constexpr unsigned long long kNoKey = ~0ull;  // inactive coordinate (above every key)

// LDS arrays of one launch, carved in the order tiny_lds_bytes counts them
struct TinyLds {
    double *x, *xb;                                // n + 1
    double *sx, *c, *l, *u, *aty, *atyb;           // n
    double *y, *yb;                                // m + 1
    double *sy, *q, *b, *axb;                      // m
    unsigned long long *tkey;                      // n + m
    double2 *tda;                                  // n + m: (d^2, a^2)
    double *tad;                                   // n + m: a d
    int *tcid;                                     // n + m: candidate breakpoints
    signed char *kind;                             // m
    double *av, *tv;                               // nnz (matrix in LDS)
    int *arp, *trp;                                // m + 1, n + 1
    unsigned short *aci, *tci;                     // nnz
    double *sn_x, *sn_sx, *sn_y, *sn_sy, *sn_q;    // the check's copy: n + 1, n, m + 1, m, m
};

__device__ TinyLds carve(unsigned char *base, int n, int m, int nnz, bool reg, bool ov) {
    TinyLds t;
    double *dp = (double *)base;
    t.x = dp; dp += n + 1;
    t.xb = dp; dp += n + 1;
    t.sx = dp; dp += n;
    t.c = dp; dp += n;
    t.l = dp; dp += n;
    t.u = dp; dp += n;
    t.aty = dp; dp += n;
    t.atyb = dp; dp += n;
    t.y = dp; dp += m + 1;
    t.yb = dp; dp += m + 1;
    t.sy = dp; dp += m;
    t.q = dp; dp += m;
    t.b = dp; dp += m;
    t.axb = dp; dp += m;
    t.tkey = (unsigned long long *)dp;
    dp += n + m;
    t.tda = (double2 *)dp;
    dp += 2 * (n + m);
    t.tad = dp; dp += n + m;
    t.tcid = (int *)dp;
    unsigned char *cp = (unsigned char *)(t.tcid + n + m);
    t.kind = (signed char *)cp;
    cp += m;
    cp = (unsigned char *)(((size_t)cp + 7) & ~(size_t)7);
    t.av = t.tv = nullptr;
    t.arp = t.trp = nullptr;
    t.aci = t.tci = nullptr;
    if (!reg) {
        dp = (double *)cp;
        t.av = dp; dp += nnz;
        t.tv = dp; dp += nnz;
        int *ip = (int *)dp;
        t.arp = ip; ip += m + 1;
        t.trp = ip; ip += n + 1;
        unsigned short *sp = (unsigned short *)ip;
        t.aci = sp; sp += nnz;
        t.tci = sp; sp += nnz;
        cp = (unsigned char *)sp;
    }
    cp = (unsigned char *)(((size_t)cp + 7) & ~(size_t)7);
    t.sn_x = t.sn_sx = t.sn_y = t.sn_sy = t.sn_q = nullptr;
    if (ov) {
        dp = (double *)cp;
        t.sn_x = dp; dp += n + 1;
        t.sn_sx = dp; dp += n;
        t.sn_y = dp; dp += m + 1;
        t.sn_sy = dp; dp += m;
        t.sn_q = dp;
    }
    return t;
}

// Sum over an aligned group of L lanes (L a power of two <= 64); every
// lane of the group ends with the same sum.  Pairs, then quads exchange by
// DPP quad permutations; once all lanes of a quad (of 8) agree, the mirror
// inside 8 (16) lanes pairs each with the other quad (half); the steps
// across rows of 16 go through the LDS crossbar.
__device__ __forceinline__ double group_sum(double s, int L) {
    if (L >= 2) s += dpp_f64<0xB1>(s);   // quad_perm [1,0,3,2]: lane ^ 1
    if (L >= 4) s += dpp_f64<0x4E>(s);   // quad_perm [2,3,0,1]: lane ^ 2
    if (L >= 8) s += dpp_f64<0x141>(s);  // row_half_mirror: 7 - lane within 8
    if (L >= 16) s += dpp_f64<0x140>(s); // row_mirror: 15 - lane within 16
    if (L >= 32) s += __shfl_xor(s, 16, 64);
    if (L >= 64) s += __shfl_xor(s, 32, 64);
    return s;
}

// Row r of a CSR matrix in LDS times the LDS vector v, by the L lanes of
// its group: lane-strided partial sums, then the group sum.
__device__ __forceinline__ double row_dot(const int *rp, const unsigned short *ci,
                                          const double *val, const double *v, int r, int lane,
                                          int L) {
    double s = 0.0;
    const int e1 = rp[r + 1];
    for (int e = rp[r] + lane; e < e1; e += L) s += val[e] * v[ci[e]];
    return group_sum(s, L);
}

// group sum with the group size known at compile time
template <int LL>
__device__ __forceinline__ double group_sum_c(double s) {
    if (LL >= 2) s += dpp_f64<0xB1>(s);
    if (LL >= 4) s += dpp_f64<0x4E>(s);
    if (LL >= 8) s += dpp_f64<0x141>(s);
    return s;
}

// the same product from the lane's entries held in registers (padding
// entries have value 0 and point at the zero after the vector's end):
// all gathers first, then the products summed as a balanced tree
template <int LL>
__device__ __forceinline__ double reg_dot(const int (&col)[K], const double (&val)[K],
                                          const double *v) {
    static_assert(K == 8, "the tree below adds eight products");
    double g[K];
#pragma unroll
    for (int k = 0; k < K; ++k) g[k] = v[col[k]];
    double p[K];
#pragma unroll
    for (int k = 0; k < K; ++k) p[k] = val[k] * g[k];
    const double s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    return group_sum_c<LL>(s);
}

// A lane's share of one row (CSR rp, ci, v in global memory) into registers
__device__ __forceinline__ void load_row(const int *rp, const int *ci, const double *v, int r,
                                         int rows, int lane, int L, int pad, int (&col)[K],
                                         double (&val)[K]) {
    int e0 = 0, e1 = 0;
    if (r < rows) {
        e0 = rp[r];
        e1 = rp[r + 1];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = e0 + lane + k * L;
        if (e < e1) {
            col[k] = ci[e];
            val[k] = v[e];
        } else {
            col[k] = pad;
            val[k] = 0.0;
        }
    }
}

// v when c, else +0.0, as a bit mask (keeps the loads of both branches
// unconditional)
__device__ __forceinline__ double keep_if(double v, bool c) {
    return __longlong_as_double(__double_as_longlong(v) & -(long long)c);
}

// This lane's share (keys q = part, part + T, ...) of the two sums of
// f at key kp: F = sum d^2 over keys <= kp, A = sum a^2 over keys > kp
__device__ __forceinline__ void f_parts(const TinyLds &t, int Nf, unsigned long long kp, int part,
                                        int T, double &F, double &A) {
    F = 0.0;
    A = 0.0;
    int q = part;
    for (; q + 3 * T < Nf; q += 4 * T) {
        unsigned long long kq[4];
        double2 da[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            kq[u] = t.tkey[q + u * T];
            da[u] = t.tda[q + u * T];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool c = kq[u] <= kp;
            F += keep_if(da[u].x, c);
            A += keep_if(da[u].y, !c);
        }
    }
    for (; q < Nf; q += T) {
        const unsigned long long kq = t.tkey[q];
        const double2 da = t.tda[q];
        const bool c = kq <= kp;
        F += keep_if(da.x, c);
        A += keep_if(da.y, !c);
    }
}

// A group of whole waves, threads [B, B + N) of the workgroup, that runs the
// check: the whole workgroup, or, when the check overlaps the iterations of
// the next block, the upper half
template <int B, int N>
struct Grp {
    static constexpr int base = B, size = N, waves = N / 64;
    static_assert(B % 64 == 0 && N % 64 == 0 && N > 0, "whole waves");
    static __device__ __forceinline__ int tid() { return (int)threadIdx.x - B; }
};

// The barrier of a group of waves: the workgroup barrier, or, for a group
// that shares the workgroup with another one running other code, a counter
// in LDS that each wave of the group raises by one and then waits on until
// every wave of the group has raised it (the count only grows, so a wave
// already at the next barrier does not disturb one still waiting).  A wait
// longer than any correct run needs stops waiting and flags the run (ends
// it as a numerical breakdown) rather than hang.
struct Barriers {
    unsigned n = 0;        // barriers passed
    unsigned *ctr = nullptr;  // the group's counter (null: workgroup barrier)
    int *fault = nullptr;  // set when a wait ran out
    int waves = 0;         // waves of the group
    bool sleep = true;     // sleep between polls (yield the SIMD to the other group)
    __device__ __forceinline__ void operator()() {
        ++n;
        if (!ctr) {
            __syncthreads();
            return;
        }
        // the same in every lane; counts wrap modulo 2^32, and a wave is
        // never more than a barrier ahead, so the signed difference decides
        const unsigned target = __builtin_amdgcn_readfirstlane(n * (unsigned)waves);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if ((threadIdx.x & 63) == 0)
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        // the count is read as one value per wave, so the wait is a scalar loop
        auto behind = [&]() {
            const unsigned seen = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
            return (int)(target - seen) > 0;
        };
        int polls = 0;
        while (behind()) {
            if (sleep) __builtin_amdgcn_s_sleep(1);
            if (++polls > (1 << 24)) {
                *fault = 1;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
};

// block_sums over the waves of group G only (sh holds G::waves * K doubles);
// the sums end in every lane of the group's first wave
template <int K, class G>
__device__ __forceinline__ void group_block_sums(double (&v)[K], double *sh, Barriers &bar) {
    static_assert(K <= 64, "one lane per value");
    const int w = G::tid() >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sh[w * K + k] = v[k];
    }
    bar();
    if (w == 0) {
        double s = 0.0;
        if (lane < K) {
#pragma unroll
            for (int i = 0; i < G::waves; ++i) s += sh[i * K + lane];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = lane_f64(s, k);
    }
    bar();
}

struct TrShared {
    double red[kWaves * 5];
    unsigned long long best;  // largest key with f <= r^2, plus one (0: none)
    unsigned long long hi;    // smallest sampled key with f > r^2 (kNoKey: none)
    int go;
    int nf;                   // breakpoints with a finite key
    int nc;                   // candidates left after the sampled bracket
    int woff[2][kWaves];      // compaction offsets of each wave's finite keys
};

constexpr unsigned long long kInfKey = 0x7FF0000000000000ull;  // key of lambda = inf

// The trust region of one slot (ts armed with r, r^2) over the N = n + m
// (<= 2 G::size) coordinates of e.  Called by every thread of group G.
template <class G, class E>
__device__ void tiny_trust_region(const E &e, TRState &ts, const TinyLds &t, TrShared &sh,
                                  Barriers &bar) {
    constexpr int GW = G::size, GN = G::waves;
    const int tid = G::tid(), w = tid >> 6, lane = threadIdx.x & 63;
    const int N = (int)e.size();
    // keys and squares of this thread's (at most two) coordinates, and the
    // sums of the full-box test (first line of Algorithm 2)
    unsigned long long key[2];
    double d2[2], a2[2], ad[2];
    bool fin[2];
    double v5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // sum d^2 (finite d), #inf d, sum a d, #bad,
                                               // sum a^2 of infinite keys
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int p = r * GW + tid;
        key[r] = kNoKey;
        d2[r] = a2[r] = ad[r] = 0.0;
        if (p < N) {
            double a, d;
            e.get(p, a, d);
            if (bad_pair(a, d)) {
                v5[3] += 1.0;
            } else if (a > 0.0) {
                key[r] = key_of(a, d);
                d2[r] = d * d;
                a2[r] = a * a;
                ad[r] = a * d;
                if (d < INFINITY) {
                    v5[0] += d2[r];
                    v5[2] += ad[r];
                } else {
                    v5[1] += 1.0;
                }
                if (key[r] >= kInfKey) v5[4] += a2[r];
            }
        }
        // a breakpoint with an infinite key is never clamped: f there is
        // the whole box, larger than r^2 once the full-box test failed
        fin[r] = key[r] < kInfKey;
        const unsigned long long bal = __ballot(fin[r]);
        if (lane == 0) sh.woff[r][w] = __popcll(bal);
    }
    group_block_sums<5, G>(v5, sh.red, bar);
    if (tid == 0) {
        int o = 0;
        for (int r = 0; r < 2; ++r)
            for (int q = 0; q < GN; ++q) {
                const int c = sh.woff[r][q];
                sh.woff[r][q] = o;
                o += c;
            }
        sh.nf = o;
        sh.go = 0;
        sh.best = 0ull;
        sh.hi = kNoKey;
        if (v5[3] > 0.0) {
            ts.nan_seen = 1;
            ts.mode = TR_ZERO;
            ts.rho = NAN;
            ts.lam = NAN;
            ts.value = NAN;
        } else if (!(ts.r > 0.0)) {
            ts.mode = TR_ZERO;
            ts.rho = 0.0;
            ts.lam = 0.0;
            ts.value = 0.0;
        } else if (v5[1] == 0.0 && v5[0] <= ts.r2) {
            ts.mode = TR_FULLBOX;
            ts.value = v5[2];
            ts.rho = v5[2] / ts.r;
            ts.lam = INFINITY;
        } else {
            sh.go = 1;
            ts.value = v5[4];  // sum a^2 over infinite keys, until the final pass
        }
    }
    bar();
    if (!sh.go) return;
    // the finite keys, compacted in coordinate order
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const unsigned long long bal = __ballot(fin[r]);
        if (fin[r]) {
            const int at = sh.woff[r][w] + __popcll(bal & lt);
            t.tkey[at] = key[r];
            t.tda[at] = make_double2(d2[r], a2[r]);
            t.tad[at] = ad[r];
        }
    }
    bar();
    const int Nf = sh.nf;
    const double Ainf = ts.value;

    // f is nondecreasing in the key, so the answer is the largest finite
    // key with f <= r^2 (equal keys give equal sums: no grouping needed).
    // f at 64 breakpoints spread over the coordinate order brackets it;
    // then f at every breakpoint strictly inside the bracket.
    const double r2 = ts.r2;
    constexpr int S = 64, TS = GW / S;
    if (Nf > S) {
        const int part = tid & (TS - 1);
        const int p = (int)((long long)(tid / TS) * Nf / S);
        const unsigned long long kp = t.tkey[p];
        double F, A;
        f_parts(t, Nf, kp, part, TS, F, A);
        F = group_sum_c<TS>(F);
        A = group_sum_c<TS>(A) + Ainf;
        if (part == 0) {
            const double lam = __longlong_as_double((long long)kp);
            if (F + lam * lam * A <= r2) atomicMax(&sh.best, kp + 1ull);
            else atomicMin(&sh.hi, kp);
        }
        bar();
    }
    {
        const unsigned long long b0 = sh.best, hi = sh.hi;
        bool inc[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int p = r * GW + tid;
            inc[r] = false;
            if (p < Nf) {
                const unsigned long long k = t.tkey[p];
                inc[r] = (b0 == 0ull || k > b0 - 1ull) && k < hi;
            }
            const unsigned long long bal = __ballot(inc[r]);
            if (lane == 0) sh.woff[r][w] = __popcll(bal);
        }
        bar();
        if (tid == 0) {
            int o = 0;
            for (int r = 0; r < 2; ++r)
                for (int q = 0; q < GN; ++q) {
                    const int c = sh.woff[r][q];
                    sh.woff[r][q] = o;
                    o += c;
                }
            sh.nc = o;
        }
        bar();
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const unsigned long long bal = __ballot(inc[r]);
            if (inc[r]) t.tcid[sh.woff[r][w] + __popcll(bal & lt)] = r * GW + tid;
        }
        bar();
    }
    const int nc = sh.nc;
    int T = 1;
    while (T < 64 && (long long)nc * (2 * T) <= GW) T <<= 1;
    const int part = tid & (T - 1);
    for (int c = tid / T; c < nc; c += GW / T) {
        const unsigned long long kp = t.tkey[t.tcid[c]];
        double F, A;
        f_parts(t, Nf, kp, part, T, F, A);
        F = group_sum(F, T);
        A = group_sum(A, T) + Ainf;
        if (part == 0) {
            const double lam = __longlong_as_double((long long)kp);
            if (F + lam * lam * A <= r2) atomicMax(&sh.best, kp + 1ull);
        }
    }
    bar();
    const unsigned long long bk = sh.best;
    const bool has = bk != 0ull;
    const unsigned long long klo = bk - 1ull;

    // F = sum d^2 (clamped), A = sum a^2 (free), AD = sum a d (clamped)
    double v3[3] = {0.0, 0.0, 0.0};
    for (int i = tid; i < Nf; i += GW) {
        const double2 da = t.tda[i];
        const double adi = t.tad[i];
        const bool c = has && t.tkey[i] <= klo;
        v3[0] += keep_if(da.x, c);
        v3[1] += keep_if(da.y, !c);
        v3[2] += keep_if(adi, c);
    }
    group_block_sums<3, G>(v3, sh.red, bar);
    if (tid == 0) {
        const double Fs = v3[0], As = v3[1] + Ainf, AD = v3[2];
        double lam, val;
        if (As > 0.0) {
            double num = ts.r2 - Fs;
            if (num < 0.0) num = 0.0;
            lam = sqrt(num / As);
            val = AD + lam * As;
        } else {
            lam = INFINITY;
            val = AD;
        }
        ts.klo = has ? klo : 0ull;
        ts.lam = lam;
        ts.value = val;
        ts.rho = val / ts.r;
        ts.mode = TR_RESOLVED;
    }
    bar();
}

// Threads of the iteration group when the check overlaps the next block's
// iterations; the check group is the rest of the workgroup
constexpr int kTinyTI = WG / 2;

// Rows of A' and A held in registers by one thread (register mode), and
// the lanes that reduce each row
struct TinyRows {
    int pc[K], dc[K];
    double pv[K], dv[K];
    int Lp, Ld, lp, gp, ld, gd;
};

// The check of Section 7 after a block of iterations, run by group G: the
// averages, then A x-bar, A'y-bar and A'y, the KKT sums and the stopping
// test, the trust regions of the normalized duality gap, the restart test
// of eq. adaptive-restart-scheme and the restart of Algorithm 1.  L views
// the state the check reads (the live arrays, or a copy of them taken at
// the end of the block when the next block already runs); the averages,
// products and trust-region work go to t.  Ends with a barrier.
template <bool REG, int LP, int LD, class G>
__device__ void tiny_check(const Dev &L, const TinyArgs &a, const TinyLds &t, DevState &sst,
                           TrShared &trs, double *red, int &armed, const TinyRows &rw,
                           Barriers &bar) {
    const int ct = G::tid();
    const int n = L.n, m = L.m;
    const long long tt = sst.t;
    for (int i = ct; i < n + m; i += G::size) average_at(L, i, tt);
    bar();
    if (REG) {
        if (rw.gd < m) {
            const double s = reg_dot<LD>(rw.dc, rw.dv, t.xb);
            if (rw.ld == 0) t.axb[rw.gd] = s;
        }
        if (rw.gp < n) {
            const double s1 = reg_dot<LP>(rw.pc, rw.pv, t.yb);
            const double s2 = reg_dot<LP>(rw.pc, rw.pv, L.y);
            if (rw.lp == 0) {
                t.atyb[rw.gp] = s1;
                t.aty[rw.gp] = s2;
            }
        }
    } else {
        for (int i = rw.gd; i < m; i += G::size / rw.Ld) {
            const double s = row_dot(t.arp, t.aci, t.av, t.xb, i, rw.ld, rw.Ld);
            if (rw.ld == 0) t.axb[i] = s;
        }
        for (int j = rw.gp; j < n; j += G::size / rw.Lp) {
            const double s1 = row_dot(t.trp, t.tci, t.tv, t.yb, j, rw.lp, rw.Lp);
            const double s2 = row_dot(t.trp, t.tci, t.tv, L.y, j, rw.lp, rw.Lp);
            if (rw.lp == 0) {
                t.atyb[j] = s1;
                t.aty[j] = s2;
            }
        }
    }
    bar();
    // KKT at z and z-bar, distances to the anchor, stopping test
    double v[kKktSums];
#pragma unroll
    for (int k = 0; k < kKktSums; ++k) v[k] = 0.0;
    const KktPoints P2{{L.x, t.xb}, {L.y, t.yb}, {L.q, t.axb}, {t.aty, t.atyb}};
    for (int i = ct; i < n + m; i += G::size) kkt_elem(L, P2, i, v);
    group_block_sums<kKktSums, G>(v, red, bar);
    if (ct < 64) {
        const int sl = kkt_conclude(L, v, a.tol, a.kkt_kind, a.omega, a.gap_slots);
        if (ct == 0) armed = sl;
    }
    bar();
    const int slots = armed;
    for (int sidx = 0; sidx < kTrSlots; ++sidx) {
        if (!(slots & (1 << sidx))) continue;
        GapElems e;
        e.n = n;
        e.m = m;
        e.c = t.c;
        e.b = t.b;
        e.l = t.l;
        e.u = t.u;
        e.kind = t.kind;
        e.x = sidx == 0 ? t.xb : L.x;
        e.y = sidx == 0 ? t.yb : L.y;
        e.ax = sidx == 0 ? t.axb : L.q;
        e.aty = sidx == 0 ? t.atyb : t.aty;
        e.sw = a.sw;
        tiny_trust_region<G>(e, sst.tr[sidx], t, trs, bar);
    }
    if (ct == 0) decide_restart(L, a.beta, a.tau0);
    bar();
    if (sst.restarted) {
        const int cand = sst.cand;
        const int mx = n > m ? n : m;
        for (int i = ct; i < mx; i += G::size) apply_restart_at(L, i, cand);
        bar();
    }
}

// OV: the check of a block runs on the upper half of the workgroup while
// the lower half already runs the next block's iterations (register mode
// only, every row within half the workgroup).  The check reads a copy of
// the state taken at the end of its block.  Each half synchronizes its own
// waves (group barriers in LDS, so neither waits on the other's steps);
// the workgroup barrier only closes each round.  The iteration waves run
// at a higher priority and poll without sleeping: the iterations are the
// longer part.  When the check restarts or stops the solve, the block run
// beside it is dropped and the state taken back from the copy, so the
// iterates and checks are exactly those of the plain order.
template <bool REG, int LP, int LD, bool OV>
__device__ __forceinline__ void tiny_body(const Dev &d, const TinyArgs &a) {
    static_assert(!OV || REG, "the overlapped check needs the rows in registers");
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ DevState sst;
    __shared__ TrShared trs;
    __shared__ double red[kWaves * kKktSums];
    __shared__ int armed;
    __shared__ unsigned gctr[2];  // OV: group barrier counters
    __shared__ int gfault;   // OV: a group barrier wait ran out
    using GC = Grp<OV ? kTinyTI : 0, OV ? WG - kTinyTI : WG>;  // the check group
    const int tid = threadIdx.x;
    const bool in_it = !OV || tid < kTinyTI;      // runs the iterations
    const int gt = in_it ? tid : tid - kTinyTI;   // index within its group
    if (OV && in_it) __builtin_amdgcn_s_setprio(3);
    const int n = d.n, m = d.m, nnz = d.nnz;
    const TinyLds t = carve(lds, n, m, nnz, REG, OV);
    if (tid == 0) sst = *d.st;
    for (int j = tid; j < n; j += WG) {
        t.x[j] = d.x[j];
        t.sx[j] = d.sx[j];
        t.c[j] = d.c[j];
        t.l[j] = d.l[j];
        t.u[j] = d.u[j];
        if (OV) {
            t.sn_x[j] = d.x[j];
            t.sn_sx[j] = d.sx[j];
        }
    }
    for (int i = tid; i < m; i += WG) {
        t.y[i] = d.y[i];
        t.sy[i] = d.sy[i];
        t.q[i] = d.q[i];
        t.b[i] = d.b[i];
        t.kind[i] = d.kind ? d.kind[i] : (signed char)0;
        if (OV) {
            t.sn_y[i] = d.y[i];
            t.sn_sy[i] = d.sy[i];
            t.sn_q[i] = d.q[i];
        }
    }
    if (tid == 0) {
        t.x[n] = 0.0;
        t.xb[n] = 0.0;
        t.y[m] = 0.0;
        t.yb[m] = 0.0;
        if (OV) {
            t.sn_x[n] = 0.0;
            t.sn_y[m] = 0.0;
        }
        gctr[0] = 0u;
        gctr[1] = 0u;
        gfault = 0;
    }
    if (!REG) {
        for (int e = tid; e < nnz; e += WG) {
            t.av[e] = d.v[e];
            t.aci[e] = (unsigned short)d.ci[e];
            t.tv[e] = d.tv[e];
            t.tci[e] = (unsigned short)d.tci[e];
        }
        for (int i = tid; i <= m; i += WG) t.arp[i] = d.rp[i];
        for (int j = tid; j <= n; j += WG) t.trp[j] = d.trp[j];
    }

    // rows in registers: LP lanes per row of A', LD per row of A (each
    // group holds its own copy when the check overlaps the iterations)
    TinyRows rw;
    rw.Lp = REG ? LP : a.Lp;
    rw.Ld = REG ? LD : a.Ld;
    rw.lp = gt & (rw.Lp - 1);
    rw.gp = gt / rw.Lp;
    rw.ld = gt & (rw.Ld - 1);
    rw.gd = gt / rw.Ld;
    const int Gp = WG / rw.Lp, Gd = WG / rw.Ld;  // rows per pass of the LDS mode
    const int Lp = rw.Lp, Ld = rw.Ld, lp = rw.lp, gp = rw.gp, ld = rw.ld, gd = rw.gd;
    const double tau = a.tau, sigma = a.sigma;
    if (REG) {
        load_row(d.trp, d.tci, d.tv, gp, n, lp, Lp, m, rw.pc, rw.pv);
        load_row(d.rp, d.ci, d.v, gd, m, ld, Ld, n, rw.dc, rw.dv);
    }
    const bool pown = REG && in_it && gp < n && lp == 0;  // owner of primal row gp
    const bool down = REG && in_it && gd < m && ld == 0;  // owner of dual row gd
    double xj = 0.0, sxj = 0.0, cj = 0.0, lj = 0.0, uj = 0.0;
    double yi = 0.0, syi = 0.0, qi = 0.0, bi = 0.0;
    int ki = 0;
    __syncthreads();
    if (pown) {
        xj = t.x[gp];
        sxj = t.sx[gp];
        cj = t.c[gp];
        lj = t.l[gp];
        uj = t.u[gp];
    }
    if (down) {
        yi = t.y[gd];
        syi = t.sy[gd];
        qi = t.q[gd];
        bi = t.b[gd];
        ki = t.kind[gd];
    }

    // the solver state as the check sees it: LDS copies of everything but
    // the anchor and the check log (with the overlap: the copy taken at
    // the end of the block being checked)
    Dev L = d;
    L.x = OV ? t.sn_x : t.x;
    L.sx = OV ? t.sn_sx : t.sx;
    L.c = t.c;
    L.l = t.l;
    L.u = t.u;
    L.xbar = t.xb;
    L.aty = t.aty;
    L.atyb = t.atyb;
    L.y = OV ? t.sn_y : t.y;
    L.sy = OV ? t.sn_sy : t.sy;
    L.q = OV ? t.sn_q : t.q;
    L.b = t.b;
    L.ybar = t.yb;
    L.axb = t.axb;
    L.kind = t.kind;
    L.st = &sst;

    // P iterations of eq. (PDHG-update) from the live state; each half-step
    // ends with a barrier (bar)
    auto iterations = [&](Barriers &bar) {
        for (int it = 0; it < a.P; ++it) {
            // x+ = proj_[l,u](x - tau (c - A'y)); sx += x+
            if (REG) {
                if (gp < n && in_it) {
                    const double aty = reg_dot<LP>(rw.pc, rw.pv, t.y);
                    if (lp == 0) {
                        const double g = cj - aty;
                        double xn = xj - tau * g;
                        if (xn < lj) xn = lj;
                        if (xn > uj) xn = uj;
                        xj = xn;
                        sxj += xn;
                        t.x[gp] = xn;
                    }
                }
            } else {
                for (int j = gp; j < n; j += Gp) {
                    const double aty = row_dot(t.trp, t.tci, t.tv, t.y, j, lp, Lp);
                    if (lp == 0) {
                        const double g = t.c[j] - aty;
                        double xn = t.x[j] - tau * g;
                        const double lo = t.l[j], hi = t.u[j];
                        if (xn < lo) xn = lo;
                        if (xn > hi) xn = hi;
                        t.x[j] = xn;
                        t.sx[j] += xn;
                    }
                }
            }
            bar();
            // y+ = proj_Y(y + sigma (b - (2 A x+ - A x))); sy += y+; q = A x+
            if (REG) {
                if (gd < m && in_it) {
                    const double ax = reg_dot<LD>(rw.dc, rw.dv, t.x);
                    if (ld == 0) {
                        double yv = yi + sigma * (bi - (2.0 * ax - qi));
                        if (ki && yv < 0.0) yv = 0.0;
                        yi = yv;
                        syi += yv;
                        qi = ax;
                        t.y[gd] = yv;
                    }
                }
            } else {
                for (int i = gd; i < m; i += Gd) {
                    const double ax = row_dot(t.arp, t.aci, t.av, t.x, i, ld, Ld);
                    if (ld == 0) {
                        double yv = t.y[i] + sigma * (t.b[i] - (2.0 * ax - t.q[i]));
                        if (t.kind[i] && yv < 0.0) yv = 0.0;
                        t.y[i] = yv;
                        t.sy[i] += yv;
                        t.q[i] = ax;
                    }
                }
            }
            bar();
        }
    };

    if (!OV) {
        for (int blk = 0; blk < a.blocks; ++blk) {
            if (sst.done) break;  // uniform: every write to sst precedes a barrier
            Barriers bar;
            iterations(bar);
            if (pown) t.sx[gp] = sxj;
            if (down) {
                t.sy[gd] = syi;
                t.q[gd] = qi;
            }
            if (tid == 0) {
                sst.k += a.P;
                sst.t += a.P;
            }
            __syncthreads();
            tiny_check<REG, LP, LD, GC>(L, a, t, sst, trs, red, armed, rw, bar);
            if (sst.restarted && pown) {
                xj = t.x[gp];
                sxj = t.sx[gp];
            }
            if (sst.restarted && down) {
                yi = t.y[gd];
                syi = t.sy[gd];
                qi = t.q[gd];
            }
            __syncthreads();
        }
    } else {
        // rounds: the iteration group runs block blk (when the budget and
        // the state allow) while the check group checks the copy taken at
        // the end of the previous block (when one is pending)
        bool pending = false;
        int blk = 0;
        Barriers gbar;
        gbar.ctr = &gctr[in_it ? 0 : 1];
        gbar.fault = &gfault;
        gbar.waves = in_it ? kTinyTI / 64 : (WG - kTinyTI) / 64;
        gbar.sleep = !in_it;
        while (true) {
            const bool run = !sst.done && blk < a.blocks;  // uniform (read after a barrier)
            if (!run && !pending) break;
            if (in_it) {
                if (run) iterations(gbar);
            } else if (pending) {
                tiny_check<REG, LP, LD, GC>(L, a, t, sst, trs, red, armed, rw, gbar);
            }
            __syncthreads();
            if (gfault) {  // uniform; correct code never gets here
                if (tid == 0) {
                    sst.numerr = 1;
                    sst.done = 1;
                }
                __syncthreads();
                break;
            }
            // the check's outcome decides whether the block just run stands
            bool keep = run;
            if (pending && (sst.done || sst.restarted)) {
                keep = false;
                for (int j = tid; j < n; j += WG) {
                    t.x[j] = t.sn_x[j];
                    t.sx[j] = t.sn_sx[j];
                }
                for (int i = tid; i < m; i += WG) {
                    t.y[i] = t.sn_y[i];
                    t.sy[i] = t.sn_sy[i];
                    t.q[i] = t.sn_q[i];
                }
            }
            if (keep) {
                if (pown) {
                    t.sn_x[gp] = xj;
                    t.sn_sx[gp] = sxj;
                }
                if (down) {
                    t.sn_y[gd] = yi;
                    t.sn_sy[gd] = syi;
                    t.sn_q[gd] = qi;
                }
            }
            __syncthreads();
            if (!keep && pending && (sst.done || sst.restarted)) {
                if (pown) {
                    xj = t.x[gp];
                    sxj = t.sx[gp];
                }
                if (down) {
                    yi = t.y[gd];
                    syi = t.sy[gd];
                    qi = t.q[gd];
                }
            }
            if (tid == 0 && keep) {
                sst.k += a.P;
                sst.t += a.P;
            }
            if (keep) ++blk;
            pending = keep;
            __syncthreads();
        }
    }

    // the state: the live arrays (with the overlap, the copy, which holds
    // the last checked point)
    const double *fx = OV ? t.sn_x : t.x, *fsx = OV ? t.sn_sx : t.sx;
    const double *fy = OV ? t.sn_y : t.y, *fsy = OV ? t.sn_sy : t.sy, *fq = OV ? t.sn_q : t.q;
    for (int j = tid; j < n; j += WG) {
        d.x[j] = fx[j];
        d.sx[j] = fsx[j];
        d.xbar[j] = t.xb[j];
        d.aty[j] = t.aty[j];
        d.atyb[j] = t.atyb[j];
    }
    for (int i = tid; i < m; i += WG) {
        d.y[i] = fy[i];
        d.sy[i] = fsy[i];
        d.q[i] = fq[i];
        d.ybar[i] = t.yb[i];
        d.axb[i] = t.axb[i];
    }
    if (tid == 0) {
        *d.st = sst;
        if (a.summary) {
            a.summary[0] = sst.k;
            a.summary[1] = (long long)sst.done | ((long long)(sst.conv_which + 1) << 8) |
                           ((long long)sst.numerr << 16);
        }
    }
}

template <bool REG, int LP, int LD, bool OV>
__global__ __launch_bounds__(WG) void k_tiny_blocks(Dev d, TinyArgs a) {
    tiny_body<REG, LP, LD, OV>(d, a);
}

// one LP per workgroup: the solver view and arguments of LP blockIdx.x
template <bool REG, int LP, int LD, bool OV>
__global__ __launch_bounds__(WG) void k_tiny_many(const Dev *__restrict__ devs,
                                                  const TinyArgs *__restrict__ args) {
    const Dev d = devs[blockIdx.x];
    const TinyArgs a = args[blockIdx.x];
    if (a.blocks > 0) tiny_body<REG, LP, LD, OV>(d, a);
}

// lanes per row with the matrix in LDS: about four entries per lane
int lanes_lds(long long nnz, long long rows) {
    const long long avg = rows > 0 ? (nnz + rows - 1) / rows : 0;
    int L = 1;
    while (L < 64 && 4ll * L < avg) L <<= 1;
    return L;
}

// lanes per row with rows in registers: the fewest (1, 2, 4 or 8) that
// hold the longest row in K entries each, or 0 when none does
int lanes_reg(long long maxlen) {
    int L = 1;
    while (L < 8 && (long long)K * L < maxlen) L <<= 1;
    return (long long)K * L < maxlen ? 0 : L;
}

// kernels by (LP, LD), both in {1, 2, 4, 8}, and OV; MANY picks the
// one-LP-per-workgroup form
template <bool MANY, int LP, bool OV>
const void *tiny_fn_ld(int Ld) {
    switch (Ld) {
    case 1: return MANY ? (const void *)k_tiny_many<true, LP, 1, OV> : (const void *)k_tiny_blocks<true, LP, 1, OV>;
    case 2: return MANY ? (const void *)k_tiny_many<true, LP, 2, OV> : (const void *)k_tiny_blocks<true, LP, 2, OV>;
    case 4: return MANY ? (const void *)k_tiny_many<true, LP, 4, OV> : (const void *)k_tiny_blocks<true, LP, 4, OV>;
    default: return MANY ? (const void *)k_tiny_many<true, LP, 8, OV> : (const void *)k_tiny_blocks<true, LP, 8, OV>;
    }
}

template <bool MANY, bool OV>
const void *tiny_fn_lp(int Lp, int Ld) {
    switch (Lp) {
    case 1: return tiny_fn_ld<MANY, 1, OV>(Ld);
    case 2: return tiny_fn_ld<MANY, 2, OV>(Ld);
    case 4: return tiny_fn_ld<MANY, 4, OV>(Ld);
    default: return tiny_fn_ld<MANY, 8, OV>(Ld);
    }
}

template <bool MANY>
const void *tiny_kernel(const TinyPlan &p) {
    if (!p.reg)
        return MANY ? (const void *)k_tiny_many<false, 0, 0, false>
                    : (const void *)k_tiny_blocks<false, 0, 0, false>;
    return p.ov ? tiny_fn_lp<MANY, true>(p.Lp, p.Ld) : tiny_fn_lp<MANY, false>(p.Lp, p.Ld);
}

}  // namespace

TinyPlan tiny_plan(const Dev &d, hipStream_t s) {
    TinyPlan p{};
    p.ok = 0;
    // PDHG_TINY=0 turns the path off, PDHG_TINY=lds keeps the matrix in LDS
    const char *env = getenv("PDHG_TINY");
    if (env && env[0] == '0') return p;
    const bool force_lds = env && env[0] == 'l';
    const int n = d.n, m = d.m;
    if (m < 1 || n < 1 || (long long)n + m > kTinyMaxCoords) return p;
    std::vector<int> rp(m + 1), trp(n + 1);
    if (hipMemcpyAsync(rp.data(), d.rp, sizeof(int) * (m + 1), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(trp.data(), d.trp, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return p;
    int amax = 0, tmax = 0;
    for (int i = 0; i < m; ++i) amax = rp[i + 1] - rp[i] > amax ? rp[i + 1] - rp[i] : amax;
    for (int j = 0; j < n; ++j) tmax = trp[j + 1] - trp[j] > tmax ? trp[j + 1] - trp[j] : tmax;
    // one row per group of lanes
    const int Lp = lanes_reg(tmax), Ld = lanes_reg(amax);
    if (Lp > 0 && Ld > 0 && (long long)n * Lp <= WG && (long long)m * Ld <= WG && !force_lds) {
        p.reg = 1;
        p.Lp = Lp;
        p.Ld = Ld;
    } else {
        p.reg = 0;
        p.Lp = lanes_lds(d.nnz, n);
        p.Ld = lanes_lds(d.nnz, m);
    }
    p.lds = tiny_lds_bytes(n, m, d.nnz, p.reg);
    if (p.lds > kTinyLdsMax) return p;
    // the check beside the next block's iterations: rows in registers,
    // every row within half the workgroup, every trust-region coordinate
    // within two per thread of the other half, and room for the copy it
    // reads (PDHG_TINY_OVERLAP=0 turns it off)
    const char *eo = getenv("PDHG_TINY_OVERLAP");
    p.ov = 0;
    if (p.reg && !(eo && eo[0] == '0') && (long long)n * p.Lp <= kTinyTI &&
        (long long)m * p.Ld <= kTinyTI && (long long)n + m <= 2ll * (WG - kTinyTI) &&
        tiny_lds_bytes(n, m, d.nnz, 1, 1) <= kTinyLdsMax) {
        p.ov = 1;
        p.lds = tiny_lds_bytes(n, m, d.nnz, 1, 1);
    }
    // the limit belongs to the kernel, shared by every handle that uses it:
    // raise it to the cap, never to one handle's size
    for (int many = 0; many < 2; ++many) {
        const void *fn = many ? tiny_kernel<true>(p) : tiny_kernel<false>(p);
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kTinyLdsMax) != hipSuccess) {
            (void)hipGetLastError();
            return p;
        }
    }
    p.ok = 1;
    return p;
}

hipError_t launch_tiny_blocks(const Dev &d, const TinyArgs &a, const TinyPlan &p, hipStream_t s) {
    const void *fn = tiny_kernel<false>(p);
    Dev dd = d;
    TinyArgs aa = a;
    void *args[] = {(void *)&dd, (void *)&aa};
    return hipLaunchKernel(fn, dim3(1), dim3(WG), args, p.lds, s);
}

hipError_t launch_tiny_many(const Dev *devs, const TinyArgs *args, int count, const TinyPlan &p,
                            size_t lds, hipStream_t s) {
    const void *fn = tiny_kernel<true>(p);
    const Dev *dv = devs;
    const TinyArgs *av = args;
    void *kargs[] = {(void *)&dv, (void *)&av};
    return hipLaunchKernel(fn, dim3(count), dim3(WG), kargs, lds, s);
}

}  // namespace pdhg
