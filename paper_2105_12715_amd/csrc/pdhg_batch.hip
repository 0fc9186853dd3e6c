// Batched restarted PDHG: many independent LPs solved by the same launches.
//
// The LPs are concatenated into one block-diagonal CSR (rows of LP i follow
// those of LP i-1, column indices shifted by its column offset), so each
// half-step of eq. PDHG-update is one SpMV launch over every LP at once
// with the update fused into the row epilogue.  Each LP keeps its own step
// sizes, iteration and restart counters, trust-region bracket and done
// flag (struct BLP).  The SpMV blocks are split per LP, so every block
// belongs to one LP: a block of a converged LP exits at once, and the
// others take their LP's step sizes from its record.  Inside each LP the
// columns are held sorted by entry count and first row (the API converts
// column vectors at the boundary), and A and A' also carry 16-bit indices
// relative to their LP when every LP is narrow enough.
//
// Per-LP reductions (KKT, radii, the normalized duality gap of eq. rhorz,
// power iteration) run over a block table: the element space of LP i
// (its n_i primal coordinates, then its m_i dual ones) is cut into chunks
// of kChunk elements, each owned by one block, and a workgroup per LP
// reduces its blocks' partial sums in a fixed order.  The trust region is
// the same radix bisection on the multiplier as the single-LP solver, with
// a histogram and a bracket per LP.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "pdhg.h"
#include "pdhg_device.h"

namespace pdhg {

constexpr int kChunk = 2048;  // elements per block of the per-LP passes
constexpr int kXcds = 8;      // accelerator dies; workgroup i runs on die i mod 8
constexpr int kBLog = 512;    // check records kept per LP

struct BLP {
    // sizes and offsets in the concatenated arrays
    int m, n, row_off, col_off;
    int blk_begin, blk_end;  // element blocks of this LP
    double eta, tau, sigma, omega, beta, sw;
    int tau0, pad0;
    // Algorithm 1 state
    long long k, t, restarts, checks;
    double rho_prev;
    int done, conv_which;
    long long conv_k;
    double kkt_cur[8], kkt_avg[8];
    double r_avg, r_cur;
    int restarted, cand, gap_slots, numerr, in_check, pad1;
    long long t_check;  // t when the last check started (window length of a restart)
    double nb2, nc2;
    // power iteration
    double pw_est, pw_prev, pw_s;
    int pw_done, pw_it;
    TRState tr[kTrSlots];
};

struct BDev {
    int count, M, N, NNZ, nblk;
    int *rp, *ci;
    double *v, *c, *b, *l, *u;
    signed char *kind;
    int *trp, *tci, *perm;
    double *tv;
    int *cursor, *long_rows;
    // column order inside each LP's column range (null: the caller's order)
    int *cperm;  // [N] internal column -> caller's column
    int *cinv;   // [N] caller's column -> internal column
    // bound classes over the whole batch, as for a single LP (bcls null: the
    // primal update reads l and u)
    const unsigned char *bcls;
    double blo[kBoundClasses], bhi[kBoundClasses];
    int nbcls;
    int *brA, *brT;
    int nblkA, nblkT;
    int *xpA, *xpT;        // workgroup -> merge-path block (XCD placement), -1: none;
                           // null: workgroup i runs block i
    int nslotA, nslotT;    // workgroups of the SpMV launches
    int *lp_row, *lp_col;
    double *tau_col, *sigma_row;  // step of each column / row's LP, 0 once it converged
    int *blk_lp, *blk_first;
    // SpMV blocks never span two LPs: LP i owns blocks blkA[i] .. blkA[i+1]-1
    // of A and blkT[i] .. of A'; lp_r0 / lp_c0 ([count + 1]) are the LPs'
    // row and column offsets.  When every LP has at most 65,536 rows and
    // columns, ci16 / tci16 hold A's column and A''s row indices relative to
    // their LP (null otherwise).
    int *blkA, *blkT, *lp_r0, *lp_c0;
    unsigned short *ci16, *tci16;
    double *x, *y, *x0, *y0, *sx, *sy, *q, *xbar, *ybar, *axb, *atyb, *aty;
    double *part;    // [nblk][kKktSums]
    double *log;     // [count][kBLog][kRec]
    BLP *lp;
    unsigned int *hcnt;  // [count][kTrSlots][2][kBuckets]
    double *hD, *hA;
    double *tpart;       // [kTrSlots][nblk][4]
    unsigned int *ccount;  // [kTrSlots][nblk]
    unsigned int *coff;    // [kTrSlots][nblk + count]
    unsigned long long *ckey;  // [kTrSlots][nblk * kChunk]
    double *ca, *cd;
    int *err;
};

__device__ __forceinline__ size_t hist_at(int lp, int slot, int half) {
    return ((size_t)(lp * kTrSlots + slot) * 2 + half) * kBuckets;
}

// element e of LP L: its index in the concatenated x (e < n) or y array
__device__ __forceinline__ bool elem_is_x(const BLP &L, int e) { return e < L.n; }

// ---------------------------------------------------------------------
// SpMV over the block-diagonal matrix; blocks of converged LPs exit
// ---------------------------------------------------------------------
// Workgroup i runs on XCD i mod 8; xp maps it to a merge-path block so that
// all blocks of one LP share an XCD (and its L2 holds that LP's gathered
// vector), or to -1 for padding.
template <class Epi>
__global__ __launch_bounds__(kWG) void k_bspmv(const int *__restrict__ rp, const int *__restrict__ ci,
                                               const double *__restrict__ v,
                                               const double *__restrict__ xin,
                                               const int *__restrict__ br, int nblk, Epi epi,
                                               const int *__restrict__ lp_of, const BLP *lps,
                                               int gate_kind, const int *__restrict__ xp,
                                               const unsigned short *__restrict__ ci16,
                                               const int *__restrict__ lp_base) {
    __shared__ SpmvShared lds;
    const int c = xp ? xp[blockIdx.x] : (int)blockIdx.x;  // null: blocks in row order
    if (c < 0) return;
    const int r0 = br[c], r1 = br[c + 1];
    if (r0 >= r1) return;
    const int a = lp_of[r0], z = lp_of[r1 - 1];
    const BLP *one = nullptr;  // the block's LP when it holds rows of one LP only
    if (a == z) {
        const BLP &L = lps[a];
        if (gate_kind == 0 ? L.done : L.pw_done) return;
        one = &L;
    }
    const int p0 = br[nblk + 1 + c], p1 = br[nblk + 2 + c];
    decltype(auto) eb = for_block(epi, one);
    // 16-bit indices within the block's LP: the gathered vector is shifted
    // to the LP's first element
    if (ci16 && one) spmv_rows(rp, ci16, v, xin + lp_base[a], r0, r1, p0, p1, eb, lds);
    else spmv_rows(rp, ci, v, xin, r0, r1, p0, p1, eb, lds);
}

// The batch's half-step epilogues: the single-LP updates with per-element
// step sizes; bounds as class bytes and the running sums in pairs of
// iterations as there (smode, sum_mode)
struct EpiPrimalB {
    const double *__restrict__ c, *__restrict__ l, *__restrict__ u;
    double *__restrict__ x, *__restrict__ sx;
    const double *__restrict__ tau;
    const unsigned char *__restrict__ cls;
    double blo[kBoundClasses], bhi[kBoundClasses];
    int smode;
    double *__restrict__ xcopy = nullptr;  // a second copy of x+ (the reverse pass's tape), or null
    __device__ __forceinline__ void operator()(int j, double aty) const { apply(j, aty, 0, 0.0); }
    // one: the block lies in one running LP, whose step is t1
    __device__ __forceinline__ void apply(int j, double aty, int one, double t1) const {
        double g = c[j] - aty;
        const double xo = x[j];
        // tau = 0 leaves a converged LP's x as it is
        double xn = xo - (one ? t1 : tau[j]) * g;
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
        if (xcopy) xcopy[j] = xn;
        if (smode == 0) sx[j] += xn;
        else if (smode == 2) sx[j] = (sx[j] + xo) + xn;
    }
};

struct EpiDualB {
    const double *__restrict__ b;
    const signed char *__restrict__ kind;
    double *__restrict__ y, *__restrict__ sy, *__restrict__ q;
    const double *__restrict__ sigma;
    int smode;
    double *__restrict__ ycopy = nullptr;
    __device__ __forceinline__ void operator()(int i, double ax) const { apply(i, ax, 0, 0.0); }
    __device__ __forceinline__ void apply(int i, double ax, int one, double s1) const {
        const double yo = y[i];
        double yv = yo + (one ? s1 : sigma[i]) * (b[i] - (2.0 * ax - q[i]));
        if (kind[i] && yv < 0.0) yv = 0.0;
        y[i] = yv;
        if (ycopy) ycopy[i] = yv;
        if (smode == 0) sy[i] += yv;
        else if (smode == 2) sy[i] = (sy[i] + yo) + yv;
        q[i] = ax;
    }
};

// The epilogue for one merge-path block: blocks inside one running LP take
// that LP's step from its record (the same value the per-element step
// arrays hold) instead of reading a step per element.
template <class Epi>
__device__ __forceinline__ const Epi &for_block(const Epi &e, const BLP *) {
    return e;
}
template <class Epi>
struct InBlock {  // an epilogue and its block's step (the epilogue is not copied)
    const Epi &e;
    int one;
    double step;
    __device__ __forceinline__ void operator()(int j, double s) const { e.apply(j, s, one, step); }
};
__device__ __forceinline__ InBlock<EpiPrimalB> for_block(const EpiPrimalB &e, const BLP *L) {
    return InBlock<EpiPrimalB>{e, L ? 1 : 0, L ? L->tau : 0.0};
}
__device__ __forceinline__ InBlock<EpiDualB> for_block(const EpiDualB &e, const BLP *L) {
    return InBlock<EpiDualB>{e, L ? 1 : 0, L ? L->sigma : 0.0};
}

static void bspmv_A(const BDev &d, const double *in, double *out, int gate_kind, hipStream_t s) {
    EpiStore e{out};
    hipLaunchKernelGGL(k_bspmv<EpiStore>, dim3(d.nslotA), dim3(kWG), 0, s, d.rp, d.ci, d.v, in,
                       d.brA, d.nblkA, e, d.lp_row, d.lp, gate_kind, d.xpA, d.ci16, d.lp_c0);
}

static void bspmv_T(const BDev &d, const double *in, double *out, int gate_kind, hipStream_t s) {
    EpiStore e{out};
    hipLaunchKernelGGL(k_bspmv<EpiStore>, dim3(d.nslotT), dim3(kWG), 0, s, d.trp, d.tci, d.tv, in,
                       d.brT, d.nblkT, e, d.lp_col, d.lp, gate_kind, d.xpT, d.tci16, d.lp_r0);
}

// The primal update from the A'y (or, for an LP restarted at its average,
// A'y-bar) the check has just computed, over the same blocks and with the
// same gate and steps as the product's launch: a block of one converged LP
// does nothing, a block of several LPs updates every row (a converged LP's
// with step 0).  The check's products ran those blocks, so every row this
// touches has the sum the product would give: bitwise the fused update.
__global__ __launch_bounds__(kWG) void k_bprimal_from_check(const int *__restrict__ br,
                                                            EpiPrimalB epi,
                                                            const int *__restrict__ lp_of,
                                                            const BLP *lps,
                                                            const int *__restrict__ xp,
                                                            const double *__restrict__ aty,
                                                            const double *__restrict__ atyb) {
    const int c = xp ? xp[blockIdx.x] : (int)blockIdx.x;
    if (c < 0) return;
    const int r0 = br[c], r1 = br[c + 1];
    if (r0 >= r1) return;
    const int a = lp_of[r0], z = lp_of[r1 - 1];
    const BLP *one = nullptr;
    if (a == z) {
        if (lps[a].done) return;
        one = &lps[a];
    }
    decltype(auto) eb = for_block(epi, one);
    for (int j = r0 + (int)threadIdx.x; j < r1; j += kWG) {
        const BLP &L = lps[lp_of[j]];
        eb(j, (L.restarted && L.cand == 0) ? atyb[j] : aty[j]);
    }
}

// one iteration; xcopy / ycopy (optional) receive copies of x+ and y+;
// from_check: right after a check, whose A'y the primal update takes
static void b_iteration(const BDev &d, int smode, hipStream_t s, double *xcopy = nullptr,
                        double *ycopy = nullptr, bool from_check = false) {
    EpiPrimalB ep{d.c, d.l, d.u, d.x, d.sx, d.tau_col, d.bcls, {}, {}, smode, xcopy};
    for (int k = 0; k < kBoundClasses; ++k) {
        ep.blo[k] = d.blo[k];
        ep.bhi[k] = d.bhi[k];
    }
    if (from_check)
        hipLaunchKernelGGL(k_bprimal_from_check, dim3(d.nslotT), dim3(kWG), 0, s, d.brT, ep,
                           d.lp_col, d.lp, d.xpT, d.aty, d.atyb);
    else
        hipLaunchKernelGGL(k_bspmv<EpiPrimalB>, dim3(d.nslotT), dim3(kWG), 0, s, d.trp, d.tci,
                           d.tv, d.y, d.brT, d.nblkT, ep, d.lp_col, d.lp, 0, d.xpT, d.tci16,
                           d.lp_r0);
    EpiDualB ed{d.b, d.kind, d.y, d.sy, d.q, d.sigma_row, smode, ycopy};
    hipLaunchKernelGGL(k_bspmv<EpiDualB>, dim3(d.nslotA), dim3(kWG), 0, s, d.rp, d.ci, d.v, d.x,
                       d.brA, d.nblkA, ed, d.lp_row, d.lp, 0, d.xpA, d.ci16, d.lp_c0);
}

// iteration counters of Algorithm 1 for the LPs still running (every LP
// of the batch takes the same iterations until it converges)
__global__ void k_badvance(BDev d, int iters) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.count) return;
    BLP &L = d.lp[i];
    if (L.done) return;
    L.k += iters;
    L.t += iters;
}

static void b_iterations(const BDev &d, long long iters, hipStream_t s, bool from_check = false) {
    if (iters <= 0) return;
    for (long long i = 0; i < iters; ++i)
        b_iteration(d, sum_mode(i, iters), s, nullptr, nullptr, from_check && i == 0);
    hipLaunchKernelGGL(k_badvance, dim3(div_up(d.count, kWG)), dim3(kWG), 0, s, d, (int)iters);
}

// per-element step sizes from the LPs (0 for converged LPs)
__global__ void k_bsteps(BDev d) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.N) {
        const BLP &L = d.lp[d.lp_col[i]];
        d.tau_col[i] = L.done ? 0.0 : L.tau;
    } else if (i < (long long)d.N + d.M) {
        const long long r = i - d.N;
        const BLP &L = d.lp[d.lp_row[r]];
        d.sigma_row[r] = L.done ? 0.0 : L.sigma;
    }
}

// ---------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------
// copy LP `lp` into the concatenated arrays
__global__ void k_bconcat(BDev d, int lpi, const int *rp, const int *ci, const double *v,
                          const double *c, const double *b, const double *l, const double *u,
                          const signed char *kind, int m, int n, int nnz, int row_off,
                          int col_off, int nnz_off) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nnz) {
        d.ci[nnz_off + i] = ci[i] + col_off;
        d.v[nnz_off + i] = v[i];
    }
    if (i < m) {
        d.rp[row_off + i] = rp[i] + nnz_off;
        d.b[row_off + i] = b[i];
        d.kind[row_off + i] = kind ? kind[i] : (signed char)0;
        d.lp_row[row_off + i] = lpi;
    }
    if (i < n) {
        d.c[col_off + i] = c[i];
        d.l[col_off + i] = l[i];
        d.u[col_off + i] = u[i];
        d.lp_col[col_off + i] = lpi;
    }
}

__global__ void k_bclose_rp(BDev d) { d.rp[d.M] = d.NNZ; }

// Block table (the layout of k_rowsplit: row starts, then entry starts) of
// the concatenated rows rp in which no block spans two LPs: LP i (rows
// off[i] .. off[i+1]-1) takes blocks blk[i] .. blk[i+1]-1, split by the
// merge-path rule over its own rows and entries.
__global__ void k_lpsplit(const int *__restrict__ rp, const int *__restrict__ off,
                          const int *__restrict__ blk, int count, int nblk, int *br) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nblk) return;
    int row = off[count];
    if (c < nblk) {
        int lo = 0, hi = count - 1;  // the LP of block c: last i with blk[i] <= c
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (blk[mid] <= c) lo = mid;
            else hi = mid - 1;
        }
        const int r0 = off[lo], rows = off[lo + 1] - r0, e0 = rp[r0];
        const long long target = (long long)(c - blk[lo]) * kUnits;
        int a = 0, b = rows;
        while (a < b) {
            const int mid = a + ((b - a) >> 1);
            if ((long long)mid + (rp[r0 + mid] - e0) >= target) b = mid;
            else a = mid + 1;
        }
        row = r0 + a;
    }
    br[c] = row;
    br[nblk + 1 + c] = rp[row];
}

// indices of a block-diagonal CSR relative to their LP: out[p] = ci[p] -
// base[lp_of[row of p]] (every LP narrower than 65,537)
__global__ void k_bidx16(const int *__restrict__ rp, const int *__restrict__ ci, int rows,
                         const int *__restrict__ lp_of, const int *__restrict__ base,
                         unsigned short *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int b0 = base[lp_of[r]];
    for (int p = rp[r]; p < rp[r + 1]; ++p) out[p] = (unsigned short)(ci[p] - b0);
}

// x = proj_X(0), y = 0, anchors, sums
__global__ void k_binit(BDev d) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.N) {
        double v = 0.0;
        if (v < d.l[i]) v = d.l[i];
        if (v > d.u[i]) v = d.u[i];
        d.x[i] = v;
        d.x0[i] = v;
        d.sx[i] = 0.0;
    }
    if (i < d.M) {
        d.y[i] = 0.0;
        d.y0[i] = 0.0;
        d.sy[i] = 0.0;
    }
}

// |b_i|^2 and |c_i|^2 per LP
__global__ __launch_bounds__(kWG) void k_bnorm_partials(BDev d) {
    __shared__ double sh[4 * 2];
    const int bb = blockIdx.x;
    const BLP &L = d.lp[d.blk_lp[bb]];
    const int first = d.blk_first[bb];
    const int E = L.n + L.m;
    const int end = first + kChunk < E ? first + kChunk : E;
    double v[2] = {0.0, 0.0};
    for (int e = first + threadIdx.x; e < end; e += kWG) {
        if (e < L.n) {
            const double cc = d.c[L.col_off + e];
            v[1] += cc * cc;
        } else {
            const double b2 = d.b[L.row_off + e - L.n];
            v[0] += b2 * b2;
        }
    }
    block_sums<2>(v, sh);
    if (threadIdx.x == 0) {
        d.part[(size_t)bb * kKktSums + 0] = v[0];
        d.part[(size_t)bb * kKktSums + 1] = v[1];
    }
}

__global__ __launch_bounds__(kWG) void k_bnorm_final(BDev d) {
    BLP &L = d.lp[blockIdx.x];
    __shared__ double sh[4 * 2];
    double out[2];
    reduce_partials<2>(d.part + (size_t)L.blk_begin * kKktSums, L.blk_end - L.blk_begin, kKktSums,
                       out, sh);
    if (threadIdx.x == 0) {
        L.nb2 = out[0];
        L.nc2 = out[1];
    }
}

// power iteration per LP (the single-LP rule, each LP stops on its own)
__global__ void k_bpw_init(BDev d) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < d.N) d.atyb[j] = 1.0 / sqrt((double)d.lp[d.lp_col[j]].n);
    if (j < d.count) {
        BLP &L = d.lp[j];
        L.pw_done = 0;
        L.pw_it = 0;
        L.pw_est = 0.0;
        L.pw_prev = 0.0;
        L.pw_s = 0.0;
    }
}

__global__ __launch_bounds__(kWG) void k_bpw_partials(BDev d) {
    __shared__ double sh[4];
    const int bb = blockIdx.x;
    const BLP &L = d.lp[d.blk_lp[bb]];
    if (L.pw_done) return;
    const int first = d.blk_first[bb];
    const int end = first + kChunk < L.n ? first + kChunk : L.n;
    double a[1] = {0.0};
    for (int e = first + threadIdx.x; e < end; e += kWG) {
        const double uu = d.aty[L.col_off + e];
        a[0] += uu * uu;
    }
    block_sums<1>(a, sh);
    if (threadIdx.x == 0) d.part[(size_t)bb * kKktSums] = a[0];
}

__global__ __launch_bounds__(kWG) void k_bpw_final(BDev d, double tol, int max_iters) {
    BLP &L = d.lp[blockIdx.x];
    if (L.pw_done) return;
    __shared__ double sh[4];
    // blocks of the LP whose chunk starts inside its x part
    int nbx = L.blk_end - L.blk_begin;
    const int need = (L.n + kChunk - 1) / kChunk;
    if (need < nbx) nbx = need;
    double tot[1];
    reduce_partials<1>(d.part + (size_t)L.blk_begin * kKktSums, nbx, kKktSums, tot, sh);
    if (threadIdx.x == 0) {
        const double sn = sqrt(tot[0]);
        if (!(sn > 0.0)) {
            L.pw_est = 0.0;
            L.pw_s = 0.0;
            L.pw_done = 1;
        } else {
            L.pw_s = sn;
            const double est = sqrt(sn);
            L.pw_est = est;
            if (L.pw_it > 0 && fabs(est - L.pw_prev) <= tol * est) L.pw_done = 2;
            L.pw_prev = est;
            L.pw_it += 1;
            if (L.pw_it >= max_iters) L.pw_done = 2;
        }
    }
}

// v = u / s for LPs still iterating (pw_done 2 marks the step that stopped)
__global__ void k_bpw_norm(BDev d) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d.N) return;
    const BLP &L = d.lp[d.lp_col[j]];
    if (L.pw_done == 1) return;
    const double sn = L.pw_s;
    if (sn > 0.0) d.atyb[j] = d.aty[j] / sn;
}

__global__ void k_bpw_settle(BDev d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.count && d.lp[i].pw_done == 2) d.lp[i].pw_done = 1;
}

// step sizes: eta given, else 0.9 / sigma_max; tau = eta / omega, sigma = eta * omega
__global__ void k_bset_steps(BDev d, const double *eta_in) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.count) return;
    BLP &L = d.lp[i];
    double eta = eta_in[i];
    if (!(eta > 0.0)) eta = L.pw_est > 0.0 ? 0.9 / L.pw_est : 1.0;
    L.eta = eta;
    L.tau = eta / L.omega;
    L.sigma = eta * L.omega;
}

// ---------------------------------------------------------------------
// check
// ---------------------------------------------------------------------
__global__ void k_bavg(BDev d) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.N) {
        const BLP &L = d.lp[d.lp_col[i]];
        if (L.done) return;
        d.xbar[i] = L.t ? d.sx[i] / (double)L.t : d.x[i];
    } else if (i < (long long)d.N + d.M) {
        const long long r = i - d.N;
        const BLP &L = d.lp[d.lp_row[r]];
        if (L.done) return;
        d.ybar[r] = L.t ? d.sy[r] / (double)L.t : d.y[r];
    }
}

__global__ __launch_bounds__(kWG) void k_bkkt_partials(BDev d) {
    const int bb = blockIdx.x;
    const BLP &L = d.lp[d.blk_lp[bb]];
    if (L.done) return;
    __shared__ double sh[4 * kKktSums];
    double v[kKktSums];
#pragma unroll
    for (int k = 0; k < kKktSums; ++k) v[k] = 0.0;
    const int first = d.blk_first[bb];
    const int E = L.n + L.m;
    const int end = first + kChunk < E ? first + kChunk : E;
    for (int e = first + threadIdx.x; e < end; e += kWG) {
        if (e < L.n) {
            const int j = L.col_off + e;
            const double cj = d.c[j], lj = d.l[j], uj = d.u[j], x0 = d.x0[j];
            const bool lf = isfinite(lj), uf = isfinite(uj);
            const double xs[2] = {d.x[j], d.xbar[j]};
            const double ats[2] = {d.aty[j], d.atyb[j]};
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
            v[S_RX2_A] += da * da;
            v[S_RX2_C] += dc * dc;
        } else {
            const int r = L.row_off + e - L.n;
            const double br = d.b[r], y0 = d.y0[r];
            const bool ge = d.kind[r] != 0;
            const double ys[2] = {d.y[r], d.ybar[r]};
            const double axs[2] = {d.q[r], d.axb[r]};
#pragma unroll
            for (int P = 0; P < 2; ++P) {
                double p = br - axs[P];
                if (ge && p < 0.0) p = 0.0;
                v[S_PRES2_C + P] += p * p;
                v[S_DOBJ_C + P] += br * ys[P];
                if (ge && ys[P] < 0.0) v[S_BV2_C + P] += ys[P] * ys[P];
            }
            const double da = ys[1] - y0, dc = ys[0] - y0;
            v[S_RY2_A] += da * da;
            v[S_RY2_C] += dc * dc;
        }
    }
    block_sums<kKktSums>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kKktSums; ++k) d.part[(size_t)bb * kKktSums + k] = v[k];
    }
}

__device__ void bkkt_point(const BLP &L, const double *S, int P, double *out) {
    const double pres2 = S[S_PRES2_C + P], dres2 = S[S_DRES2_C + P];
    const double pobj = S[S_POBJ_C + P], dobj = S[S_DOBJ_C + P], bv2 = S[S_BV2_C + P];
    const double pres = sqrt(pres2), dres = sqrt(dres2);
    const double gap = pobj - dobj;
    const double rel_p = pres / (1.0 + sqrt(L.nb2));
    const double rel_d = dres / (1.0 + sqrt(L.nc2));
    const double rel_g = fabs(gap) / (1.0 + fabs(pobj) + fabs(dobj));
    double rel = rel_p;
    if (rel_d > rel) rel = rel_d;
    if (rel_g > rel) rel = rel_g;
    const double gpos = gap > 0.0 ? gap : 0.0;
    double mx = pres;
    if (dres > mx) mx = dres;
    if (fabs(gap) > mx) mx = fabs(gap);
    out[1] = rel;
    out[2] = pres;
    out[3] = dres;
    out[4] = pobj;
    out[5] = dobj;
    out[6] = sqrt(bv2 + pres2 + dres2 + gpos * gpos);
    out[7] = mx;
}

__device__ __forceinline__ double bkkt_pick(const double *k8, int kind) {
    if (kind == 1) return k8[6];
    if (kind == 2) return k8[7];
    return k8[1];
}

__global__ __launch_bounds__(kWG) void k_bkkt_final(BDev d, double tol, int kkt_kind, int gap_slots) {
    const int lpi = blockIdx.x;
    BLP &L = d.lp[lpi];
    if (L.done) return;
    __shared__ double sh[4 * kKktSums];
    __shared__ int armed;
    double S[kKktSums];
    reduce_partials<kKktSums>(d.part + (size_t)L.blk_begin * kKktSums, L.blk_end - L.blk_begin,
                              kKktSums, S, sh);
    if (threadIdx.x == 0) {
        L.in_check = 1;
        L.restarted = 0;
        L.cand = 0;
        L.t_check = L.t;
        bkkt_point(L, S, 0, L.kkt_cur);
        bkkt_point(L, S, 1, L.kkt_avg);
        const double kc = bkkt_pick(L.kkt_cur, kkt_kind), ka = bkkt_pick(L.kkt_avg, kkt_kind);
        L.kkt_cur[0] = kc;
        L.kkt_avg[0] = ka;
        bool bad = false;
        for (int k = 0; k < kKktSums; ++k) bad |= !isfinite(S[k]);
        L.numerr = bad ? 1 : 0;
        const int conv = (tol > 0.0 && (kc <= tol || ka <= tol)) ? 1 : 0;
        L.conv_which = -1;
        if (conv) {
            L.done = 1;
            L.conv_which = (ka <= kc) ? 1 : 0;
            L.conv_k = L.k;
        }
        L.r_avg = sqrt(L.omega * S[S_RX2_A] + S[S_RY2_A] / L.omega);
        L.r_cur = sqrt(L.omega * S[S_RX2_C] + S[S_RY2_C] / L.omega);
        int slots = 0;
        if (!conv && !bad && L.t > 0) slots = gap_slots;
        L.gap_slots = slots;
        for (int sidx = 0; sidx < kTrSlots; ++sidx) {
            TRState &ts = L.tr[sidx];
            ts.mode = TR_IDLE;
            ts.rho = 0.0;
            ts.lam = 0.0;
            if (slots & (1 << sidx)) {
                ts.mode = TR_SEARCH;
                ts.r = sidx == 0 ? L.r_avg : L.r_cur;
                ts.r2 = ts.r * ts.r;
                ts.F_acc = 0.0;
                ts.A_acc = 0.0;
                ts.prefix = 0ull;
                ts.klo = 0ull;
                ts.level = 0;
                ts.count = 0u;
                ts.ncomp = 0u;
                ts.nan_seen = 0;
                ts.cap = kChunk;
            }
        }
        armed = slots;
    }
    __syncthreads();
    for (int sidx = 0; sidx < kTrSlots; ++sidx) {
        if (!(armed & (1 << sidx))) continue;
        const size_t h0 = hist_at(lpi, sidx, 0);
        for (int b = threadIdx.x; b < kBuckets; b += kWG) {
            d.hcnt[h0 + b] = 0u;
            d.hD[h0 + b] = 0.0;
            d.hA[h0 + b] = 0.0;
        }
    }
}

// coordinate (a, d) pair of element e of LP L for the gap at slot 0 (z-bar)
// or slot 1 (z): the same formulas as the single-LP solver
__device__ __forceinline__ void bgap_elem(const BDev &d, const BLP &L, int slot, int e, double &a,
                                          double &dd) {
    if (e < L.n) {
        const int j = L.col_off + e;
        const double xv = slot == 0 ? d.xbar[j] : d.x[j];
        const double at = slot == 0 ? d.atyb[j] : d.aty[j];
        const double g = d.c[j] - at;
        double dist = 0.0;
        if (g > 0.0) dist = xv - d.l[j];
        else if (g < 0.0) dist = d.u[j] - xv;
        if (dist < 0.0) dist = 0.0;
        a = fabs(g) / L.sw;
        dd = dist * L.sw;
    } else {
        const int r = L.row_off + e - L.n;
        const double yv = slot == 0 ? d.ybar[r] : d.y[r];
        const double ax = slot == 0 ? d.axb[r] : d.q[r];
        const double g = ax - d.b[r];
        const double lo = d.kind[r] ? 0.0 : -INFINITY;
        double dist = 0.0;
        if (g > 0.0) dist = yv - lo;
        else if (g < 0.0) dist = INFINITY;
        if (dist < 0.0) dist = 0.0;
        a = fabs(g) * L.sw;
        dd = dist / L.sw;
    }
}

__device__ __forceinline__ int blk_end_elem(const BDev &d, const BLP &L, int bb) {
    const int first = d.blk_first[bb];
    const int E = L.n + L.m;
    return first + kChunk < E ? first + kChunk : E;
}

__global__ __launch_bounds__(kWG) void k_btr_hist0(BDev d, int slot) {
    const int bb = blockIdx.x;
    const BLP &L = d.lp[d.blk_lp[bb]];
    const TRState &ts = L.tr[slot];
    if (!L.in_check || ts.mode != TR_SEARCH || ts.level != 0) return;
    __shared__ unsigned int scnt[kBuckets];
    __shared__ double sD[kBuckets], sA[kBuckets];
    __shared__ double sh[4 * 4];
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        scnt[b] = 0u;
        sD[b] = 0.0;
        sA[b] = 0.0;
    }
    __syncthreads();
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int end = blk_end_elem(d, L, bb);
    for (int e = d.blk_first[bb] + threadIdx.x; e < end; e += kWG) {
        double a, dd;
        bgap_elem(d, L, slot, e, a, dd);
        if (bad_pair(a, dd)) {
            v[3] += 1.0;
        } else if (a > 0.0) {
            const unsigned long long key = key_of(a, dd);
            const int b = (int)(key >> 52);
            atomicAdd(&scnt[b], 1u);
            atomicAdd(&sA[b], a * a);
            if (dd < INFINITY) {
                atomicAdd(&sD[b], dd * dd);
                v[0] += dd * dd;
                v[2] += a * dd;
            } else {
                v[1] += 1.0;
            }
        }
    }
    __syncthreads();
    const size_t h0 = hist_at(d.blk_lp[bb], slot, 0);
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        if (scnt[b]) {
            atomicAdd(&d.hcnt[h0 + b], scnt[b]);
            atomicAdd(&d.hD[h0 + b], sD[b]);
            atomicAdd(&d.hA[h0 + b], sA[b]);
        }
    }
    block_sums<4>(v, sh);
    if (threadIdx.x == 0) {
        double *tp = d.tpart + ((size_t)slot * d.nblk + bb) * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) tp[k] = v[k];
    }
}

__device__ void bzero_hist(const BDev &d, int lpi, int slot, int half) {
    const size_t h = hist_at(lpi, slot, half);
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        d.hcnt[h + b] = 0u;
        d.hD[h + b] = 0.0;
        d.hA[h + b] = 0.0;
    }
}

__global__ __launch_bounds__(kWG) void k_btr_decide0(BDev d, int slot) {
    const int lpi = blockIdx.x;
    BLP &L = d.lp[lpi];
    if (!L.in_check || L.tr[slot].mode != TR_SEARCH || L.tr[slot].level != 0) return;
    __shared__ TRState sts;
    __shared__ ChooseShared cs;
    __shared__ double sh[4 * 4];
    __shared__ int go;
    if (threadIdx.x == 0) sts = L.tr[slot];
    double tot[4];
    reduce_partials<4>(d.tpart + ((size_t)slot * d.nblk + L.blk_begin) * 4,
                       L.blk_end - L.blk_begin, 4, tot, sh);
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
            sts.mode = TR_FULLBOX;
            sts.value = tot[2];
            sts.rho = tot[2] / sts.r;
            sts.lam = INFINITY;
        } else {
            go = 1;
        }
    }
    __syncthreads();
    const size_t h0 = hist_at(lpi, slot, 0);
    if (go) choose_bucket(sts, d.hcnt + h0, d.hD + h0, d.hA + h0, kBuckets, 0, cs);
    bzero_hist(d, lpi, slot, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        sts.ncomp = 0u;
        L.tr[slot] = sts;
    }
}

// level 1 + compaction of the bracket's members into the block's region
__global__ __launch_bounds__(kWG) void k_btr_pass1(BDev d, int slot) {
    const int bb = blockIdx.x;
    const int lpi = d.blk_lp[bb];
    const BLP &L = d.lp[lpi];
    const TRState &ts = L.tr[slot];
    if (!L.in_check || ts.mode != TR_SEARCH || ts.level != 1) return;
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
    const unsigned long long top = ts.prefix >> 52;
    const size_t region = ((size_t)slot * d.nblk + bb) * kChunk;
    const int end = blk_end_elem(d, L, bb);
    for (int e = d.blk_first[bb] + threadIdx.x; e < end; e += kWG) {
        double a, dd;
        bgap_elem(d, L, slot, e, a, dd);
        if (bad_pair(a, dd) || !(a > 0.0)) continue;
        const unsigned long long key = key_of(a, dd);
        if ((key >> 52) != top) continue;
        const int b = (int)((key >> 41) & (kBuckets - 1));
        atomicAdd(&scnt[b], 1u);
        atomicAdd(&sD[b], dd * dd);
        atomicAdd(&sA[b], a * a);
        const unsigned int q = atomicAdd(&nloc, 1u);
        d.ckey[region + q] = key;
        d.ca[region + q] = a;
        d.cd[region + q] = dd;
    }
    __syncthreads();
    const size_t h1 = hist_at(lpi, slot, 1);
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        if (scnt[b]) {
            atomicAdd(&d.hcnt[h1 + b], scnt[b]);
            atomicAdd(&d.hD[h1 + b], sD[b]);
            atomicAdd(&d.hA[h1 + b], sA[b]);
        }
    }
    if (threadIdx.x == 0) d.ccount[(size_t)slot * d.nblk + bb] = nloc;
}

// exclusive prefix of the LP's block counts into coff (one entry per block
// plus the LP's total); the total is returned through LDS
__device__ unsigned int bscan_counts(const BDev &d, const BLP &L, int lpi, int slot,
                                     unsigned int *sh) {
    const int nb = L.blk_end - L.blk_begin;
    const unsigned int *cnt = d.ccount + (size_t)slot * d.nblk + L.blk_begin;
    unsigned int *off = d.coff + (size_t)slot * (d.nblk + d.count) + L.blk_begin + lpi;
    __shared__ unsigned int carry;
    if (threadIdx.x == 0) carry = 0u;
    __syncthreads();
    for (int base = 0; base < nb; base += kWG) {
        const int i = base + threadIdx.x;
        const unsigned int v = i < nb ? cnt[i] : 0u;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kWG; o <<= 1) {
            unsigned int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0u;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) off[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += sh[kWG - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[nb] = carry;
    __syncthreads();
    return carry;
}

__global__ __launch_bounds__(kWG) void k_btr_decide1(BDev d, int slot) {
    const int lpi = blockIdx.x;
    BLP &L = d.lp[lpi];
    if (!L.in_check || L.tr[slot].mode != TR_SEARCH || L.tr[slot].level != 1) return;
    __shared__ TRState sts;
    __shared__ ChooseShared cs;
    __shared__ unsigned int shs[kWG];
    if (threadIdx.x == 0) sts = L.tr[slot];
    const unsigned int total = bscan_counts(d, L, lpi, slot, shs);
    if (threadIdx.x == 0) sts.ncomp = total;
    __syncthreads();
    const size_t h1 = hist_at(lpi, slot, 1);
    choose_bucket(sts, d.hcnt + h1, d.hD + h1, d.hA + h1, kBuckets, 1, cs);
    bzero_hist(d, lpi, slot, 0);
    __syncthreads();
    if (threadIdx.x == 0) L.tr[slot] = sts;
}

constexpr unsigned int kBFinishMax = 65536;

__global__ __launch_bounds__(kWG) void k_btr_cpass(BDev d, int slot, int level) {
    const int bb = blockIdx.x;
    const int lpi = d.blk_lp[bb];
    const BLP &L = d.lp[lpi];
    const TRState &ts = L.tr[slot];
    if (!L.in_check || ts.mode != TR_SEARCH || ts.level != level || ts.count <= kBFinishMax) return;
    __shared__ unsigned int scnt[kBuckets];
    __shared__ double sD[kBuckets], sA[kBuckets];
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        scnt[b] = 0u;
        sD[b] = 0.0;
        sA[b] = 0.0;
    }
    __syncthreads();
    const int shift = shift_of(level), above = shift_of(level - 1);
    const unsigned long long want = ts.prefix >> above;
    const size_t region = ((size_t)slot * d.nblk + bb) * kChunk;
    unsigned int cnt = d.ccount[(size_t)slot * d.nblk + bb];
    if (cnt > (unsigned int)kChunk) cnt = kChunk;
    for (unsigned int q = threadIdx.x; q < cnt; q += kWG) {
        const unsigned long long key = d.ckey[region + q];
        if ((key >> above) != want) continue;
        const int b = (int)((key >> shift) & (kBuckets - 1));
        const double a = d.ca[region + q], dd = d.cd[region + q];
        atomicAdd(&scnt[b], 1u);
        atomicAdd(&sD[b], dd * dd);
        atomicAdd(&sA[b], a * a);
    }
    __syncthreads();
    const size_t h = hist_at(lpi, slot, level & 1);
    for (int b = threadIdx.x; b < kBuckets; b += kWG) {
        if (scnt[b]) {
            atomicAdd(&d.hcnt[h + b], scnt[b]);
            atomicAdd(&d.hD[h + b], sD[b]);
            atomicAdd(&d.hA[h + b], sA[b]);
        }
    }
}

__global__ __launch_bounds__(kWG) void k_btr_cdecide(BDev d, int slot, int level) {
    const int lpi = blockIdx.x;
    BLP &L = d.lp[lpi];
    const TRState &ts0 = L.tr[slot];
    if (!L.in_check || ts0.mode != TR_SEARCH || ts0.level != level || ts0.count <= kBFinishMax)
        return;
    __shared__ TRState sts;
    __shared__ ChooseShared cs;
    if (threadIdx.x == 0) sts = L.tr[slot];
    __syncthreads();
    const size_t h = hist_at(lpi, slot, level & 1);
    choose_bucket(sts, d.hcnt + h, d.hD + h, d.hA + h, kBuckets, level, cs);
    bzero_hist(d, lpi, slot, 1 - (level & 1));
    __syncthreads();
    if (threadIdx.x == 0) L.tr[slot] = sts;
}

__global__ __launch_bounds__(kWG) void k_btr_finish(BDev d, int slot) {
    const int lpi = blockIdx.x;
    BLP &L = d.lp[lpi];
    if (!L.in_check || L.tr[slot].mode != TR_SEARCH) return;
    __shared__ TRState sts;
    __shared__ ChooseShared cs;
    __shared__ unsigned int scnt[kBuckets];
    __shared__ double sD[kBuckets], sA[kBuckets];
    if (threadIdx.x == 0) sts = L.tr[slot];
    __syncthreads();
    const int nb = L.blk_end - L.blk_begin;
    const unsigned int *off = d.coff + (size_t)slot * (d.nblk + d.count) + L.blk_begin + lpi;
    unsigned int total = off[nb];
    const unsigned long long room = (unsigned long long)nb * kChunk;
    if ((unsigned long long)total > room) total = (unsigned int)room;
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
            int lo = 0, hi = nb - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (off[mid] <= idx) lo = mid;
                else hi = mid - 1;
            }
            const unsigned int within = idx - off[lo];
            if (within >= (unsigned int)kChunk) continue;
            const size_t at = ((size_t)slot * d.nblk + L.blk_begin + lo) * kChunk + within;
            const unsigned long long key = d.ckey[at];
            if ((key >> above) != want) continue;
            const int b = (int)((key >> shift) & (unsigned long long)(nbuck - 1));
            const double a = d.ca[at], dd = d.cd[at];
            atomicAdd(&scnt[b], 1u);
            atomicAdd(&sD[b], dd * dd);
            atomicAdd(&sA[b], a * a);
        }
        __syncthreads();
        choose_bucket(sts, scnt, sD, sA, nbuck, level, cs);
    }
    if (threadIdx.x == 0) L.tr[slot] = sts;
}

__global__ __launch_bounds__(kWG) void k_btr_final_partials(BDev d, int slot) {
    const int bb = blockIdx.x;
    const BLP &L = d.lp[d.blk_lp[bb]];
    const TRState &ts = L.tr[slot];
    if (!L.in_check || ts.mode != TR_RESOLVED) return;
    __shared__ double sh[4 * 3];
    const unsigned long long klo = ts.klo;
    double v[3] = {0.0, 0.0, 0.0};
    const int end = blk_end_elem(d, L, bb);
    for (int e = d.blk_first[bb] + threadIdx.x; e < end; e += kWG) {
        double a, dd;
        bgap_elem(d, L, slot, e, a, dd);
        if (bad_pair(a, dd) || !(a > 0.0)) continue;
        if (key_of(a, dd) <= klo) {
            v[0] += dd * dd;
            v[2] += a * dd;
        } else {
            v[1] += a * a;
        }
    }
    block_sums<3>(v, sh);
    if (threadIdx.x == 0) {
        double *tp = d.tpart + ((size_t)slot * d.nblk + bb) * 4;
#pragma unroll
        for (int k = 0; k < 3; ++k) tp[k] = v[k];
    }
}

__global__ __launch_bounds__(kWG) void k_btr_final(BDev d, int slot) {
    BLP &L = d.lp[blockIdx.x];
    if (!L.in_check || L.tr[slot].mode != TR_RESOLVED) return;
    __shared__ double sh[4 * 3];
    double tot[3];
    reduce_partials<3>(d.tpart + ((size_t)slot * d.nblk + L.blk_begin) * 4,
                       L.blk_end - L.blk_begin, 4, tot, sh);
    if (threadIdx.x == 0) {
        TRState &ts = L.tr[slot];
        const double F = tot[0], A = tot[1], AD = tot[2];
        double lam, val;
        if (A > 0.0) {
            double num = ts.r2 - F;
            if (num < 0.0) num = 0.0;
            lam = sqrt(num / A);
            val = AD + lam * A;
        } else {
            lam = INFINITY;
            val = AD;
        }
        ts.lam = lam;
        ts.value = val;
        ts.rho = val / ts.r;
    }
}

static void b_gap(const BDev &d, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_btr_hist0, dim3(d.nblk), dim3(kWG), 0, s, d, slot);
    hipLaunchKernelGGL(k_btr_decide0, dim3(d.count), dim3(kWG), 0, s, d, slot);
    hipLaunchKernelGGL(k_btr_pass1, dim3(d.nblk), dim3(kWG), 0, s, d, slot);
    hipLaunchKernelGGL(k_btr_decide1, dim3(d.count), dim3(kWG), 0, s, d, slot);
    for (int level = 2; level <= 3; ++level) {
        hipLaunchKernelGGL(k_btr_cpass, dim3(d.nblk), dim3(kWG), 0, s, d, slot, level);
        hipLaunchKernelGGL(k_btr_cdecide, dim3(d.count), dim3(kWG), 0, s, d, slot, level);
    }
    hipLaunchKernelGGL(k_btr_finish, dim3(d.count), dim3(kWG), 0, s, d, slot);
    hipLaunchKernelGGL(k_btr_final_partials, dim3(d.nblk), dim3(kWG), 0, s, d, slot);
    hipLaunchKernelGGL(k_btr_final, dim3(d.count), dim3(kWG), 0, s, d, slot);
}

// restart decision per LP (eq. adaptive-restart-scheme, Remark rem:flexible)
__global__ void k_bdecide(BDev d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.count) return;
    BLP &L = d.lp[i];
    if (!L.in_check) return;
    double rec[kRec];
    rec[0] = (double)L.k;
    rec[1] = (double)L.t;
    rec[2] = (double)L.restarts;
    rec[3] = L.kkt_cur[0];
    rec[4] = L.kkt_avg[0];
    rec[5] = 0.0;
    rec[6] = 0.0;
    rec[7] = 0.0;
    rec[8] = -1.0;
    rec[9] = 0.0;
    rec[10] = 0.0;
    rec[11] = (double)L.conv_which;
    rec[12] = L.rho_prev;
    rec[13] = 0.0;
    const int slots = L.gap_slots;
    if (slots & 1) {
        rec[5] = L.r_avg;
        rec[6] = L.tr[0].rho;
        rec[13] = L.tr[0].lam;
        if (L.tr[0].nan_seen) L.numerr = 1;
    }
    if (slots & 2) {
        rec[7] = L.r_cur;
        rec[8] = L.tr[1].rho;
        if (L.tr[1].nan_seen) L.numerr = 1;
    }
    if ((slots & 1) && !L.done && !L.numerr) {
        const double rho_a = L.tr[0].rho;
        double rho_c = rho_a;
        int cand = 0;
        if ((slots & 2) && L.tr[1].rho < rho_a) {
            cand = 1;
            rho_c = L.tr[1].rho;
        }
        bool restart;
        if (L.restarts == 0) restart = L.t >= (long long)L.tau0;
        else restart = rho_c <= L.beta * L.rho_prev;
        rec[10] = (double)cand;
        if (restart) {
            rec[9] = 1.0;
            L.restarted = 1;
            L.cand = cand;
            L.restarts += 1;
            L.t = 0;
            L.rho_prev = rho_c;
        }
    }
    double *dst = d.log + ((size_t)i * kBLog + (size_t)(L.checks % kBLog)) * kRec;
    for (int q = 0; q < kRec; ++q) dst[q] = rec[q];
    L.checks += 1;
    L.in_check = 0;
}

__global__ void k_bapply(BDev d) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.N) {
        const BLP &L = d.lp[d.lp_col[i]];
        d.tau_col[i] = L.done ? 0.0 : L.tau;
        if (!L.restarted) return;
        if (L.cand == 0) {
            const double v = d.xbar[i];
            d.x[i] = v;
            d.x0[i] = v;
        } else {
            d.x0[i] = d.x[i];
        }
        d.sx[i] = 0.0;
    } else if (i < (long long)d.N + d.M) {
        const long long r = i - d.N;
        const BLP &L = d.lp[d.lp_row[r]];
        d.sigma_row[r] = L.done ? 0.0 : L.sigma;
        if (!L.restarted) return;
        if (L.cand == 0) {
            const double v = d.ybar[r];
            d.y[r] = v;
            d.y0[r] = v;
            d.q[r] = d.axb[r];
        } else {
            d.y0[r] = d.y[r];
        }
        d.sy[r] = 0.0;
    }
}

__global__ void k_breset(BDev d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.count) d.lp[i].in_check = 0;
}

static void b_check(const BDev &d, double tol, int kkt_kind, int slots, hipStream_t s) {
    const long long NM = (long long)d.N + d.M;
    hipLaunchKernelGGL(k_bavg, dim3(div_up(NM, kWG)), dim3(kWG), 0, s, d);
    bspmv_A(d, d.xbar, d.axb, 0, s);
    bspmv_T(d, d.ybar, d.atyb, 0, s);
    bspmv_T(d, d.y, d.aty, 0, s);
    hipLaunchKernelGGL(k_bkkt_partials, dim3(d.nblk), dim3(kWG), 0, s, d);
    hipLaunchKernelGGL(k_bkkt_final, dim3(d.count), dim3(kWG), 0, s, d, tol, kkt_kind, slots);
    if (slots & 1) b_gap(d, 0, s);
    if (slots & 2) b_gap(d, 1, s);
    hipLaunchKernelGGL(k_bdecide, dim3(div_up(d.count, 64)), dim3(64), 0, s, d);
    hipLaunchKernelGGL(k_bapply, dim3(div_up(NM, kWG)), dim3(kWG), 0, s, d);
}

__global__ void k_bget(BDev d, int lpi, int which, double *ox, double *oy) {
    const BLP &L = d.lp[lpi];
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long t = L.t;
    const bool sol_avg = L.conv_which == 1;
    if (i < L.n) {
        const int j = d.cinv ? d.cinv[L.col_off + (int)i] : L.col_off + (int)i;
        double v;
        if (which == 0) v = d.x[j];
        else if (which == 1) v = t ? d.sx[j] / (double)t : d.x[j];
        else if (which == 2) v = d.x0[j];
        else v = sol_avg ? d.xbar[j] : d.x[j];
        ox[i] = v;
    }
    if (i < L.m) {
        const int r = L.row_off + (int)i;
        double v;
        if (which == 0) v = d.y[r];
        else if (which == 1) v = t ? d.sy[r] / (double)t : d.y[r];
        else if (which == 2) v = d.y0[r];
        else v = sol_avg ? d.ybar[r] : d.y[r];
        oy[i] = v;
    }
}

// ---------------------------------------------------------------------
// Differentiation of K unrolled iterations (reverse sweep with frozen
// projection masks and restart decisions).  Forward per iteration:
//   u = x - tau (c - A'y), x+ = proj_X(u); w = 2x+ - x,
//   v = y + sigma (b - A w), y+ = proj_Y(v); S_x += x+, S_y += y+,
// and at a restart to the average x = S_x / T (Algorithm 1).
// Reverse of one iteration, with xh, yh the adjoints of x+, y+ from later
// iterations and Sxh, Syh those of the running sums:
//   vh = mask_y (yh + Syh);                    b^ += sigma vh
//   wh = -sigma A' vh;  uh = mask_x (xh + Sxh + 2 wh);  c^ += -tau uh
//   xh <- -wh + uh;     yh <- vh + tau A uh
//   A^_ij += -sigma vh_i (2x+_j - x_j) + tau y_i uh_j
// ---------------------------------------------------------------------
struct Tape {
    double *cx, *cy, *cq;   // checkpoints (x, y, A x) at every window start
    int *ev;                // [nwin][count] restart after the window: 0 none, 1 average, 2 current
    long long *evT;         // window length of that restart
    double *sx, *sy;        // recomputed iterates of one window: [(P+1)][N], [(P+1)][M]
    double *xh, *yh, *sxh, *syh, *vh;
    double2 *uw;            // per column: (uh, 2 x+ - x) for the A^ entries
    double *gc;             // dL/dc in the internal column order (permuted columns only)
    // the batch's state at the end of the forward call (x, y, A x, running
    // sums, per-LP records), put back after the reverse sweep, which
    // recomputes the windows through the live iterate arrays
    double *ex, *ey, *eq, *esx, *esy;
    BLP *elp;
    int nwin, P;
    long long K;
};

__global__ void k_breset_lps(BDev d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.count) return;
    BLP &L = d.lp[i];
    L.k = 0;
    L.t = 0;
    L.restarts = 0;
    L.checks = 0;
    L.rho_prev = 0.0;
    L.done = 0;
    L.conv_which = -1;
    L.conv_k = -1;
    L.restarted = 0;
    L.cand = 0;
    L.in_check = 0;
    L.numerr = 0;
    L.t_check = 0;
    for (int sidx = 0; sidx < kTrSlots; ++sidx) L.tr[sidx].mode = TR_IDLE;
}

__global__ void k_record_events(BDev d, int *ev, long long *evT) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.count) return;
    const BLP &L = d.lp[i];
    ev[i] = L.restarted ? (L.cand ? 2 : 1) : 0;
    evT[i] = L.t_check;
}

__global__ void k_adj_event(BDev d, const int *ev, const long long *evT, double *xh, double *yh,
                            double *sxh, double *syh) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.N) {
        const int lp = d.lp_col[i];
        const int e = ev[lp];
        if (e == 1) {
            sxh[i] = xh[i] / (double)evT[lp];
            xh[i] = 0.0;
        } else if (e == 2) {
            sxh[i] = 0.0;
        }
    } else if (i < (long long)d.N + d.M) {
        const long long r = i - d.N;
        const int lp = d.lp_row[r];
        const int e = ev[lp];
        if (e == 1) {
            syh[r] = yh[r] / (double)evT[lp];
            yh[r] = 0.0;
        } else if (e == 2) {
            syh[r] = 0.0;
        }
    }
}

__global__ void k_adj_dual(BDev d, const double *yt, const double *yh, const double *syh,
                           double *vh, double *gb) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.M) return;
    const BLP &L = d.lp[d.lp_row[i]];
    const bool inside = !d.kind[i] || yt[i] > 0.0;
    const double v = inside ? yh[i] + syh[i] : 0.0;
    vh[i] = v;
    gb[i] += L.sigma * v;
}

// the A' product of the reverse step with the primal adjoint fused; it
// also leaves (uh_j, 2 x+_j - x_j) side by side for the A rows, which then
// gather both with one load
struct EpiAdjPrimal {
    const double *__restrict__ xt, *__restrict__ xprev, *__restrict__ l, *__restrict__ u;
    double *__restrict__ xh, *__restrict__ sxh, *__restrict__ gc;
    double2 *__restrict__ uw;
    const int *__restrict__ lpc;
    const BLP *lp;
    __device__ __forceinline__ void operator()(int j, double atv) const {
        const BLP &L = lp[lpc[j]];
        const double wh = -L.sigma * atv;
        const double tot = xh[j] + sxh[j] + 2.0 * wh;
        const double xtj = xt[j];
        const bool inside = l[j] < xtj && xtj < u[j];
        const double uu = inside ? tot : 0.0;
        uw[j] = make_double2(uu, 2.0 * xtj - xprev[j]);
        gc[j] += -L.tau * uu;
        xh[j] = -wh + uu;
    }
};

// rows of A: yh_i = vh_i + tau (A uh)_i and the A^ entries of the row
// (uw_j = (uh_j, 2 x+_j - x_j))
__global__ __launch_bounds__(kWG) void k_adj_rows(BDev d, const double2 *__restrict__ uw,
                                                  const double *__restrict__ yprev,
                                                  const double *__restrict__ vh, double *yh,
                                                  double *gA) {
    __shared__ double sp[kLdsProducts], sw[kLdsProducts], su[kLdsProducts];
    const int r0 = d.brA[blockIdx.x], r1 = d.brA[blockIdx.x + 1];
    if (r0 >= r1) return;
    const int *rp = d.rp, *ci = d.ci;
    const double *v = d.v;
    const int tid = threadIdx.x;
    const int p0 = rp[r0], p1 = rp[r1], nb = p1 - p0, R = r1 - r0;
    if (nb <= kLdsProducts) {
        // all index and value loads of a thread, then all its gathers
        int col[kPerThread];
        double val[kPerThread];
        double2 g[kPerThread];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int e = tid + k * kWG;
            if (e < nb) {
                col[k] = ci[p0 + e];
                val[k] = v[p0 + e];
            }
        }
#pragma unroll
        for (int k = 0; k < kPerThread; ++k)
            if (tid + k * kWG < nb) g[k] = uw[col[k]];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int e = tid + k * kWG;
            if (e < nb) {
                sp[e] = val[k] * g[k].x;
                sw[e] = g[k].y;
                su[e] = g[k].x;
            }
        }
        __syncthreads();
        const int avg = nb / R;
        int L = 1;
        while (L < 64 && 2 * L <= avg) L <<= 1;
        const int G = kWG / L, lane = tid & (L - 1), grp = tid / L;
        for (int rr = grp; rr < R; rr += G) {
            const int row = r0 + rr;
            const BLP &LP = d.lp[d.lp_row[row]];
            const double sig = LP.sigma, tau = LP.tau, vr = vh[row], yr = yprev[row];
            const int s0 = rp[row] - p0, s1 = rp[row + 1] - p0;
            double s = 0.0;
            for (int e = s0 + lane; e < s1; e += L) {
                s += sp[e];
                gA[p0 + e] += -sig * vr * sw[e] + tau * yr * su[e];
            }
            for (int off = L >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
            if (lane == 0) yh[row] = vr + tau * s;
        }
    } else {
        const int wave = tid >> 6, lane = tid & 63;
        for (int row = r0 + wave; row < r1; row += kWG / 64) {
            const BLP &LP = d.lp[d.lp_row[row]];
            const double sig = LP.sigma, tau = LP.tau, vr = vh[row], yr = yprev[row];
            double s = 0.0;
            for (int p = rp[row] + lane; p < rp[row + 1]; p += 64) {
                const double2 g = uw[ci[p]];
                s += v[p] * g.x;
                gA[p] += -sig * vr * g.y + tau * yr * g.x;
            }
            s = wave_sum(s);
            if (lane == 0) yh[row] = vr + tau * s;
        }
    }
}

__global__ void k_fill_d(double *a, long long len, double v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) a[i] = v;
}

// refresh A' values after new A values (entries keep their positions)
__global__ void k_bgather_tv(BDev d) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < d.NNZ) d.tv[q] = d.v[d.perm[q]];
}

// ---------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------
struct BLayout {
    size_t total;
    size_t o_lp, o_err, o_rp, o_ci, o_v, o_c, o_b, o_l, o_u, o_kind, o_trp, o_tci, o_perm, o_tv;
    size_t o_xpA, o_xpT;
    size_t o_cperm, o_cinv, o_bcls, o_blkA, o_blkT, o_lpr0, o_lpc0, o_ci16, o_tci16;
    size_t o_cursor, o_long, o_brA, o_brT, o_lprow, o_lpcol, o_tau, o_sig, o_blklp, o_blkfirst, o_vn, o_vm;
    size_t o_part, o_log, o_hcnt, o_hD, o_hA, o_tpart, o_ccount, o_coff, o_ckey, o_ca, o_cd;
    int M, N, NNZ, nblk, nblkA, nblkT;
};

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

static bool b_layout(int count, const int64_t *m, const int64_t *n, const int64_t *nnz,
                     BLayout *L) {
    if (count < 1 || count > (1 << 20)) return false;
    long long M = 0, N = 0, Z = 0, nblk = 0;
    for (int i = 0; i < count; ++i) {
        if (m[i] < 0 || n[i] < 1 || nnz[i] < 0) return false;
        M += m[i];
        N += n[i];
        Z += nnz[i];
        long long E = n[i] + m[i];
        nblk += (E + kChunk - 1) / kChunk;
    }
    const long long lim = 0x7fffffffLL - 4096;
    if (M > lim || N > lim || Z > lim || nblk > lim / kChunk) return false;
    L->M = (int)M;
    L->N = (int)N;
    L->NNZ = (int)Z;
    L->nblk = (int)nblk;
    // blocks per LP (no block spans two LPs)
    long long nbA = 0, nbT = 0;
    for (int i = 0; i < count; ++i) {
        nbA += nblocks_for((int)m[i], (int)nnz[i]);
        nbT += nblocks_for((int)n[i], (int)nnz[i]);
    }
    if (nbA > lim / kUnits || nbT > lim / kUnits) return false;
    L->nblkA = (int)nbA;
    L->nblkT = (int)nbT;
    const size_t M1 = (size_t)(M > 0 ? M : 1), N1 = (size_t)N, Z1 = (size_t)(Z > 0 ? Z : 1);
    size_t o = 0;
    auto put = [&](size_t &off, size_t bytes) {
        off = o;
        o += al(bytes);
    };
    put(L->o_lp, sizeof(BLP) * (size_t)count);
    put(L->o_err, sizeof(int) * 16);
    put(L->o_rp, sizeof(int) * (M1 + 1));
    put(L->o_ci, sizeof(int) * Z1);
    put(L->o_v, sizeof(double) * Z1);
    put(L->o_c, sizeof(double) * N1);
    put(L->o_b, sizeof(double) * M1);
    put(L->o_l, sizeof(double) * N1);
    put(L->o_u, sizeof(double) * N1);
    put(L->o_kind, M1);
    put(L->o_trp, sizeof(int) * (N1 + 1));
    put(L->o_tci, sizeof(int) * Z1);
    put(L->o_perm, sizeof(int) * Z1);
    put(L->o_tv, sizeof(double) * Z1);
    put(L->o_cperm, sizeof(int) * N1);
    put(L->o_cinv, sizeof(int) * N1);
    put(L->o_bcls, N1);
    put(L->o_blkA, sizeof(int) * ((size_t)count + 1));
    put(L->o_blkT, sizeof(int) * ((size_t)count + 1));
    put(L->o_lpr0, sizeof(int) * ((size_t)count + 1));
    put(L->o_lpc0, sizeof(int) * ((size_t)count + 1));
    put(L->o_ci16, sizeof(unsigned short) * Z1);
    put(L->o_tci16, sizeof(unsigned short) * Z1);
    put(L->o_cursor, sizeof(int) * N1);
    put(L->o_long, sizeof(int) * N1);
    put(L->o_brA, sizeof(int) * 2 * ((size_t)L->nblkA + 1));  // block tables (k_rowsplit)
    put(L->o_brT, sizeof(int) * 2 * ((size_t)L->nblkT + 1));
    put(L->o_xpA, sizeof(int) * kXcds * ((size_t)L->nblkA + 1));
    put(L->o_xpT, sizeof(int) * kXcds * ((size_t)L->nblkT + 1));
    put(L->o_lprow, sizeof(int) * M1);
    put(L->o_lpcol, sizeof(int) * N1);
    put(L->o_tau, sizeof(double) * N1);
    put(L->o_sig, sizeof(double) * M1);
    put(L->o_blklp, sizeof(int) * (size_t)nblk);
    put(L->o_blkfirst, sizeof(int) * (size_t)nblk);
    put(L->o_vn, al(sizeof(double) * N1) * 6);
    put(L->o_vm, al(sizeof(double) * M1) * 6);
    put(L->o_part, sizeof(double) * (size_t)nblk * kKktSums);
    put(L->o_log, sizeof(double) * (size_t)count * kBLog * kRec);
    put(L->o_hcnt, sizeof(unsigned int) * (size_t)count * kTrSlots * 2 * kBuckets);
    put(L->o_hD, sizeof(double) * (size_t)count * kTrSlots * 2 * kBuckets);
    put(L->o_hA, sizeof(double) * (size_t)count * kTrSlots * 2 * kBuckets);
    put(L->o_tpart, sizeof(double) * kTrSlots * (size_t)nblk * 4);
    put(L->o_ccount, sizeof(unsigned int) * kTrSlots * (size_t)nblk);
    put(L->o_coff, sizeof(unsigned int) * kTrSlots * ((size_t)nblk + count));
    put(L->o_ckey, sizeof(unsigned long long) * kTrSlots * (size_t)nblk * kChunk);
    put(L->o_ca, sizeof(double) * kTrSlots * (size_t)nblk * kChunk);
    put(L->o_cd, sizeof(double) * kTrSlots * (size_t)nblk * kChunk);
    L->total = o;
    return true;
}

// Placement of merge-path blocks on XCDs.  br (host copy, nblk + 1 row
// starts) and off (LP row starts, count + 1) give each non-empty block the
// LP of its first row; LPs go to XCDs largest first, each to the XCD with
// the fewest blocks so far; workgroup 8 j + x then runs the j-th block of
// XCD x (-1 past the end of its list).  Returns the workgroup count.
static int place_blocks(const std::vector<int> &br, const std::vector<int> &off, int count,
                        std::vector<int> &xp) {
    const int nblk = (int)br.size() - 1;
    std::vector<std::vector<int>> of_lp((size_t)count);
    for (int c = 0, lp = 0; c < nblk; ++c) {
        const int r0 = br[c];
        if (r0 >= br[c + 1]) continue;
        while (lp + 1 < count && off[lp + 1] <= r0) ++lp;
        of_lp[lp].push_back(c);
    }
    std::vector<int> order((size_t)count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return of_lp[a].size() > of_lp[b].size();
    });
    std::vector<std::vector<int>> lists(kXcds);
    for (int i : order) {
        int best = 0;
        for (int x = 1; x < kXcds; ++x)
            if (lists[x].size() < lists[best].size()) best = x;
        lists[best].insert(lists[best].end(), of_lp[i].begin(), of_lp[i].end());
    }
    size_t len = 0;
    for (const auto &l : lists) len = l.size() > len ? l.size() : len;
    if (len == 0) len = 1;
    xp.assign(len * kXcds, -1);
    for (int x = 0; x < kXcds; ++x)
        for (size_t j = 0; j < lists[x].size(); ++j) xp[j * kXcds + x] = lists[x][j];
    return (int)xp.size();
}

// Column order of the concatenated matrix, inside each LP's own column
// range: columns by entry count, largest first, equal counts by the row of
// their first entry (two stable counting passes per LP), as for a single
// LP.  Rows next to each other then gather columns next to each other in
// A x and rows of A' next to each other gather nearby y in A'y.  The
// block-diagonal structure and every LP's column range stay as they are.
// Runs after the concatenation and before the transpose, whose scratch
// (trp, cursor, tci) and the not yet initialised x0, sx, xbar it borrows.
static int b_order_columns(BDev &d, const std::vector<BLP> &hl, int *cperm, int *cinv,
                           hipStream_t s) {
    d.cperm = d.cinv = nullptr;
    const int N = d.N, M = d.M;
    if (N < 2 || d.NNZ == 0 || M == 0) return PDHG_OK;
    launch_col_counts(d.ci, d.NNZ, N, d.trp, s);
    launch_first_rows(d.rp, d.ci, M, N, d.NNZ, d.cursor, s);
    std::vector<int> cnt((size_t)N + 1), first((size_t)N);
    if (hipMemcpyAsync(cnt.data(), d.trp, sizeof(int) * ((size_t)N + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(first.data(), d.cursor, sizeof(int) * (size_t)N, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PDHG_E_HIP;
    std::vector<int> order((size_t)N), inv((size_t)N), by_first, fstart, start;
    bool ident = true;
    for (const BLP &L : hl) {
        const int co = L.col_off, n = L.n, ro = L.row_off, m = L.m;
        // key of a column: its first row inside the LP, m when it is empty
        auto key = [&](int j) { return first[(size_t)co + j] >= M ? m : first[(size_t)co + j] - ro; };
        by_first.assign((size_t)n, 0);
        fstart.assign((size_t)m + 2, 0);
        for (int j = 0; j < n; ++j) fstart[(size_t)key(j) + 1] += 1;
        for (int r = 0; r <= m; ++r) fstart[(size_t)r + 1] += fstart[r];
        for (int j = 0; j < n; ++j) by_first[(size_t)fstart[(size_t)key(j)]++] = j;
        int cmax = 0;
        for (int j = 0; j < n; ++j) cmax = cnt[(size_t)co + j + 1] > cmax ? cnt[(size_t)co + j + 1] : cmax;
        start.assign((size_t)cmax + 2, 0);
        for (int j = 0; j < n; ++j) start[(size_t)(cmax - cnt[(size_t)co + j + 1]) + 1] += 1;
        for (int k = 0; k <= cmax; ++k) start[(size_t)k + 1] += start[k];
        for (int t = 0; t < n; ++t) {
            const int j = by_first[(size_t)t];
            const int q = start[(size_t)(cmax - cnt[(size_t)co + j + 1])]++;
            order[(size_t)co + q] = co + j;
            inv[(size_t)co + j] = co + q;
            ident &= (q == j);
        }
    }
    if (ident) return PDHG_OK;
    if (hipMemcpyAsync(cperm, order.data(), sizeof(int) * (size_t)N, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(cinv, inv.data(), sizeof(int) * (size_t)N, hipMemcpyHostToDevice, s) != hipSuccess)
        return PDHG_E_HIP;
    launch_permute_cols(d.ci, d.NNZ, cinv, d.tci, d.c, d.l, d.u, cperm, N, d.x0, d.sx, d.xbar, s);
    const size_t nb = sizeof(double) * (size_t)N;
    if (hipMemcpyAsync(d.ci, d.tci, sizeof(int) * (size_t)d.NNZ, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d.c, d.x0, nb, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d.l, d.sx, nb, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d.u, d.xbar, nb, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)  // the host vectors above leave scope
        return PDHG_E_HIP;
    d.cperm = cperm;
    d.cinv = cinv;
    return hipGetLastError() == hipSuccess ? PDHG_OK : PDHG_E_HIP;
}

// Bound classes of the concatenated columns: at most kBoundClasses distinct
// (l, u) pairs (bit for bit) over the whole batch give each column a class
// byte, which the primal update reads instead of l and u.
static int b_bound_classes(BDev &d, unsigned char *dev, hipStream_t s) {
    d.bcls = nullptr;
    const size_t N = (size_t)d.N;
    std::vector<unsigned long long> lo(N), hi(N);
    if (hipMemcpyAsync(lo.data(), d.l, sizeof(double) * N, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hi.data(), d.u, sizeof(double) * N, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PDHG_E_HIP;
    std::vector<unsigned char> cls(N);
    unsigned long long kl[kBoundClasses], ku[kBoundClasses];
    int nc = 0;
    for (size_t j = 0; j < N; ++j) {
        int k = 0;
        while (k < nc && (kl[k] != lo[j] || ku[k] != hi[j])) ++k;
        if (k == nc) {
            if (nc == kBoundClasses) return PDHG_OK;
            kl[nc] = lo[j];
            ku[nc] = hi[j];
            ++nc;
        }
        cls[j] = (unsigned char)k;
    }
    for (int k = 0; k < kBoundClasses; ++k) {
        const int q = k < nc ? k : 0;
        memcpy(&d.blo[k], &kl[q], sizeof(double));
        memcpy(&d.bhi[k], &ku[q], sizeof(double));
    }
    if (hipMemcpyAsync(dev, cls.data(), N, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)  // the host vector above leaves scope
        return PDHG_E_HIP;
    d.bcls = dev;
    d.nbcls = nc;
    return PDHG_OK;
}

}  // namespace pdhg

using namespace pdhg;

struct pdhg_batch_handle {
    BDev d;
    hipStream_t stream, cap;
    int count;
    int mode, period, kkt_kind;
    hipGraphExec_t gexec;
    hipGraphExec_t gexec_r;  // the same block, its first primal update from the check's A'y
    double g_tol;
    bool g_valid;
    bool reuse;              // PDHG_CHECK_REUSE=0 at creation: never take the check's A'y
    bool fresh;              // the last step on the batch was a check
    std::vector<int> pw_used;
    // the tape of the last unrolled forward call, while nothing has changed
    // the batch since (the backward recomputes its windows from it)
    const void *tape_of = nullptr;
    int64_t tape_K = -1;
    bool tape_ok = false;
    // the SpMV schedules (pdhg_batch_set_schedule): the XCD placement lists
    // and the 16-bit indices built at creation
    int *xpA_x = nullptr, *xpT_x = nullptr;
    int nslotA_x = 0, nslotT_x = 0;
    unsigned short *ci16_x = nullptr, *tci16_x = nullptr;
    int placement = 1, index16 = 0;
};

#define BCK(expr)                                  \
    do {                                           \
        if ((expr) != hipSuccess) return PDHG_E_HIP; \
    } while (0)

static int b_last_error() { return hipGetLastError() == hipSuccess ? PDHG_OK : PDHG_E_HIP; }

static int b_read_lps(pdhg_batch_t *h, std::vector<BLP> &out) {
    out.resize((size_t)h->count);
    BCK(hipMemcpyAsync(out.data(), h->d.lp, sizeof(BLP) * (size_t)h->count, hipMemcpyDeviceToHost,
                       h->stream));
    BCK(hipStreamSynchronize(h->stream));
    return PDHG_OK;
}

static int b_slots(int mode) {
    if (mode == PDHG_RESTART_ADAPTIVE) return 1;
    if (mode == PDHG_RESTART_FLEXIBLE) return 3;
    return 0;
}

extern "C" {

size_t pdhg_batch_workspace_bytes(int32_t count, const int64_t *m, const int64_t *n,
                                  const int64_t *nnz) {
    if (!m || !n || !nnz) return 0;
    BLayout L;
    if (!b_layout(count, m, n, nnz, &L)) return 0;
    return L.total;
}

int pdhg_batch_create(int32_t count, const pdhg_lp *lps, const pdhg_params *prm,
                      void *workspace, size_t workspace_bytes, void *stream, pdhg_batch_t **out) {
    if (!out) return PDHG_E_INVALID;
    *out = nullptr;
    if (count < 1 || !lps) return PDHG_E_INVALID;
    std::vector<int64_t> ms(count), ns(count), zs(count);
    std::vector<pdhg_params> P(count);
    for (int i = 0; i < count; ++i) {
        const pdhg_lp &lp = lps[i];
        ms[i] = lp.m;
        ns[i] = lp.n;
        zs[i] = lp.nnz;
        if (!lp.row_ptr || !lp.c || !lp.l || !lp.u) return PDHG_E_INVALID;
        if (lp.nnz > 0 && (!lp.col_idx || !lp.vals)) return PDHG_E_INVALID;
        if (lp.m > 0 && !lp.b) return PDHG_E_INVALID;
        if (prm) P[i] = prm[i];
        else pdhg_default_params(&P[i]);
        const pdhg_params &p = P[i];
        if (!(p.omega > 0.0) || !isfinite(p.omega) || !(p.beta > 0.0) || !(p.beta < 1.0) ||
            p.check_period < 1 || p.tau0 < 1 || p.kkt_kind < 0 || p.kkt_kind > 2 ||
            isnan(p.eta) || isinf(p.eta) || p.restart_mode < 0 || p.restart_mode > 2 ||
            p.method != PDHG_METHOD_PDHG)
            return PDHG_E_INVALID;
        if (p.restart_mode != P[0].restart_mode || p.check_period != P[0].check_period ||
            p.kkt_kind != P[0].kkt_kind)
            return PDHG_E_INVALID;
    }
    BLayout L;
    if (!b_layout(count, ms.data(), ns.data(), zs.data(), &L)) return PDHG_E_INVALID;
    if (!workspace || ((uintptr_t)workspace & 255u) || workspace_bytes < L.total)
        return PDHG_E_WORKSPACE;
    pdhg_batch_t *h = new (std::nothrow) pdhg_batch_handle();
    if (!h) return PDHG_E_HIP;
    h->stream = (hipStream_t)stream;
    h->cap = nullptr;
    h->gexec = nullptr;
    h->gexec_r = nullptr;
    h->g_valid = false;
    h->fresh = false;
    {
        const char *e = getenv("PDHG_CHECK_REUSE");
        h->reuse = !(e && e[0] == '0');
    }
    h->count = count;
    h->mode = P[0].restart_mode;
    h->period = P[0].check_period;
    h->kkt_kind = P[0].kkt_kind;
    char *ws = (char *)workspace;
    BDev &d = h->d;
    memset(&d, 0, sizeof(d));
    d.count = count;
    d.M = L.M;
    d.N = L.N;
    d.NNZ = L.NNZ;
    d.nblk = L.nblk;
    d.nblkA = L.nblkA;
    d.nblkT = L.nblkT;
    d.lp = (BLP *)(ws + L.o_lp);
    d.err = (int *)(ws + L.o_err);
    d.rp = (int *)(ws + L.o_rp);
    d.ci = (int *)(ws + L.o_ci);
    d.v = (double *)(ws + L.o_v);
    d.c = (double *)(ws + L.o_c);
    d.b = (double *)(ws + L.o_b);
    d.l = (double *)(ws + L.o_l);
    d.u = (double *)(ws + L.o_u);
    d.kind = (signed char *)(ws + L.o_kind);
    d.trp = (int *)(ws + L.o_trp);
    d.tci = (int *)(ws + L.o_tci);
    d.perm = (int *)(ws + L.o_perm);
    d.tv = (double *)(ws + L.o_tv);
    d.cursor = (int *)(ws + L.o_cursor);
    d.long_rows = (int *)(ws + L.o_long);
    d.brA = (int *)(ws + L.o_brA);
    d.brT = (int *)(ws + L.o_brT);
    d.xpA = (int *)(ws + L.o_xpA);
    d.xpT = (int *)(ws + L.o_xpT);
    d.lp_row = (int *)(ws + L.o_lprow);
    d.lp_col = (int *)(ws + L.o_lpcol);
    d.tau_col = (double *)(ws + L.o_tau);
    d.sigma_row = (double *)(ws + L.o_sig);
    d.blk_lp = (int *)(ws + L.o_blklp);
    d.blk_first = (int *)(ws + L.o_blkfirst);
    d.blkA = (int *)(ws + L.o_blkA);
    d.blkT = (int *)(ws + L.o_blkT);
    d.lp_r0 = (int *)(ws + L.o_lpr0);
    d.lp_c0 = (int *)(ws + L.o_lpc0);
    d.ci16 = d.tci16 = nullptr;
    const size_t sn = al(sizeof(double) * (size_t)L.N), sm = al(sizeof(double) * (size_t)(L.M > 0 ? L.M : 1));
    double **vn[6] = {&d.x, &d.x0, &d.sx, &d.xbar, &d.atyb, &d.aty};
    double **vm[6] = {&d.y, &d.y0, &d.sy, &d.q, &d.ybar, &d.axb};
    for (int k = 0; k < 6; ++k) {
        *vn[k] = (double *)(ws + L.o_vn + k * sn);
        *vm[k] = (double *)(ws + L.o_vm + k * sm);
    }
    d.part = (double *)(ws + L.o_part);
    d.log = (double *)(ws + L.o_log);
    d.hcnt = (unsigned int *)(ws + L.o_hcnt);
    d.hD = (double *)(ws + L.o_hD);
    d.hA = (double *)(ws + L.o_hA);
    d.tpart = (double *)(ws + L.o_tpart);
    d.ccount = (unsigned int *)(ws + L.o_ccount);
    d.coff = (unsigned int *)(ws + L.o_coff);
    d.ckey = (unsigned long long *)(ws + L.o_ckey);
    d.ca = (double *)(ws + L.o_ca);
    d.cd = (double *)(ws + L.o_cd);

    // host-side tables: per-LP offsets and the element-block table
    std::vector<BLP> hl((size_t)count);
    std::vector<int> blk_lp, blk_first;
    std::vector<double> etas((size_t)count);
    int roff = 0, coff_ = 0;
    for (int i = 0; i < count; ++i) {
        BLP &b = hl[i];
        memset(&b, 0, sizeof(BLP));
        b.m = (int)ms[i];
        b.n = (int)ns[i];
        b.row_off = roff;
        b.col_off = coff_;
        b.blk_begin = (int)blk_lp.size();
        const int E = b.n + b.m;
        for (int f = 0; f < E; f += kChunk) {
            blk_lp.push_back(i);
            blk_first.push_back(f);
        }
        b.blk_end = (int)blk_lp.size();
        b.omega = P[i].omega;
        b.beta = P[i].beta;
        b.sw = sqrt(P[i].omega);
        b.tau0 = P[i].tau0;
        b.conv_which = -1;
        b.conv_k = -1;
        etas[i] = P[i].eta;
        roff += b.m;
        coff_ += b.n;
    }
    int rc = PDHG_OK;
    hipStream_t s = h->stream;
    double *eta_keep = d.log;  // requested step sizes; the log is written only by checks
    do {
        if (hipMemsetAsync(d.err, 0, sizeof(int) * 16, s) != hipSuccess) { rc = PDHG_E_HIP; break; }
        // validate every LP with the single-LP validation kernel
        for (int i = 0; i < count; ++i) {
            Dev vd;
            memset(&vd, 0, sizeof(vd));
            vd.m = (int)ms[i];
            vd.n = (int)ns[i];
            vd.nnz = (int)zs[i];
            vd.rp = lps[i].row_ptr;
            vd.ci = lps[i].col_idx;
            vd.v = lps[i].vals;
            vd.c = lps[i].c;
            vd.b = lps[i].b;
            vd.l = lps[i].l;
            vd.u = lps[i].u;
            vd.kind = (const signed char *)lps[i].row_kind;
            vd.err = d.err;
            launch_validate(vd, s);
        }
        int err = 0;
        if (hipMemcpyAsync(&err, d.err, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { rc = PDHG_E_HIP; break; }
        if (err) { rc = PDHG_E_INVALID; break; }
        if (hipMemcpyAsync(d.lp, hl.data(), sizeof(BLP) * (size_t)count, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(d.blk_lp, blk_lp.data(), sizeof(int) * blk_lp.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(d.blk_first, blk_first.data(), sizeof(int) * blk_first.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(eta_keep, etas.data(), sizeof(double) * (size_t)count, hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = PDHG_E_HIP;
            break;
        }
        // per-LP block ranges of the SpMV splits and the LPs' offsets
        std::vector<int> hblkA((size_t)count + 1), hblkT((size_t)count + 1);
        std::vector<int> hr0((size_t)count + 1), hc0((size_t)count + 1);
        long long wide = 0;
        hblkA[0] = hblkT[0] = 0;
        for (int i = 0; i < count; ++i) {
            hblkA[(size_t)i + 1] = hblkA[i] + nblocks_for((int)ms[i], (int)zs[i]);
            hblkT[(size_t)i + 1] = hblkT[i] + nblocks_for((int)ns[i], (int)zs[i]);
            hr0[i] = hl[i].row_off;
            hc0[i] = hl[i].col_off;
            wide = std::max(wide, (long long)std::max(ms[i], ns[i]));
        }
        hr0[count] = L.M;
        hc0[count] = L.N;
        if (hblkA[count] != d.nblkA || hblkT[count] != d.nblkT) {
            rc = PDHG_E_INVALID;
            break;
        }
        if (hipMemcpyAsync(d.blkA, hblkA.data(), sizeof(int) * hblkA.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(d.blkT, hblkT.data(), sizeof(int) * hblkT.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(d.lp_r0, hr0.data(), sizeof(int) * hr0.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(d.lp_c0, hc0.data(), sizeof(int) * hc0.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {  // the host vectors above leave scope
            rc = PDHG_E_HIP;
            break;
        }
        long long nz_off = 0;
        for (int i = 0; i < count; ++i) {
            const BLP &b = hl[i];
            long long mx = zs[i];
            if (b.m > mx) mx = b.m;
            if (b.n > mx) mx = b.n;
            if (mx > 0)
                hipLaunchKernelGGL(k_bconcat, dim3(div_up(mx, kWG)), dim3(kWG), 0, s, d, i,
                                   lps[i].row_ptr, lps[i].col_idx, lps[i].vals, lps[i].c, lps[i].b,
                                   lps[i].l, lps[i].u, (const signed char *)lps[i].row_kind, b.m,
                                   b.n, (int)zs[i], b.row_off, b.col_off, (int)nz_off);
            nz_off += zs[i];
        }
        hipLaunchKernelGGL(k_bclose_rp, dim3(1), dim3(1), 0, s, d);
        if ((rc = b_order_columns(d, hl, (int *)(ws + L.o_cperm), (int *)(ws + L.o_cinv), s)) != PDHG_OK)
            break;
        if ((rc = b_bound_classes(d, (unsigned char *)(ws + L.o_bcls), s)) != PDHG_OK) break;
        // explicit A' of the block-diagonal matrix and the SpMV row splits
        Dev td;
        memset(&td, 0, sizeof(td));
        td.m = d.M;
        td.n = d.N;
        td.nnz = d.NNZ;
        td.rp = d.rp;
        td.ci = d.ci;
        td.v = d.v;
        td.trp = d.trp;
        td.tci = d.tci;
        td.perm = d.perm;
        td.tv = d.tv;
        td.cursor = d.cursor;
        td.long_rows = d.long_rows;
        td.err = d.err;
        hipLaunchKernelGGL(k_lpsplit, dim3(div_up(d.nblkA + 1, kWG)), dim3(kWG), 0, s, d.rp, d.lp_r0,
                           d.blkA, count, d.nblkA, d.brA);
        launch_transpose(td, s);
        hipLaunchKernelGGL(k_lpsplit, dim3(div_up(d.nblkT + 1, kWG)), dim3(kWG), 0, s, d.trp, d.lp_c0,
                           d.blkT, count, d.nblkT, d.brT);
        if (d.NNZ > 0 && wide <= 65536) {
            unsigned short *a16 = (unsigned short *)(ws + L.o_ci16), *t16 = (unsigned short *)(ws + L.o_tci16);
            if (d.M > 0)
                hipLaunchKernelGGL(k_bidx16, dim3(div_up(d.M, kWG)), dim3(kWG), 0, s, d.rp, d.ci, d.M,
                                   d.lp_row, d.lp_c0, a16);
            hipLaunchKernelGGL(k_bidx16, dim3(div_up(d.N, kWG)), dim3(kWG), 0, s, d.trp, d.tci, d.N,
                               d.lp_col, d.lp_r0, t16);
            d.ci16 = a16;
            d.tci16 = t16;
        }
        {
            std::vector<int> hbrA((size_t)d.nblkA + 1), hbrT((size_t)d.nblkT + 1);
            std::vector<int> roffs((size_t)count + 1), coffs((size_t)count + 1);
            for (int i = 0; i < count; ++i) {
                roffs[i] = hl[i].row_off;
                coffs[i] = hl[i].col_off;
            }
            roffs[count] = d.M;
            coffs[count] = d.N;
            if (hipMemcpyAsync(hbrA.data(), d.brA, sizeof(int) * hbrA.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(hbrT.data(), d.brT, sizeof(int) * hbrT.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) { rc = PDHG_E_HIP; break; }
            std::vector<int> xa, xt;
            d.nslotA = place_blocks(hbrA, roffs, count, xa);
            d.nslotT = place_blocks(hbrT, coffs, count, xt);
            // the lists hold each block at most once: within kXcds (nblk + 1) slots
            if ((size_t)d.nslotA > (size_t)kXcds * ((size_t)d.nblkA + 1) ||
                (size_t)d.nslotT > (size_t)kXcds * ((size_t)d.nblkT + 1)) { rc = PDHG_E_INVALID; break; }
            if (hipMemcpyAsync(d.xpA, xa.data(), sizeof(int) * xa.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(d.xpT, xt.data(), sizeof(int) * xt.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) { rc = PDHG_E_HIP; break; }
            h->xpA_x = d.xpA;
            h->xpT_x = d.xpT;
            h->nslotA_x = d.nslotA;
            h->nslotT_x = d.nslotT;
            h->ci16_x = d.ci16;
            h->tci16_x = d.tci16;
            h->placement = 1;
            h->index16 = d.ci16 ? 1 : 0;
        }
        hipLaunchKernelGGL(k_bnorm_partials, dim3(d.nblk), dim3(kWG), 0, s, d);
        hipLaunchKernelGGL(k_bnorm_final, dim3(count), dim3(kWG), 0, s, d);
        const long long NM = (long long)d.N + d.M;
        hipLaunchKernelGGL(k_binit, dim3(div_up(NM, kWG)), dim3(kWG), 0, s, d);
        bspmv_A(d, d.x, d.q, 0, s);
        if ((rc = b_last_error()) != PDHG_OK) break;
        // power iteration for the LPs without a given step size
        bool need_pw = false;
        for (int i = 0; i < count; ++i) need_pw |= !(etas[i] > 0.0);
        h->pw_used.assign((size_t)count, 0);
        if (need_pw) {
            const int pw_max = P[0].power_iters > 0 ? P[0].power_iters : 1000;
            const double pw_tol = P[0].power_tol > 0.0 ? P[0].power_tol : 1e-10;
            hipLaunchKernelGGL(k_bpw_init, dim3(div_up(d.N > count ? d.N : count, kWG)), dim3(kWG), 0, s, d);
            std::vector<BLP> cur;
            bool all = false;
            while (!all && rc == PDHG_OK) {
                for (int q = 0; q < 25; ++q) {
                    bspmv_A(d, d.atyb, d.axb, 1, s);
                    bspmv_T(d, d.axb, d.aty, 1, s);
                    hipLaunchKernelGGL(k_bpw_partials, dim3(d.nblk), dim3(kWG), 0, s, d);
                    hipLaunchKernelGGL(k_bpw_final, dim3(count), dim3(kWG), 0, s, d, pw_tol, pw_max);
                    hipLaunchKernelGGL(k_bpw_norm, dim3(div_up(d.N, kWG)), dim3(kWG), 0, s, d);
                    hipLaunchKernelGGL(k_bpw_settle, dim3(div_up(count, kWG)), dim3(kWG), 0, s, d);
                }
                if ((rc = b_last_error()) != PDHG_OK) break;
                if ((rc = b_read_lps(h, cur)) != PDHG_OK) break;
                all = true;
                for (int i = 0; i < count; ++i) all &= cur[i].pw_done != 0;
            }
            if (rc != PDHG_OK) break;
            for (int i = 0; i < count; ++i) h->pw_used[i] = cur[i].pw_it;
        }
        hipLaunchKernelGGL(k_bset_steps, dim3(div_up(count, kWG)), dim3(kWG), 0, s, d, eta_keep);
        hipLaunchKernelGGL(k_bsteps, dim3(div_up((long long)d.N + d.M, kWG)), dim3(kWG), 0, s, d);
        if ((rc = b_last_error()) != PDHG_OK) break;
        if (hipStreamSynchronize(s) != hipSuccess) { rc = PDHG_E_HIP; break; }
        if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) { rc = PDHG_E_HIP; break; }
    } while (0);
    if (rc != PDHG_OK) {
        if (h->cap) (void)hipStreamDestroy(h->cap);
        delete h;
        return rc;
    }
    *out = h;
    return PDHG_OK;
}

void pdhg_batch_destroy(pdhg_batch_t *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->gexec_r) (void)hipGraphExecDestroy(h->gexec_r);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    delete h;
}

int pdhg_batch_step(pdhg_batch_t *h, int64_t iters) {
    if (!h || iters < 0) return PDHG_E_INVALID;
    h->tape_ok = false;
    if (iters > 0) h->fresh = false;
    b_iterations(h->d, iters, h->stream);
    return b_last_error();
}

static int b_build_graph(pdhg_batch_t *h, double tol) {
    if (h->g_valid && h->g_tol == tol) return PDHG_OK;
    hipGraphExec_t *ex[2] = {&h->gexec, &h->gexec_r};
    for (int v = 0; v < 2; ++v)
        if (*ex[v]) {
            (void)hipGraphExecDestroy(*ex[v]);
            *ex[v] = nullptr;
        }
    h->g_valid = false;
    for (int v = 0; v < (h->reuse ? 2 : 1); ++v) {
        hipGraph_t g = nullptr;
        BCK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        b_iterations(h->d, h->period, h->cap, v == 1);
        b_check(h->d, tol, h->kkt_kind, b_slots(h->mode), h->cap);
        if (hipStreamEndCapture(h->cap, &g) != hipSuccess) return PDHG_E_HIP;
        hipError_t e = hipGraphInstantiate(ex[v], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            *ex[v] = nullptr;
            return PDHG_E_HIP;
        }
    }
    h->g_tol = tol;
    h->g_valid = true;
    return PDHG_OK;
}

int pdhg_batch_solve(pdhg_batch_t *h, int64_t max_iters, double tol, pdhg_result *results) {
    if (!h || max_iters < 0 || isnan(tol)) return PDHG_E_INVALID;
    h->tape_ok = false;
    int rc;
    std::vector<BLP> cur;
    hipLaunchKernelGGL(k_breset, dim3(div_up(h->count, kWG)), dim3(kWG), 0, h->stream, h->d);
    if ((rc = b_read_lps(h, cur))) return rc;
    // every LP of a batch has run the same iterations until it converged;
    // the schedule follows the LPs that are still running
    long long k = -1;
    bool all_done = true;
    for (int i = 0; i < h->count; ++i)
        if (!cur[i].done) {
            all_done = false;
            if (k < 0) k = cur[i].k;
        }
    if (all_done) k = 0;
    const int64_t P = h->period;
    const int64_t k_end = k + max_iters;
    while (!all_done && k < k_end) {
        if (k % P == 0 && k_end - k >= P) {
            if ((rc = b_build_graph(h, tol))) return rc;
            int64_t blocks = (k_end - k) / P, batch = 1;
            while (blocks > 0 && !all_done) {
                const int64_t nb = batch < blocks ? batch : blocks;
                for (int64_t q = 0; q < nb; ++q) {
                    BCK(hipGraphLaunch(h->fresh && h->gexec_r ? h->gexec_r : h->gexec,
                                       h->stream));
                    h->fresh = true;
                }
                if ((rc = b_read_lps(h, cur))) return rc;
                blocks -= nb;
                k += nb * P;
                all_done = true;
                for (int i = 0; i < h->count; ++i) {
                    if (cur[i].numerr) return PDHG_E_NUMERICAL;
                    all_done &= cur[i].done != 0;
                }
                if (batch < 64) batch *= 2;
            }
            continue;
        }
        const int64_t to_check = P - (k % P);
        const int64_t sstep = to_check < k_end - k ? to_check : k_end - k;
        b_iterations(h->d, sstep, h->stream);
        if (sstep > 0) h->fresh = false;
        k += sstep;
        if (k % P == 0) {
            b_check(h->d, tol, h->kkt_kind, b_slots(h->mode), h->stream);
            if ((rc = b_last_error())) return rc;
            h->fresh = true;
        }
        if ((rc = b_read_lps(h, cur))) return rc;
        all_done = true;
        for (int i = 0; i < h->count; ++i) {
            if (cur[i].numerr) return PDHG_E_NUMERICAL;
            all_done &= cur[i].done != 0;
        }
    }
    if ((rc = b_read_lps(h, cur))) return rc;
    bool every = true;
    for (int i = 0; i < h->count; ++i) {
        const BLP &L = cur[i];
        every &= L.conv_which >= 0;
        if (!results) continue;
        pdhg_result &r = results[i];
        r.iterations = L.k;
        r.restarts = L.restarts;
        r.which_point = L.conv_which;
        if (L.conv_which >= 0) {
            const double *k8 = L.conv_which == 1 ? L.kkt_avg : L.kkt_cur;
            r.status = PDHG_OK;
            r.kkt = k8[0];
            r.pobj = k8[4];
            r.dobj = k8[5];
        } else {
            r.status = PDHG_NOT_CONVERGED;
            r.kkt = L.kkt_cur[0];
            r.pobj = L.kkt_cur[4];
            r.dobj = L.kkt_cur[5];
        }
    }
    return every ? PDHG_OK : PDHG_NOT_CONVERGED;
}

int pdhg_batch_get_iterate(pdhg_batch_t *h, int32_t index, int32_t which, double *x, double *y) {
    if (!h || index < 0 || index >= h->count || which < 0 || which > 3 || !x) return PDHG_E_INVALID;
    std::vector<BLP> cur;
    int rc = b_read_lps(h, cur);
    if (rc) return rc;
    const BLP &L = cur[index];
    if (L.m > 0 && !y) return PDHG_E_INVALID;
    const int mx = L.n > L.m ? L.n : L.m;
    hipLaunchKernelGGL(k_bget, dim3(div_up(mx, kWG)), dim3(kWG), 0, h->stream, h->d, index, which, x, y);
    return b_last_error();
}

int pdhg_batch_set_schedule(pdhg_batch_t *h, int32_t placement, int32_t index16) {
    if (!h || (placement != 0 && placement != 1) || (index16 != 0 && index16 != 1) ||
        (index16 && !h->ci16_x))
        return PDHG_E_INVALID;
    BDev &d = h->d;
    d.xpA = placement ? h->xpA_x : nullptr;
    d.xpT = placement ? h->xpT_x : nullptr;
    d.nslotA = placement ? h->nslotA_x : d.nblkA;
    d.nslotT = placement ? h->nslotT_x : d.nblkT;
    d.ci16 = index16 ? h->ci16_x : nullptr;
    d.tci16 = index16 ? h->tci16_x : nullptr;
    h->placement = placement;
    h->index16 = index16;
    h->g_valid = false;  // the recorded graph holds the old launch arguments
    h->fresh = false;
    return PDHG_OK;
}

int pdhg_batch_autotune(pdhg_batch_t *h, int32_t iters, pdhg_batch_tune *out) {
    if (!h || iters < 1 || iters > 10000) return PDHG_E_INVALID;
    h->fresh = false;
    pdhg_batch_tune r;
    memset(&r, 0, sizeof(r));
    hipStream_t s = h->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return PDHG_E_HIP;
    }
    int rc = PDHG_OK, best_p = h->placement, best_i = h->index16, k = 0;
    double best = INFINITY;
    for (int pl = 1; pl >= 0 && rc == PDHG_OK; --pl) {
        for (int ix = h->ci16_x ? 1 : 0; ix >= 0 && rc == PDHG_OK; --ix) {
            (void)pdhg_batch_set_schedule(h, pl, ix);
            const BDev &d = h->d;
            // A'y and A x of the current point into the check's scratch
            // vectors (rewritten by every check before use)
            bspmv_T(d, d.y, d.aty, 0, s);
            bspmv_A(d, d.x, d.axb, 0, s);
            float ms = 0.f;
            if (hipEventRecord(e0, s) != hipSuccess) rc = PDHG_E_HIP;
            for (int q = 0; q < iters && rc == PDHG_OK; ++q) {
                bspmv_T(d, d.y, d.aty, 0, s);
                bspmv_A(d, d.x, d.axb, 0, s);
            }
            if (rc == PDHG_OK && (hipEventRecord(e1, s) != hipSuccess ||
                                  hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = PDHG_E_HIP;
            if (rc == PDHG_OK) rc = b_last_error();
            if (rc != PDHG_OK) break;
            const double per = (double)ms / iters;
            r.tried_placement[k] = pl;
            r.tried_index16[k] = ix;
            r.ms[k] = per;
            ++k;
            if (per < best) {
                best = per;
                best_p = pl;
                best_i = ix;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    r.candidates = k;
    (void)pdhg_batch_set_schedule(h, best_p, best_i);
    r.placement = h->placement;
    r.index16 = h->index16;
    if (out) *out = r;
    return rc;
}

int pdhg_batch_get_info(pdhg_batch_t *h, int32_t index, pdhg_info *out) {
    if (!h || index < 0 || index >= h->count || !out) return PDHG_E_INVALID;
    std::vector<BLP> cur;
    int rc = b_read_lps(h, cur);
    if (rc) return rc;
    const BLP &L = cur[index];
    out->eta = L.eta;
    out->tau = L.tau;
    out->sigma = L.sigma;
    out->sigma_max = L.pw_est;
    out->k = L.k;
    out->t = L.t;
    out->restarts = L.restarts;
    out->rho_prev = L.rho_prev;
    out->checks = L.checks;
    out->power_iters_used = h->pw_used.empty() ? 0 : h->pw_used[index];
    out->one_workgroup = 0;
    out->bound_classes = h->d.nbcls;
    return PDHG_OK;
}

int pdhg_batch_get_check_log(pdhg_batch_t *h, int32_t index, pdhg_check_record *out, int64_t max,
                             int64_t *count) {
    if (!h || index < 0 || index >= h->count || max < 0 || (max > 0 && !out)) return PDHG_E_INVALID;
    std::vector<BLP> cur;
    int rc = b_read_lps(h, cur);
    if (rc) return rc;
    const long long checks = cur[index].checks;
    const int64_t have = checks < kBLog ? checks : kBLog;
    const int64_t nret = have < max ? have : max;
    for (int64_t q = 0; q < nret; ++q) {
        const long long idx = checks - nret + q;
        const double *src = h->d.log + ((size_t)index * kBLog + (size_t)(idx % kBLog)) * kRec;
        BCK(hipMemcpyAsync(out[q].v, src, sizeof(double) * kRec, hipMemcpyDeviceToHost, h->stream));
    }
    BCK(hipStreamSynchronize(h->stream));
    if (count) *count = nret;
    return PDHG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------
// unrolled forward / reverse
// ---------------------------------------------------------------------
static bool tape_carve(const pdhg_batch_t *h, int64_t K, char *base, Tape *t, size_t *total) {
    if (K < 0 || K > (int64_t)1 << 40) return false;
    const BDev &d = h->d;
    const long long P = h->period;
    const long long nwin = (K + P - 1) / P;
    const size_t N = (size_t)d.N, M = (size_t)(d.M > 0 ? d.M : 1), C = (size_t)d.count;
    size_t o = 0;
    auto put = [&](size_t bytes) {
        size_t at = o;
        o += al(bytes);
        return at;
    };
    const size_t ocx = put(sizeof(double) * N * (size_t)(nwin > 0 ? nwin : 1));
    const size_t ocy = put(sizeof(double) * M * (size_t)(nwin > 0 ? nwin : 1));
    const size_t ocq = put(sizeof(double) * M * (size_t)(nwin > 0 ? nwin : 1));
    const size_t oev = put(sizeof(int) * C * (size_t)(nwin > 0 ? nwin : 1));
    const size_t oet = put(sizeof(long long) * C * (size_t)(nwin > 0 ? nwin : 1));
    const size_t osx = put(sizeof(double) * N * (size_t)(P + 1));
    const size_t osy = put(sizeof(double) * M * (size_t)(P + 1));
    const size_t oxh = put(sizeof(double) * N), oyh = put(sizeof(double) * M);
    const size_t osxh = put(sizeof(double) * N), osyh = put(sizeof(double) * M);
    const size_t ovh = put(sizeof(double) * M), ouw = put(sizeof(double2) * N);
    const size_t ogc = d.cinv ? put(sizeof(double) * N) : 0;
    const size_t oex = put(sizeof(double) * N), oey = put(sizeof(double) * M);
    const size_t oeq = put(sizeof(double) * M), oesx = put(sizeof(double) * N);
    const size_t oesy = put(sizeof(double) * M), oelp = put(sizeof(BLP) * C);
    *total = o;
    if (base && t) {
        t->cx = (double *)(base + ocx);
        t->cy = (double *)(base + ocy);
        t->cq = (double *)(base + ocq);
        t->ev = (int *)(base + oev);
        t->evT = (long long *)(base + oet);
        t->sx = (double *)(base + osx);
        t->sy = (double *)(base + osy);
        t->xh = (double *)(base + oxh);
        t->yh = (double *)(base + oyh);
        t->sxh = (double *)(base + osxh);
        t->syh = (double *)(base + osyh);
        t->vh = (double *)(base + ovh);
        t->uw = (double2 *)(base + ouw);
        t->gc = d.cinv ? (double *)(base + ogc) : nullptr;
        t->ex = (double *)(base + oex);
        t->ey = (double *)(base + oey);
        t->eq = (double *)(base + oeq);
        t->esx = (double *)(base + oesx);
        t->esy = (double *)(base + oesy);
        t->elp = (BLP *)(base + oelp);
        t->nwin = (int)nwin;
        t->P = (int)P;
        t->K = K;
    }
    return true;
}

extern "C" {

// copy the batch's end-of-forward state into the tape (save) or back
static hipError_t save_end_state(const BDev &d, const Tape &t, bool save, hipStream_t s) {
    const size_t N = (size_t)d.N, M = (size_t)d.M;
    struct {
        double *live, *kept;
        size_t len;
    } v[5] = {{d.x, t.ex, N}, {d.y, t.ey, M}, {d.q, t.eq, M}, {d.sx, t.esx, N}, {d.sy, t.esy, M}};
    for (auto &e : v) {
        if (!e.len) continue;
        hipError_t r = hipMemcpyAsync(save ? e.kept : e.live, save ? e.live : e.kept,
                                      sizeof(double) * e.len, hipMemcpyDeviceToDevice, s);
        if (r != hipSuccess) return r;
    }
    return hipMemcpyAsync(save ? (void *)t.elp : (void *)d.lp, save ? (void *)d.lp : (void *)t.elp,
                          sizeof(BLP) * (size_t)d.count, hipMemcpyDeviceToDevice, s);
}

size_t pdhg_batch_tape_bytes(pdhg_batch_t *h, int64_t K) {
    if (!h) return 0;
    size_t total = 0;
    if (!tape_carve(h, K, nullptr, nullptr, &total)) return 0;
    return total;
}

int pdhg_batch_set_data(pdhg_batch_t *h, const double *c, const double *b, const double *vals) {
    if (!h || !c || (h->d.M > 0 && !b) || (h->d.NNZ > 0 && !vals)) return PDHG_E_INVALID;
    h->fresh = false;
    h->tape_ok = false;
    const BDev &d = h->d;
    hipStream_t s = h->stream;
    if (d.cperm) launch_gather(c, d.cperm, d.N, d.c, s);
    else BCK(hipMemcpyAsync(d.c, c, sizeof(double) * (size_t)d.N, hipMemcpyDeviceToDevice, s));
    if (d.M > 0) BCK(hipMemcpyAsync(d.b, b, sizeof(double) * (size_t)d.M, hipMemcpyDeviceToDevice, s));
    if (d.NNZ > 0) {
        BCK(hipMemcpyAsync(d.v, vals, sizeof(double) * (size_t)d.NNZ, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_bgather_tv, dim3(div_up(d.NNZ, kWG)), dim3(kWG), 0, s, d);
    }
    hipLaunchKernelGGL(k_bnorm_partials, dim3(d.nblk), dim3(kWG), 0, s, d);
    hipLaunchKernelGGL(k_bnorm_final, dim3(d.count), dim3(kWG), 0, s, d);
    return b_last_error();
}

int pdhg_batch_unrolled_forward(pdhg_batch_t *h, int64_t K, void *tape, size_t tape_bytes,
                                double *xK) {
    if (!h) return PDHG_E_INVALID;
    h->fresh = false;
    Tape t;
    size_t need = 0;
    if (!tape_carve(h, K, (char *)tape, &t, &need)) return PDHG_E_INVALID;
    if (!tape || ((uintptr_t)tape & 255u) || tape_bytes < need) return PDHG_E_WORKSPACE;
    h->tape_ok = false;
    const BDev &d = h->d;
    hipStream_t s = h->stream;
    const long long NM = (long long)d.N + d.M;
    // every LP back to its initial point with fresh counters
    hipLaunchKernelGGL(k_breset_lps, dim3(div_up(d.count, kWG)), dim3(kWG), 0, s, d);
    hipLaunchKernelGGL(k_binit, dim3(div_up(NM, kWG)), dim3(kWG), 0, s, d);
    bspmv_A(d, d.x, d.q, 0, s);
    hipLaunchKernelGGL(k_bsteps, dim3(div_up(NM, kWG)), dim3(kWG), 0, s, d);
    const size_t N = (size_t)d.N, M = (size_t)d.M;
    for (int w = 0; w < t.nwin; ++w) {
        BCK(hipMemcpyAsync(t.cx + w * N, d.x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        if (M) {
            BCK(hipMemcpyAsync(t.cy + w * M, d.y, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
            BCK(hipMemcpyAsync(t.cq + w * M, d.q, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
        }
        const long long len = (K - (long long)w * t.P) < t.P ? (K - (long long)w * t.P) : t.P;
        b_iterations(d, len, s);
        if (len == t.P) {
            b_check(d, 0.0, h->kkt_kind, b_slots(h->mode), s);
            hipLaunchKernelGGL(k_record_events, dim3(div_up(d.count, kWG)), dim3(kWG), 0, s, d,
                               t.ev + (size_t)w * d.count, t.evT + (size_t)w * d.count);
        } else {
            BCK(hipMemsetAsync(t.ev + (size_t)w * d.count, 0, sizeof(int) * (size_t)d.count, s));
        }
        int rc = b_last_error();
        if (rc) return rc;
    }
    if (xK && d.cinv) launch_gather(d.x, d.cinv, d.N, xK, s);
    else if (xK) BCK(hipMemcpyAsync(xK, d.x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    BCK(save_end_state(d, t, true, s));
    const int rc = b_last_error();
    if (rc == PDHG_OK) {
        h->tape_of = tape;
        h->tape_K = K;
        h->tape_ok = true;
    }
    return rc;
}

int pdhg_batch_unrolled_backward(pdhg_batch_t *h, int64_t K, void *tape, size_t tape_bytes,
                                 const double *dLdx, double *gc, double *gb, double *gA) {
    if (!h || !dLdx || !gc || (h->d.M > 0 && !gb) || (h->d.NNZ > 0 && !gA)) return PDHG_E_INVALID;
    h->fresh = false;
    Tape t;
    size_t need = 0;
    if (!tape_carve(h, K, (char *)tape, &t, &need)) return PDHG_E_INVALID;
    if (!tape || ((uintptr_t)tape & 255u) || tape_bytes < need) return PDHG_E_WORKSPACE;
    // the tape must come from the last forward call, with nothing changed
    // since: the windows are recomputed from the batch's current data
    if (!h->tape_ok || tape != h->tape_of || K != h->tape_K) return PDHG_E_INVALID;
    const BDev &d = h->d;
    hipStream_t s = h->stream;
    const size_t N = (size_t)d.N, M = (size_t)d.M;
    const long long NM = (long long)d.N + d.M;
    // dL/dx in, dL/dc out in the caller's column order; the sweep runs in
    // the internal one (gA follows the entries, which keep their places)
    if (d.cperm) launch_gather(dLdx, d.cperm, d.N, t.xh, s);
    else BCK(hipMemcpyAsync(t.xh, dLdx, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    double *gcw = d.cinv ? t.gc : gc;
    hipLaunchKernelGGL(k_fill_d, dim3(div_up(d.N, kWG)), dim3(kWG), 0, s, t.sxh, (long long)d.N, 0.0);
    hipLaunchKernelGGL(k_fill_d, dim3(div_up(d.N, kWG)), dim3(kWG), 0, s, gcw, (long long)d.N, 0.0);
    if (M) {
        hipLaunchKernelGGL(k_fill_d, dim3(div_up(d.M, kWG)), dim3(kWG), 0, s, t.yh, (long long)d.M, 0.0);
        hipLaunchKernelGGL(k_fill_d, dim3(div_up(d.M, kWG)), dim3(kWG), 0, s, t.syh, (long long)d.M, 0.0);
        hipLaunchKernelGGL(k_fill_d, dim3(div_up(d.M, kWG)), dim3(kWG), 0, s, gb, (long long)d.M, 0.0);
    }
    if (d.NNZ) hipLaunchKernelGGL(k_fill_d, dim3(div_up(d.NNZ, kWG)), dim3(kWG), 0, s, gA, (long long)d.NNZ, 0.0);
    for (int w = t.nwin - 1; w >= 0; --w) {
        const long long len = (K - (long long)w * t.P) < t.P ? (K - (long long)w * t.P) : t.P;
        if (len == t.P)
            hipLaunchKernelGGL(k_adj_event, dim3(div_up(NM, kWG)), dim3(kWG), 0, s, d,
                               t.ev + (size_t)w * d.count, t.evT + (size_t)w * d.count, t.xh,
                               t.yh, t.sxh, t.syh);
        // recompute the window from its checkpoint, keeping every iterate
        BCK(hipMemcpyAsync(d.x, t.cx + w * N, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        BCK(hipMemcpyAsync(t.sx, d.x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        if (M) {
            BCK(hipMemcpyAsync(d.y, t.cy + w * M, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
            BCK(hipMemcpyAsync(d.q, t.cq + w * M, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
            BCK(hipMemcpyAsync(t.sy, d.y, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
        }
        // After the forward call no LP has stopped (its checks have no
        // stopping test), so every block runs and the epilogues write the
        // whole iterate into the tape.
        for (long long q = 1; q <= len; ++q)
            b_iteration(d, 0, s, t.sx + q * N, M ? t.sy + q * M : nullptr);
        for (long long q = len; q >= 1; --q) {
            const double *xt = t.sx + q * N, *xp = t.sx + (q - 1) * N;
            const double *yt = t.sy + q * M, *yp = t.sy + (q - 1) * M;
            if (M)
                hipLaunchKernelGGL(k_adj_dual, dim3(div_up(d.M, kWG)), dim3(kWG), 0, s, d, yt,
                                   t.yh, t.syh, t.vh, gb);
            EpiAdjPrimal ep{xt, xp, d.l, d.u, t.xh, t.sxh, gcw, t.uw, d.lp_col, d.lp};
            hipLaunchKernelGGL(k_spmv<EpiAdjPrimal>, dim3(d.nblkT), dim3(kWG), 0, s, d.trp, d.tci,
                               d.tv, t.vh, d.brT, d.nblkT, ep, (const int *)nullptr, 0);
            if (M)
                hipLaunchKernelGGL(k_adj_rows, dim3(d.nblkA), dim3(kWG), 0, s, d,
                                   (const double2 *)t.uw, yp, t.vh, t.yh, gA);
        }
        int rc = b_last_error();
        if (rc) return rc;
    }
    if (d.cinv) launch_gather(t.gc, d.cinv, d.N, gc, s);
    // the batch is left where the forward call left it (x_K, its running
    // sums and counters), so later calls continue from there
    BCK(save_end_state(d, t, false, s));
    return b_last_error();
}

}  // extern "C"
