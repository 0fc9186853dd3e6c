// HIP kernels of the restarted-PDHG library for gfx950 (MI355X).
//
// Hot path (two products per iteration, eq. PDHG-update):
//   over the explicit A' :  x+ = clamp(x - tau (c - A'y)), sx += x+
//   over A               :  q = A x+, y+ = proj(y + sigma (b - (2q - q_prev))),
//                           sy += y+, q_prev = q
// A(2x+ - x) is formed as 2 A x+ - A x from the cached A x of the previous
// half-step, so each iteration streams A and A' once and gathers x+ and y
// once per stored entry.  The extragradient method (eq.
// extra-gradient-update) uses the same products four times per iteration.
//
// SpMV schedule: rows are cut into merge-path blocks of kUnits (1024)
// rows+entries (a row belongs to the block its start falls in), so each
// workgroup owns whole rows and the per-row epilogue is fused.  A block
// stages its products value * vector[col] in 16 KB of LDS with coalesced
// non-temporal loads of the matrix, then groups of
// L lanes (L a power of two near the block's mean row length) reduce one
// row each with a fixed butterfly.  Every sum has a fixed order, so results
// are reproducible run to run.  Blocks whose entries exceed the LDS stage
// fall back to one wave per row straight from HBM.
//
// Column slabs: when the gathered vector is larger than one XCD's L2, the
// matrix is also kept split by column into S slabs whose slice of the
// vector fits an L2, and the product runs one slab per launch: every XCD
// then gathers from the same 4 MB slice.  The first slabs leave their row
// sums in an accumulator (added in slab order), and the last slab's launch
// applies the epilogue to the full sum.
//
// The normalized duality gap (eq. rhorz) needs the multiplier lambda* of the
// linear trust region of Section 6.3.1.  The GPU finds it by bisection on
// the multiplier over the IEEE bit patterns of the breakpoints d_i / a_i
// (monotone for non-negative doubles): 2048-way radix levels narrow the
// bracket containing lambda*, then lambda* = sqrt((r^2 - F)/A) on the
// breakpoint-free bracket, the closing formula of Algorithm 2.
#include "pdhg_device.h"

#include <math.h>
#include <stdlib.h>

namespace pdhg {

// Extragradient step (eq. extra-gradient-update) with F(z) = (c - A'y, Ax - b):
// the target z~ = proj_Z(z - D F(z)) (first two products), then
// z+ = proj_Z(z - D F(z~)) (last two); the sums of Algorithm 1 take z~.
struct EpiEgmTargetX {
    const double *__restrict__ c, *__restrict__ l, *__restrict__ u;
    const double *__restrict__ x;
    double *__restrict__ xt;
    double tau;
    __device__ __forceinline__ void operator()(int j, double aty) const {
        double v = x[j] - tau * (c[j] - aty);
        const double lo = l[j], hi = u[j];
        if (v < lo) v = lo;
        if (v > hi) v = hi;
        xt[j] = v;
    }
};

struct EpiEgmTargetY {
    const double *__restrict__ b;
    const signed char *__restrict__ kind;
    const double *__restrict__ y;
    double *__restrict__ yt;
    double sigma;
    __device__ __forceinline__ void operator()(int i, double ax) const {
        double v = y[i] - sigma * (ax - b[i]);
        if (kind && kind[i] && v < 0.0) v = 0.0;
        yt[i] = v;
    }
};

struct EpiEgmX {
    const double *__restrict__ c, *__restrict__ l, *__restrict__ u;
    double *__restrict__ x;
    const double *__restrict__ xt;
    double *__restrict__ sx;
    double tau;
    DevState *st;
    __device__ __forceinline__ void operator()(int j, double aty) const {
        double v = x[j] - tau * (c[j] - aty);
        const double lo = l[j], hi = u[j];
        if (v < lo) v = lo;
        if (v > hi) v = hi;
        x[j] = v;
        sx[j] += xt[j];
        if (j == 0) {  // iteration counters of Algorithm 1
            st->k += 1;
            st->t += 1;
        }
    }
};

struct EpiEgmY {
    const double *__restrict__ b;
    const signed char *__restrict__ kind;
    double *__restrict__ y;
    const double *__restrict__ yt;
    double *__restrict__ sy;
    double sigma;
    __device__ __forceinline__ void operator()(int i, double ax) const {
        double v = y[i] - sigma * (ax - b[i]);
        if (kind && kind[i] && v < 0.0) v = 0.0;
        y[i] = v;
        sy[i] += yt[i];
    }
};

int nblocks_for(int rows, int nnz) {
    long long u = (long long)rows + nnz;
    int nb = div_up(u, kUnits);
    return nb < 1 ? 1 : nb;
}

// Block table of a merge-path split, 2 (nblk + 1) ints: br[c] = first row
// i in [0, rows] with i + rp[i] >= c * kUnits (br[nblk] = rows), and
// br[nblk + 1 + c] = rp[br[c]], the block's first entry, so that a block
// finds its rows and its entries in one round of loads.
__global__ void k_rowsplit(const int *__restrict__ rp, int rows, int nblk, int *br) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nblk) return;
    int lo = rows;
    if (c < nblk) {
        long long target = (long long)c * kUnits;
        int hi = rows;
        lo = 0;
        while (lo < hi) {
            int mid = lo + ((hi - lo) >> 1);
            if ((long long)mid + rp[mid] >= target) hi = mid;
            else lo = mid + 1;
        }
    }
    br[c] = lo;
    br[nblk + 1 + c] = rp[lo];
}

void launch_rowsplit(const int *rp, int rows, int nnz, int nblk, int *br, hipStream_t s) {
    (void)nnz;
    hipLaunchKernelGGL(k_rowsplit, dim3(div_up(nblk + 1, kWG)), dim3(kWG), 0, s, rp, rows, nblk, br);
}

// k_rowsplit for row starts that begin at rp[0] (a row range): the merge
// path counts rp[i] - rp[0] entries before row i; the entry starts stored
// are rp's own values
__global__ void k_rowsplit_range(const int *__restrict__ rp, int rows, int nblk, int *br) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nblk) return;
    const int base = rp[0];
    int lo = rows;
    if (c < nblk) {
        long long target = (long long)c * kUnits;
        int hi = rows;
        lo = 0;
        while (lo < hi) {
            int mid = lo + ((hi - lo) >> 1);
            if ((long long)mid + (rp[mid] - base) >= target) hi = mid;
            else lo = mid + 1;
        }
    }
    br[c] = lo;
    br[nblk + 1 + c] = rp[lo];
}

void launch_rowsplit_range(const int *rp, int rows, int nblk, int *br, hipStream_t s) {
    hipLaunchKernelGGL(k_rowsplit_range, dim3(div_up(nblk + 1, kWG)), dim3(kWG), 0, s, rp, rows,
                       nblk, br);
}

// per slab, the smallest and the largest row (+ 1) holding one of its
// entries; range is preset to (rows, -1) per slab
__global__ void k_slab_ranges(Slabs sb, int *range) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sb.rows) return;
    for (int q = 0; q < sb.S; ++q) {
        const int *a = sb.srp + (size_t)q * (sb.rows + 1);
        if (a[i + 1] > a[i]) {
            atomicMin(&range[2 * q], i);
            atomicMax(&range[2 * q + 1], i + 1);
        }
    }
}

__global__ void k_slab_ranges_init(int *range, int S, int rows) {
    const int q = threadIdx.x;
    if (q < S) {
        range[2 * q] = rows;
        range[2 * q + 1] = -1;
    }
}

void launch_slab_ranges(const Slabs &sb, int *range, hipStream_t s) {
    hipLaunchKernelGGL(k_slab_ranges_init, dim3(1), dim3(kSlabMax), 0, s, range, sb.S, sb.rows);
    if (sb.rows > 0)
        hipLaunchKernelGGL(k_slab_ranges, dim3(div_up(sb.rows, kWG)), dim3(kWG), 0, s, sb, range);
}

// Each merge-path block's entries sorted by column: the key of an entry is
// column << kPkSlotBits | its place in the block, unique within the block,
// so an ascending bitonic sort of the keys in LDS gives one definite order
// (columns ascending, then places).  Padding keys (all ones) sort last; a
// real key can only equal them as the block's largest, whose slot then
// holds that same value.  Blocks longer than the LDS stage (the one-wave-
// per-row path of spmv_rows) keep their order.
__global__ __launch_bounds__(kWG) void k_sort_blocks(const int *__restrict__ rp,
                                                     const int *__restrict__ ci,
                                                     const double *__restrict__ v,
                                                     const int *__restrict__ br, int nblk,
                                                     unsigned *__restrict__ pk,
                                                     double *__restrict__ sv) {
    __shared__ unsigned key[kLdsProducts];
    (void)rp;
    const int b = blockIdx.x, tid = threadIdx.x;
    const int p0 = br[nblk + 1 + b], p1 = br[nblk + 2 + b];
    const int nb = p1 - p0;
    if (nb <= 0) return;
    if (nb > kLdsProducts) {
        for (int e = tid; e < nb; e += kWG) {
            pk[p0 + e] = ((unsigned)ci[p0 + e] << kPkSlotBits) | ((unsigned)e & kPkSlotMask);
            sv[p0 + e] = v[p0 + e];
        }
        return;
    }
    int P2 = 1;
    while (P2 < nb) P2 <<= 1;
    for (int e = tid; e < P2; e += kWG)
        key[e] = e < nb ? (((unsigned)ci[p0 + e] << kPkSlotBits) | (unsigned)e) : 0xFFFFFFFFu;
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P2; i += kWG) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned a = key[i], c = key[l];
                    const bool up = (i & k) == 0;
                    if ((a > c) == up) {
                        key[i] = c;
                        key[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < nb; e += kWG) {
        const unsigned w = key[e];
        pk[p0 + e] = w;
        sv[p0 + e] = v[p0 + (int)(w & kPkSlotMask)];
    }
}

void launch_sort_blocks(const int *rp, const int *ci, const double *v, const int *br, int nblk,
                        unsigned *pk, double *sv, hipStream_t s) {
    if (nblk > 0)
        hipLaunchKernelGGL(k_sort_blocks, dim3(nblk), dim3(kWG), 0, s, rp, ci, v, br, nblk, pk,
                           sv);
}

// One slab at a time, each launch over its row range (Slabs): row r of
// the range is row lo[sl] + r of the matrix.  Its sum goes to acc when an
// earlier range holds nothing of the row (or is added to acc otherwise);
// the launch of the last range holding the row applies the epilogue to the
// full sum instead.  The sums of a row are added in slab order, so every
// row gets the same value as with all rows in every launch (a row with no
// entries in a slab adds +0.0 there, which changes no sum but the sign of
// a zero one, and the update rounds it the same).
template <class Epi>
struct EpiSlab {
    Epi inner;
    double *acc;
    int lo;      // first row of this launch's range
    int before;  // rows at or past it are in no earlier range
    int after;   // rows below it are in no later range
    __device__ __forceinline__ void operator()(int r, double s) const {
        const int j = lo + r;
        const double t = j >= before ? s : acc[j] + s;
        if (j < after) inner(j, t);
        else acc[j] = t;
    }
};

template <class Epi, int WG = kWG>
__global__ __launch_bounds__(WG) void k_slab_one(Slabs sb, int sl, const double *__restrict__ xin,
                                                 Epi epi, const int *skip, int lbias) {
    __shared__ SpmvShared lds;
    // the gate and the slab's metadata are loaded together
    const long long *me = sb.smeta + 4 * sl;
    const int b = blockIdx.x, nb = (int)me[3];
    const int off = skip ? *skip : 0;
    if (off || b >= nb) return;
    const int *br = sb.sbr + me[2];
    const int r0 = br[b], r1 = br[b + 1];
    if (r0 >= r1) return;
    spmv_rows<Epi, int, false, WG>(sb.srp + me[0] + sb.lo[sl], sb.sci + me[1], sb.sv + me[1],
                                   xin + (size_t)sl * sb.W, r0, r1, br[nb + 1 + b], br[nb + 2 + b],
                                   epi, lds, lbias);
}

// the slabs one after the other, each row's update fused into the last
// launch whose range holds it
template <class Epi, int WG>
static void slabs_in_turn(const Slabs &sb, const double *in, const Epi &e, const int *skip,
                          int lbias, hipStream_t s) {
    for (int sl = 0; sl < sb.S; ++sl)
        hipLaunchKernelGGL((k_slab_one<EpiSlab<Epi>, WG>), dim3(sb.nbmax), dim3(WG), 0, s, sb, sl,
                           in, EpiSlab<Epi>{e, sb.spart, sb.lo[sl], sb.before[sl], sb.after[sl]},
                           skip, lbias);
}

template <class Epi, int WG>
static void product_A_wg(const Dev &d, const double *in, const Epi &e, const int *skip,
                         hipStream_t s) {
    if (d.slA.S > 1) {
        slabs_in_turn<Epi, WG>(d.slA, in, e, skip, d.lbA, s);
        return;
    }
    if (d.apk) {
        hipLaunchKernelGGL((k_spmv<Epi, unsigned, true, WG>), dim3(d.nblkA), dim3(WG), 0, s, d.rp,
                           d.apk, d.asv, in, d.brA, d.nblkA, e, skip, d.lbA);
        return;
    }
    hipLaunchKernelGGL((k_spmv<Epi, int, false, WG>), dim3(d.nblkA), dim3(WG), 0, s, d.rp, d.ci,
                       d.v, in, d.brA, d.nblkA, e, skip, d.lbA);
}

// workgroup size of the single-LP products (Dev::swg)
template <class Epi>
static void product_A(const Dev &d, const double *in, const Epi &e, const int *skip,
                      hipStream_t s) {
    if (d.m == 0) return;
    if (d.swgA == 128) product_A_wg<Epi, 128>(d, in, e, skip, s);
    else product_A_wg<Epi, kWG>(d, in, e, skip, s);
}

// the same over the rows of A' (explicit transpose)
template <class Epi, int WG>
static void product_T_wg(const Dev &d, const double *in, const Epi &e, const int *skip,
                         hipStream_t s) {
    if (d.slT.S > 1) {
        slabs_in_turn<Epi, WG>(d.slT, in, e, skip, d.lbT, s);
        return;
    }
    hipLaunchKernelGGL((k_spmv<Epi, int, false, WG>), dim3(d.nblkT), dim3(WG), 0, s, d.trp,
                       d.tci, d.tv, in, d.brT, d.nblkT, e, skip, d.lbT);
}

template <class Epi>
static void product_T(const Dev &d, const double *in, const Epi &e, const int *skip,
                      hipStream_t s) {
    if (d.swgT == 128) product_T_wg<Epi, 128>(d, in, e, skip, s);
    else product_T_wg<Epi, kWG>(d, in, e, skip, s);
}

void launch_primal(const Dev &d, double tau, int smode, hipStream_t s) {
    EpiPrimal e{d.c, d.l, d.u, d.x, d.sx, tau, d.st, d.bcls, {}, {}, smode};
    for (int k = 0; k < kBoundClasses; ++k) {
        e.blo[k] = d.blo[k];
        e.bhi[k] = d.bhi[k];
    }
    product_T(d, d.y, e, &d.st->done, s);
}

// The primal update of eq. (PDHG-update) from an A'y the check has just
// computed: A'y of the current y, or A'y-bar when the check restarted at
// the average (y became y-bar).  The row sums are those the product would
// give (the same launches computed them), so the update is bitwise the
// fused one.
__global__ __launch_bounds__(kWG) void k_primal_from_check(Dev d, EpiPrimal e) {
    if (d.st->done) return;
    const int j = blockIdx.x * kWG + threadIdx.x;
    if (j >= d.n) return;
    const bool bar = d.st->restarted && d.st->cand == 0;
    e(j, bar ? d.atyb[j] : d.aty[j]);
}

void launch_primal_from_check(const Dev &d, double tau, int smode, hipStream_t s) {
    EpiPrimal e{d.c, d.l, d.u, d.x, d.sx, tau, d.st, d.bcls, {}, {}, smode};
    for (int k = 0; k < kBoundClasses; ++k) {
        e.blo[k] = d.blo[k];
        e.bhi[k] = d.bhi[k];
    }
    hipLaunchKernelGGL(k_primal_from_check, dim3(div_up(d.n, kWG)), dim3(kWG), 0, s, d, e);
}

void launch_dual(const Dev &d, double sigma, int smode, hipStream_t s) {
    product_A(d, d.x, EpiDual{d.b, d.kind, d.y, d.sy, d.q, sigma, smode}, &d.st->done, s);
}

void launch_egm(const Dev &d, double tau, double sigma, int part, hipStream_t s) {
    const int *gate = &d.st->done;
    if (part < 0 || part == 0)
        product_T(d, d.y, EpiEgmTargetX{d.c, d.l, d.u, d.x, d.xt, tau}, gate, s);
    if (part < 0 || part == 1)
        product_A(d, d.x, EpiEgmTargetY{d.b, d.kind, d.y, d.yt, sigma}, gate, s);
    if (part < 0 || part == 2)
        product_T(d, d.yt, EpiEgmX{d.c, d.l, d.u, d.x, d.xt, d.sx, tau, d.st}, gate, s);
    if (part < 0 || part == 3)
        product_A(d, d.xt, EpiEgmY{d.b, d.kind, d.y, d.yt, d.sy, sigma}, gate, s);
}

static void spmv_A_gated(const Dev &d, const double *in, double *out, const int *skip,
                         hipStream_t s) {
    product_A(d, in, EpiStore{out}, skip, s);
}

// --- building the slabs (once, at create) ---------------------------------
// srp[s][i + 1] = entries of row i that fall in slab s (scanned afterwards)
__global__ void k_slab_count(Slabs sb, const int *__restrict__ rp, const int *__restrict__ ci) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sb.rows) return;
    int cnt[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) cnt[q] = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int sl = ci[p] / sb.W;
#pragma unroll
        for (int q = 0; q < 8; ++q) cnt[q] += (sl == q) ? 1 : 0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (q < sb.S) {
            sb.srp[(size_t)q * (sb.rows + 1) + i + 1] = cnt[q];
            if (i == 0) sb.srp[(size_t)q * (sb.rows + 1)] = 0;
        }
}

// place every entry of row i in its slab, keeping the row's order
__global__ void k_slab_scatter(Slabs sb, const int *__restrict__ rp, const int *__restrict__ ci,
                               const double *__restrict__ v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sb.rows) return;
    int run[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) run[q] = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int c = ci[p];
        const int sl = c / sb.W;
        int r = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (sl == q) r = run[q]++;
        const long long pos = sb.smeta[4 * sl + 1] + sb.srp[(size_t)sl * (sb.rows + 1) + i] + r;
        sb.sci[pos] = c - sl * sb.W;
        sb.sv[pos] = v[p];
    }
}

static void spmv_T_gated(const Dev &d, const double *in, double *out, const int *skip,
                         hipStream_t s) {
    product_T(d, in, EpiStore{out}, skip, s);
}

void launch_spmv_A(const Dev &d, const double *in, double *out, hipStream_t s,
                   const int *skip) {
    spmv_A_gated(d, in, out, skip, s);
}

void launch_spmv_T(const Dev &d, const double *in, double *out, hipStream_t s,
                   const int *skip) {
    spmv_T_gated(d, in, out, skip, s);
}

// ---------------------------------------------------------------------
// setup: validation, transpose, initial point, norms
// ---------------------------------------------------------------------
enum { ERR_RP = 1, ERR_COL = 2, ERR_VAL = 4, ERR_BOUND = 8, ERR_C = 16, ERR_B = 32, ERR_KIND = 64 };

__global__ void k_validate(Dev d) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long g0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int err = 0;
    for (long long i = g0; i <= d.m; i += stride) {
        int a = d.rp[i];
        if (i == 0 && a != 0) err |= ERR_RP;
        if (a < 0 || a > d.nnz) err |= ERR_RP;
        if (i < d.m && d.rp[i + 1] < a) err |= ERR_RP;
        if (i == d.m && a != d.nnz) err |= ERR_RP;
    }
    for (long long p = g0; p < d.nnz; p += stride) {
        int cc = d.ci[p];
        if (cc < 0 || cc >= d.n) err |= ERR_COL;
        if (!isfinite(d.v[p])) err |= ERR_VAL;
    }
    for (long long j = g0; j < d.n; j += stride) {
        double lo = d.l[j], hi = d.u[j];
        if (isnan(lo) || isnan(hi) || !(lo <= hi) || lo == INFINITY || hi == -INFINITY)
            err |= ERR_BOUND;
        if (!isfinite(d.c[j])) err |= ERR_C;
    }
    for (long long i = g0; i < d.m; i += stride) {
        if (!isfinite(d.b[i])) err |= ERR_B;
        if (d.kind && (d.kind[i] != 0 && d.kind[i] != 1)) err |= ERR_KIND;
    }
    if (err) atomicOr(d.err, err);
}

void launch_validate(const Dev &d, hipStream_t s) {
    long long mx = d.nnz;
    if (d.m + 1 > mx) mx = d.m + 1;
    if (d.n > mx) mx = d.n;
    int g = div_up(mx, kWG);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_validate, dim3(g), dim3(kWG), 0, s, d);
}

__global__ void k_fill_int(int *a, long long len, int val) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) a[i] = val;
}

__global__ void k_count_cols(const int *__restrict__ ci, int nnz, int *cnt /* n+1 */) {
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) atomicAdd(&cnt[ci[p] + 1], 1);
}

// In-place inclusive scan of chunks of 2048 ints; chunk totals to bsum.
constexpr int kScanChunk = 2048;
__global__ __launch_bounds__(kWG) void k_scan_chunks(int *a, long long len, int *bsum) {
    __shared__ int sh[kScanChunk];
    const long long base = (long long)blockIdx.x * kScanChunk;
    for (int e = threadIdx.x; e < kScanChunk; e += kWG)
        sh[e] = (base + e < len) ? a[base + e] : 0;
    __syncthreads();
    // each thread scans 8 consecutive entries, then a scan of thread totals
    __shared__ int tot[kWG];
    int loc[8];
    int s = 0;
    for (int k = 0; k < 8; ++k) {
        s += sh[threadIdx.x * 8 + k];
        loc[k] = s;
    }
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kWG; off <<= 1) {
        int t = threadIdx.x >= off ? tot[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += t;
        __syncthreads();
    }
    int pre = threadIdx.x ? tot[threadIdx.x - 1] : 0;
    for (int k = 0; k < 8; ++k) {
        long long i = base + threadIdx.x * 8 + k;
        if (i < len) a[i] = loc[k] + pre;
    }
    if (threadIdx.x == kWG - 1) bsum[blockIdx.x] = tot[kWG - 1];
}

// exclusive scan of nb chunk totals by one workgroup (sequential in chunks)
__global__ __launch_bounds__(kWG) void k_scan_sums(int *bsum, int nb) {
    __shared__ int tot[kWG];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += kWG) {
        int i = base + threadIdx.x;
        int v = i < nb ? bsum[i] : 0;
        tot[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kWG; off <<= 1) {
            int t = threadIdx.x >= off ? tot[threadIdx.x - off] : 0;
            __syncthreads();
            tot[threadIdx.x] += t;
            __syncthreads();
        }
        int excl = tot[threadIdx.x] - v + carry;
        if (i < nb) bsum[i] = excl;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot[kWG - 1];
        __syncthreads();
    }
}

__global__ void k_scan_add(int *a, long long len, const int *boff) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) a[i] += boff[i / kScanChunk];
}

// each entry p of A (row i, column j) takes the next free slot of column j
__global__ void k_scatter(const int *__restrict__ rp, const int *__restrict__ ci, int m, int nnz,
                          int *cursor, int *tci, int *perm) {
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    // row of entry p: last i with rp[i] <= p
    int lo = 0, hi = m - 1;
    while (lo < hi) {
        int mid = lo + ((hi - lo + 1) >> 1);
        if (rp[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    int q = atomicAdd(&cursor[ci[p]], 1);
    tci[q] = lo;
    perm[q] = (int)p;
}

// Order each row of A' by increasing entry index of A (= increasing row of
// A).  Short rows: insertion sort by one thread.  Long rows are listed.
constexpr int kShortRow = 32;
constexpr int kBitonic = 4096;
__global__ void k_sort_short(const int *__restrict__ trp, int n, int *tci, int *perm,
                             int *long_rows, int *nlong) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int a = trp[j], b = trp[j + 1];
    int len = b - a;
    if (len <= 1) return;
    if (len > kShortRow) {
        int slot = atomicAdd(nlong, 1);
        long_rows[slot] = j;
        return;
    }
    for (int i = a + 1; i < b; ++i) {
        int kp = perm[i], kt = tci[i];
        int q = i - 1;
        while (q >= a && perm[q] > kp) {
            perm[q + 1] = perm[q];
            tci[q + 1] = tci[q];
            --q;
        }
        perm[q + 1] = kp;
        tci[q + 1] = kt;
    }
}

__global__ __launch_bounds__(kWG) void k_sort_long(const int *__restrict__ trp,
                                                   const int *__restrict__ long_rows,
                                                   const int *__restrict__ nlong, int *tci,
                                                   int *perm) {
    __shared__ int key[kBitonic];
    __shared__ int val[kBitonic];
    const int cnt = *nlong;
    for (int w = blockIdx.x; w < cnt; w += gridDim.x) {
        const int j = long_rows[w];
        const int a = trp[j], len = trp[j + 1] - a;
        if (len <= kBitonic) {
            int P = 1;
            while (P < len) P <<= 1;
            for (int e = threadIdx.x; e < P; e += kWG) {
                key[e] = e < len ? perm[a + e] : 0x7fffffff;
                val[e] = e < len ? tci[a + e] : 0;
            }
            __syncthreads();
            for (int k = 2; k <= P; k <<= 1) {
                for (int jj = k >> 1; jj > 0; jj >>= 1) {
                    for (int i = threadIdx.x; i < P; i += kWG) {
                        int ixj = i ^ jj;
                        if (ixj > i) {
                            bool up = (i & k) == 0;
                            int ki = key[i], kj = key[ixj];
                            if ((ki > kj) == up) {
                                key[i] = kj;
                                key[ixj] = ki;
                                int t = val[i];
                                val[i] = val[ixj];
                                val[ixj] = t;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (int e = threadIdx.x; e < len; e += kWG) {
                perm[a + e] = key[e];
                tci[a + e] = val[e];
            }
            __syncthreads();
        }
    }
}

// Rows longer than the LDS stage (columns of A with more than 4096
// entries): one workgroup per row sorts it by merging.  First every chunk
// of 4096 entries is sorted in LDS (bitonic, as above); then runs of width
// w are merged pairwise, 2w, 4w, ..., ping-ponging between (perm, tci) and
// a scratch array of (key, value) pairs: an entry's place in the merged
// run is its index in its own run plus the number of smaller keys in the
// partner run (a binary search; keys are distinct entry indices of A).
// O(len log^2 len) per row.
__device__ __forceinline__ int count_below(const int *keys, int stride, int lo, int hi, int k) {
    // number of keys[lo..hi) (element q at keys[q * stride]) smaller than k
    int a = lo, b = hi;
    while (a < b) {
        const int mid = a + ((b - a) >> 1);
        if (keys[(long long)mid * stride] < k) a = mid + 1;
        else b = mid;
    }
    return a - lo;
}

__global__ __launch_bounds__(kWG) void k_sort_huge(const int *__restrict__ trp,
                                                   const int *__restrict__ long_rows,
                                                   const int *__restrict__ nlong, int *tci,
                                                   int *perm, int2 *scratch) {
    __shared__ int key[kBitonic];
    __shared__ int val[kBitonic];
    const int cnt = *nlong;
    for (int w = blockIdx.x; w < cnt; w += gridDim.x) {
        const int j = long_rows[w];
        const int a = trp[j], len = trp[j + 1] - a;
        if (len <= kBitonic) continue;
        // 1. sort each chunk of kBitonic entries in place
        for (int c0 = 0; c0 < len; c0 += kBitonic) {
            const int clen = len - c0 < kBitonic ? len - c0 : kBitonic;
            for (int e = threadIdx.x; e < kBitonic; e += kWG) {
                key[e] = e < clen ? perm[a + c0 + e] : 0x7fffffff;
                val[e] = e < clen ? tci[a + c0 + e] : 0;
            }
            __syncthreads();
            for (int k = 2; k <= kBitonic; k <<= 1) {
                for (int jj = k >> 1; jj > 0; jj >>= 1) {
                    for (int i = threadIdx.x; i < kBitonic; i += kWG) {
                        const int ixj = i ^ jj;
                        if (ixj > i) {
                            const bool up = (i & k) == 0;
                            const int ki = key[i], kj = key[ixj];
                            if ((ki > kj) == up) {
                                key[i] = kj;
                                key[ixj] = ki;
                                const int t = val[i];
                                val[i] = val[ixj];
                                val[ixj] = t;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (int e = threadIdx.x; e < clen; e += kWG) {
                perm[a + c0 + e] = key[e];
                tci[a + c0 + e] = val[e];
            }
            __syncthreads();
        }
        // 2. merge runs of width rw into runs of 2 rw
        bool in_scratch = false;  // where the current runs live
        for (int rw = kBitonic; rw < len; rw <<= 1) {
            const int *skey = in_scratch ? &scratch[a].x : perm + a;
            const int *sval = in_scratch ? &scratch[a].y : tci + a;
            const int stride = in_scratch ? 2 : 1;
            for (int e = threadIdx.x; e < len; e += kWG) {
                const int run = e / rw, i = e - run * rw;
                const int pair0 = (run & ~1) * rw;
                const int partner = run ^ 1;
                const int p0 = partner * rw;
                const int p1 = p0 + rw < len ? p0 + rw : len;
                const int k = skey[(long long)e * stride], v = sval[(long long)e * stride];
                const int below = p0 < len ? count_below(skey, stride, p0, p1, k) : 0;
                const int dst = pair0 + i + below;
                if (in_scratch) {
                    perm[a + dst] = k;
                    tci[a + dst] = v;
                } else {
                    scratch[a + dst] = make_int2(k, v);
                }
            }
            __syncthreads();
            in_scratch = !in_scratch;
        }
        if (in_scratch) {
            for (int e = threadIdx.x; e < len; e += kWG) {
                const int2 kv = scratch[a + e];
                perm[a + e] = kv.x;
                tci[a + e] = kv.y;
            }
        }
        __syncthreads();
    }
}

__global__ void k_gather_vals(const int *__restrict__ perm, const double *__restrict__ v, int nnz,
                              double *tv) {
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) tv[q] = v[perm[q]];
}

__global__ void k_fill_zero(double *a, long long len) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) a[i] = 0.0;
}

__global__ void k_copy_int(const int *__restrict__ a, int *b, long long len) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) b[i] = a[i];
}

void launch_transpose(const Dev &d, hipStream_t s) {
    const int n = d.n, nnz = d.nnz, m = d.m;
    hipLaunchKernelGGL(k_fill_int, dim3(div_up(n + 1, kWG)), dim3(kWG), 0, s, d.trp,
                       (long long)n + 1, 0);
    if (nnz > 0)
        hipLaunchKernelGGL(k_count_cols, dim3(div_up(nnz, kWG)), dim3(kWG), 0, s, d.ci, nnz,
                           d.trp);
    // inclusive scan of trp[0..n] (trp[0] = 0) gives the row starts of A'
    const long long len = (long long)n + 1;
    const int nchunk = div_up(len, kScanChunk);
    int *bsum = d.long_rows;  // n >= nchunk; reused before the sort needs it
    hipLaunchKernelGGL(k_scan_chunks, dim3(nchunk), dim3(kWG), 0, s, d.trp, len, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kWG), 0, s, bsum, nchunk);
    hipLaunchKernelGGL(k_scan_add, dim3(div_up(len, kWG)), dim3(kWG), 0, s, d.trp, len, bsum);
    if (nnz == 0) return;
    hipLaunchKernelGGL(k_copy_int, dim3(div_up(n, kWG)), dim3(kWG), 0, s, d.trp, d.cursor,
                       (long long)n);
    hipLaunchKernelGGL(k_scatter, dim3(div_up(nnz, kWG)), dim3(kWG), 0, s, d.rp, d.ci, m, nnz,
                       d.cursor, d.tci, d.perm);
    int *nlong = d.err + 1;
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, s, nlong, 1LL, 0);
    hipLaunchKernelGGL(k_sort_short, dim3(div_up(n, kWG)), dim3(kWG), 0, s, d.trp, n, d.tci,
                       d.perm, d.long_rows, nlong);
    hipLaunchKernelGGL(k_sort_long, dim3(1024), dim3(kWG), 0, s, d.trp, d.long_rows, nlong,
                       d.tci, d.perm);
    int2 *scratch = reinterpret_cast<int2 *>(d.tv);  // tv is filled afterwards
    hipLaunchKernelGGL(k_sort_huge, dim3(1024), dim3(kWG), 0, s, d.trp, d.long_rows, nlong,
                       d.tci, d.perm, scratch);
    hipLaunchKernelGGL(k_gather_vals, dim3(div_up(nnz, kWG)), dim3(kWG), 0, s, d.perm, d.v, nnz,
                       d.tv);
}

void launch_slab_count(const Slabs &sb, const int *rp, const int *ci, int *scratch,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_slab_count, dim3(div_up(sb.rows, kWG)), dim3(kWG), 0, s, sb, rp, ci);
    // inclusive scan of each slab's rows + 1 counts gives its row starts
    const long long len = (long long)sb.rows + 1;
    const int nchunk = div_up(len, kScanChunk);
    for (int q = 0; q < sb.S; ++q) {
        int *a = sb.srp + (size_t)q * (sb.rows + 1);
        hipLaunchKernelGGL(k_scan_chunks, dim3(nchunk), dim3(kWG), 0, s, a, len, scratch);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kWG), 0, s, scratch, nchunk);
        hipLaunchKernelGGL(k_scan_add, dim3(div_up(len, kWG)), dim3(kWG), 0, s, a, len, scratch);
    }
}

void launch_slab_fill(const Slabs &sb, const int *rp, const int *ci, const double *v,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_slab_scatter, dim3(div_up(sb.rows, kWG)), dim3(kWG), 0, s, sb, rp, ci, v);
}

// --- column order (set-up and the API's conversions) ----------------------
// first[j] = the smallest row holding an entry of column j (m for an empty
// column); one thread per entry finds its row by bisection of the row starts
__global__ void k_first_rows(const int *__restrict__ rp, const int *__restrict__ ci, int m,
                             int nnz, int *first) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int lo = 0, hi = m - 1;  // last row r with rp[r] <= e
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    atomicMin(&first[ci[e]], lo);
}

// last[j] = the largest row holding an entry of column j (-1 for an empty
// column), as k_first_rows
__global__ void k_last_rows(const int *__restrict__ rp, const int *__restrict__ ci, int m,
                            int nnz, int *last) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int lo = 0, hi = m - 1;  // last row r with rp[r] <= e
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    atomicMax(&last[ci[e]], lo);
}

void launch_last_rows(const int *rp, const int *ci, int m, int n, int nnz, int *last,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3(div_up(n, kWG)), dim3(kWG), 0, s, last, (long long)n, -1);
    if (nnz > 0 && m > 0)
        hipLaunchKernelGGL(k_last_rows, dim3(div_up(nnz, kWG)), dim3(kWG), 0, s, rp, ci, m, nnz,
                           last);
}

void launch_first_rows(const int *rp, const int *ci, int m, int n, int nnz, int *first,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3(div_up(n, kWG)), dim3(kWG), 0, s, first, (long long)n, m);
    if (nnz > 0 && m > 0)
        hipLaunchKernelGGL(k_first_rows, dim3(div_up(nnz, kWG)), dim3(kWG), 0, s, rp, ci, m, nnz,
                           first);
}

void launch_col_counts(const int *ci, int nnz, int n, int *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3(div_up(n + 1, kWG)), dim3(kWG), 0, s, cnt,
                       (long long)n + 1, 0);
    if (nnz > 0)
        hipLaunchKernelGGL(k_count_cols, dim3(div_up(nnz, kWG)), dim3(kWG), 0, s, ci, nnz, cnt);
}

__global__ void k_permute_cols(const int *__restrict__ ci, int nnz, const int *__restrict__ cinv,
                               int *ci2, const double *__restrict__ c,
                               const double *__restrict__ l, const double *__restrict__ u,
                               const int *__restrict__ cperm, int n, double *c2, double *l2,
                               double *u2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nnz) ci2[i] = cinv[ci[i]];
    if (i < n) {
        const int j = cperm[i];
        c2[i] = c[j];
        l2[i] = l[j];
        u2[i] = u[j];
    }
}

void launch_permute_cols(const int *ci, int nnz, const int *cinv, int *ci2, const double *c,
                         const double *l, const double *u, const int *cperm, int n, double *c2,
                         double *l2, double *u2, hipStream_t s) {
    const long long mx = nnz > n ? nnz : n;
    hipLaunchKernelGGL(k_permute_cols, dim3(div_up(mx, kWG)), dim3(kWG), 0, s, ci, nnz, cinv, ci2,
                       c, l, u, cperm, n, c2, l2, u2);
}

__global__ void k_gather(const double *__restrict__ in, const int *__restrict__ idx, long long n,
                         double *out) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = in[idx[q]];
}

void launch_gather(const double *in, const int *idx, long long n, double *out, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_gather, dim3(div_up(n, kWG)), dim3(kWG), 0, s, in, idx, n, out);
}

// row lengths of A' in the caller's column order: orp[j + 1] (orp[0] = 0)
__global__ void k_tout_counts(const int *__restrict__ trp, const int *__restrict__ cinv, int n,
                              int *orp) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) orp[0] = 0;
    if (j < n) {
        const int q = cinv[j];
        orp[j + 1] = trp[q + 1] - trp[q];
    }
}

__global__ void k_tout_copy(const int *__restrict__ trp, const int *__restrict__ tci,
                            const double *__restrict__ tv, const int *__restrict__ tperm,
                            const int *__restrict__ cinv, int n, const int *__restrict__ orp,
                            int *oci, double *ov, int *operm) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int q = cinv[j];
    const int src = trp[q], len = trp[q + 1] - trp[q], dst = orp[j];
    for (int k = 0; k < len; ++k) {
        if (oci) oci[dst + k] = tci[src + k];
        if (ov) ov[dst + k] = tv[src + k];
        if (operm) operm[dst + k] = tperm[src + k];
    }
}

void launch_transpose_out(const Dev &d, int *orp, int *oci, double *ov, int *operm,
                          hipStream_t s) {
    const int n = d.n;
    hipLaunchKernelGGL(k_tout_counts, dim3(div_up(n, kWG)), dim3(kWG), 0, s, d.trp, d.cinv, n, orp);
    const long long len = (long long)n + 1;
    const int nchunk = div_up(len, kScanChunk);
    int *bsum = d.long_rows;  // n >= nchunk
    hipLaunchKernelGGL(k_scan_chunks, dim3(nchunk), dim3(kWG), 0, s, orp, len, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kWG), 0, s, bsum, nchunk);
    hipLaunchKernelGGL(k_scan_add, dim3(div_up(len, kWG)), dim3(kWG), 0, s, orp, len, bsum);
    if (d.nnz > 0)
        hipLaunchKernelGGL(k_tout_copy, dim3(div_up(n, kWG)), dim3(kWG), 0, s, d.trp, d.tci, d.tv,
                           d.perm, d.cinv, n, orp, oci, ov, operm);
}

// x = proj_X(0), x0 = x, y = y0 = 0, sums 0, counters 0
__global__ void k_init_point(Dev d) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.n) {
        double v = 0.0;
        if (v < d.l[i]) v = d.l[i];
        if (v > d.u[i]) v = d.u[i];
        d.x[i] = v;
        d.x0[i] = v;
        d.sx[i] = 0.0;
    }
    if (i < d.m) {
        d.y[i] = 0.0;
        d.y0[i] = 0.0;
        d.sy[i] = 0.0;
    }
    if (i == 0) {
        DevState *st = d.st;
        st->k = 0;
        st->t = 0;
        st->restarts = 0;
        st->checks = 0;
        st->rho_prev = 0.0;
        st->done = 0;
        st->conv_which = -1;
        st->conv_k = -1;
        st->restarted = 0;
        st->cand = 0;
        st->gap_slots = 0;
        st->numerr = 0;
        st->in_check = 0;
        for (int sidx = 0; sidx < kTrSlots; ++sidx) st->tr[sidx].mode = TR_IDLE;
    }
}

void launch_init_point(const Dev &d, hipStream_t s) {
    long long mx = d.n > d.m ? d.n : d.m;
    hipLaunchKernelGGL(k_init_point, dim3(div_up(mx, kWG)), dim3(kWG), 0, s, d);
    if (d.m > 0) launch_spmv_A(d, d.x, d.q, s);
}

// |b|^2 and |c|^2 (deterministic), stored in the state
__global__ __launch_bounds__(kWG) void k_norm_partials(Dev d) {
    __shared__ double sh[4 * 2];
    double v[2] = {0.0, 0.0};
    const long long stride = (long long)gridDim.x * kWG;
    for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < (long long)d.n + d.m;
         i += stride) {
        if (i < d.n) v[1] += d.c[i] * d.c[i];
        else {
            double bb = d.b[i - d.n];
            v[0] += bb * bb;
        }
    }
    block_sums<2>(v, sh);
    if (threadIdx.x == 0) {
        d.part[blockIdx.x * kKktSums + 0] = v[0];
        d.part[blockIdx.x * kKktSums + 1] = v[1];
    }
}

__global__ __launch_bounds__(kWG) void k_norm_final(Dev d, int nb) {
    __shared__ double sh[4 * 2];
    double out[2];
    reduce_partials<2>(d.part, nb, kKktSums, out, sh);
    if (threadIdx.x == 0) {
        d.st->nb2 = out[0];
        d.st->nc2 = out[1];
    }
}

int red_grid(long long N) {
    int g = div_up(N, kWG);
    if (g > kRedBlocks) g = kRedBlocks;
    if (g < 1) g = 1;
    return g;
}

void launch_norms(const Dev &d, hipStream_t s) {
    int g = red_grid((long long)d.n + d.m);
    hipLaunchKernelGGL(k_norm_partials, dim3(g), dim3(kWG), 0, s, d);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kWG), 0, s, d, g);
}

// ---------------------------------------------------------------------
// check: averages, KKT, radii
// ---------------------------------------------------------------------
__global__ void k_reset_done(DevState *st) {
    st->done = 0;
    st->in_check = 0;
}

__global__ void k_average(Dev d) {
    if (d.st->done) return;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    average_at(d, i, d.st->t);
}

void launch_average(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_average, dim3(div_up((long long)d.n + d.m, kWG)), dim3(kWG), 0, s, d);
}

__global__ __launch_bounds__(kWG) void k_kkt_partials(Dev d, KktPoints P2, int gated) {
    if (gated && d.st->done) return;
    __shared__ double sh[4 * kKktSums];
    double v[kKktSums];
#pragma unroll
    for (int k = 0; k < kKktSums; ++k) v[k] = 0.0;
    const long long N = (long long)d.n + d.m;
    const long long stride = (long long)gridDim.x * kWG;
    for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < N; i += stride)
        kkt_elem(d, P2, i, v);
    block_sums<kKktSums>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kKktSums; ++k) d.part[(size_t)blockIdx.x * kKktSums + k] = v[k];
    }
}

void launch_kkt_partials(const Dev &d, hipStream_t s) {
    int g = red_grid((long long)d.n + d.m);
    KktPoints P2{{d.x, d.xbar}, {d.y, d.ybar}, {d.q, d.axb}, {d.aty, d.atyb}};
    hipLaunchKernelGGL(k_kkt_partials, dim3(g), dim3(kWG), 0, s, d, P2, 1);
}

// KKT of one held point into st->kkt_eval, leaving the solver state alone
__global__ __launch_bounds__(kWG) void k_kkt_eval(Dev d, int nb) {
    __shared__ double sh[4 * kKktSums];
    double S[kKktSums];
    reduce_partials<kKktSums>(d.part, nb, kKktSums, S, sh);
    if (threadIdx.x == 0) kkt_point(d, S, 0, d.st->kkt_eval);
}

void launch_kkt_eval(const Dev &d, int which, hipStream_t s) {
    launch_copy_point(d, which, d.gx, d.gy, s);
    launch_spmv_A(d, d.gx, d.gax, s);
    launch_spmv_T(d, d.gy, d.gaty, s);
    int g = red_grid((long long)d.n + d.m);
    KktPoints P2{{d.gx, d.gx}, {d.gy, d.gy}, {d.gax, d.gax}, {d.gaty, d.gaty}};
    hipLaunchKernelGGL(k_kkt_partials, dim3(g), dim3(kWG), 0, s, d, P2, 0);
    hipLaunchKernelGGL(k_kkt_eval, dim3(1), dim3(kWG), 0, s, d, g);
}


// Stopping test and the radii; arms the trust-region slots.
__global__ __launch_bounds__(kWG) void k_kkt_final(Dev d, int nb, double tol, int kkt_kind,
                                                   double omega, int gap_slots) {
    DevState *st = d.st;
    if (st->done) return;
    __shared__ double sh[4 * kKktSums];
    __shared__ int armed;
    double S[kKktSums];
    reduce_partials<kKktSums>(d.part, nb, kKktSums, S, sh);
    if (threadIdx.x < 64) {
        const int sl = kkt_conclude(d, S, tol, kkt_kind, omega, gap_slots);
        if (threadIdx.x == 0) armed = sl;
    }
    __syncthreads();
    // clear level-0 histograms of the armed slots
    for (int sidx = 0; sidx < kTrSlots; ++sidx) {
        if (!(armed & (1 << sidx))) continue;
        const TRWork &w = d.tr[sidx];
        for (int b = threadIdx.x; b < kBuckets; b += kWG) {
            w.hcnt[b] = 0u;
            w.hD[b] = 0.0;
            w.hA[b] = 0.0;
        }
    }
}

void launch_kkt_final(const Dev &d, double tol, int kkt_kind, int gap_slots, hipStream_t s) {
    int g = red_grid((long long)d.n + d.m);
    hipLaunchKernelGGL(k_kkt_final, dim3(1), dim3(kWG), 0, s, d, g, tol, kkt_kind, d.omega,
                       gap_slots);
}

void launch_reset_done(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_done, dim3(1), dim3(1), 0, s, d.st);
}

// ---------------------------------------------------------------------
// power iteration on A'A for sigma_max(A) (Section 7 step size):
// v = 1/sqrt(n); repeat w = A v, u = A'w, s = |u|, v = u/s, est = sqrt(s)
// until |est - prev| <= tol est or max_iters products.
// ---------------------------------------------------------------------
__global__ void k_power_init(Dev d) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < d.n) d.atyb[j] = 1.0 / sqrt((double)d.n);
    if (j == 0) {
        d.st->pw_done = 0;
        d.st->pw_it = 0;
        d.st->pw_est = 0.0;
        d.st->pw_prev = 0.0;
        d.st->pw_s = 0.0;
    }
}

void launch_power_init(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_power_init, dim3(div_up(d.n, kWG)), dim3(kWG), 0, s, d);
}

__global__ __launch_bounds__(kWG) void k_sq_partials(const double *v, long long N, double *part,
                                                     const int *gate) {
    if (gate && *gate) return;
    __shared__ double sh[4];
    double a[1] = {0.0};
    for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < N;
         i += (long long)gridDim.x * kWG)
        a[0] += v[i] * v[i];
    block_sums<1>(a, sh);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * kKktSums] = a[0];
}

__global__ __launch_bounds__(kWG) void k_power_final(Dev d, int nb, double tol, int max_iters) {
    DevState *st = d.st;
    if (st->pw_done) return;
    __shared__ double sh[4];
    double tot[1];
    reduce_partials<1>(d.part, nb, kKktSums, tot, sh);
    if (threadIdx.x == 0) {
        const double sn = sqrt(tot[0]);
        if (!(sn > 0.0)) {
            st->pw_est = 0.0;
            st->pw_s = 0.0;
            st->pw_done = 1;
        } else {
            st->pw_s = sn;
            const double est = sqrt(sn);
            st->pw_est = est;
            if (st->pw_it > 0 && fabs(est - st->pw_prev) <= tol * est) st->pw_done = 1;
            st->pw_prev = est;
            st->pw_it += 1;
            if (st->pw_it >= max_iters) st->pw_done = 1;
        }
    }
}

__global__ void k_power_norm(Dev d) {
    const double sn = d.st->pw_s;
    if (!(sn > 0.0)) return;
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < d.n) d.atyb[j] = d.aty[j] / sn;
}

// one power-iteration product pair; every kernel skips once converged
void launch_power_step(const Dev &d, double tol, int max_iters, hipStream_t s) {
    const int *gate = &d.st->pw_done;
    spmv_A_gated(d, d.atyb, d.axb, gate, s);
    spmv_T_gated(d, d.axb, d.aty, gate, s);
    const int g = red_grid(d.n);
    hipLaunchKernelGGL(k_sq_partials, dim3(g), dim3(kWG), 0, s, d.aty, (long long)d.n, d.part,
                       gate);
    hipLaunchKernelGGL(k_power_final, dim3(1), dim3(kWG), 0, s, d, g, tol, max_iters);
    hipLaunchKernelGGL(k_power_norm, dim3(div_up(d.n, kWG)), dim3(kWG), 0, s, d);
}

// ---------------------------------------------------------------------
// measurement yardsticks: a plain streaming copy (the HBM ceiling the
// half-steps are set against) and a plain gather out[i] = val[i] x[idx[i]]
// (the access pattern of a product's gathers without its rows)
// ---------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_copy_yard(const double4 *__restrict__ src,
                                                   double4 *__restrict__ dst, long long n4,
                                                   const double *__restrict__ s1,
                                                   double *__restrict__ d1, long long n) {
    const long long stride = (long long)gridDim.x * kWG;
    for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < n4; i += stride)
        dst[i] = src[i];
    // the last n mod 4 elements
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)(n - 4 * n4))
        d1[4 * n4 + threadIdx.x] = s1[4 * n4 + threadIdx.x];
}

// 32 bytes per lane and 16,384 workgroups: the fastest plain copy found on
// MI355X (sweeps of 8-32 bytes per lane and 1,024-16,384 workgroups)
void launch_copy_yard(const double *src, double *dst, long long n, hipStream_t s) {
    const long long n4 = n / 4;
    long long g = (n4 + kWG - 1) / kWG;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_copy_yard, dim3((unsigned)g), dim3(kWG), 0, s, (const double4 *)src,
                       (double4 *)dst, n4, src, dst, n);
}

constexpr int kYardPer = 8;  // gathers in flight per thread, as in the SpMV stage
__global__ __launch_bounds__(kWG) void k_gather_yard(const int *__restrict__ idx,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ out, long long n) {
    const long long base = (long long)blockIdx.x * kWG * kYardPer + threadIdx.x;
    int c[kYardPer];
    double v[kYardPer], g[kYardPer];
#pragma unroll
    for (int k = 0; k < kYardPer; ++k) {
        const long long e = base + (long long)k * kWG;
        if (e < n) {
            c[k] = ld_matrix(idx + e);
            v[k] = ld_matrix(val + e);
        }
    }
#pragma unroll
    for (int k = 0; k < kYardPer; ++k)
        if (base + (long long)k * kWG < n) g[k] = x[c[k]];
#pragma unroll
    for (int k = 0; k < kYardPer; ++k) {
        const long long e = base + (long long)k * kWG;
        if (e < n) out[e] = v[k] * g[k];
    }
}

// gathers alone: thread t adds x at the indices of entries t, t + kWG, ...
// (4 per thread, from an index stream, or, with idx null, from Fibonacci
// hashing of the entry number into a window of 2^lg doubles) and stores one
// sum; no values, no rows, no update
constexpr int kGatherOnly = 4;
__global__ __launch_bounds__(kWG) void k_gather_only(const int *__restrict__ idx,
                                                     const double *__restrict__ x, long long n,
                                                     int lg, double *__restrict__ out) {
    const long long base = (long long)blockIdx.x * kWG * kGatherOnly + threadIdx.x;
    int c[kGatherOnly];
#pragma unroll
    for (int k = 0; k < kGatherOnly; ++k) {
        const long long e = min(base + (long long)k * kWG, n - 1);
        c[k] = idx ? ld_matrix(idx + e)
                   : (int)(((unsigned long long)e * 0x9E3779B97F4A7C15ull) >> (64 - lg));
    }
    double g[kGatherOnly];
#pragma unroll
    for (int k = 0; k < kGatherOnly; ++k) g[k] = x[c[k]];
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < kGatherOnly; ++k)
        if (base + (long long)k * kWG < n) sum += g[k];
    out[(long long)blockIdx.x * kWG + threadIdx.x] = sum;
}

long long gather_only_outputs(long long n) {
    const long long per = (long long)kWG * kGatherOnly;
    return (n + per - 1) / per * kWG;
}

void launch_gather_only(const int *idx, const double *x, long long n, int lg, double *out,
                        hipStream_t s) {
    const long long per = (long long)kWG * kGatherOnly;
    const long long g = (n + per - 1) / per;
    if (g > 0) hipLaunchKernelGGL(k_gather_only, dim3((unsigned)g), dim3(kWG), 0, s, idx, x, n, lg, out);
}

void launch_gather_yard(const int *idx, const double *val, const double *x, double *out,
                        long long n, hipStream_t s) {
    const long long per = (long long)kWG * kYardPer;
    const long long g = (n + per - 1) / per;
    if (g < 1) return;
    hipLaunchKernelGGL(k_gather_yard, dim3((unsigned)g), dim3(kWG), 0, s, idx, val, x, out, n);
}

}  // namespace pdhg
