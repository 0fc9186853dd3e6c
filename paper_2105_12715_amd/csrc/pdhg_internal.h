// Internal declarations shared by the kernels and the C ABI of the
// restarted-PDHG library.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pdhg {

constexpr int kWG = 256;             // threads per workgroup (4 wave64)
// SpMV block size in rows + nnz (a build parameter for tuning sweeps)
#ifndef PDHG_SPMV_UNITS
#define PDHG_SPMV_UNITS 1024
#endif
constexpr int kUnits = PDHG_SPMV_UNITS;
constexpr int kLdsProducts = 2 * kUnits;  // products staged in LDS per SpMV block
static_assert(kLdsProducts <= 65535, "row starts are staged as 16-bit offsets");
// Blocks stored sorted by column (Dev::apk): one 32-bit word per entry,
// column << kPkSlotBits | slot, with the slot the entry's place in its block
// (so a block holds at most 2^kPkSlotBits staged entries)
constexpr int kPkSlotBits = 11;
constexpr unsigned kPkSlotMask = (1u << kPkSlotBits) - 1u;
constexpr int64_t kPkMaxCols = 1ll << (32 - kPkSlotBits);
inline bool sorted_blocks_fit(int64_t cols) {
    return kLdsProducts <= (1 << kPkSlotBits) && cols <= kPkMaxCols;
}
constexpr int kRedBlocks = 1024;     // max blocks of a partial-sum reduction
constexpr int kKktSums = 14;         // partial sums of the KKT / radius pass
constexpr int kBuckets = 2048;       // radix buckets of the multiplier search
constexpr int kTrSlots = 2;          // trust-region evaluations per check
constexpr int kLogCap = 4096;        // check records kept on the device
constexpr int kRec = 14;             // doubles per check record
constexpr int kBoundClasses = 4;     // distinct (l, u) pairs held as a class byte

// KKT partial-sum slots
enum {
    S_PRES2_C = 0, S_PRES2_A, S_DRES2_C, S_DRES2_A, S_POBJ_C, S_POBJ_A,
    S_DOBJ_C, S_DOBJ_A, S_BV2_C, S_BV2_A, S_RX2_A, S_RY2_A, S_RX2_C, S_RY2_C
};

// trust-region evaluation modes
enum { TR_IDLE = 0, TR_SEARCH = 1, TR_RESOLVED = 2, TR_FULLBOX = 3, TR_ZERO = 4 };

struct TRState {
    double r, r2;          // radius and its square
    double F_acc, A_acc;   // sums of d^2 below / a^2 above the bracket
    double rho, lam;       // results
    double value;          // r * rho
    unsigned long long prefix;  // key bits fixed so far
    unsigned long long klo;     // key of the bracket's lower end
    int mode;              // TR_*
    int level;             // radix level reached
    unsigned int count;    // elements inside the bracket
    unsigned int ncomp;    // compacted elements (after the level-1 pass)
    int nan_seen;
    int cap;               // compaction region length per block
};

struct DevState {
    long long k, t, restarts, checks;
    double rho_prev;
    int done;              // a solve converged: later graph kernels do nothing
    int conv_which;        // -1 none, 0 current, 1 average
    long long conv_k;
    double kkt_cur[8];     // picked, rel, pres, dres, pobj, dobj, paper_abs, max_abs
    double kkt_avg[8];
    double kkt_eval[8];    // stand-alone KKT evaluation
    double r_avg, r_cur;
    int restarted, cand;   // outcome of the last check
    int gap_slots;         // bitmask of trust-region slots to evaluate
    int numerr;            // NaN/Inf seen in a check
    int in_check;          // a check is in progress (set by the KKT pass)
    int pad1;
    double nb2, nc2;       // |b|^2 and |c|^2
    // power iteration
    double pw_est, pw_prev, pw_s;
    int pw_done, pw_it;
    TRState tr[kTrSlots];
};

// Trust-region scratch carved from a workspace.
struct TRWork {
    unsigned int *hcnt;    // [2][kBuckets]
    double *hD, *hA;       // [2][kBuckets]
    double *part;          // [kRedBlocks][4]
    unsigned int *ccount;  // [kRedBlocks] compacted elements per block
    unsigned int *coff;    // [kRedBlocks + 1] their exclusive prefix
    unsigned long long *ckey;  // [N + kRedBlocks * kWG] compacted keys, one region per block
    double *ca, *cd;       // same length
    unsigned int *fcount;  // members of the bracket gathered for the last levels
    unsigned long long *fkey;  // [kFinishMax] their keys
    double *fa, *fd;       // [kFinishMax]
};
// bracket size from which the last levels run in one workgroup
constexpr unsigned int kFinishMax = 65536;

// A sparse matrix (CSR, rows x cols) split into S column slabs of width W:
// slab s holds the entries with column in [s W, (s+1) W), in CSR of its own
// with local column indices, and its own merge-path block table.
//
// Each slab's launch runs over a range of rows [lo[s], hi[s]) holding every
// row with an entry in that slab.  The ranges are widened so that those of
// slabs 0..s always cover [0, before[s + 1]) and those of slabs s..S-1
// cover [after[s - 1], rows) with no gap: a row of launch s is then the
// row's first launch iff it is at or past before[s] (the end of the
// earlier ranges), and its last iff it lies below after[s] (the start of
// the later ones).  The first launch writes the row's partial sum to the
// accumulator (or, when it is also the last, applies the update to it
// directly), later launches add to it, and the last applies the update.
constexpr int kSlabMax = 8;
struct Slabs {
    int S, W, nbmax, rows;
    int *srp;                  // [S][rows + 1] row starts within each slab
    int *sci;                  // [nnz] local column index
    double *sv;                // [nnz]
    int *sbr;                  // block tables of every slab over its row range (k_rowsplit)
    long long *smeta;          // [S][4]: row-start offset, entry offset, block offset, blocks
    double *spart;             // [rows] running sum of the slabs done so far
    int lo[kSlabMax], hi[kSlabMax];  // row range of each slab's launch
    int before[kSlabMax];      // end of the ranges of slabs < s (0 for s = 0)
    int after[kSlabMax];       // start of the ranges of slabs > s (rows for s = S - 1)
};

// Device-side view of one LP and its solver state.
struct Dev {
    int m, n, nnz;
    const int *rp, *ci;
    const double *v;
    const double *c, *b, *l, *u;
    const signed char *kind;   // may be null
    // transpose
    int *trp, *tci, *perm;
    double *tv;
    int *cursor;               // n, setup scratch
    int *long_rows;            // n, setup scratch
    // merge-path block row starts
    int *brA, *brT;            // block tables: 2 (nblk + 1) ints (k_rowsplit)
    int nblkA, nblkT;
    // vectors
    double *x, *y, *x0, *y0, *sx, *sy, *q;
    double *xbar, *ybar, *axb, *atyb, *aty;
    double *gx, *gy, *gax, *gaty;   // scratch point of the stand-alone gap
    double *xt, *yt;           // extragradient target point z~
    double *part;              // [kRedBlocks][kKktSums]
    double *log;               // [kLogCap][kRec]
    DevState *st;
    TRWork tr[kTrSlots];
    int *err;                  // validation flags; err[1] counts long A' rows
    double omega;              // primal weight (norm of the gap and radii)
    Slabs slA;                 // A by column slabs (gathers x), for A x
    Slabs slT;                 // A' by column slabs (gathers y), for A' y
    int lbA, lbT;              // lanes-per-row bias of the A x and A'y blocks (-1, 0, +1)
    // Column order.  Columns are kept sorted by entry count (largest first,
    // ties by the row of their first entry), so the most gathered entries
    // of x share cache lines, neighbouring rows of A gather neighbouring
    // columns, and blocks of A' hold rows of similar length.  ci, c, l, u
    // above are then the reordered copies; iterates cross the API in the
    // caller's order.
    int permuted;              // 0: the caller's order is already sorted
    const int *cperm;          // [n] internal column q -> caller's column
    const int *cinv;           // [n] caller's column j -> internal column
    // Bound classes: when the columns' (l, u) pairs take at most
    // kBoundClasses distinct values, bcls[j] names column j's pair in
    // blo/bhi and the primal update reads that byte instead of l and u
    // (which stay for the checks).  Null otherwise.
    const unsigned char *bcls;
    double blo[kBoundClasses], bhi[kBoundClasses];
    int nbcls;                 // distinct pairs in use (0 with bcls null)
    // A with each merge-path block's entries sorted by column (k_sort_blocks):
    // the lanes of a wave that gather the same cache line of x are then
    // neighbours and share one request.  Null when A runs over column slabs
    // or has too many columns for the packed word.
    const unsigned *apk;       // [nnz] column << kPkSlotBits | slot
    const double *asv;         // [nnz] values in the same order
    int swgA, swgT;            // threads per workgroup of A x and A'y: 128 or kWG
};

// Column slabs: each slab's slice of the gathered vector is meant to fit
// one XCD's 4 MB L2; the slabs run one launch after the other.
// S = 1 (plain merge-path SpMV) when the gathered vector fits one L2 or the
// set-up scan of the slab row starts would not fit its n-int scratch.
inline int slab_count_for(int64_t rows, int64_t gathered, int64_t scratch_ints,
                          int64_t slice_bytes = 4ll << 20) {
    const int64_t bytes = gathered * 8;
    if (rows < 1 || (rows + 1 + 2047) / 2048 > scratch_ints) return 1;
    int S = 1;
    while (S < 8 && (int64_t)S * slice_bytes < bytes) S <<= 1;
    return S;
}

// Threads per workgroup of a product's launches: 128 when the launch has
// many blocks (more than fill the chip at kWG threads) of few rows each
// (one pass of the epilogue over the block's rows), so each thread keeps
// twice the entries in flight; kWG otherwise (a short grid keeps all its
// threads, and blocks of many rows keep the epilogue to a pass or two).
inline int spmv_threads_for(int64_t rows, int64_t nblk) {
    return (nblk >= 2048 && rows <= 128 * nblk) ? 128 : kWG;
}

// Slab counts the workspace reserves room for when a product uses slabs at
// all (the tuner may try any power of two up to it)
inline int slab_reserve_for(int64_t rows, int64_t gathered, int64_t scratch_ints,
                            int64_t slice_bytes) {
    return slab_count_for(rows, gathered, scratch_ints, slice_bytes) > 1 ? kSlabMax : 1;
}

// Primal-weight search: W <= kWMax copies of non-restarted PDHG sharing A
constexpr int kWMax = 16;
constexpr int kWSums = 5;      // |p|^2, |d|^2, pobj, dobj, bound violation^2
struct WArgs {
    int m, n, W;
    int egm;                   // 1: extragradient copies, 0: PDHG
    const int *rp, *ci, *trp, *tci;
    const double *v, *tv, *c, *b, *l, *u;
    const signed char *kind;
    const DevState *st;        // |b|^2 and |c|^2 of the LP
    const int *cinv;           // caller's column -> internal column, or null
    double *x, *aty;           // [n][W]
    double *y, *q;             // [m][W]; q = A x of the latest x
    double *xt, *yt;           // [n][W], [m][W]: extragradient targets
    double *part;              // [W][kRedBlocks][kWSums]
    double *out;               // [W][8] KKT parts
    double tau[kWMax], sigma[kWMax];
};
size_t wsearch_bytes(int64_t m, int64_t n, int W);
void wsearch_carve(char *ws, int64_t m, int64_t n, int W, WArgs *a);
void launch_w_init(const WArgs &a, hipStream_t s);
void launch_w_iter(const WArgs &a, hipStream_t s);
void launch_w_kkt(const WArgs &a, hipStream_t s);
void launch_w_extract(const WArgs &a, double *xo, double *yo, hipStream_t s);

// Workspace layout: offsets (bytes) of every region for given sizes.
struct Layout {
    size_t total;
    size_t o_state, o_err, o_trp, o_tci, o_perm, o_tv, o_cursor, o_long;
    size_t o_brA, o_brT, o_vec_n[8], o_vec_m[8], o_part, o_log;
    size_t o_slab[2][6];       // srp, sci, sv, sbr, smeta, spart of slA, slT
    size_t o_xt, o_yt;
    size_t o_ci2, o_cperm, o_cinv, o_c2, o_l2, o_u2, o_bcls;
    size_t o_apk, o_asv;       // A's blocks sorted by column (empty when they cannot be packed)
    size_t o_tr[kTrSlots];
};
bool make_layout(int64_t m, int64_t n, int64_t nnz, Layout *L);
size_t tr_work_bytes(int64_t N);
void carve_tr(char *base, int64_t N, TRWork *w);

// ---------------------------------------------------------------------
// Launchers (all enqueue on `s`, never synchronize).
// ---------------------------------------------------------------------
int nblocks_for(int rows, int nnz);

// setup
void launch_validate(const Dev &d, hipStream_t s);
void launch_transpose(const Dev &d, hipStream_t s);
void launch_rowsplit(const int *rp, int rows, int nnz, int nblk, int *br, hipStream_t s);
// the merge-path blocks of the CSR (rp, ci, v) with table br (k_rowsplit),
// each block's entries sorted by column into pk (column << kPkSlotBits |
// place in the block) and sv; blocks too long for the LDS stage keep their
// order
void launch_sort_blocks(const int *rp, const int *ci, const double *v, const int *br, int nblk,
                        unsigned *pk, double *sv, hipStream_t s);
void launch_init_point(const Dev &d, hipStream_t s);
// column slabs (when sb.S > 1) of the CSR (rp, ci, v): row starts of every
// slab (scan scratch: div_up(rows + 1, 2048) ints), then the entries
void launch_slab_count(const Slabs &sb, const int *rp, const int *ci, int *scratch,
                       hipStream_t s);
void launch_slab_fill(const Slabs &sb, const int *rp, const int *ci, const double *v,
                      hipStream_t s);
void launch_norms(const Dev &d, hipStream_t s);   // |b|^2, |c|^2 into part[0..1]
// column counts of the caller's A into cnt[1..n] (cnt[0] = 0)
void launch_col_counts(const int *ci, int nnz, int n, int *cnt, hipStream_t s);
// first[j] = smallest row with an entry in column j (m if none), j < n
void launch_first_rows(const int *rp, const int *ci, int m, int n, int nnz, int *first,
                       hipStream_t s);
// last[j] = largest row with an entry in column j (-1 if none), j < n
void launch_last_rows(const int *rp, const int *ci, int m, int n, int nnz, int *last,
                      hipStream_t s);
// range[2q], range[2q + 1] = smallest row and largest row + 1 with an entry
// in slab q (rows, -1 for an empty slab), from the slab row starts
void launch_slab_ranges(const Slabs &sb, int *range, hipStream_t s);
// merge-path block table of the rows [0, rows) of a CSR whose row starts rp
// need not begin at 0 (a row range of a larger matrix)
void launch_rowsplit_range(const int *rp, int rows, int nblk, int *br, hipStream_t s);
// ci2 = cinv[ci]; c2, l2, u2 = c, l, u in the internal column order
void launch_permute_cols(const int *ci, int nnz, const int *cinv, int *ci2, const double *c,
                         const double *l, const double *u, const int *cperm, int n, double *c2,
                         double *l2, double *u2, hipStream_t s);
// out[q] = in[idx[q]], q < n
void launch_gather(const double *in, const int *idx, long long n, double *out, hipStream_t s);
// A' in the caller's column order from the internal one (row j <- row cinv[j])
void launch_transpose_out(const Dev &d, int *orp, int *oci, double *ov, int *operm,
                          hipStream_t s);

// iteration
// Half-steps of eq. PDHG-update with the running sums of Algorithm 1.
// smode (sum_mode below): 0 adds the new iterate to S, 1 leaves S for the
// next iteration, 2 adds the previous iterate and then the new one.
void launch_primal(const Dev &d, double tau, int smode, hipStream_t s);
// the primal update from the A'y (or A'y-bar) of the check just done
void launch_primal_from_check(const Dev &d, double tau, int smode, hipStream_t s);
void launch_dual(const Dev &d, double sigma, int smode, hipStream_t s);
// How iteration i of a run of `iters` iterations updates the running sums:
// in pairs, so S is read and written every other iteration; a run of odd
// length ends with a single addition.  Every run leaves S complete, and
// (S + x_i) + x_{i+1} rounds exactly as two additions one after the other.
inline int sum_mode(int64_t i, int64_t iters) {
    if ((i & 1) == 0) return i + 1 < iters ? 1 : 0;
    return 2;
}
// one extragradient iteration (part < 0), or one of its four products
// (0: target x~, 1: target y~, 2: x+, 3: y+), for timing
void launch_egm(const Dev &d, double tau, double sigma, int part, hipStream_t s);
// out = A in / A' in; skip (device flag, may be null) turns the launch into a no-op
void launch_spmv_A(const Dev &d, const double *in, double *out, hipStream_t s,
                   const int *skip = nullptr);
void launch_spmv_T(const Dev &d, const double *in, double *out, hipStream_t s,
                   const int *skip = nullptr);

// two points for the KKT / radius pass: [0] current, [1] average
struct KktPoints {
    const double *x[2], *y[2], *ax[2], *aty[2];
};

// check
void launch_average(const Dev &d, hipStream_t s);
void launch_reset_done(const Dev &d, hipStream_t s);
void launch_kkt_partials(const Dev &d, hipStream_t s);
// KKT parts of a held point (0 current, 1 average, 2 anchor, 3 solution) into st->kkt_eval
void launch_kkt_eval(const Dev &d, int which, hipStream_t s);
void launch_kkt_final(const Dev &d, double tol, int kkt_kind, int gap_slots, hipStream_t s);
// trust region of slot 0 (point z-bar) or 1 (point z), if armed
void launch_gap(const Dev &d, int slot, hipStream_t s);
void launch_decide(const Dev &d, int mode, double beta, int tau0, hipStream_t s);
void launch_apply(const Dev &d, hipStream_t s);
void launch_fixed_restart(const Dev &d, hipStream_t s);
// which: 0 current, 1 average (from the sums), 2 anchor, 3 solution
void launch_copy_point(const Dev &d, int which, double *x, double *y, hipStream_t s);
void launch_set_point(const Dev &d, const double *x, const double *y, hipStream_t s);
// gap at a held point (0 current, 1 average, 2 anchor) with radius r
// (r < 0: distance to the anchor); result in st->tr[0]
void launch_gap_point(const Dev &d, int which, double r, hipStream_t s);

// power iteration
void launch_power_init(const Dev &d, hipStream_t s);
void launch_power_step(const Dev &d, double tol, int max_iters, hipStream_t s);
// shared reductions
int red_grid(long long N);

// measurement yardsticks (plain streaming copy of n doubles; plain gather
// out[i] = val[i] x[idx[i]], i < n)
void launch_copy_yard(const double *src, double *dst, long long n, hipStream_t s);
void launch_gather_yard(const int *idx, const double *val, const double *x, double *out,
                        long long n, hipStream_t s);
// gathers only (4 per thread, one sum stored per thread): x[idx[i]], i < n,
// or with idx null x at hashed indices in [0, 2^lg); outputs: doubles of out
long long gather_only_outputs(long long n);
void launch_gather_only(const int *idx, const double *x, long long n, int lg, double *out,
                        hipStream_t s);

// stand-alone trust region on raw (a, d)
void launch_tr_raw(int64_t N, const double *a, const double *dd, double r,
                   const TRWork &w, TRState *st, hipStream_t s);

// ---------------------------------------------------------------------
// One-workgroup solver for LPs whose iteration vectors (and, unless every
// row fits the registers of its lanes, the matrix) fit one CU's LDS: whole
// blocks of iterations plus their checks in one launch.
// ---------------------------------------------------------------------
constexpr int kTinyWG = 512;                 // threads of the one workgroup
constexpr int kTinyMaxCoords = 2 * kTinyWG;  // n + m (two trust-region coordinates per thread)
constexpr int kTinyK = 8;                    // matrix entries per lane held in registers
constexpr size_t kTinyLdsMax = 148u << 10;   // dynamic LDS bytes (static LDS + this <= 160 KB)
struct TinyPlan {
    int ok;                // the LP fits
    int reg;               // 1: matrix rows in registers, 0: matrix in LDS
    int ov;                // 1: each check overlaps the next block's iterations
    int Lp, Ld;            // lanes per row of A' (primal) and of A (dual)
    size_t lds;            // dynamic LDS bytes
};
struct TinyArgs {
    double tau, sigma, tol, beta, omega, sw;  // sw = sqrt(omega)
    int P, tau0, kkt_kind, gap_slots, blocks;
    int Lp, Ld;
    long long *summary;    // may be null: [0] = k, [1] = done | (conv_which + 1) << 8 | numerr << 16
};
// LDS bytes of the one-workgroup solver: doubles x, x-bar (n + 1 each, the
// last a zero that padded matrix entries point at), sx, c, l, u, A'y,
// A'y-bar (n each), y, y-bar (m + 1 each), sy, q, b, A x-bar (m each);
// trust-region keys, d^2, a^2 and a d (n + m each) and candidate indices
// (n + m ints); m bytes of row kinds; and,
// with the matrix in LDS, the values of A and A' (nnz doubles each), their
// row starts (ints) and 16-bit column indices; with the overlapped check,
// the copy of x (n + 1), sx (n), y (m + 1), sy and q (m each) it reads
__host__ __device__ inline size_t tiny_lds_bytes(long long n, long long m, long long nnz,
                                                 int reg, int ov = 0) {
    long long b = 8 * (8 * n + 6 * m + 4) + 36 * (n + m) + m;
    b = (b + 7) & ~7ll;
    if (!reg) b += 16 * nnz + 4 * (n + m + 2) + 4 * nnz;
    b = (b + 7) & ~7ll;
    if (ov) b += 8 * (2 * n + 3 * m + 2);
    return (size_t)((b + 15) & ~15ll);
}
// plan for an LP already on the device (reads its row starts)
TinyPlan tiny_plan(const Dev &d, hipStream_t s);
hipError_t launch_tiny_blocks(const Dev &d, const TinyArgs &a, const TinyPlan &p, hipStream_t s);
// count LPs at once, one workgroup each (devs, args in device memory); all
// of them planned with the kernel of p (same mode and lanes), lds the
// largest of their LDS sizes
hipError_t launch_tiny_many(const Dev *devs, const TinyArgs *args, int count, const TinyPlan &p,
                            size_t lds, hipStream_t s);

}  // namespace pdhg
