// C ABI of the restarted-PDHG library (declared in include/pdhg.h).
//
// The host side only orders launches: every arithmetic step runs in the
// kernels.  State that decides control flow (iteration counters, restart
// count, the converged flag) lives on the device so that a block of
// `check_period` iterations plus its check can be recorded once as a HIP
// graph and replayed; the host reads one status word per batch of replays.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "pdhg.h"
#include "pdhg_internal.h"

using namespace pdhg;

struct pdhg_handle {
    Dev d;
    hipStream_t stream;
    hipStream_t cap;        // private stream used only to record graphs
    pdhg_params prm;
    double eta, tau, sigma, sigma_max;
    int64_t pw_used;
    hipGraphExec_t gexec;   // one block of iterations plus its check
    hipGraphExec_t gexec_r; // the same, its first primal update from the last check's A'y
    double g_tol;
    bool g_valid;
    bool reuse;             // blocks right after a check take A'y from it (PDHG)
    bool fresh;             // the last step on the state was a check of this path
    TinyPlan tiny;          // one-workgroup solver, when the LP fits one CU's LDS
    int slab_cap[2];        // slab counts the workspace has room for (A, A')
};

#define CK(expr)                                   \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return PDHG_E_HIP;   \
    } while (0)

namespace pdhg {

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Target bytes of the gathered vector per column slab: one XCD's L2 (4 MiB)
// unless PDHG_SLAB_BYTES overrides it (a tuning knob; read at every
// workspace-size query and create, so keep it fixed between the two).
static int64_t slab_slice_bytes() {
    const char *e = getenv("PDHG_SLAB_BYTES");
    if (e && *e) {
        const long long v = atoll(e);
        if (v >= (64ll << 10) && v <= (1ll << 30)) return v;
    }
    return 4ll << 20;
}

// A's merge-path blocks sorted by column (k_sort_blocks) unless
// PDHG_SORTED_BLOCKS=0 (read at create; the plain layout gives bitwise the
// same sums, so tests compare the two)
static bool sorted_blocks_wanted() {
    const char *e = getenv("PDHG_SORTED_BLOCKS");
    return !(e && e[0] == '0');
}

// threads per workgroup of a single-LP product (spmv_threads_for);
// PDHG_SPMV_WG=128 or 256 sets both products instead (read at create)
static int spmv_wg_for(int64_t rows, int64_t nblk) {
    const char *e = getenv("PDHG_SPMV_WG");
    if (e && atoi(e) == 128) return 128;
    if (e && atoi(e) == 256) return kWG;
    return spmv_threads_for(rows, nblk);
}

size_t tr_work_bytes(int64_t N) {
    size_t b = 0;
    b += al(sizeof(unsigned int) * 2 * kBuckets);
    b += al(sizeof(double) * 2 * kBuckets) * 2;
    b += al(sizeof(double) * kRedBlocks * 4);
    b += al(sizeof(unsigned int) * kRedBlocks) + al(sizeof(unsigned int) * (kRedBlocks + 1));
    size_t n1 = (size_t)(N > 0 ? N : 1) + (size_t)kRedBlocks * kWG;
    b += al(sizeof(unsigned long long) * n1);
    b += al(sizeof(double) * n1) * 2;
    b += al(sizeof(unsigned int));
    b += al(sizeof(unsigned long long) * kFinishMax);
    b += al(sizeof(double) * kFinishMax) * 2;
    return b;
}

void carve_tr(char *base, int64_t N, TRWork *w) {
    size_t o = 0;
    size_t n1 = (size_t)(N > 0 ? N : 1) + (size_t)kRedBlocks * kWG;
    w->hcnt = (unsigned int *)(base + o);
    o += al(sizeof(unsigned int) * 2 * kBuckets);
    w->hD = (double *)(base + o);
    o += al(sizeof(double) * 2 * kBuckets);
    w->hA = (double *)(base + o);
    o += al(sizeof(double) * 2 * kBuckets);
    w->part = (double *)(base + o);
    o += al(sizeof(double) * kRedBlocks * 4);
    w->ccount = (unsigned int *)(base + o);
    o += al(sizeof(unsigned int) * kRedBlocks);
    w->coff = (unsigned int *)(base + o);
    o += al(sizeof(unsigned int) * (kRedBlocks + 1));
    w->ckey = (unsigned long long *)(base + o);
    o += al(sizeof(unsigned long long) * n1);
    w->ca = (double *)(base + o);
    o += al(sizeof(double) * n1);
    w->cd = (double *)(base + o);
    o += al(sizeof(double) * n1);
    w->fcount = (unsigned int *)(base + o);
    o += al(sizeof(unsigned int));
    w->fkey = (unsigned long long *)(base + o);
    o += al(sizeof(unsigned long long) * kFinishMax);
    w->fa = (double *)(base + o);
    o += al(sizeof(double) * kFinishMax);
    w->fd = (double *)(base + o);
}

bool make_layout(int64_t m, int64_t n, int64_t nnz, Layout *L) {
    if (m < 0 || n < 1 || nnz < 0) return false;
    const int64_t lim = 0x7fffffffLL - 4096;
    if (m > lim || n > lim || nnz > lim || m + nnz > 0x7fffffffLL * 2) return false;
    const size_t n1 = (size_t)n, m1 = (size_t)(m > 0 ? m : 1), z1 = (size_t)(nnz > 0 ? nnz : 1);
    size_t o = 0;
    L->o_state = o;
    o += al(sizeof(DevState));
    L->o_err = o;
    o += al(sizeof(int) * 16);
    L->o_trp = o;
    o += al(sizeof(int) * (n1 + 1));
    L->o_tci = o;
    o += al(sizeof(int) * z1);
    L->o_perm = o;
    o += al(sizeof(int) * z1);
    L->o_tv = o;
    o += al(sizeof(double) * z1);
    L->o_cursor = o;
    o += al(sizeof(int) * n1);
    L->o_long = o;
    o += al(sizeof(int) * n1);
    const int nbA = nblocks_for((int)m, (int)nnz), nbT = nblocks_for((int)n, (int)nnz);
    L->o_brA = o;  // block tables: row starts, then entry starts (k_rowsplit)
    o += al(sizeof(int) * 2 * ((size_t)nbA + 1));
    L->o_brT = o;
    o += al(sizeof(int) * 2 * ((size_t)nbT + 1));
    for (int k = 0; k < 8; ++k) {
        L->o_vec_n[k] = o;
        o += al(sizeof(double) * n1);
    }
    for (int k = 0; k < 8; ++k) {
        L->o_vec_m[k] = o;
        o += al(sizeof(double) * m1);
    }
    L->o_xt = o;
    o += al(sizeof(double) * n1);
    L->o_yt = o;
    o += al(sizeof(double) * m1);
    // column order: reordered col_idx, the permutation both ways, c, l, u
    L->o_ci2 = o;
    o += al(sizeof(int) * z1);
    L->o_cperm = o;
    o += al(sizeof(int) * n1);
    L->o_cinv = o;
    o += al(sizeof(int) * n1);
    L->o_c2 = o;
    o += al(sizeof(double) * n1);
    L->o_l2 = o;
    o += al(sizeof(double) * n1);
    L->o_u2 = o;
    o += al(sizeof(double) * n1);
    L->o_bcls = o;
    o += al(n1);
    const bool pk = sorted_blocks_fit(n);
    L->o_apk = o;
    o += al(pk ? sizeof(unsigned) * z1 : 0);
    L->o_asv = o;
    o += al(pk ? sizeof(double) * z1 : 0);
    L->o_part = o;
    o += al(sizeof(double) * kRedBlocks * kKktSums);
    L->o_log = o;
    o += al(sizeof(double) * kLogCap * kRec);
    for (int sidx = 0; sidx < kTrSlots; ++sidx) {
        L->o_tr[sidx] = o;
        o += tr_work_bytes((int64_t)n1 + (int64_t)(m > 0 ? m : 0));
    }
    // column slabs of A and of A' (empty regions when one slab covers the
    // gathered vector)
    const int64_t rows_of[2] = {m, n}, gath_of[2] = {n, m};
    for (int t = 0; t < 2; ++t) {
        const int S = slab_reserve_for(rows_of[t], gath_of[t], n, slab_slice_bytes());
        const size_t Ss = S > 1 ? (size_t)S : 0, zS = S > 1 ? z1 : 0;
        const size_t r1 = (size_t)(rows_of[t] > 0 ? rows_of[t] : 1);
        const int nb = t == 0 ? nbA : nbT;
        const size_t sz[6] = {sizeof(int) * Ss * (r1 + 1), sizeof(int) * zS, sizeof(double) * zS,
                              sizeof(int) * Ss * 2 * ((size_t)nb + 1), sizeof(long long) * 4 * Ss,
                              sizeof(double) * (S > 1 ? r1 : 0)};
        for (int k = 0; k < 6; ++k) {
            L->o_slab[t][k] = o;
            o += al(sz[k]);
        }
    }
    L->total = o;
    return true;
}

}  // namespace pdhg

static int gap_slots_for(int mode) {
    if (mode == PDHG_RESTART_ADAPTIVE) return 1;
    if (mode == PDHG_RESTART_FLEXIBLE) return 3;
    return 0;
}

// the check of Section 7, enqueued on s (also used while recording graphs)
static void enqueue_check(pdhg_t *h, double tol, hipStream_t s) {
    const Dev &d = h->d;
    const int *gate = &d.st->done;
    // the extragradient iterations leave no A x of the current point behind
    if (h->prm.method == PDHG_METHOD_EGM) launch_spmv_A(d, d.x, d.q, s, gate);
    launch_average(d, s);
    launch_spmv_A(d, d.xbar, d.axb, s, gate);
    launch_spmv_T(d, d.ybar, d.atyb, s, gate);
    launch_spmv_T(d, d.y, d.aty, s, gate);
    launch_kkt_partials(d, s);
    const int slots = gap_slots_for(h->prm.restart_mode);
    launch_kkt_final(d, tol, h->prm.kkt_kind, slots, s);
    if (slots & 1) launch_gap(d, 0, s);
    if (slots & 2) launch_gap(d, 1, s);
    launch_decide(d, h->prm.restart_mode, h->prm.beta, h->prm.tau0, s);
    launch_apply(d, s);
}

// from_check: the iterations start right after a check, whose A'y (or
// A'y-bar after a restart at the average) the first primal update takes
// instead of the product
static void enqueue_iters(pdhg_t *h, int64_t iters, hipStream_t s, bool from_check = false) {
    for (int64_t i = 0; i < iters; ++i) {
        if (h->prm.method == PDHG_METHOD_EGM) {
            launch_egm(h->d, h->tau, h->sigma, -1, s);
        } else {
            const int sm = sum_mode(i, iters);
            if (i == 0 && from_check) launch_primal_from_check(h->d, h->tau, sm, s);
            else launch_primal(h->d, h->tau, sm, s);
            launch_dual(h->d, h->sigma, sm, s);
        }
    }
}

static int read_state(pdhg_t *h, DevState *out) {
    CK(hipMemcpyAsync(out, h->d.st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    CK(hipStreamSynchronize(h->stream));
    return PDHG_OK;
}

static int last_error() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PDHG_OK : PDHG_E_HIP;
}

extern "C" {

void pdhg_default_params(pdhg_params *p) {
    if (!p) return;
    p->eta = 0.0;
    p->omega = 1.0;
    p->beta = exp(-1.0);
    p->check_period = 30;
    p->tau0 = 1;
    p->restart_mode = PDHG_RESTART_ADAPTIVE;
    p->fixed_len = 0;
    p->kkt_kind = PDHG_KKT_RELATIVE;
    p->power_iters = 1000;
    p->power_tol = 1e-10;
    p->method = PDHG_METHOD_PDHG;
}

size_t pdhg_workspace_bytes(int64_t m, int64_t n, int64_t nnz) {
    Layout L;
    if (!make_layout(m, n, nnz, &L)) return 0;
    return L.total;
}

const char *pdhg_strerror(int code) {
    switch (code) {
    case PDHG_OK: return "ok";
    case PDHG_NOT_CONVERGED: return "iteration budget used without reaching the tolerance";
    case PDHG_E_INVALID: return "invalid argument or malformed LP data";
    case PDHG_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case PDHG_E_HIP: return "HIP runtime error";
    case PDHG_E_NUMERICAL: return "NaN or Inf in the iterates";
    default: return "unknown code";
    }
}

// Split the CSR (rp, ci, v) with nblk merge-path blocks into sb.S column
// slabs (see slab_count_for); one host round trip for the entry count of
// every slab.
// Each slab's launch covers the rows from the first to the last one with an
// entry in the slab (PDHG_SLAB_RANGES=0: every row, for comparisons); the
// first range starts at row 0, the last ends at the last row, and the last
// range is stretched down over any row no range holds (rows without
// entries), so every row has a launch that applies its update.
static bool slab_ranges_wanted() {
    const char *e = getenv("PDHG_SLAB_RANGES");
    return !(e && e[0] == '0');
}

static void fit_slab_bounds(Slabs &sb) {
    const int S = sb.S;
    int end = 0;
    for (int q = 0; q < S; ++q) {
        sb.before[q] = end;
        if (sb.hi[q] > end) end = sb.hi[q];
    }
    int beg = sb.rows;
    for (int q = S - 1; q >= 0; --q) {
        sb.after[q] = beg;
        if (sb.lo[q] < beg) beg = sb.lo[q];
    }
    for (int q = S; q < kSlabMax; ++q) {
        sb.before[q] = sb.rows;
        sb.after[q] = sb.rows;
    }
}

static void fit_slab_ranges(Slabs &sb, const int *range) {
    const int S = sb.S, rows = sb.rows;
    const bool want = slab_ranges_wanted();
    for (int q = 0; q < kSlabMax; ++q) {
        sb.lo[q] = 0;
        sb.hi[q] = q < S ? rows : 0;
    }
    if (!want) {
        fit_slab_bounds(sb);
        return;
    }
    for (int q = 0; q < S; ++q) {
        int lo = range[2 * q], hi = range[2 * q + 1];
        if (hi < 0) lo = hi = 0;  // no entries in this slab
        if (q == 0) lo = 0;
        if (q == S - 1) hi = rows;
        sb.lo[q] = lo;
        sb.hi[q] = hi > lo ? hi : lo;
    }
    // widen: the ranges of slabs 0..q cover [0, end) with no gap, and those
    // of slabs q..S-1 cover [start, rows) with no gap
    int end = sb.hi[0];
    for (int q = 1; q < S; ++q) {
        if (sb.lo[q] > end) sb.lo[q] = end;
        if (sb.hi[q] > end) end = sb.hi[q];
    }
    int beg = sb.lo[S - 1];
    for (int q = S - 2; q >= 0; --q) {
        if (sb.hi[q] < beg) sb.hi[q] = beg;
        if (sb.lo[q] < beg) beg = sb.lo[q];
    }
}

static int build_slabs(Slabs &sb, const int *rp, const int *ci, const double *v, int nnz,
                       int nblk, int *scratch, hipStream_t s) {
    launch_slab_count(sb, rp, ci, scratch, s);
    launch_slab_ranges(sb, scratch, s);
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int range[2 * kSlabMax];
    for (int q = 0; q < sb.S; ++q)
        CK(hipMemcpyAsync(&cnt[q], sb.srp + (size_t)q * (sb.rows + 1) + sb.rows, sizeof(int),
                          hipMemcpyDeviceToHost, s));
    CK(hipMemcpyAsync(range, scratch, sizeof(int) * 2 * sb.S, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    fit_slab_ranges(sb, range);
    fit_slab_bounds(sb);
    long long meta[32];
    long long eoff = 0, boff = 0;
    int nbmax = 0;
    for (int q = 0; q < sb.S; ++q) {
        const int nb = nblocks_for(sb.hi[q] - sb.lo[q], cnt[q]);
        meta[4 * q + 0] = (long long)q * (sb.rows + 1);
        meta[4 * q + 1] = eoff;
        meta[4 * q + 2] = boff;
        meta[4 * q + 3] = nb;
        eoff += cnt[q];
        boff += 2 * (nb + 1);
        if (nb > nbmax) nbmax = nb;
    }
    // every entry lands in exactly one slab; the block tables fit their region
    if (eoff != nnz || boff > (long long)sb.S * 2 * (nblk + 1)) return PDHG_E_INVALID;
    CK(hipMemcpyAsync(sb.smeta, meta, sizeof(long long) * 4 * sb.S, hipMemcpyHostToDevice, s));
    CK(hipStreamSynchronize(s));
    sb.nbmax = nbmax;
    launch_slab_fill(sb, rp, ci, v, s);
    for (int q = 0; q < sb.S; ++q)
        launch_rowsplit_range(sb.srp + meta[4 * q] + sb.lo[q], sb.hi[q] - sb.lo[q],
                              (int)meta[4 * q + 3], sb.sbr + meta[4 * q + 2], s);
    return last_error();
}

// Sort the columns by entry count, largest first (a stable counting sort
// on the host), and switch the device view to the reordered copies.  With
// most entries in the first columns, the x that the A x products gather is
// mostly one L2-sized region; when that region holds at least 60% of the
// entries, A x skips its column slabs.
static int order_columns(Dev &d, const Layout &L, char *ws, hipStream_t s) {
    d.permuted = 0;
    if (d.n < 2 || d.nnz == 0) return PDHG_OK;
    const int n = d.n, m = d.m;
    int *cnt_dev = d.trp;     // n + 1 ints, rebuilt by the transpose afterwards
    int *first_dev = d.cursor;  // n ints of transpose scratch, free until then
    launch_col_counts(d.ci, d.nnz, n, cnt_dev, s);
    launch_first_rows(d.rp, d.ci, m, n, d.nnz, first_dev, s);
    std::vector<int> cnt((size_t)n + 1), first((size_t)n);
    CK(hipMemcpyAsync(cnt.data(), cnt_dev, sizeof(int) * ((size_t)n + 1), hipMemcpyDeviceToHost,
                      s));
    CK(hipMemcpyAsync(first.data(), first_dev, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    // Columns by entry count, largest first; equal counts by their first row,
    // so that rows next to each other gather columns next to each other in
    // A x, and rows of A' next to each other gather nearby y in A'y (two
    // stable counting passes: first row, then count).
    std::vector<int> by_first((size_t)n);
    {
        std::vector<int> fstart((size_t)m + 2, 0);
        for (int j = 0; j < n; ++j) fstart[(size_t)first[j] + 1] += 1;
        for (int r = 0; r <= m; ++r) fstart[(size_t)r + 1] += fstart[r];
        for (int j = 0; j < n; ++j) by_first[(size_t)fstart[first[j]]++] = j;
    }
    int cmax = 0;
    for (int j = 0; j < n; ++j) cmax = cnt[j + 1] > cmax ? cnt[j + 1] : cmax;
    std::vector<int> start((size_t)cmax + 2, 0);
    for (int j = 0; j < n; ++j) start[(size_t)(cmax - cnt[j + 1]) + 1] += 1;
    for (int k = 0; k <= cmax; ++k) start[k + 1] += start[k];
    std::vector<int> by_count((size_t)n);
    for (int t = 0; t < n; ++t) {
        const int j = by_first[(size_t)t];
        by_count[(size_t)start[(size_t)(cmax - cnt[j + 1])]++] = j;
    }
    // When A'y runs over two column slabs of y, the columns go in three
    // regions (each in the order above): those whose rows all lie in the
    // first slab of y, those with rows in both, those with rows all in the
    // second (then empty columns).  A'y's first launch then covers the rows
    // of A' up to the end of the middle region and its second launch the
    // rows from the start of the middle region, and only the middle region
    // goes through the accumulator of the slabs (Slabs).
    std::vector<int> cls((size_t)n, 0);
    const char *reg_env = getenv("PDHG_COLUMN_REGIONS");
    const bool regions = d.slT.S == 2 && d.m > 0 && !(reg_env && reg_env[0] == '0');
    if (regions) {
        int *last_dev = d.long_rows;  // n ints of transpose scratch, free until then
        launch_last_rows(d.rp, d.ci, m, n, d.nnz, last_dev, s);
        std::vector<int> last((size_t)n);
        CK(hipMemcpyAsync(last.data(), last_dev, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost,
                          s));
        CK(hipStreamSynchronize(s));
        const int W = d.slT.W;
        for (int j = 0; j < n; ++j)
            cls[(size_t)j] = cnt[j + 1] == 0 ? 3 : last[j] < W ? 0 : first[j] >= W ? 2 : 1;
    }
    std::vector<int> cstart(5, 0);
    for (int j = 0; j < n; ++j) cstart[(size_t)cls[(size_t)j] + 1] += 1;
    for (int k = 0; k < 4; ++k) cstart[k + 1] += cstart[k];
    const int ncls0 = regions ? cstart[1] : 0;  // where the middle region starts
    std::vector<int> order((size_t)n), inv((size_t)n);
    bool ident = true;
    for (int t = 0; t < n; ++t) {
        const int j = by_count[(size_t)t];
        const int q = cstart[(size_t)cls[(size_t)j]]++;
        order[q] = j;
        inv[j] = q;
        ident &= (q == j);
    }
    // share of the entries in the L2-sized run of columns where the most
    // gathered ones start (the first column, or the middle region): when
    // the hot columns hold most of them, A x gathers from one L2 without
    // slabs
    const long long w0 = slab_slice_bytes() / 8;
    long long hot = 0;
    for (long long q = ncls0; q < n && q < ncls0 + w0; ++q) hot += cnt[(size_t)order[q] + 1];
    if (d.slA.S > 1 && 10 * hot >= 6 * (long long)d.nnz) d.slA.S = 1;
    if (ident) return PDHG_OK;
    int *ci2 = (int *)(ws + L.o_ci2);
    int *cperm = (int *)(ws + L.o_cperm), *cinv = (int *)(ws + L.o_cinv);
    double *c2 = (double *)(ws + L.o_c2), *l2 = (double *)(ws + L.o_l2);
    double *u2 = (double *)(ws + L.o_u2);
    CK(hipMemcpyAsync(cperm, order.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(cinv, inv.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, s));
    launch_permute_cols(d.ci, d.nnz, cinv, ci2, d.c, d.l, d.u, cperm, n, c2, l2, u2, s);
    CK(hipStreamSynchronize(s));  // the host vectors above leave scope
    d.ci = ci2;
    d.c = c2;
    d.l = l2;
    d.u = u2;
    d.cperm = cperm;
    d.cinv = cinv;
    d.permuted = 1;
    return last_error();
}

// Bound classes: when the columns' (l, u) pairs (compared bit for bit)
// take at most kBoundClasses distinct values, each column gets a one-byte
// class and the primal update reads that byte instead of 16 bytes of bounds.
// LPs with more distinct pairs keep reading l and u.
static int bound_classes(Dev &d, const Layout &L, char *ws, hipStream_t s) {
    d.bcls = nullptr;
    d.nbcls = 0;
    const int n = d.n;
    std::vector<unsigned long long> lo((size_t)n), hi((size_t)n);
    CK(hipMemcpyAsync(lo.data(), d.l, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, s));
    CK(hipMemcpyAsync(hi.data(), d.u, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    std::vector<unsigned char> cls((size_t)n);
    unsigned long long kl[kBoundClasses], ku[kBoundClasses];
    int nc = 0;
    for (int j = 0; j < n; ++j) {
        int k = 0;
        while (k < nc && (kl[k] != lo[(size_t)j] || ku[k] != hi[(size_t)j])) ++k;
        if (k == nc) {
            if (nc == kBoundClasses) return PDHG_OK;
            kl[nc] = lo[(size_t)j];
            ku[nc] = hi[(size_t)j];
            ++nc;
        }
        cls[(size_t)j] = (unsigned char)k;
    }
    for (int k = 0; k < kBoundClasses; ++k) {
        const int q = k < nc ? k : 0;
        memcpy(&d.blo[k], &kl[q], sizeof(double));
        memcpy(&d.bhi[k], &ku[q], sizeof(double));
    }
    unsigned char *dev = (unsigned char *)(ws + L.o_bcls);
    CK(hipMemcpyAsync(dev, cls.data(), (size_t)n, hipMemcpyHostToDevice, s));
    CK(hipStreamSynchronize(s));  // the host vector above leaves scope
    d.bcls = dev;
    d.nbcls = nc;
    return PDHG_OK;
}

int pdhg_create(const pdhg_lp *lp, const pdhg_params *prm_in, void *workspace,
                size_t workspace_bytes, void *stream, pdhg_t **out) {
    if (!out) return PDHG_E_INVALID;
    *out = nullptr;
    if (!lp) return PDHG_E_INVALID;
    pdhg_params prm;
    if (prm_in) prm = *prm_in;
    else pdhg_default_params(&prm);
    if (!(prm.omega > 0.0) || !isfinite(prm.omega) || !(prm.beta > 0.0) || !(prm.beta < 1.0) ||
        prm.check_period < 1 || prm.tau0 < 1 || prm.restart_mode < 0 || prm.restart_mode > 3 ||
        (prm.restart_mode == PDHG_RESTART_FIXED && prm.fixed_len < 1) || prm.kkt_kind < 0 ||
        prm.kkt_kind > 2 || isnan(prm.eta) || isinf(prm.eta) ||
        (prm.method != PDHG_METHOD_PDHG && prm.method != PDHG_METHOD_EGM))
        return PDHG_E_INVALID;
    if (prm.power_iters < 1) prm.power_iters = 1000;
    if (!(prm.power_tol > 0.0)) prm.power_tol = 1e-10;
    Layout L;
    if (!make_layout(lp->m, lp->n, lp->nnz, &L)) return PDHG_E_INVALID;
    if (!lp->row_ptr || !lp->c || !lp->l || !lp->u) return PDHG_E_INVALID;
    if (lp->nnz > 0 && (!lp->col_idx || !lp->vals)) return PDHG_E_INVALID;
    if (lp->m > 0 && !lp->b) return PDHG_E_INVALID;
    if (!workspace || ((uintptr_t)workspace & 255u) || workspace_bytes < L.total)
        return PDHG_E_WORKSPACE;

    pdhg_t *h = new (std::nothrow) pdhg_handle();
    if (!h) return PDHG_E_HIP;
    h->stream = (hipStream_t)stream;
    h->prm = prm;
    h->g_valid = false;
    h->gexec = nullptr;
    h->gexec_r = nullptr;
    h->fresh = false;
    {
        // PDHG_CHECK_REUSE=0: every primal half-step runs its product
        const char *e = getenv("PDHG_CHECK_REUSE");
        h->reuse = !(e && e[0] == '0');
    }
    h->cap = nullptr;
    char *ws = (char *)workspace;
    Dev &d = h->d;
    memset(&d, 0, sizeof(d));
    d.m = (int)lp->m;
    d.n = (int)lp->n;
    d.nnz = (int)lp->nnz;
    d.rp = lp->row_ptr;
    d.ci = lp->col_idx;
    d.v = lp->vals;
    d.c = lp->c;
    d.b = lp->b;
    d.l = lp->l;
    d.u = lp->u;
    d.kind = (const signed char *)lp->row_kind;
    d.st = (DevState *)(ws + L.o_state);
    d.err = (int *)(ws + L.o_err);
    d.trp = (int *)(ws + L.o_trp);
    d.tci = (int *)(ws + L.o_tci);
    d.perm = (int *)(ws + L.o_perm);
    d.tv = (double *)(ws + L.o_tv);
    d.cursor = (int *)(ws + L.o_cursor);
    d.long_rows = (int *)(ws + L.o_long);
    d.nblkA = nblocks_for(d.m, d.nnz);
    d.nblkT = nblocks_for(d.n, d.nnz);
    d.brA = (int *)(ws + L.o_brA);
    d.brT = (int *)(ws + L.o_brT);
    double *vn[8], *vm[8];
    for (int k = 0; k < 8; ++k) {
        vn[k] = (double *)(ws + L.o_vec_n[k]);
        vm[k] = (double *)(ws + L.o_vec_m[k]);
    }
    d.x = vn[0]; d.x0 = vn[1]; d.sx = vn[2]; d.xbar = vn[3];
    d.atyb = vn[4]; d.aty = vn[5]; d.gx = vn[6]; d.gaty = vn[7];
    d.y = vm[0]; d.y0 = vm[1]; d.sy = vm[2]; d.q = vm[3];
    d.ybar = vm[4]; d.axb = vm[5]; d.gy = vm[6]; d.gax = vm[7];
    d.xt = (double *)(ws + L.o_xt);
    d.yt = (double *)(ws + L.o_yt);
    d.part = (double *)(ws + L.o_part);
    d.log = (double *)(ws + L.o_log);
    for (int sidx = 0; sidx < kTrSlots; ++sidx)
        carve_tr(ws + L.o_tr[sidx], (int64_t)d.n + d.m, &d.tr[sidx]);
    d.omega = prm.omega;
    Slabs *sl[2] = {&d.slA, &d.slT};
    const int rows_of[2] = {d.m, d.n}, gath_of[2] = {d.n, d.m};
    for (int t = 0; t < 2; ++t) {
        Slabs &sb = *sl[t];
        sb.S = slab_count_for(rows_of[t], gath_of[t], d.n, slab_slice_bytes());
        sb.W = (int)(((long long)gath_of[t] + sb.S - 1) / sb.S);
        h->slab_cap[t] = slab_reserve_for(rows_of[t], gath_of[t], d.n, slab_slice_bytes());
        sb.rows = rows_of[t];
        sb.nbmax = 0;
        sb.srp = (int *)(ws + L.o_slab[t][0]);
        sb.sci = (int *)(ws + L.o_slab[t][1]);
        sb.sv = (double *)(ws + L.o_slab[t][2]);
        sb.sbr = (int *)(ws + L.o_slab[t][3]);
        sb.smeta = (long long *)(ws + L.o_slab[t][4]);
        sb.spart = (double *)(ws + L.o_slab[t][5]);
    }

    int rc = PDHG_OK;
    do {
        hipStream_t s = h->stream;
        if (hipMemsetAsync(d.st, 0, sizeof(DevState), s) != hipSuccess ||
            hipMemsetAsync(d.err, 0, sizeof(int) * 16, s) != hipSuccess) {
            rc = PDHG_E_HIP;
            break;
        }
        launch_validate(d, s);
        int err[2] = {0, 0};
        if (hipMemcpyAsync(err, d.err, sizeof(err), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = PDHG_E_HIP;
            break;
        }
        if (err[0]) {
            rc = PDHG_E_INVALID;
            break;
        }
        if ((rc = order_columns(d, L, ws, s)) != PDHG_OK) break;
        if ((rc = bound_classes(d, L, ws, s)) != PDHG_OK) break;
        launch_rowsplit(d.rp, d.m, d.nnz, d.nblkA, d.brA, s);
        if (sorted_blocks_fit(d.n) && d.nnz > 0 && d.m > 0 && sorted_blocks_wanted()) {
            unsigned *apk = (unsigned *)(ws + L.o_apk);
            double *asv = (double *)(ws + L.o_asv);
            launch_sort_blocks(d.rp, d.ci, d.v, d.brA, d.nblkA, apk, asv, s);
            d.apk = apk;
            d.asv = asv;
        }
        launch_transpose(d, s);
        launch_rowsplit(d.trp, d.n, d.nnz, d.nblkT, d.brT, s);
        if (d.slA.S > 1 && (rc = build_slabs(d.slA, d.rp, d.ci, d.v, d.nnz, d.nblkA,
                                             d.long_rows, s)) != PDHG_OK)
            break;
        if (d.slT.S > 1 && (rc = build_slabs(d.slT, d.trp, d.tci, d.tv, d.nnz, d.nblkT,
                                             d.long_rows, s)) != PDHG_OK)
            break;
        d.swgA = spmv_wg_for(d.m, d.slA.S > 1 ? d.slA.nbmax : d.nblkA);
        d.swgT = spmv_wg_for(d.n, d.slT.S > 1 ? d.slT.nbmax : d.nblkT);
        launch_norms(d, s);
        launch_init_point(d, s);
        if ((rc = last_error()) != PDHG_OK) break;
        h->sigma_max = 0.0;
        h->pw_used = 0;
        if (prm.eta > 0.0) {
            h->eta = prm.eta;
        } else {
            launch_power_init(d, s);
            DevState hs;
            int done = 0;
            while (!done) {
                for (int q = 0; q < 25; ++q) launch_power_step(d, prm.power_tol, prm.power_iters, s);
                if ((rc = last_error()) != PDHG_OK) break;
                if ((rc = read_state(h, &hs)) != PDHG_OK) break;
                done = hs.pw_done;
            }
            if (rc != PDHG_OK) break;
            h->sigma_max = hs.pw_est;
            h->pw_used = hs.pw_it;
            h->eta = h->sigma_max > 0.0 ? 0.9 / h->sigma_max : 1.0;
        }
        h->tau = h->eta / prm.omega;
        h->sigma = h->eta * prm.omega;
        h->tiny = tiny_plan(d, s);
        if (hipStreamSynchronize(s) != hipSuccess) {
            rc = PDHG_E_HIP;
            break;
        }
        if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) {
            rc = PDHG_E_HIP;
            break;
        }
    } while (0);
    if (rc != PDHG_OK) {
        if (h->cap) (void)hipStreamDestroy(h->cap);
        delete h;
        return rc;
    }
    *out = h;
    return PDHG_OK;
}

void pdhg_destroy(pdhg_t *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->gexec_r) (void)hipGraphExecDestroy(h->gexec_r);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    delete h;
}

// plain iterations; fixed-length restarts happen when t reaches fixed_len
static int run_iters(pdhg_t *h, int64_t iters, int64_t *t_host) {
    if (iters > 0) h->fresh = false;
    if (h->prm.restart_mode != PDHG_RESTART_FIXED) {
        enqueue_iters(h, iters, h->stream);
        return last_error();
    }
    const int64_t T = h->prm.fixed_len;
    while (iters > 0) {
        int64_t sstep = T - *t_host;
        if (sstep > iters) sstep = iters;
        enqueue_iters(h, sstep, h->stream);
        iters -= sstep;
        *t_host += sstep;
        if (*t_host >= T) {
            launch_fixed_restart(h->d, h->stream);
            *t_host = 0;
        }
    }
    return last_error();
}

int pdhg_step(pdhg_t *h, int64_t iters) {
    if (!h || iters < 0) return PDHG_E_INVALID;
    launch_reset_done(h->d, h->stream);
    int64_t t_host = 0;
    if (h->prm.restart_mode == PDHG_RESTART_FIXED) {
        DevState hs;
        int rc = read_state(h, &hs);
        if (rc) return rc;
        t_host = hs.t;
    }
    return run_iters(h, iters, &t_host);
}

static void fill_record(const double *rec, pdhg_check_record *out) {
    if (out) memcpy(out->v, rec, sizeof(double) * kRec);
}

static int read_last_record(pdhg_t *h, const DevState &hs, double *rec) {
    if (hs.checks <= 0) return PDHG_E_INVALID;
    const double *src = h->d.log + (size_t)((hs.checks - 1) % kLogCap) * kRec;
    CK(hipMemcpyAsync(rec, src, sizeof(double) * kRec, hipMemcpyDeviceToHost, h->stream));
    CK(hipStreamSynchronize(h->stream));
    return PDHG_OK;
}

int pdhg_restart_check(pdhg_t *h, double tol, int32_t *converged, int32_t *restarted,
                       double *rho, pdhg_check_record *rec) {
    if (!h || isnan(tol)) return PDHG_E_INVALID;
    launch_reset_done(h->d, h->stream);
    enqueue_check(h, tol, h->stream);
    int rc = last_error();
    if (rc) return rc;
    h->fresh = true;
    DevState hs;
    if ((rc = read_state(h, &hs))) return rc;
    double r[kRec];
    if ((rc = read_last_record(h, hs, r))) return rc;
    if (converged) *converged = hs.conv_which >= 0 ? 1 : 0;
    if (restarted) *restarted = (int32_t)r[9];
    if (rho) *rho = r[6];
    fill_record(r, rec);
    if (hs.numerr) return PDHG_E_NUMERICAL;
    return PDHG_OK;
}

int pdhg_kkt_error(pdhg_t *h, int32_t which, pdhg_kkt *out) {
    if (!h || which < 0 || which > 3 || !out) return PDHG_E_INVALID;
    launch_kkt_eval(h->d, which, h->stream);
    int rc = last_error();
    if (rc) return rc;
    DevState hs;
    if ((rc = read_state(h, &hs))) return rc;
    const double *k8 = hs.kkt_eval;
    out->kkt_rel = k8[1];
    out->primal_res = k8[2];
    out->dual_res = k8[3];
    out->pobj = k8[4];
    out->dobj = k8[5];
    out->kkt_paper_abs = k8[6];
    out->kkt_max_abs = k8[7];
    out->kkt = h->prm.kkt_kind == 1 ? k8[6] : (h->prm.kkt_kind == 2 ? k8[7] : k8[1]);
    return PDHG_OK;
}

int pdhg_gap(pdhg_t *h, int32_t which, double r, double *rho, double *r_used, double *lambda) {
    if (!h || which < 0 || which > 3 || isnan(r)) return PDHG_E_INVALID;
    launch_gap_point(h->d, which, r, h->stream);
    int rc = last_error();
    if (rc) return rc;
    DevState hs;
    if ((rc = read_state(h, &hs))) return rc;
    if (rho) *rho = hs.tr[0].rho;
    if (r_used) *r_used = hs.tr[0].r;
    if (lambda) *lambda = hs.tr[0].lam;
    if (hs.tr[0].nan_seen) return PDHG_E_NUMERICAL;
    return PDHG_OK;
}

// record one block: check_period iterations followed by the check
static int build_graph(pdhg_t *h, double tol) {
    if (h->g_valid && h->g_tol == tol) return PDHG_OK;
    hipGraphExec_t *ex[2] = {&h->gexec, &h->gexec_r};
    for (int v = 0; v < 2; ++v)
        if (*ex[v]) {
            (void)hipGraphExecDestroy(*ex[v]);
            *ex[v] = nullptr;
        }
    h->g_valid = false;
    for (int v = 0; v < 2; ++v) {
        if (v == 1 && !(h->reuse && h->prm.method == PDHG_METHOD_PDHG)) break;
        hipGraph_t g = nullptr;
        CK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        enqueue_iters(h, h->prm.check_period, h->cap, v == 1);
        enqueue_check(h, tol, h->cap);
        hipError_t e = hipStreamEndCapture(h->cap, &g);
        if (e != hipSuccess) return PDHG_E_HIP;
        e = hipGraphInstantiate(ex[v], g, nullptr, nullptr, 0);
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

static int finish_result(pdhg_t *h, const DevState &hs, pdhg_result *out) {
    if (!out) return PDHG_OK;
    out->iterations = hs.k;
    out->restarts = hs.restarts;
    if (hs.conv_which >= 0) {
        const double *k8 = hs.conv_which == 1 ? hs.kkt_avg : hs.kkt_cur;
        out->status = PDHG_OK;
        out->which_point = hs.conv_which;
        out->kkt = k8[0];
        out->pobj = k8[4];
        out->dobj = k8[5];
        return PDHG_OK;
    }
    pdhg_kkt kk;
    int rc = pdhg_kkt_error(h, PDHG_POINT_CURRENT, &kk);
    if (rc) return rc;
    out->status = PDHG_NOT_CONVERGED;
    out->which_point = -1;
    out->kkt = kk.kkt;
    out->pobj = kk.pobj;
    out->dobj = kk.dobj;
    return PDHG_OK;
}

// Plain iterations up to the next check point (or k_end if sooner), then the
// check when it falls there: the eager part of pdhg_solve.
// Blocks of iterations plus check per round before the host reads the
// state: rounds of 1, 2, 4, ... up to these.  A one-workgroup launch runs
// its blocks in one kernel (and stops at convergence by itself), so long
// rounds cost nothing; the graph path queues one replay per block.
constexpr int64_t kTinyBatchMax = 1024;
constexpr int64_t kGraphBatchMax = 64;

static int solve_eager_step(pdhg_t *h, int64_t *k, int64_t k_end, double tol, int64_t *t_host,
                            bool *conv) {
    const int64_t P = h->prm.check_period;
    const int64_t to_check = P - (*k % P);
    const int64_t sstep = to_check < k_end - *k ? to_check : k_end - *k;
    int rc;
    if ((rc = run_iters(h, sstep, t_host))) return rc;
    *k += sstep;
    if (*k % P == 0) {
        enqueue_check(h, tol, h->stream);
        if ((rc = last_error())) return rc;
        h->fresh = true;
        DevState hs;
        if ((rc = read_state(h, &hs))) return rc;
        if (hs.numerr) return PDHG_E_NUMERICAL;
        *conv = hs.conv_which >= 0 && hs.done;
        *t_host = hs.t;
    }
    return PDHG_OK;
}

static bool one_workgroup(const pdhg_t *h) {
    return h->tiny.ok && h->prm.method == PDHG_METHOD_PDHG &&
           h->prm.restart_mode != PDHG_RESTART_FIXED && h->prm.check_period <= INT32_MAX;
}

static TinyArgs tiny_args(const pdhg_t *h, double tol, int blocks) {
    TinyArgs ta{};
    ta.tau = h->tau;
    ta.sigma = h->sigma;
    ta.tol = tol;
    ta.beta = h->prm.beta;
    ta.omega = h->d.omega;
    ta.sw = sqrt(h->d.omega);
    ta.P = (int)h->prm.check_period;
    ta.tau0 = h->prm.tau0;
    ta.kkt_kind = h->prm.kkt_kind;
    ta.gap_slots = gap_slots_for(h->prm.restart_mode);
    ta.blocks = blocks;
    ta.Lp = h->tiny.Lp;
    ta.Ld = h->tiny.Ld;
    ta.summary = nullptr;
    return ta;
}

int pdhg_solve(pdhg_t *h, int64_t max_iters, double tol, pdhg_result *out) {
    if (!h || max_iters < 0 || isnan(tol)) return PDHG_E_INVALID;
    int rc;
    launch_reset_done(h->d, h->stream);
    DevState hs;
    if ((rc = read_state(h, &hs))) return rc;
    const int64_t P = h->prm.check_period;
    int64_t k = hs.k, t_host = hs.t;
    const int64_t k_end = k + max_iters;
    bool conv = false;
    const bool use_graph = h->prm.restart_mode != PDHG_RESTART_FIXED;
    while (k < k_end && !conv) {
        if (use_graph && k % P == 0 && k_end - k >= P) {
            // replay whole blocks; the device skips everything after convergence
            const bool tiny = one_workgroup(h);
            TinyArgs ta = tiny_args(h, tol, 0);
            if (!tiny && (rc = build_graph(h, tol))) return rc;
            int64_t blocks = (k_end - k) / P;
            int64_t batch = 1;
            double kkt_prev = 0.0;  // the smaller KKT of the last round's last check
            while (blocks > 0 && !conv) {
                int64_t nb = batch < blocks ? batch : blocks;
                if (tiny) {
                    ta.blocks = (int)nb;
                    CK(launch_tiny_blocks(h->d, ta, h->tiny, h->stream));
                    h->fresh = false;
                } else {
                    for (int64_t q = 0; q < nb; ++q) {
                        CK(hipGraphLaunch(h->fresh && h->gexec_r ? h->gexec_r : h->gexec,
                                          h->stream));
                        h->fresh = true;
                    }
                }
                if ((rc = read_state(h, &hs))) return rc;
                if (hs.numerr) return PDHG_E_NUMERICAL;
                blocks -= nb;
                k += nb * P;
                conv = hs.conv_which >= 0 && hs.done;
                if (batch < (tiny ? kTinyBatchMax : kGraphBatchMax)) batch *= 2;
                // Replays queued past convergence still launch every kernel
                // (each returns at once): near the tolerance, size the next
                // round by the KKT's decay over this one, at half the blocks
                // that rate would need
                if (!tiny && tol > 0.0 && !conv) {
                    const double kk = fmin(hs.kkt_cur[0], hs.kkt_avg[0]);
                    if (kkt_prev > 0.0 && kk > tol && kk < kkt_prev) {
                        const double need = log(tol / kk) / (log(kk / kkt_prev) / (double)nb);
                        const int64_t cap = need < 2.0 ? 1 : (int64_t)(0.5 * need);
                        if (batch > cap) batch = cap;
                    }
                    kkt_prev = kk;
                }
            }
            continue;
        }
        if ((rc = solve_eager_step(h, &k, k_end, tol, &t_host, &conv))) return rc;
    }
    if ((rc = read_state(h, &hs))) return rc;
    if ((rc = finish_result(h, hs, out))) return rc;
    return conv ? PDHG_OK : PDHG_NOT_CONVERGED;
}

static size_t many_bytes(int64_t count) {
    return al(sizeof(Dev) * (size_t)count) + al(sizeof(TinyArgs) * (size_t)count) +
           al(sizeof(long long) * 2 * (size_t)count);
}

size_t pdhg_solve_many_workspace_bytes(int32_t count) {
    return count > 0 ? many_bytes(count) : 0;
}

int pdhg_solve_many(pdhg_t *const *hs, int32_t count, int64_t max_iters, double tol,
                    void *workspace, size_t workspace_bytes, pdhg_result *out) {
    if (count < 0 || (count > 0 && !hs) || max_iters < 0 || isnan(tol)) return PDHG_E_INVALID;
    if (count == 0) return PDHG_OK;
    {
        std::vector<const pdhg_t *> seen(hs, hs + count);
        std::sort(seen.begin(), seen.end());
        for (int32_t i = 0; i < count; ++i)
            if (!seen[i] || (i > 0 && seen[i] == seen[i - 1])) return PDHG_E_INVALID;
    }
    if (!workspace || workspace_bytes < many_bytes(count)) return PDHG_E_INVALID;
    char *ws = (char *)workspace;
    Dev *ddev = (Dev *)ws;
    TinyArgs *dargs = (TinyArgs *)(ws + al(sizeof(Dev) * (size_t)count));
    long long *dsum = (long long *)(ws + al(sizeof(Dev) * (size_t)count) +
                                    al(sizeof(TinyArgs) * (size_t)count));
    hipStream_t s = hs[0]->stream;
    bool all_conv = true;
    std::vector<int64_t> k(count), kend(count), t_host(count);
    std::vector<char> conv(count, 0), joint(count, 0);
    int rc;
    for (int32_t i = 0; i < count; ++i) {
        pdhg_t *h = hs[i];
        if (!one_workgroup(h)) {
            rc = pdhg_solve(h, max_iters, tol, out ? &out[i] : nullptr);
            if (rc != PDHG_OK && rc != PDHG_NOT_CONVERGED) return rc;
            all_conv &= rc == PDHG_OK;
            continue;
        }
        launch_reset_done(h->d, h->stream);
        DevState st;
        if ((rc = read_state(h, &st))) return rc;
        k[i] = st.k;
        t_host[i] = st.t;
        kend[i] = k[i] + max_iters;
        const int64_t P = h->prm.check_period;
        bool c = false;
        // up to the first check point, as pdhg_solve does
        if (k[i] % P != 0 && k[i] < kend[i] &&
            (rc = solve_eager_step(h, &k[i], kend[i], tol, &t_host[i], &c)))
            return rc;
        conv[i] = c;
        joint[i] = !c && kend[i] - k[i] >= P;
        CK(hipStreamSynchronize(h->stream));
    }
    // whole blocks of every remaining handle, one workgroup each, a group of
    // handles sharing one kernel per launch; rounds of 1, 2, 4, ... kTinyBatchMax blocks
    for (int32_t lead = 0; lead < count; ++lead) {
        if (!joint[lead]) continue;
        const TinyPlan &pl = hs[lead]->tiny;
        std::vector<int32_t> g;
        size_t lds = 0;
        for (int32_t i = lead; i < count; ++i) {
            const TinyPlan &q = hs[i]->tiny;
            if (joint[i] && q.reg == pl.reg && q.ov == pl.ov &&
                (!pl.reg || (q.Lp == pl.Lp && q.Ld == pl.Ld))) {
                g.push_back(i);
                lds = q.lds > lds ? q.lds : lds;
                joint[i] = 0;
            }
        }
        const int ng = (int)g.size();
        std::vector<Dev> hdev(ng);
        std::vector<TinyArgs> harg(ng);
        std::vector<long long> hsum(2 * (size_t)ng);
        for (int j = 0; j < ng; ++j) hdev[j] = hs[g[j]]->d;
        CK(hipMemcpyAsync(ddev, hdev.data(), sizeof(Dev) * ng, hipMemcpyHostToDevice, s));
        std::vector<char> live(ng, 1);
        int nlive = ng;
        int64_t batch = 1;
        while (nlive > 0) {
            for (int j = 0; j < ng; ++j) {
                pdhg_t *h = hs[g[j]];
                const int64_t P = h->prm.check_period;
                int64_t nb = live[j] ? (kend[g[j]] - k[g[j]]) / P : 0;
                if (nb > batch) nb = batch;
                harg[j] = tiny_args(h, tol, (int)nb);
                harg[j].summary = dsum + 2 * j;
            }
            CK(hipMemcpyAsync(dargs, harg.data(), sizeof(TinyArgs) * ng, hipMemcpyHostToDevice, s));
            CK(launch_tiny_many(ddev, dargs, ng, pl, lds, s));
            for (int j = 0; j < ng; ++j) hs[g[j]]->fresh = false;
            CK(hipMemcpyAsync(hsum.data(), dsum, sizeof(long long) * 2 * ng,
                              hipMemcpyDeviceToHost, s));
            CK(hipStreamSynchronize(s));
            for (int j = 0; j < ng; ++j) {
                if (!live[j] || harg[j].blocks == 0) continue;
                const int32_t i = g[j];
                const long long f = hsum[2 * (size_t)j + 1];
                if ((f >> 16) & 1) return PDHG_E_NUMERICAL;
                // a converged handle stops at the check that converged
                const bool c = (f & 0xff) && ((f >> 8) & 0xff) > 0;
                k[i] = hsum[2 * (size_t)j];
                conv[i] = c;
                if (c || kend[i] - k[i] < hs[i]->prm.check_period) {
                    live[j] = 0;
                    --nlive;
                }
            }
            if (batch < kTinyBatchMax) batch *= 2;
        }
    }
    // the iterations after the last whole block, and the results
    for (int32_t i = 0; i < count; ++i) {
        pdhg_t *h = hs[i];
        if (!one_workgroup(h)) continue;
        bool c = conv[i];
        while (!c && k[i] < kend[i])
            if ((rc = solve_eager_step(h, &k[i], kend[i], tol, &t_host[i], &c))) return rc;
        DevState st;
        if ((rc = read_state(h, &st))) return rc;
        if ((rc = finish_result(h, st, out ? &out[i] : nullptr))) return rc;
        all_conv &= c;
    }
    return all_conv ? PDHG_OK : PDHG_NOT_CONVERGED;
}

// ---------------------------------------------------------------------
// tuning of the column slabs per matrix
// ---------------------------------------------------------------------
// slab count S of A (t = 0) or A' (t = 1), rebuilding the slabs; the
// recorded graph holds the old launches, so it is dropped
static int set_slabs(pdhg_t *h, int t, int S) {
    Dev &d = h->d;
    Slabs &sb = t == 0 ? d.slA : d.slT;
    if (S == sb.S) return PDHG_OK;
    if (S < 1 || S > h->slab_cap[t]) return PDHG_E_INVALID;
    const int gath = t == 0 ? d.n : d.m;
    h->g_valid = false;
    h->fresh = false;  // A'y of the last check was summed in the old layout
    sb.S = S;
    sb.W = (int)(((long long)gath + S - 1) / S);
    if (S == 1) return PDHG_OK;
    return t == 0 ? build_slabs(sb, d.rp, d.ci, d.v, d.nnz, d.nblkA, d.long_rows, h->stream)
                  : build_slabs(sb, d.trp, d.tci, d.tv, d.nnz, d.nblkT, d.long_rows, h->stream);
}

// mean time of one product A x (t = 0) or A'y (t = 1) of the current point,
// written to scratch vectors: the solver state is left alone
static int time_product(pdhg_t *h, int t, int iters, double *ms) {
    const Dev &d = h->d;
    hipStream_t s = h->stream;
    auto once = [&]() {
        if (t == 0) launch_spmv_A(d, d.x, d.gax, s);
        else launch_spmv_T(d, d.y, d.gaty, s);
    };
    once();  // warm-up
    hipEvent_t a = nullptr, b = nullptr;
    int rc = PDHG_OK;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = PDHG_E_HIP;
    if (rc == PDHG_OK && hipEventRecord(a, s) != hipSuccess) rc = PDHG_E_HIP;
    for (int i = 0; i < iters && rc == PDHG_OK; ++i) once();
    if (rc == PDHG_OK && hipEventRecord(b, s) != hipSuccess) rc = PDHG_E_HIP;
    if (rc == PDHG_OK) rc = last_error();
    float el = 0.f;
    if (rc == PDHG_OK && (hipEventSynchronize(b) != hipSuccess ||
                          hipEventElapsedTime(&el, a, b) != hipSuccess))
        rc = PDHG_E_HIP;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (rc == PDHG_OK) *ms = el / (double)iters;
    return rc;
}

// signature of a matrix for the tuning cache: sizes and 32 sampled row
// starts of A and of A' (FNV-1a)
static int matrix_signature(pdhg_t *h, uint64_t *sig) {
    const Dev &d = h->d;
    uint64_t f = 1469598103934665603ull;
    auto mix = [&](long long v) {
        for (int k = 0; k < 8; ++k) {
            f ^= (uint64_t)((v >> (8 * k)) & 0xff);
            f *= 1099511628211ull;
        }
    };
    mix(d.m);
    mix(d.n);
    mix(d.nnz);
    const int *arrs[2] = {d.rp, d.trp};
    const int rows[2] = {d.m, d.n};
    for (int t = 0; t < 2; ++t) {
        int v[32];
        for (int q = 0; q < 32; ++q)
            CK(hipMemcpyAsync(&v[q], arrs[t] + (long long)rows[t] * q / 31, sizeof(int),
                              hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
        for (int q = 0; q < 32; ++q) mix(v[q]);
    }
    *sig = f;
    return PDHG_OK;
}

struct TuneChoice {
    int slabs[2], lbias[2], threads[2];  // [0] A x, [1] A'y
};
static std::mutex g_tune_mu;
static std::map<uint64_t, TuneChoice> g_tune_cache;

static void set_lbias(pdhg_t *h, int t, int b) {
    int &cur = t == 0 ? h->d.lbA : h->d.lbT;
    if (cur != b) h->g_valid = h->fresh = false;  // the recorded block holds the old value
    cur = b;
}

static void set_threads(pdhg_t *h, int t, int wg) {
    int &cur = t == 0 ? h->d.swgA : h->d.swgT;
    if (cur != wg) h->g_valid = h->fresh = false;  // the recorded block holds the old launches
    cur = wg;
}

int pdhg_autotune(pdhg_t *h, int32_t iters, int32_t use_cache, pdhg_tune *out) {
    if (!h || iters < 1 || iters > 10000) return PDHG_E_INVALID;
    pdhg_tune r;
    memset(&r, 0, sizeof(r));
    int rc;
    uint64_t sig = 0;
    if ((rc = matrix_signature(h, &sig))) return rc;
    bool cached = false;
    TuneChoice choice{{h->d.slA.S, h->d.slT.S}, {h->d.lbA, h->d.lbT}, {h->d.swgA, h->d.swgT}};
    if (use_cache) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(sig);
        if (it != g_tune_cache.end()) {
            cached = true;
            choice = it->second;
        }
    }
    if (cached) {
        for (int t = 0; t < 2; ++t) {
            if ((rc = set_slabs(h, t, choice.slabs[t]))) return rc;
            set_lbias(h, t, choice.lbias[t]);
            set_threads(h, t, choice.threads[t]);
        }
        r.from_cache = 1;
    } else {
        int *tried[2] = {r.tried_A, r.tried_At};
        double *ms[2] = {r.ms_A, r.ms_At};
        int *ncand[2] = {&r.candidates_A, &r.candidates_At};
        double *msl[2] = {r.ms_lanes_A, r.ms_lanes_At};
        for (int t = 0; t < 2; ++t) {
            // 1. column slabs (when the gathered vector exceeds one L2),
            //    with the lanes rule as it is
            set_lbias(h, t, 0);
            int best = t == 0 ? h->d.slA.S : h->d.slT.S;
            if (h->slab_cap[t] > 1) {
                double bt = 0.0;
                for (int S = 1; S <= h->slab_cap[t] && *ncand[t] < 4; S <<= 1) {
                    double m = 0.0;
                    if ((rc = set_slabs(h, t, S)) || (rc = time_product(h, t, iters, &m)))
                        return rc;
                    tried[t][*ncand[t]] = S;
                    ms[t][*ncand[t]] = m;
                    ++*ncand[t];
                    if (*ncand[t] == 1 || m < bt) {
                        bt = m;
                        best = S;
                    }
                }
                if ((rc = set_slabs(h, t, best))) return rc;
            }
            choice.slabs[t] = best;
            // 2. lanes per row one power of two below, at and above the rule
            int bb = 0;
            double bl = 0.0;
            for (int k = 0; k < 3; ++k) {
                const int b = k - 1;
                set_lbias(h, t, b);
                double m = 0.0;
                if ((rc = time_product(h, t, iters, &m))) return rc;
                msl[t][k] = m;
                if (k == 0 || m < bl) {
                    bl = m;
                    bb = b;
                }
            }
            set_lbias(h, t, bb);
            choice.lbias[t] = bb;
            // 3. threads per workgroup: kWG or 128 (twice the entries per
            //    thread), with that slab count and lanes rule
            double *mst = t == 0 ? r.ms_threads_A : r.ms_threads_At;
            const int wgs[2] = {kWG, 128};
            int bw = kWG;
            double bwt = 0.0;
            for (int k = 0; k < 2; ++k) {
                set_threads(h, t, wgs[k]);
                double m = 0.0;
                if ((rc = time_product(h, t, iters, &m))) return rc;
                mst[k] = m;
                if (k == 0 || m < bwt) {
                    bwt = m;
                    bw = wgs[k];
                }
            }
            set_threads(h, t, bw);
            choice.threads[t] = bw;
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[sig] = choice;
    }
    CK(hipStreamSynchronize(h->stream));
    r.slabs_A = h->d.slA.S;
    r.slabs_At = h->d.slT.S;
    r.lanes_bias_A = h->d.lbA;
    r.lanes_bias_At = h->d.lbT;
    r.threads_A = h->d.swgA;
    r.threads_At = h->d.swgT;
    if (out) *out = r;
    return last_error();
}

int pdhg_set_schedule(pdhg_t *h, int32_t slabs_A, int32_t slabs_At, int32_t lanes_bias_A,
                      int32_t lanes_bias_At) {
    if (!h) return PDHG_E_INVALID;
    const int sl[2] = {slabs_A, slabs_At}, lb[2] = {lanes_bias_A, lanes_bias_At};
    for (int t = 0; t < 2; ++t) {
        const int S = sl[t];
        if (S < 1 || (S & (S - 1)) || S > h->slab_cap[t] || lb[t] < -1 || lb[t] > 1)
            return PDHG_E_INVALID;
    }
    for (int t = 0; t < 2; ++t) {
        const int rc = set_slabs(h, t, sl[t]);
        if (rc) return rc;
        set_lbias(h, t, lb[t]);
    }
    return last_error();
}

int pdhg_get_iterate(pdhg_t *h, int32_t which, double *x, double *y) {
    if (!h || which < 0 || which > 3 || !x || (h->d.m > 0 && !y)) return PDHG_E_INVALID;
    const Dev &d = h->d;
    if (d.permuted) {
        launch_copy_point(d, which, d.gx, y, h->stream);
        launch_gather(d.gx, d.cinv, d.n, x, h->stream);
    } else {
        launch_copy_point(d, which, x, y, h->stream);
    }
    return last_error();
}

int pdhg_set_iterate(pdhg_t *h, const double *x, const double *y) {
    if (!h || !x || (h->d.m > 0 && !y)) return PDHG_E_INVALID;
    h->fresh = false;
    const Dev &d = h->d;
    if (d.permuted) {
        launch_gather(x, d.cperm, d.n, d.gx, h->stream);
        launch_set_point(d, d.gx, y, h->stream);
    } else {
        launch_set_point(d, x, y, h->stream);
    }
    return last_error();
}

// --- checkpoint of the solver state (Algorithm 1's restart state) ----------
// Blob layout, each region 256-byte aligned: header, DevState (counters k,
// t, n, checks, rho_prev and the last check's results), then x, y, x0, y0,
// S_x, S_y, q = A x, x-bar, y-bar (the solution point when the average
// converged) in the library's internal column order, then the check log.
namespace {
constexpr uint64_t kStateMagic = 0x31415453474844ull;  // "DHGSTA1"
struct StateHeader {
    uint64_t magic;
    int64_t m, n, nnz;
    uint64_t sig;                 // matrix signature (sizes, sampled row starts)
    int32_t method, restart_mode, check_period, kkt_kind;
    double eta, omega;
    int64_t bytes;
};
struct StateLayout {
    size_t hdr, st, vec[9], log, total;
};
StateLayout state_layout(const Dev &d) {
    StateLayout L;
    size_t o = 0;
    L.hdr = o;
    o += al(sizeof(StateHeader));
    L.st = o;
    o += al(sizeof(DevState));
    const int64_t len[9] = {d.n, d.m, d.n, d.m, d.n, d.m, d.m, d.n, d.m};
    for (int q = 0; q < 9; ++q) {
        L.vec[q] = o;
        o += al(sizeof(double) * (size_t)(len[q] > 0 ? len[q] : 1));
    }
    L.log = o;
    o += al(sizeof(double) * (size_t)kLogCap * kRec);
    L.total = o;
    return L;
}
}  // namespace

size_t pdhg_state_bytes(pdhg_t *h) { return h ? state_layout(h->d).total : 0; }

int pdhg_get_state(pdhg_t *h, void *state, size_t bytes) {
    if (!h || !state) return PDHG_E_INVALID;
    const Dev &d = h->d;
    const StateLayout L = state_layout(d);
    if (bytes < L.total || ((uintptr_t)state & 255)) return PDHG_E_WORKSPACE;
    StateHeader hd{};
    hd.magic = kStateMagic;
    hd.m = d.m;
    hd.n = d.n;
    hd.nnz = d.nnz;
    int rc = matrix_signature(h, &hd.sig);
    if (rc) return rc;
    hd.method = h->prm.method;
    hd.restart_mode = h->prm.restart_mode;
    hd.check_period = h->prm.check_period;
    hd.kkt_kind = h->prm.kkt_kind;
    hd.eta = h->eta;
    hd.omega = d.omega;
    hd.bytes = (int64_t)L.total;
    char *b = (char *)state;
    CK(hipMemcpyAsync(b + L.hdr, &hd, sizeof(hd), hipMemcpyHostToDevice, h->stream));
    CK(hipMemcpyAsync(b + L.st, d.st, sizeof(DevState), hipMemcpyDeviceToDevice, h->stream));
    const double *src[9] = {d.x, d.y, d.x0, d.y0, d.sx, d.sy, d.q, d.xbar, d.ybar};
    const int64_t len[9] = {d.n, d.m, d.n, d.m, d.n, d.m, d.m, d.n, d.m};
    for (int q = 0; q < 9; ++q)
        if (len[q] > 0)
            CK(hipMemcpyAsync(b + L.vec[q], src[q], sizeof(double) * (size_t)len[q],
                              hipMemcpyDeviceToDevice, h->stream));
    CK(hipMemcpyAsync(b + L.log, d.log, sizeof(double) * (size_t)kLogCap * kRec,
                      hipMemcpyDeviceToDevice, h->stream));
    CK(hipStreamSynchronize(h->stream));  // the header came from host memory
    return PDHG_OK;
}

int pdhg_set_state(pdhg_t *h, const void *state, size_t bytes) {
    if (!h || !state) return PDHG_E_INVALID;
    h->fresh = false;
    Dev &d = h->d;
    const StateLayout L = state_layout(d);
    if (bytes < L.total || ((uintptr_t)state & 255)) return PDHG_E_WORKSPACE;
    const char *b = (const char *)state;
    StateHeader hd;
    CK(hipMemcpyAsync(&hd, b + L.hdr, sizeof(hd), hipMemcpyDeviceToHost, h->stream));
    CK(hipStreamSynchronize(h->stream));
    uint64_t sig = 0;
    int rc = matrix_signature(h, &sig);
    if (rc) return rc;
    if (hd.magic != kStateMagic || hd.m != d.m || hd.n != d.n || hd.nnz != d.nnz ||
        hd.sig != sig || hd.method != h->prm.method ||
        hd.restart_mode != h->prm.restart_mode || hd.check_period != h->prm.check_period ||
        hd.kkt_kind != h->prm.kkt_kind || hd.bytes != (int64_t)L.total ||
        !(hd.eta > 0.0) || !(hd.omega > 0.0))
        return PDHG_E_INVALID;
    // the step sizes belong to the state: a resumed run takes the same steps
    if (hd.eta != h->eta || hd.omega != d.omega) {
        h->eta = hd.eta;
        h->prm.omega = hd.omega;
        d.omega = hd.omega;
        h->tau = hd.eta / hd.omega;
        h->sigma = hd.eta * hd.omega;
        h->g_valid = false;  // the recorded block holds the old step sizes
    }
    CK(hipMemcpyAsync(d.st, b + L.st, sizeof(DevState), hipMemcpyDeviceToDevice, h->stream));
    double *dst[9] = {d.x, d.y, d.x0, d.y0, d.sx, d.sy, d.q, d.xbar, d.ybar};
    const int64_t len[9] = {d.n, d.m, d.n, d.m, d.n, d.m, d.m, d.n, d.m};
    for (int q = 0; q < 9; ++q)
        if (len[q] > 0)
            CK(hipMemcpyAsync(dst[q], b + L.vec[q], sizeof(double) * (size_t)len[q],
                              hipMemcpyDeviceToDevice, h->stream));
    CK(hipMemcpyAsync(d.log, b + L.log, sizeof(double) * (size_t)kLogCap * kRec,
                      hipMemcpyDeviceToDevice, h->stream));
    CK(hipStreamSynchronize(h->stream));
    return PDHG_OK;
}

size_t pdhg_weight_search_workspace_bytes(int64_t m, int64_t n, int32_t count) {
    if (m < 0 || n < 1 || count < 1 || count > kWMax) return 0;
    return wsearch_bytes(m, n, count);
}

int pdhg_weight_search(pdhg_t *h, const double *omega, int32_t count, int64_t iters,
                       void *workspace, size_t workspace_bytes, pdhg_kkt *kkt,
                       int32_t *best, double *x_out, double *y_out) {
    if (!h || !omega || !kkt || count < 1 || count > kWMax || iters < 0) return PDHG_E_INVALID;
    for (int w = 0; w < count; ++w)
        if (!(omega[w] > 0.0) || !isfinite(omega[w])) return PDHG_E_INVALID;
    h->fresh = false;
    const Dev &d = h->d;
    if (!workspace || ((uintptr_t)workspace & 255u) ||
        workspace_bytes < wsearch_bytes(d.m, d.n, count))
        return PDHG_E_WORKSPACE;
    WArgs a;
    memset(&a, 0, sizeof(a));
    a.m = d.m;
    a.n = d.n;
    a.W = count;
    a.egm = h->prm.method == PDHG_METHOD_EGM ? 1 : 0;
    a.rp = d.rp;
    a.ci = d.ci;
    a.v = d.v;
    a.trp = d.trp;
    a.tci = d.tci;
    a.tv = d.tv;
    a.c = d.c;
    a.b = d.b;
    a.l = d.l;
    a.u = d.u;
    a.kind = d.kind;
    a.st = d.st;
    a.cinv = d.permuted ? d.cinv : nullptr;
    wsearch_carve((char *)workspace, d.m, d.n, count, &a);
    for (int w = 0; w < count; ++w) {
        a.tau[w] = h->eta / omega[w];
        a.sigma[w] = h->eta * omega[w];
    }
    hipStream_t s = h->stream;
    launch_w_init(a, s);
    int rc = last_error();
    if (rc) return rc;
    // blocks of iterations replayed as one graph, the rest launched directly
    const int64_t blk = 50;
    if (iters >= 2 * blk) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        CK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        for (int64_t i = 0; i < blk; ++i) launch_w_iter(a, h->cap);
        CK(hipStreamEndCapture(h->cap, &g));
        hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return PDHG_E_HIP;
        for (int64_t i = 0; i + blk <= iters && e == hipSuccess; i += blk)
            e = hipGraphLaunch(ge, s);
        (void)hipStreamSynchronize(s);
        (void)hipGraphExecDestroy(ge);
        if (e != hipSuccess) return PDHG_E_HIP;
        for (int64_t i = iters - iters % blk; i < iters; ++i) launch_w_iter(a, s);
    } else {
        for (int64_t i = 0; i < iters; ++i) launch_w_iter(a, s);
    }
    launch_w_kkt(a, s);
    if (x_out || y_out) launch_w_extract(a, x_out, d.m > 0 ? y_out : nullptr, s);
    if ((rc = last_error())) return rc;
    double out[kWMax * 8];
    CK(hipMemcpyAsync(out, a.out, sizeof(double) * 8 * count, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    int32_t bw = -1;
    for (int w = 0; w < count; ++w) {
        const double *o = out + 8 * w;
        pdhg_kkt &k = kkt[w];
        k.kkt_rel = o[0];
        k.primal_res = o[1];
        k.dual_res = o[2];
        k.pobj = o[3];
        k.dobj = o[4];
        k.kkt_paper_abs = o[5];
        k.kkt_max_abs = o[6];
        k.kkt = o[5];
        if (!isnan(o[5]) && (bw < 0 || o[5] < out[8 * bw + 5])) bw = w;
    }
    if (best) *best = bw;
    return PDHG_OK;
}

int pdhg_set_primal_weight(pdhg_t *h, double omega) {
    if (!h || !(omega > 0.0) || !isfinite(omega)) return PDHG_E_INVALID;
    h->prm.omega = omega;
    h->d.omega = omega;
    h->tau = h->eta / omega;
    h->sigma = h->eta * omega;
    h->g_valid = false;  // the recorded block holds the old step sizes
    h->fresh = false;
    launch_init_point(h->d, h->stream);
    return last_error();
}

int pdhg_get_info(pdhg_t *h, pdhg_info *out) {
    if (!h || !out) return PDHG_E_INVALID;
    DevState hs;
    int rc = read_state(h, &hs);
    if (rc) return rc;
    out->eta = h->eta;
    out->tau = h->tau;
    out->sigma = h->sigma;
    out->sigma_max = h->sigma_max;
    out->k = hs.k;
    out->t = hs.t;
    out->restarts = hs.restarts;
    out->rho_prev = hs.rho_prev;
    out->checks = hs.checks;
    out->power_iters_used = h->pw_used;
    out->one_workgroup = 0;
    if (h->tiny.ok && h->prm.method == PDHG_METHOD_PDHG &&
        h->prm.restart_mode != PDHG_RESTART_FIXED)
        out->one_workgroup = h->tiny.reg ? (h->tiny.ov ? 3 : 1) : 2;
    out->bound_classes = h->d.nbcls;
    return PDHG_OK;
}

int pdhg_get_check_log(pdhg_t *h, pdhg_check_record *out, int64_t max, int64_t *count) {
    if (!h || max < 0 || (max > 0 && !out)) return PDHG_E_INVALID;
    DevState hs;
    int rc = read_state(h, &hs);
    if (rc) return rc;
    int64_t have = hs.checks < kLogCap ? hs.checks : kLogCap;
    int64_t nret = have < max ? have : max;
    for (int64_t q = 0; q < nret; ++q) {
        int64_t idx = hs.checks - nret + q;
        const double *src = h->d.log + (size_t)(idx % kLogCap) * kRec;
        CK(hipMemcpyAsync(out[q].v, src, sizeof(double) * kRec, hipMemcpyDeviceToHost, h->stream));
    }
    CK(hipStreamSynchronize(h->stream));
    if (count) *count = nret;
    return PDHG_OK;
}

int pdhg_matvec(pdhg_t *h, int32_t transpose, const double *in, double *out) {
    if (!h || !in || !out || (transpose != 0 && transpose != 1)) return PDHG_E_INVALID;
    const Dev &d = h->d;
    if (!d.permuted) {
        if (transpose) launch_spmv_T(d, in, out, h->stream);
        else launch_spmv_A(d, in, out, h->stream);
    } else if (transpose) {
        launch_spmv_T(d, in, d.gaty, h->stream);
        launch_gather(d.gaty, d.cinv, d.n, out, h->stream);
    } else {
        launch_gather(in, d.cperm, d.n, d.gx, h->stream);
        launch_spmv_A(d, d.gx, out, h->stream);
    }
    return last_error();
}

int pdhg_get_transpose(pdhg_t *h, int32_t *t_row_ptr, int32_t *t_col_idx, double *t_vals,
                       int32_t *perm) {
    if (!h || !t_row_ptr) return PDHG_E_INVALID;
    const Dev &d = h->d;
    if (d.permuted) {
        launch_transpose_out(d, t_row_ptr, t_col_idx, t_vals, perm, h->stream);
        return last_error();
    }
    CK(hipMemcpyAsync(t_row_ptr, d.trp, sizeof(int) * ((size_t)d.n + 1), hipMemcpyDeviceToDevice,
                      h->stream));
    if (d.nnz > 0) {
        if (t_col_idx)
            CK(hipMemcpyAsync(t_col_idx, d.tci, sizeof(int) * (size_t)d.nnz,
                              hipMemcpyDeviceToDevice, h->stream));
        if (t_vals)
            CK(hipMemcpyAsync(t_vals, d.tv, sizeof(double) * (size_t)d.nnz,
                              hipMemcpyDeviceToDevice, h->stream));
        if (perm)
            CK(hipMemcpyAsync(perm, d.perm, sizeof(int) * (size_t)d.nnz, hipMemcpyDeviceToDevice,
                              h->stream));
    }
    return PDHG_OK;
}

int pdhg_time_iterations(pdhg_t *h, int64_t iters, double *ms_primal, double *ms_dual) {
    if (!h || iters < 1 || iters > 100000) return PDHG_E_INVALID;
    launch_reset_done(h->d, h->stream);
    // products per iteration: A'y then A x (PDHG); A'y, A x, A'y~, A x~ (EGM)
    const bool egm = h->prm.method == PDHG_METHOD_EGM;
    const int nseg = egm ? 4 : 2;
    const int64_t ne = nseg * iters + 1;
    hipEvent_t *ev = new (std::nothrow) hipEvent_t[ne];
    if (!ev) return PDHG_E_HIP;
    int64_t made = 0;
    int rc = PDHG_OK;
    for (; made < ne; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) {
            rc = PDHG_E_HIP;
            break;
        }
    if (rc == PDHG_OK) {
        hipStream_t s = h->stream;
        if (hipEventRecord(ev[0], s) != hipSuccess) rc = PDHG_E_HIP;
        for (int64_t i = 0; i < iters && rc == PDHG_OK; ++i) {
            for (int p = 0; p < nseg && rc == PDHG_OK; ++p) {
                if (egm) launch_egm(h->d, h->tau, h->sigma, p, s);
                else if (p == 0) launch_primal(h->d, h->tau, sum_mode(i, iters), s);
                else launch_dual(h->d, h->sigma, sum_mode(i, iters), s);
                if (hipEventRecord(ev[nseg * i + p + 1], s) != hipSuccess) rc = PDHG_E_HIP;
            }
        }
        if (rc == PDHG_OK) rc = last_error();
        if (rc == PDHG_OK && hipStreamSynchronize(s) != hipSuccess) rc = PDHG_E_HIP;
        double tp = 0.0, td = 0.0;
        for (int64_t q = 0; q + 1 < ne && rc == PDHG_OK; ++q) {
            float a = 0.f;
            if (hipEventElapsedTime(&a, ev[q], ev[q + 1]) != hipSuccess) rc = PDHG_E_HIP;
            if ((q % nseg) % 2 == 0) tp += a;
            else td += a;
        }
        if (rc == PDHG_OK) {
            if (ms_primal) *ms_primal = tp / (double)iters;
            if (ms_dual) *ms_dual = td / (double)iters;
        }
    }
    for (int64_t q = 0; q < made; ++q) (void)hipEventDestroy(ev[q]);
    delete[] ev;
    return rc;
}

// mean time of `reps` launches enqueued on s by `launch`, in ms
}  // extern "C"
template <class F>
static int time_launches(hipStream_t s, int32_t reps, F launch, double *ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PDHG_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = PDHG_E_HIP;
    if (rc == PDHG_OK) {
        launch();  // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) rc = PDHG_E_HIP;
        for (int32_t r = 0; r < reps && rc == PDHG_OK; ++r) launch();
        if (rc == PDHG_OK && hipEventRecord(e1, s) != hipSuccess) rc = PDHG_E_HIP;
        if (rc == PDHG_OK) rc = last_error();
        if (rc == PDHG_OK && hipEventSynchronize(e1) != hipSuccess) rc = PDHG_E_HIP;
        float a = 0.f;
        if (rc == PDHG_OK && hipEventElapsedTime(&a, e0, e1) != hipSuccess) rc = PDHG_E_HIP;
        if (rc == PDHG_OK && ms) *ms = a / (double)reps;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

extern "C" {
int pdhg_time_copy(const double *src, double *dst, int64_t n, int32_t reps, void *stream,
                   double *ms) {
    if (!src || !dst || n < 1 || reps < 1 || reps > 1000 || ((uintptr_t)src & 31) ||
        ((uintptr_t)dst & 31))
        return PDHG_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    return time_launches(s, reps, [&] { launch_copy_yard(src, dst, n, s); }, ms);
}

int pdhg_time_gather(const int32_t *idx, const double *val, const double *x, double *out,
                     int64_t n, int32_t reps, void *stream, double *ms) {
    if (!idx || !val || !x || !out || n < 1 || n > 0x7fffffffLL || reps < 1 || reps > 1000)
        return PDHG_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    return time_launches(s, reps, [&] { launch_gather_yard(idx, val, x, out, n, s); }, ms);
}

int64_t pdhg_gather_only_outputs(int64_t n) {
    if (n < 1 || n > 0x7fffffffLL) return 0;
    return gather_only_outputs(n);
}

int pdhg_time_gather_only(const int32_t *idx, int64_t n, const double *x, int64_t xlen,
                          double *out, int32_t reps, void *stream, double *ms) {
    if (!x || !out || n < 1 || n > 0x7fffffffLL || reps < 1 || reps > 1000 || xlen < 1 ||
        xlen > 0x7fffffffLL)
        return PDHG_E_INVALID;
    int lg = 0;
    if (!idx) {
        if (xlen < 2 || (xlen & (xlen - 1))) return PDHG_E_INVALID;
        while ((1ll << lg) < xlen) ++lg;
    }
    hipStream_t s = (hipStream_t)stream;
    return time_launches(s, reps, [&] { launch_gather_only(idx, x, n, lg, out, s); }, ms);
}

size_t pdhg_trust_region_workspace_bytes(int64_t N) {
    if (N < 0 || N > 0x7fffffffLL) return 0;
    return al(sizeof(TRState)) + tr_work_bytes(N);
}

int pdhg_linear_trust_region(int64_t N, const double *a, const double *d, double r,
                             void *workspace, size_t workspace_bytes, void *stream, double *value,
                             double *lambda) {
    if (N < 0 || N > 0x7fffffffLL || isnan(r) || (N > 0 && (!a || !d))) return PDHG_E_INVALID;
    const size_t need = pdhg_trust_region_workspace_bytes(N);
    if (!workspace || ((uintptr_t)workspace & 255u) || workspace_bytes < need)
        return PDHG_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    TRState *ts = (TRState *)ws;
    TRWork w;
    carve_tr(ws + al(sizeof(TRState)), N, &w);
    launch_tr_raw(N, a, d, r, w, ts, s);
    int rc = last_error();
    if (rc) return rc;
    TRState hts;
    CK(hipMemcpyAsync(&hts, ts, sizeof(TRState), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (hts.nan_seen) return PDHG_E_INVALID;
    if (value) *value = hts.value;
    if (lambda) *lambda = hts.lam;
    return PDHG_OK;
}

}  // extern "C"

// --- the same trust region with library-owned scratch ---------------------
// For callers that cannot allocate device memory.  The scratch lives in a
// file-scope device array; host code must not pass the array's name to a
// kernel (in host code it is a stand-in, not a device address): each device
// holds its own copy, whose address hipGetSymbolAddress gives once per
// device, with that device current.
namespace {
constexpr size_t kTrStaticBytes = 14u << 20;  // holds the scratch of PDHG_TR_STATIC_MAX_N
static __device__ __align__(256) unsigned char scratch[kTrStaticBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // per device: the array's device address

// device address of the current device's copy of `scratch` (nullptr on
// failure); set up on the first call on each device
void *device_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {
int pdhg_linear_trust_region_static(int64_t N, const double *a, const double *d, double r,
                                    void *stream, double *value, double *lambda) {
    if (N < 0 || N > PDHG_TR_STATIC_MAX_N || isnan(r) || (N > 0 && (!a || !d)))
        return PDHG_E_INVALID;
    const size_t need = pdhg_trust_region_workspace_bytes(N);
    if (need == 0 || need > kTrStaticBytes) return PDHG_E_WORKSPACE;
    void *ws = device_scratch();
    if (!ws) return PDHG_E_HIP;
    // every value the kernels read is written by them first (k_tr_arm
    // clears the first histograms; the later levels clear their own), so
    // what an earlier call left in the array does not matter
    return pdhg_linear_trust_region(N, a, d, r, ws, kTrStaticBytes, stream, value, lambda);
}
}  // extern "C"
