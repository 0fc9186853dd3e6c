// Primal-weight search (Section 7, experimental setup): W copies of
// non-restarted PDHG (or extragradient) that differ only in the primal
// weight omega_w (primal step eta / omega_w, dual step eta * omega_w), run
// side by side so that every product streams A or A' once for all W copies.
//
// Vectors are stored interleaved, [row][W]: the W values a gathered entry
// needs are adjacent (W <= 16 doubles, one or two cache lines), so the
// gather cost of an SpMV is paid once per entry instead of once per copy.
// A group of 16 lanes works on one row of A or A'; lane w < W owns copy w.
#include "pdhg_device.h"

namespace pdhg {

constexpr int kLanesW = 16;                 // lanes per row (>= kWMax)
constexpr int kRowsPerBlockW = kWG / kLanesW;
static_assert(kWMax <= kLanesW, "one lane per copy");

size_t wsearch_bytes(int64_t m, int64_t n, int W) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t n1 = (size_t)n, m1 = (size_t)(m > 0 ? m : 1), w = (size_t)W;
    return al(sizeof(double) * n1 * w) * 3 + al(sizeof(double) * m1 * w) * 3 +
           al(sizeof(double) * (size_t)kRedBlocks * kWMax * kWSums) +
           al(sizeof(double) * kWMax * 8);
}

void wsearch_carve(char *ws, int64_t m, int64_t n, int W, WArgs *a) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t n1 = (size_t)n, m1 = (size_t)(m > 0 ? m : 1), w = (size_t)W;
    size_t o = 0;
    a->x = (double *)(ws + o);
    o += al(sizeof(double) * n1 * w);
    a->aty = (double *)(ws + o);
    o += al(sizeof(double) * n1 * w);
    a->y = (double *)(ws + o);
    o += al(sizeof(double) * m1 * w);
    a->q = (double *)(ws + o);
    o += al(sizeof(double) * m1 * w);
    a->xt = (double *)(ws + o);
    o += al(sizeof(double) * n1 * w);
    a->yt = (double *)(ws + o);
    o += al(sizeof(double) * m1 * w);
    a->part = (double *)(ws + o);
    o += al(sizeof(double) * (size_t)kRedBlocks * kWMax * kWSums);
    a->out = (double *)(ws + o);
}

// What a row's W sums feed:
//   0: x+ = proj_X(x - tau_w (c - A'y))            (row of A', eq. PDHG-update)
//   1: y+ = proj_Y(y + sigma_w (b - (2 A x+ - q))), q = A x+   (row of A)
//   2: aty = A'y                                   (row of A')
//   3: q = A x                                     (row of A)
// and for the extragradient method (eq. extra-gradient-update):
//   4: x~ = proj_X(x - tau_w (c - A'y))            (row of A')
//   5: y~ = proj_Y(y - sigma_w (A x - b))          (row of A)
//   6: x+ = proj_X(x - tau_w (c - A'y~))           (row of A', gathers y~)
//   7: y+ = proj_Y(y - sigma_w (A x~ - b))         (row of A, gathers x~)
template <int Mode>
__global__ __launch_bounds__(kWG) void k_w_spmv(WArgs a) {
    constexpr bool T = (Mode == 0 || Mode == 2 || Mode == 4 || Mode == 6);
    const int row = blockIdx.x * kRowsPerBlockW + (int)(threadIdx.x / kLanesW);
    const int w = threadIdx.x % kLanesW;
    const int rows = T ? a.n : a.m;
    if (row >= rows || w >= a.W) return;
    const int *__restrict__ rp = T ? a.trp : a.rp;
    const int *__restrict__ ci = T ? a.tci : a.ci;
    const double *__restrict__ v = T ? a.tv : a.v;
    const double *__restrict__ vin =
        Mode == 6 ? a.yt : (Mode == 7 ? a.xt : (T ? a.y : a.x));
    const int W = a.W;
    const int p0 = rp[row], p1 = rp[row + 1];
    double s = 0.0;
    int p = p0;
    // four independent gathers in flight; the sum keeps the entry order
    for (; p + 4 <= p1; p += 4) {
        const int c0 = ci[p], c1 = ci[p + 1], c2 = ci[p + 2], c3 = ci[p + 3];
        const double v0 = v[p], v1 = v[p + 1], v2 = v[p + 2], v3 = v[p + 3];
        const double g0 = vin[(size_t)c0 * W + w], g1 = vin[(size_t)c1 * W + w];
        const double g2 = vin[(size_t)c2 * W + w], g3 = vin[(size_t)c3 * W + w];
        s += v0 * g0;
        s += v1 * g1;
        s += v2 * g2;
        s += v3 * g3;
    }
    for (; p < p1; ++p) s += v[p] * vin[(size_t)ci[p] * W + w];
    const size_t e = (size_t)row * W + w;
    if (Mode == 0) {
        double xn = a.x[e] - a.tau[w] * (a.c[row] - s);
        const double lo = a.l[row], hi = a.u[row];
        if (xn < lo) xn = lo;
        if (xn > hi) xn = hi;
        a.x[e] = xn;
    } else if (Mode == 1) {
        double yn = a.y[e] + a.sigma[w] * (a.b[row] - (2.0 * s - a.q[e]));
        if (a.kind && a.kind[row] && yn < 0.0) yn = 0.0;
        a.y[e] = yn;
        a.q[e] = s;
    } else if (Mode == 2) {
        a.aty[e] = s;
    } else if (Mode == 3) {
        a.q[e] = s;
    } else if (Mode == 4 || Mode == 6) {
        double xn = a.x[e] - a.tau[w] * (a.c[row] - s);
        const double lo = a.l[row], hi = a.u[row];
        if (xn < lo) xn = lo;
        if (xn > hi) xn = hi;
        if (Mode == 4) a.xt[e] = xn;
        else a.x[e] = xn;
    } else {
        double yn = a.y[e] - a.sigma[w] * (s - a.b[row]);
        if (a.kind && a.kind[row] && yn < 0.0) yn = 0.0;
        if (Mode == 5) a.yt[e] = yn;
        else a.y[e] = yn;
    }
}

// x = proj_X(0), y = 0 for every copy
__global__ void k_w_init(WArgs a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nx = (long long)a.n * a.W, ny = (long long)a.m * a.W;
    if (i < nx) {
        const int j = (int)(i / a.W);
        double v = 0.0;
        if (v < a.l[j]) v = a.l[j];
        if (v > a.u[j]) v = a.u[j];
        a.x[i] = v;
    }
    if (i < ny) a.y[i] = 0.0;
}

template <int Mode>
static void w_spmv(const WArgs &a, hipStream_t s) {
    const int rows = (Mode == 0 || Mode == 2 || Mode == 4 || Mode == 6) ? a.n : a.m;
    if (rows == 0) return;
    hipLaunchKernelGGL(k_w_spmv<Mode>, dim3(div_up(rows, kRowsPerBlockW)), dim3(kWG), 0, s, a);
}

void launch_w_init(const WArgs &a, hipStream_t s) {
    const long long mx = (long long)(a.n > a.m ? a.n : a.m) * a.W;
    hipLaunchKernelGGL(k_w_init, dim3(div_up(mx, kWG)), dim3(kWG), 0, s, a);
    w_spmv<3>(a, s);
}

void launch_w_iter(const WArgs &a, hipStream_t s) {
    if (a.egm) {
        w_spmv<4>(a, s);
        w_spmv<5>(a, s);
        w_spmv<6>(a, s);
        w_spmv<7>(a, s);
        return;
    }
    w_spmv<0>(a, s);
    w_spmv<1>(a, s);
}

// KKT sums of copy w = blockIdx.y (the formulas of the single-LP check)
__global__ __launch_bounds__(kWG) void k_w_kkt_partials(WArgs a) {
    __shared__ double sh[4 * kWSums];
    const int w = blockIdx.y, W = a.W;
    double v[kWSums];
#pragma unroll
    for (int k = 0; k < kWSums; ++k) v[k] = 0.0;
    const long long N = (long long)a.n + a.m;
    const long long stride = (long long)gridDim.x * kWG;
    for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < N; i += stride) {
        if (i < a.n) {
            const int j = (int)i;
            const double cj = a.c[j], lj = a.l[j], uj = a.u[j];
            const double xp = a.x[(size_t)j * W + w];
            const double rc = cj - a.aty[(size_t)j * W + w];
            const bool lf = isfinite(lj), uf = isfinite(uj);
            double lam;
            if (lf && uf) lam = rc;
            else if (lf) lam = rc > 0.0 ? rc : 0.0;
            else if (uf) lam = rc < 0.0 ? rc : 0.0;
            else lam = 0.0;
            const double dr = rc - lam;
            v[1] += dr * dr;
            double dob = 0.0;
            if (lam > 0.0) dob += lj * lam;
            if (lam < 0.0) dob += uj * lam;
            v[3] += dob;
            v[2] += cj * xp;
            double bv = 0.0;
            if (xp < lj) bv = lj - xp;
            if (xp > uj) bv = xp - uj;
            v[4] += bv * bv;
        } else {
            const int r = (int)(i - a.n);
            const double br = a.b[r];
            const bool ge = a.kind && a.kind[r];
            const double yr = a.y[(size_t)r * W + w];
            double p = br - a.q[(size_t)r * W + w];
            if (ge && p < 0.0) p = 0.0;
            v[0] += p * p;
            v[3] += br * yr;
            if (ge && yr < 0.0) v[4] += yr * yr;
        }
    }
    block_sums<kWSums>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kWSums; ++k)
            a.part[((size_t)w * kRedBlocks + blockIdx.x) * kWSums + k] = v[k];
    }
}

// out[w][0..7] = kkt_rel, |p|, |d|, pobj, dobj, paper_abs, max_abs, finite
__global__ __launch_bounds__(kWG) void k_w_kkt_final(WArgs a, int nb) {
    __shared__ double sh[4 * kWSums];
    const int w = blockIdx.x;
    double S[kWSums];
    reduce_partials<kWSums>(a.part + (size_t)w * kRedBlocks * kWSums, nb, kWSums, S, sh);
    if (threadIdx.x == 0) {
        const double pres = sqrt(S[0]), dres = sqrt(S[1]);
        const double pobj = S[2], dobj = S[3];
        const double gap = pobj - dobj;
        const double rel_p = pres / (1.0 + sqrt(a.st->nb2));
        const double rel_d = dres / (1.0 + sqrt(a.st->nc2));
        const double rel_g = fabs(gap) / (1.0 + fabs(pobj) + fabs(dobj));
        double rel = rel_p;
        if (rel_d > rel) rel = rel_d;
        if (rel_g > rel) rel = rel_g;
        const double gpos = gap > 0.0 ? gap : 0.0;
        double mx = pres;
        if (dres > mx) mx = dres;
        if (fabs(gap) > mx) mx = fabs(gap);
        double *o = a.out + (size_t)w * 8;
        o[0] = rel;
        o[1] = pres;
        o[2] = dres;
        o[3] = pobj;
        o[4] = dobj;
        o[5] = sqrt(S[4] + S[0] + S[1] + gpos * gpos);
        o[6] = mx;
        bool fin = true;
        for (int k = 0; k < kWSums; ++k) fin &= (bool)isfinite(S[k]);
        o[7] = fin ? 1.0 : 0.0;
    }
}

void launch_w_kkt(const WArgs &a, hipStream_t s) {
    if (a.egm) w_spmv<3>(a, s);  // the extragradient iterations keep no A x
    w_spmv<2>(a, s);
    int g = div_up((long long)a.n + a.m, kWG);
    if (g > kRedBlocks) g = kRedBlocks;
    hipLaunchKernelGGL(k_w_kkt_partials, dim3(g, a.W), dim3(kWG), 0, s, a);
    hipLaunchKernelGGL(k_w_kkt_final, dim3(a.W), dim3(kWG), 0, s, a, g);
}

// copy w of the interleaved iterates into plain vectors (x_out[w n + j]),
// columns back in the caller's order
__global__ void k_w_extract(WArgs a, double *xo, double *yo) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nx = (long long)a.n * a.W, ny = (long long)a.m * a.W;
    if (xo && i < nx) {
        const long long w = i / a.n, j = i % a.n;
        const long long q = a.cinv ? a.cinv[j] : j;
        xo[i] = a.x[q * a.W + w];
    }
    if (yo && i < ny) {
        const long long w = i / a.m, r = i % a.m;
        yo[i] = a.y[r * a.W + w];
    }
}

void launch_w_extract(const WArgs &a, double *xo, double *yo, hipStream_t s) {
    const long long mx = (long long)(a.n > a.m ? a.n : a.m) * a.W;
    hipLaunchKernelGGL(k_w_extract, dim3(div_up(mx, kWG)), dim3(kWG), 0, s, a, xo, yo);
}

}  // namespace pdhg
