// Plan-time kernels: Gauss-Legendre nodes/weights and the P̄_n^m tables.
//
// Everything here runs in FP64 on the device.  The nodes are Newton roots of
// P_nlat polished in double-double so that each stored node is the double
// nearest to the true root; the tables follow the standard three-term
// recurrence in n for each fixed m from the sectoral seed P̄_m^m.  The paper
// (Section 3.1.1) keeps all such data resident on the GPU.
#include <cmath>

#include "shtx_internal.h"

namespace shtx {

namespace {

// ---------------------------------------------------------------------------
// double-double arithmetic (hi + lo, |lo| <= ulp(hi) / 2)
//
// The error-free transformations below need every product rounded exactly
// once where it is written: contracting a product into a later add (which the
// GPU compiler does by default) makes the error terms inconsistent, so
// contraction is off from here to the end of the node kernel.
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
struct dd {
    double hi, lo;
};

__device__ inline dd quick_two_sum(double a, double b)
{
    double s = a + b;
    return {s, b - (s - a)};
}

__device__ inline dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

__device__ inline dd two_prod(double a, double b)
{
    double p = a * b;
    return {p, fma(a, b, -p)};
}

__device__ inline dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

__device__ inline dd dd_neg(dd a) { return {-a.hi, -a.lo}; }

__device__ inline dd dd_mul(dd a, dd b)
{
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}

__device__ inline dd dd_mul_d(dd a, double b)
{
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}

__device__ inline dd dd_div(dd a, dd b)
{
    double q1 = a.hi / b.hi;
    dd r = dd_add(a, dd_neg(dd_mul_d(b, q1)));
    double q2 = r.hi / b.hi;
    r = dd_add(r, dd_neg(dd_mul_d(b, q2)));
    double q3 = r.hi / b.hi;
    dd q = quick_two_sum(q1, q2);
    return dd_add(q, dd{q3, 0.0});
}

// P_n(x) and P_{n-1}(x) (unnormalised Legendre polynomials) in double-double
// at a double-double abscissa, by l P_l = (2l-1) x P_{l-1} - (l-1) P_{l-2}.
__device__ void legendre_dd(int n, dd x, dd *pn, dd *pn1)
{
    dd p0 = {1.0, 0.0}, p1 = x;
    for (int l = 2; l <= n; ++l) {
        dd t = dd_mul_d(dd_mul(p1, x), (double)(2 * l - 1));
        t = dd_add(t, dd_neg(dd_mul_d(p0, (double)(l - 1))));
        dd p2 = dd_div(t, dd{(double)l, 0.0});
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *pn1 = p0;
}

// P'_n(x) = n (x P_n - P_{n-1}) / (x^2 - 1) in double-double.
__device__ dd dlegendre_dd(int n, dd x, dd pn, dd pn1)
{
    dd num = dd_mul_d(dd_add(dd_mul(x, pn), dd_neg(pn1)), (double)n);
    dd den = dd_add(dd_mul(x, x), dd{-1.0, 0.0});
    return dd_div(num, den);
}

// One thread per northern node j < nlat / 2.
__global__ void k_gauss_nodes(int nlat, double *mu, double *w)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nlat / 2) return;
    double x = cos(M_PI * (j + 0.75) / (nlat + 0.5));
    for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int l = 2; l <= nlat; ++l) {
            double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
            p0 = p1;
            p1 = p2;
        }
        double dp = nlat * (x * p1 - p0) / (x * x - 1.0);
        double dx = p1 / dp;
        x -= dx;
        if (fabs(dx) < 1e-16) break;
    }
    // Two Newton steps in double-double; the normalised hi word is then the
    // double nearest to the root.
    dd r = {x, 0.0};
    for (int it = 0; it < 2; ++it) {
        dd pn, pn1;
        legendre_dd(nlat, r, &pn, &pn1);
        dd dp = dlegendre_dd(nlat, r, pn, pn1);
        r = dd_add(r, dd_neg(dd_div(pn, dp)));
    }
    dd pn, pn1;
    legendre_dd(nlat, r, &pn, &pn1);
    dd dp = dlegendre_dd(nlat, r, pn, pn1);
    // w = 2 / ((1 - x)(1 + x) P'(x)^2) at the double-double root
    dd omx = dd_add(dd{1.0, 0.0}, dd_neg(r));
    dd opx = dd_add(dd{1.0, 0.0}, r);
    dd den = dd_mul(dd_mul(omx, opx), dd_mul(dp, dp));
    dd wq = dd_div(dd{2.0, 0.0}, den);
    mu[j] = r.hi;
    w[j] = wq.hi;
    mu[nlat - 1 - j] = -r.hi;
    w[nlat - 1 - j] = wq.hi;
}

#pragma clang fp contract(fast)

// Sectoral seeds P̄_m^m(mu_j) = prod_{k<=m} sqrt((2k+1)/(2k)) s_j, one thread per
// northern ring, s_j = sqrt((1 - mu_j)(1 + mu_j)), kept as q 2^E with q in
// [1/2, 1) (frexp after every factor): near the poles the product leaves the
// double range for large m (m log10(1/s) > 300) while the recurrence in n can
// bring P̄_n^m back to order one before n reaches the truncation (TCo1999).
__global__ void k_sectoral(int nl, int trunc, const double *mu, double *diag, int *diag_e)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nl) return;
    double x = mu[j];
    double s = sqrt((1.0 - x) * (1.0 + x));
    double q = 1.0;
    int E = 0;
    double *d = diag + (int64_t)j * (trunc + 1);
    int *de = diag_e + (int64_t)j * (trunc + 1);
    d[0] = 1.0;
    de[0] = 0;
    for (int k = 1; k <= trunc; ++k) {
        int e;
        q = frexp(q * (sqrt((2.0 * k + 1.0) / (2.0 * k)) * s), &e);
        E += e;
        d[k] = q;
        de[k] = E;
    }
}

__device__ inline unsigned short bf16_rne(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ inline float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Column recurrence over n for one (m, ring).  MODE 0: per-m max |P̄| only;
// MODE 1: store FP64; MODE 2: store FP32; MODE 3: store split BF16 hi + lo
// scaled by 2^e_m, e_m putting the block's largest entry in [1/2, 1); MODE 4:
// store split IEEE half hi + lo scaled by 2^e_m, the largest entry in
// [2^13, 2^14) (half's 5-bit exponent: entries that small relative to the
// block's largest lose their lo half to the subnormal range, a loss relative
// to that largest entry of at most 2^-38).  Both table layouts are written:
// kr = [p][k][r] and rk = [p][r][k] (k = (n - m - p) / 2).
template <int MODE>
__global__ void k_legendre_table(int trunc, const double *mu, const double *diag, const int *diag_e, MBlock *mbs,
                                 unsigned long long *mmax, void *tab_kr, void *tab_rk,
                                 void *lo_kr, void *lo_rk)
{
    const int m = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const MBlock b = mbs[m];
    // exponent: max * 2^e in [2^(t-1), 2^t), t = 0 (BF16) or 14 (IEEE half)
    constexpr int t_top = MODE == 4 ? 14 : 0;
    if (MODE >= 3 && r == 0 && blockIdx.x == 0) {
        double mx = __longlong_as_double((long long)mmax[m]);
        int E = 0;
        if (mx > 0.0) frexp(mx, &E);
        mbs[m].e = t_top - E;
    }
    if (r >= b.R) return;
    const int j = b.j0 + r;
    const double x = mu[j];
    double scale = 1.0;
    if (MODE >= 3) {
        double mx = __longlong_as_double((long long)mmax[m]);
        int E = 0;
        if (mx > 0.0) frexp(mx, &E);
        scale = ldexp(1.0, t_top - E);
    }
    double vmax = 0.0;
    auto put = [&](int n, double v) {
        if (MODE == 0) {
            vmax = fmax(vmax, fabs(v));
            return;
        }
        int t = n - m, par = t & 1, k = t >> 1;
        int64_t ikr = b.off_kr + (int64_t)par * b.Kp * b.Rp + (int64_t)k * b.Rp + r;
        int64_t irk = b.off_rk + (int64_t)par * b.Rp * b.Kp + (int64_t)r * b.Kp + k;
        if (MODE == 1) {
            ((double *)tab_kr)[ikr] = v;
            ((double *)tab_rk)[irk] = v;
        } else if (MODE == 2) {
            ((float *)tab_kr)[ikr] = (float)v;
            ((float *)tab_rk)[irk] = (float)v;
        } else if (MODE == 3) {
            double vs = v * scale;
            unsigned short hi = bf16_rne((float)vs);
            unsigned short lo = bf16_rne((float)(vs - (double)bf16_to_f(hi)));
            ((unsigned short *)tab_kr)[ikr] = hi;
            ((unsigned short *)tab_rk)[irk] = hi;
            ((unsigned short *)lo_kr)[ikr] = lo;
            ((unsigned short *)lo_rk)[irk] = lo;
        } else {
            double vs = v * scale;
            _Float16 h = (_Float16)(float)vs;
            _Float16 l = (_Float16)(float)(vs - (double)h);
            unsigned short hi = __builtin_bit_cast(unsigned short, h);
            unsigned short lo = __builtin_bit_cast(unsigned short, l);
            ((unsigned short *)tab_kr)[ikr] = hi;
            ((unsigned short *)tab_rk)[irk] = hi;
            ((unsigned short *)lo_kr)[ikr] = lo;
            ((unsigned short *)lo_rk)[irk] = lo;
        }
    };
    // the column runs on values scaled by 2^-E (E <= 0 from the seed; a power
    // of two commutes with rounding), rescaled by 2^-600 whenever it exceeds
    // 2^600; each stored value is ldexp(p, E)
    double p0 = diag[(int64_t)j * (trunc + 1) + m];
    int E = diag_e[(int64_t)j * (trunc + 1) + m];
    put(m, ldexp(p0, E));
    if (m < trunc) {
        double p1 = sqrt(2.0 * m + 3.0) * x * p0;
        put(m + 1, ldexp(p1, E));
        for (int n = m + 2; n <= trunc; ++n) {
            double nn = (double)n * n, mm = (double)m * m;
            double a = sqrt((4.0 * nn - 1.0) / (nn - mm));
            double bb = sqrt((2.0 * n + 1.0) * (n - 1.0 - m) * (n - 1.0 + m) / ((2.0 * n - 3.0) * (nn - mm)));
            double p2 = a * x * p1 - bb * p0;
            if (fabs(p2) > 0x1p600) {
                p1 *= 0x1p-600;
                p2 *= 0x1p-600;
                E += 600;
            }
            put(n, ldexp(p2, E));
            p0 = p1;
            p1 = p2;
        }
    }
    if (MODE == 0 && vmax > 0.0) atomicMax(mmax + m, (unsigned long long)__double_as_longlong(vmax));
}

}  // namespace

hipError_t launch_gauss_nodes(int nlat, double *mu, double *w, hipStream_t s)
{
    if (nlat < 2 || nlat % 2) return hipErrorInvalidValue;
    int half = nlat / 2;
    k_gauss_nodes<<<(half + 127) / 128, 128, 0, s>>>(nlat, mu, w);
    return hipGetLastError();
}

hipError_t launch_legendre_tables(Plan &p, hipStream_t s)
{
    const int NL = p.nlat / 2, N = p.trunc;
    if (p.mb.size() != (size_t)N + 1) return hipErrorInvalidValue;
    // host check: every table write of every (m, r) lands inside the allocation
    for (const MBlock &b : p.mb) {
        if (b.R > b.Rp || b.K0 > b.Kp || b.j0 + b.R > NL) return hipErrorInvalidValue;
        if (b.off_kr + 2 * (int64_t)b.Kp * b.Rp > p.tab_elems) return hipErrorInvalidValue;
    }
    size_t el = p.prec == SHTX_FP64 ? 8 : p.prec == SHTX_FP32 ? 4 : 2;
    hipError_t e = hipMemsetAsync(p.d_tab_kr, 0, el * p.tab_elems, s);
    if (e == hipSuccess) e = hipMemsetAsync(p.d_tab_rk, 0, el * p.tab_elems, s);
    if (e == hipSuccess && p.d_tab_kr_lo) e = hipMemsetAsync(p.d_tab_kr_lo, 0, el * p.tab_elems, s);
    if (e == hipSuccess && p.d_tab_rk_lo) e = hipMemsetAsync(p.d_tab_rk_lo, 0, el * p.tab_elems, s);
    if (e == hipSuccess) e = hipMemsetAsync(p.d_mmax, 0, sizeof(unsigned long long) * (N + 1), s);
    if (e != hipSuccess) return e;
    k_sectoral<<<(NL + 127) / 128, 128, 0, s>>>(NL, N, p.d_mu, p.d_diag, p.d_diag_e);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    dim3 grid((NL + 127) / 128, N + 1);
    if (p.prec == SHTX_FP64) {
        k_legendre_table<1><<<grid, 128, 0, s>>>(N, p.d_mu, p.d_diag, p.d_diag_e, p.d_mb, p.d_mmax, p.d_tab_kr,
                                                  p.d_tab_rk, nullptr, nullptr);
    } else if (p.prec == SHTX_FP32) {
        k_legendre_table<2><<<grid, 128, 0, s>>>(N, p.d_mu, p.d_diag, p.d_diag_e, p.d_mb, p.d_mmax, p.d_tab_kr,
                                                  p.d_tab_rk, nullptr, nullptr);
    } else {
        k_legendre_table<0><<<grid, 128, 0, s>>>(N, p.d_mu, p.d_diag, p.d_diag_e, p.d_mb, p.d_mmax, nullptr,
                                                  nullptr, nullptr, nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (p.prec == SHTX_FP16X3)
            k_legendre_table<4><<<grid, 128, 0, s>>>(N, p.d_mu, p.d_diag, p.d_diag_e, p.d_mb, p.d_mmax, p.d_tab_kr,
                                                      p.d_tab_rk, p.d_tab_kr_lo, p.d_tab_rk_lo);
        else
            k_legendre_table<3><<<grid, 128, 0, s>>>(N, p.d_mu, p.d_diag, p.d_diag_e, p.d_mb, p.d_mmax, p.d_tab_kr,
                                                      p.d_tab_rk, p.d_tab_kr_lo, p.d_tab_rk_lo);
    }
    return hipGetLastError();
}

}  // namespace shtx
