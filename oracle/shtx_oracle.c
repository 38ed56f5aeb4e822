/*
 * Plain FP64 CPU oracle for the spherical-harmonic transform pair.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load this library.  It
 * shares no source, header, table or helper with the HIP library; the two
 * meet only through arrays produced by the seeded input generator.
 *
 * What it computes.  The paper (Section 3, "Spectral Transform - Spherical
 * Harmonics Dwarf", and Section 2.2.2, which names the IFS spectral transform
 * as the workload) gives no formula for the transform, so this file writes
 * out the textbook definitions in their plainest form:
 *
 *   nodes    mu_j = roots of the Legendre polynomial P_nlat, descending,
 *            found by Newton iteration and polished in quad precision so
 *            that each double is the one nearest to the true root;
 *            w_j = 2 / ((1 - mu_j^2) P'_nlat(mu_j)^2)  (Gauss-Legendre).
 *   P̄_n^m   normalised so that (1/2) * integral_{-1}^{1} (P̄_n^m)^2 dmu = 1,
 *            no Condon-Shortley phase, built by the standard three-term
 *            recurrence in n for each fixed m.
 *   inverse  F_m(mu_j) = sum_{n=m}^{N} a_n^m P̄_n^m(mu_j)               (m <= M_j)
 *            g_{j,k}   = sum_{m=0}^{M_j} c_m Re(F_m(mu_j) e^{i m lambda_k})
 *            c_0 = 1, c_m = 2 (m >= 1), lambda_k = 2 pi k / nlon_j.
 *   direct   G_m(mu_j) = (1/nlon_j) sum_k g_{j,k} e^{-i m lambda_k}      (m <= M_j)
 *            a_n^m     = (1/2) sum_{j : M_j >= m} w_j G_m(mu_j) P̄_n^m(mu_j)
 *            Im a_n^0 := 0.
 *   adjoints (Euclidean inner products on (Re, Im) of the stored triangle
 *            and on raw grid values)
 *            inv_adj(y)_n^m   = sum_{j : M_j >= m} P̄_n^m(mu_j) c_m
 *                                 sum_k y_{j,k} e^{-i m lambda_k},  Im(.)_n^0 := 0
 *            dir_adj(b)_{j,k} = (w_j / (2 nlon_j)) sum_{m=0}^{M_j}
 *                                 Re((sum_n b_n^m P̄_n^m(mu_j)) e^{i m lambda_k}).
 *   cutoff   M_j = min(N, floor((nlon_j - 1) / 2)): the largest wavenumber a
 *            ring of nlon_j points carries without aliasing.
 *
 * Every sum is evaluated as written: the Fourier step is a naive DFT over a
 * per-ring twiddle table, the Legendre step a plain dot product over n, with
 * no even/odd folding, no blocking and no FFT.  Both hemispheres are
 * evaluated directly (no use of the equatorial symmetry).
 *
 * Layouts (shared with the tests only):
 *   spectral  [nfld][nspec] complex (re, im interleaved), m-major, n
 *             ascending: index(m, n) = m (2N + 3 - m) / 2 + (n - m).
 *   grid      [nfld][npts] real, rings concatenated north to south, each
 *             ring starting at lambda = 0.
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ----------------------------------------------------------------------- */
/* Grid geometry                                                            */
/* ----------------------------------------------------------------------- */

/* Octahedral reduced Gaussian grid O_nl: 2 nl rings; the i-th ring from the
 * nearer pole (i = 0 .. nl-1) has 20 + 4 i points.  The paper names the
 * TCo (cubic-octahedral) resolutions in Section 3.1.4.1 and Section 3.2.2. */
void oracle_octahedral_nlon(int nl, int32_t *nlon)
{
    for (int j = 0; j < 2 * nl; ++j) {
        int i = j < nl ? j : 2 * nl - 1 - j;
        nlon[j] = 20 + 4 * i;
    }
}

/* Ring cutoff M_j = min(N, floor((nlon - 1) / 2)). */
int oracle_ring_cutoff(int trunc, int nlon)
{
    int m = (nlon - 1) / 2;
    return m < trunc ? m : trunc;
}

int64_t oracle_nspec(int trunc) { return (int64_t)(trunc + 1) * (trunc + 2) / 2; }

static int64_t spec_index(int trunc, int m, int n)
{
    return (int64_t)m * (2 * trunc + 3 - m) / 2 + (n - m);
}

/* ----------------------------------------------------------------------- */
/* Gauss-Legendre nodes and weights                                         */
/* ----------------------------------------------------------------------- */

/* P_n(x) and P_{n-1}(x) of the unnormalised Legendre polynomials by
 * l P_l = (2l - 1) x P_{l-1} - (l - 1) P_{l-2}. */
static void legendre_poly_d(int n, double x, double *pn, double *pn1)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *pn = 1.0; *pn1 = 0.0; return; }
    for (int l = 2; l <= n; ++l) {
        double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *pn1 = p0;
}

static void legendre_poly_q(int n, __float128 x, __float128 *pn, __float128 *pn1)
{
    __float128 p0 = 1, p1 = x;
    if (n == 0) { *pn = 1; *pn1 = 0; return; }
    for (int l = 2; l <= n; ++l) {
        __float128 p2 = ((__float128)(2 * l - 1) * x * p1 - (__float128)(l - 1) * p0) / l;
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *pn1 = p0;
}

/* mu[nlat] descending and w[nlat].  Newton in double from the classical
 * guess cos(pi (j + 3/4) / (nlat + 1/2)), then Newton in quad precision until
 * the step is below 1e-30, then one rounding to double: each mu_j is the
 * double nearest to the true root.  The southern half mirrors the northern. */
void oracle_gauss(int nlat, double *mu, double *w)
{
    int half = (nlat + 1) / 2;
#pragma omp parallel for schedule(dynamic, 8)
    for (int j = 0; j < half; ++j) {
        double x = cos(M_PI * (j + 0.75) / (nlat + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, p1;
            legendre_poly_d(nlat, x, &p, &p1);
            double dp = nlat * (x * p - p1) / (x * x - 1.0);
            double dx = p / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        __float128 xq = x, dpq = 1;
        for (int it = 0; it < 8; ++it) {
            __float128 p, p1;
            legendre_poly_q(nlat, xq, &p, &p1);
            dpq = (__float128)nlat * (xq * p - p1) / (xq * xq - 1);
            __float128 dx = p / dpq;
            xq -= dx;
            if (fabsq(dx) < 1e-30Q) break;
        }
        {
            __float128 p, p1;
            legendre_poly_q(nlat, xq, &p, &p1);
            dpq = (__float128)nlat * (xq * p - p1) / (xq * xq - 1);
        }
        if ((nlat & 1) && j == half - 1) xq = 0; /* odd nlat: exact middle root */
        __float128 wq = 2 / ((1 - xq) * (1 + xq) * dpq * dpq);
        mu[j] = (double)xq;
        w[j] = (double)wq;
        mu[nlat - 1 - j] = xq == 0 ? 0.0 : -(double)xq;
        w[nlat - 1 - j] = (double)wq;
    }
}

/* ----------------------------------------------------------------------- */
/* Normalised associated Legendre functions                                 */
/* ----------------------------------------------------------------------- */

/* out[n - m] = P̄_n^m(mu) for n = m .. trunc, with s = sqrt((1-mu)(1+mu)):
 *   P̄_0^0 = 1,  P̄_m^m = sqrt((2m+1)/(2m)) s P̄_{m-1}^{m-1},
 *   P̄_{m+1}^m = sqrt(2m+3) mu P̄_m^m,
 *   P̄_n^m = a_nm mu P̄_{n-1}^m - b_nm P̄_{n-2}^m,
 *   a_nm = sqrt((4n^2 - 1) / (n^2 - m^2)),
 *   b_nm = sqrt((2n+1)(n-1-m)(n-1+m) / ((2n-3)(n^2 - m^2))).
 *
 * Extended exponent.  Near the poles the sectoral value P̄_m^m ~ s^m leaves
 * the double range for large m (m log10(1/s) > 300) while the recurrence in
 * n can bring P̄_n^m back to order one before n reaches the truncation (at
 * N = 1999 values up to about 5 would be lost, at N = 1279 at most 1e-62).
 * The column is therefore carried as q 2^E: the sectoral product is
 * renormalised by frexp after every factor, the recurrence runs on the
 * scaled values q (scaling by a power of two commutes with rounding, so
 * nothing changes where the plain recurrence stays in range), q is rescaled
 * by 2^-600 whenever it exceeds 2^600, and each output is ldexp(q, E): zero
 * or subnormal while 2^E is that small. */
static void legendre_column(int trunc, int m, double mu, double s, double *out)
{
    double q = 1.0;
    int E = 0;
    for (int k = 1; k <= m; ++k) {
        int e;
        q = frexp(q * (sqrt((2.0 * k + 1.0) / (2.0 * k)) * s), &e);
        E += e;
    }
    out[0] = ldexp(q, E);
    if (m == trunc) return;
    double q0 = q, q1 = sqrt(2.0 * m + 3.0) * mu * q;
    out[1] = ldexp(q1, E);
    for (int n = m + 2; n <= trunc; ++n) {
        double nn = (double)n * n, mm = (double)m * m;
        double a = sqrt((4.0 * nn - 1.0) / (nn - mm));
        double b = sqrt((2.0 * n + 1.0) * (n - 1.0 - m) * (n - 1.0 + m) / ((2.0 * n - 3.0) * (nn - mm)));
        double q2 = a * mu * q1 - b * q0;
        if (fabs(q2) > 0x1p600) {
            q1 *= 0x1p-600;
            q2 *= 0x1p-600;
            E += 600;
        }
        out[n - m] = ldexp(q2, E);
        q0 = q1;
        q1 = q2;
    }
}

/* P̄_n^m(mu_i) for n = m..trunc at each of npt abscissae: out[i][n - m]. */
void oracle_legendre(int trunc, int m, int npt, const double *mu, double *out)
{
    for (int i = 0; i < npt; ++i) {
        double s = sqrt((1.0 - mu[i]) * (1.0 + mu[i]));
        legendre_column(trunc, m, mu[i], s, out + (int64_t)i * (trunc - m + 1));
    }
}

/* ----------------------------------------------------------------------- */
/* Fourier twiddles                                                         */
/* ----------------------------------------------------------------------- */

/* tab[2r], tab[2r+1] = cos, sin of 2 pi r / n, r = 0 .. n-1, evaluated in
 * long double and rounded once; e^{i m lambda_k} = tab[(m k) mod n]. */
static void twiddle_table(int n, double *tab)
{
    for (int r = 0; r < n; ++r) {
        long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)r / (long double)n;
        tab[2 * r] = (double)cosl(a);
        tab[2 * r + 1] = (double)sinl(a);
    }
}

/* Naive real synthesis on one ring of n points:
 *   g_k = sum_{m=0}^{M} fac_m Re(F_m e^{2 pi i m k / n}),
 * fac_0 = 1 and fac_m = fac_pos (m >= 1).  F holds M+1 complex values. */
void oracle_ring_synth(int n, int M, double fac_pos, const double *F, double *g)
{
    double *tab = malloc(sizeof(double) * 2 * (size_t)n);
    twiddle_table(n, tab);
    for (int k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int m = 0; m <= M; ++m) {
            int r = (int)(((int64_t)m * k) % n);
            double fac = m > 0 ? fac_pos : 1.0;
            /* Re(F e^{i m lambda}) = Re F cos - Im F sin */
            acc += fac * (F[2 * m] * tab[2 * r] - F[2 * m + 1] * tab[2 * r + 1]);
        }
        g[k] = acc;
    }
    free(tab);
}

/* Naive real analysis on one ring of n points:
 *   G_m = sum_{k=0}^{n-1} g_k e^{-2 pi i m k / n},  m = 0 .. M. */
void oracle_ring_dft(int n, int M, const double *g, double *G)
{
    double *tab = malloc(sizeof(double) * 2 * (size_t)n);
    twiddle_table(n, tab);
    for (int m = 0; m <= M; ++m) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < n; ++k) {
            int r = (int)(((int64_t)m * k) % n);
            /* g e^{-i m lambda} = g (cos - i sin) */
            re += g[k] * tab[2 * r];
            im -= g[k] * tab[2 * r + 1];
        }
        G[2 * m] = re;
        G[2 * m + 1] = im;
    }
    free(tab);
}

/* ----------------------------------------------------------------------- */
/* Synthesis: spectral -> grid                                              */
/* ----------------------------------------------------------------------- */

/* g_{j,k} = ring_scale_j * sum_{m=0}^{M_j} fac_m Re(F_m(mu_j) e^{i m lambda_k}),
 * F_m(mu_j) = sum_n a_n^m P̄_n^m(mu_j).  The inverse transform takes
 * fac_m = c_m and ring_scale_j = 1; the adjoint of the direct transform takes
 * fac_m = 1 and ring_scale_j = w_j / (2 nlon_j).  Parallel over rings. */
static void synthesis(int trunc, int nlat, const int32_t *nlon, int nfld,
                      const double *spec, double *grid, int fac_is_cm, int weighted)
{
    double *mu = malloc(sizeof(double) * nlat), *w = malloc(sizeof(double) * nlat);
    int64_t *off = malloc(sizeof(int64_t) * (nlat + 1));
    int64_t nspec = oracle_nspec(trunc);
    oracle_gauss(nlat, mu, w);
    off[0] = 0;
    for (int j = 0; j < nlat; ++j) off[j + 1] = off[j] + nlon[j];
    int64_t npts = off[nlat];

#pragma omp parallel
    {
        double *pcol = malloc(sizeof(double) * (trunc + 1));
        double *four = malloc(sizeof(double) * 2 * (size_t)nfld * (trunc + 1));
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < nlat; ++j) {
            int n_j = nlon[j];
            int M = oracle_ring_cutoff(trunc, n_j);
            double x = mu[j], s = sqrt((1.0 - x) * (1.0 + x));
            double ring_scale = weighted ? w[j] / (2.0 * n_j) : 1.0;
            for (int m = 0; m <= M; ++m) {
                legendre_column(trunc, m, x, s, pcol);
                for (int f = 0; f < nfld; ++f) {
                    const double *a = spec + 2 * ((int64_t)f * nspec + spec_index(trunc, m, m));
                    double re = 0.0, im = 0.0;
                    for (int n = m; n <= trunc; ++n) {
                        re += a[2 * (n - m)] * pcol[n - m];
                        im += a[2 * (n - m) + 1] * pcol[n - m];
                    }
                    four[2 * ((int64_t)f * (trunc + 1) + m)] = re;
                    four[2 * ((int64_t)f * (trunc + 1) + m) + 1] = im;
                }
            }
            for (int f = 0; f < nfld; ++f) {
                double *g = grid + (int64_t)f * npts + off[j];
                oracle_ring_synth(n_j, M, fac_is_cm ? 2.0 : 1.0, four + 2 * (int64_t)f * (trunc + 1), g);
                for (int k = 0; k < n_j; ++k) g[k] *= ring_scale;
            }
        }
        free(pcol);
        free(four);
    }
    free(mu);
    free(w);
    free(off);
}

/* ----------------------------------------------------------------------- */
/* Analysis: grid -> spectral                                               */
/* ----------------------------------------------------------------------- */

/* Step 1 (parallel over rings): G_m(mu_j) = dft_scale_j fac_m sum_k g_{j,k}
 * e^{-i m lambda_k} for m <= M_j.  Step 2 (parallel over m):
 * a_n^m = sum_{j : M_j >= m} quad_j G_m(mu_j) P̄_n^m(mu_j), then Im a_n^0 := 0.
 * The direct transform takes dft_scale_j = 1/nlon_j, fac_m = 1 and
 * quad_j = w_j / 2; the adjoint of the inverse takes dft_scale_j = 1,
 * fac_m = c_m and quad_j = 1. */
static void analysis(int trunc, int nlat, const int32_t *nlon, int nfld,
                     const double *grid, double *spec, int adjoint)
{
    double *mu = malloc(sizeof(double) * nlat), *w = malloc(sizeof(double) * nlat);
    int64_t *off = malloc(sizeof(int64_t) * (nlat + 1));
    int64_t *goff = malloc(sizeof(int64_t) * (nlat + 1));
    int64_t nspec = oracle_nspec(trunc);
    oracle_gauss(nlat, mu, w);
    off[0] = 0;
    goff[0] = 0;
    for (int j = 0; j < nlat; ++j) {
        off[j + 1] = off[j] + nlon[j];
        goff[j + 1] = goff[j] + oracle_ring_cutoff(trunc, nlon[j]) + 1;
    }
    int64_t npts = off[nlat], nfour = goff[nlat];
    /* G[f][goff[j] + m] complex */
    double *G = malloc(sizeof(double) * 2 * (size_t)nfld * (size_t)nfour);

#pragma omp parallel
    {
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < nlat; ++j) {
            int n_j = nlon[j];
            int M = oracle_ring_cutoff(trunc, n_j);
            double dft_scale = adjoint ? 1.0 : 1.0 / n_j;
            for (int f = 0; f < nfld; ++f) {
                const double *g = grid + (int64_t)f * npts + off[j];
                double *Gf = G + 2 * ((int64_t)f * nfour + goff[j]);
                oracle_ring_dft(n_j, M, g, Gf);
                for (int m = 0; m <= M; ++m) {
                    double fac = (adjoint && m > 0) ? 2.0 : 1.0;
                    Gf[2 * m] *= dft_scale * fac;
                    Gf[2 * m + 1] *= dft_scale * fac;
                }
            }
        }
    }

#pragma omp parallel
    {
        double *pcol = malloc(sizeof(double) * (trunc + 1));
        double *acc = malloc(sizeof(double) * 2 * (size_t)nfld * (trunc + 1));
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m <= trunc; ++m) {
            int K = trunc - m + 1;
            memset(acc, 0, sizeof(double) * 2 * (size_t)nfld * K);
            for (int j = 0; j < nlat; ++j) {
                if (oracle_ring_cutoff(trunc, nlon[j]) < m) continue;
                double x = mu[j], s = sqrt((1.0 - x) * (1.0 + x));
                double quad = adjoint ? 1.0 : 0.5 * w[j];
                legendre_column(trunc, m, x, s, pcol);
                for (int f = 0; f < nfld; ++f) {
                    const double *Gf = G + 2 * ((int64_t)f * nfour + goff[j] + m);
                    double gre = quad * Gf[0], gim = quad * Gf[1];
                    double *af = acc + 2 * (int64_t)f * K;
                    for (int t = 0; t < K; ++t) {
                        af[2 * t] += gre * pcol[t];
                        af[2 * t + 1] += gim * pcol[t];
                    }
                }
            }
            for (int f = 0; f < nfld; ++f) {
                double *a = spec + 2 * ((int64_t)f * nspec + spec_index(trunc, m, m));
                const double *af = acc + 2 * (int64_t)f * K;
                for (int t = 0; t < K; ++t) {
                    a[2 * t] = af[2 * t];
                    a[2 * t + 1] = (m == 0) ? 0.0 : af[2 * t + 1];
                }
            }
        }
        free(pcol);
        free(acc);
    }
    free(G);
    free(mu);
    free(w);
    free(off);
    free(goff);
}

/* ----------------------------------------------------------------------- */
/* Public entry points                                                       */
/* ----------------------------------------------------------------------- */

static void set_threads(int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

/* Inverse transform: spec[nfld][nspec] complex -> grid[nfld][npts]. */
void oracle_inv(int trunc, int nlat, const int32_t *nlon, int nfld,
                const double *spec, double *grid, int nthreads)
{
    set_threads(nthreads);
    synthesis(trunc, nlat, nlon, nfld, spec, grid, 1, 0);
}

/* Direct transform: grid[nfld][npts] -> spec[nfld][nspec] complex. */
void oracle_dir(int trunc, int nlat, const int32_t *nlon, int nfld,
                const double *grid, double *spec, int nthreads)
{
    set_threads(nthreads);
    analysis(trunc, nlat, nlon, nfld, grid, spec, 0);
}

/* Adjoint of the inverse transform: grid -> spectral. */
void oracle_inv_adj(int trunc, int nlat, const int32_t *nlon, int nfld,
                    const double *grid, double *spec, int nthreads)
{
    set_threads(nthreads);
    analysis(trunc, nlat, nlon, nfld, grid, spec, 1);
}

/* Adjoint of the direct transform: spectral -> grid. */
void oracle_dir_adj(int trunc, int nlat, const int32_t *nlon, int nfld,
                    const double *spec, double *grid, int nthreads)
{
    set_threads(nthreads);
    synthesis(trunc, nlat, nlon, nfld, spec, grid, 0, 1);
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* ----------------------------------------------------------------------- */
/* Wind from vorticity and divergence                                       */
/* ----------------------------------------------------------------------- */

/* H_n^m(mu) = (1 - mu^2) dP̄_n^m/dmu for n = m .. trunc at one abscissa, from
 * the derivative identity of the normalised functions
 *   (1 - mu^2) dP̄_n^m/dmu = -n mu P̄_n^m + (2n + 1) eps_n^m P̄_{n-1}^m,
 *   eps_n^m = sqrt((n^2 - m^2) / (4 n^2 - 1)),  P̄_{m-1}^m := 0. */
void oracle_legendre_deriv(int trunc, int m, double mu, double *out)
{
    double *p = malloc(sizeof(double) * (trunc - m + 1));
    double s = sqrt((1.0 - mu) * (1.0 + mu));
    legendre_column(trunc, m, mu, s, p);
    for (int n = m; n <= trunc; ++n) {
        double eps = sqrt(((double)n * n - (double)m * m) / (4.0 * n * n - 1.0));
        double prev = n > m ? p[n - m - 1] : 0.0;
        out[n - m] = -n * mu * p[n - m] + (2.0 * n + 1.0) * eps * prev;
    }
    free(p);
}

/* Wind images on the unit sphere from spectral vorticity zeta and divergence
 * D (truncation trunc, [nfld][nspec] each):
 *   psi_n^m = -zeta_n^m / (n (n + 1)),  chi_n^m = -D_n^m / (n (n + 1))  (n >= 1;
 *            0 for n = 0), the streamfunction and velocity potential;
 *   U = u cos(phi) = d chi / d lambda - (1 - mu^2) d psi / d mu,
 *   V = v cos(phi) = d psi / d lambda + (1 - mu^2) d chi / d mu,
 * evaluated as the real fields sum_m c_m Re(X_m(mu_j) e^{i m lambda_k}) with
 *   U_m(mu) = sum_n (i m chi_n^m P̄_n^m(mu) - psi_n^m H_n^m(mu)),
 *   V_m(mu) = sum_n (i m psi_n^m P̄_n^m(mu) + chi_n^m H_n^m(mu)),
 * m <= M_j (ring cutoff of the truncation), Im of the m = 0 coefficients
 * ignored.  grid is [2 nfld][npts]: U of field f in row f, V in row nfld + f. */
void oracle_uv(int trunc, int nlat, const int32_t *nlon, int nfld,
               const double *vor, const double *dvg, double *grid, int nthreads)
{
    set_threads(nthreads);
    double *mu = malloc(sizeof(double) * nlat), *w = malloc(sizeof(double) * nlat);
    int64_t *off = malloc(sizeof(int64_t) * (nlat + 1));
    int64_t nspec = oracle_nspec(trunc);
    oracle_gauss(nlat, mu, w);
    off[0] = 0;
    for (int j = 0; j < nlat; ++j) off[j + 1] = off[j] + nlon[j];
    int64_t npts = off[nlat];

#pragma omp parallel
    {
        double *pcol = malloc(sizeof(double) * (trunc + 1));
        double *hcol = malloc(sizeof(double) * (trunc + 1));
        double *fu = malloc(sizeof(double) * 2 * (size_t)nfld * (trunc + 1));
        double *fv = malloc(sizeof(double) * 2 * (size_t)nfld * (trunc + 1));
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < nlat; ++j) {
            int n_j = nlon[j];
            int M = oracle_ring_cutoff(trunc, n_j);
            double x = mu[j], s = sqrt((1.0 - x) * (1.0 + x));
            for (int m = 0; m <= M; ++m) {
                legendre_column(trunc, m, x, s, pcol);
                oracle_legendre_deriv(trunc, m, x, hcol);
                for (int f = 0; f < nfld; ++f) {
                    const double *z = vor + 2 * ((int64_t)f * nspec + spec_index(trunc, m, m));
                    const double *d = dvg + 2 * ((int64_t)f * nspec + spec_index(trunc, m, m));
                    double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
                    for (int n = (m > 0 ? m : 1); n <= trunc; ++n) {
                        double inv_l = -1.0 / ((double)n * (n + 1));
                        double psr = inv_l * z[2 * (n - m)], psi = m == 0 ? 0.0 : inv_l * z[2 * (n - m) + 1];
                        double chr = inv_l * d[2 * (n - m)], chi = m == 0 ? 0.0 : inv_l * d[2 * (n - m) + 1];
                        double P = pcol[n - m], H = hcol[n - m];
                        /* i m chi P - psi H */
                        ur += -m * chi * P - psr * H;
                        ui += m * chr * P - psi * H;
                        /* i m psi P + chi H */
                        vr += -m * psi * P + chr * H;
                        vi += m * psr * P + chi * H;
                    }
                    fu[2 * ((int64_t)f * (trunc + 1) + m)] = ur;
                    fu[2 * ((int64_t)f * (trunc + 1) + m) + 1] = ui;
                    fv[2 * ((int64_t)f * (trunc + 1) + m)] = vr;
                    fv[2 * ((int64_t)f * (trunc + 1) + m) + 1] = vi;
                }
            }
            for (int f = 0; f < nfld; ++f) {
                oracle_ring_synth(n_j, M, 2.0, fu + 2 * (int64_t)f * (trunc + 1), grid + (int64_t)f * npts + off[j]);
                oracle_ring_synth(n_j, M, 2.0, fv + 2 * (int64_t)f * (trunc + 1),
                                  grid + (int64_t)(nfld + f) * npts + off[j]);
            }
        }
        free(pcol);
        free(hcol);
        free(fu);
        free(fv);
    }
    free(mu);
    free(w);
    free(off);
}
