/*
 * The C ABI used from C alone (no Python, no torch): a plan, device buffers
 * from the HIP runtime, one inverse and one direct transform, checked
 * against closed forms of the textbook definition the header states.
 *
 *   field 0: a_1^0 = 1            ->  g = P̄_1^0(mu)          = sqrt(3) mu
 *   field 1: a_1^1 = 1/2 + i/4    ->  g = 2 Re(a_1^1 e^{i lambda}) P̄_1^1(mu)
 *                                     = (cos lambda - sin lambda / 2) sqrt(3/2) sqrt(1 - mu^2)
 * (unit mean-square normalisation, no Condon-Shortley phase), then the
 * direct transform must return the two spectra.  Usage: roundtrip fp64|fp32;
 * prints the errors and exits 0 when they are within the form's bound.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "shtx.h"

static const double kPi = 3.14159265358979323846;

#define CHECK(x)                                                           \
    do {                                                                   \
        int rc_ = (x);                                                     \
        if (rc_ != 0) {                                                    \
            fprintf(stderr, "%s failed: %d (%s)\n", #x, rc_, shtx_strerror(rc_)); \
            return 2;                                                      \
        }                                                                  \
    } while (0)
#define HIPCHECK(x)                                                        \
    do {                                                                   \
        if ((x) != hipSuccess) {                                           \
            fprintf(stderr, "%s failed\n", #x);                            \
            return 2;                                                      \
        }                                                                  \
    } while (0)

int main(int argc, char **argv)
{
    const int dbl = argc > 1 && strcmp(argv[1], "fp64") == 0;
    const int N = 31, nlat = 64, nfld = 2;
    const double tol = dbl ? 1e-13 : 1e-6;
    shtx_plan p = NULL;
    CHECK(shtx_plan_create(&p, N, SHTX_GRID_OCTAHEDRAL, nlat, 0, nfld, dbl ? SHTX_FP64 : SHTX_FP32, 0u, NULL));
    shtx_info info;
    CHECK(shtx_plan_info(p, &info));
    const long nspec = info.nspec, npts = info.npts;
    const size_t el = dbl ? sizeof(double) : sizeof(float);

    double *mu = malloc(sizeof(double) * nlat), *w = malloc(sizeof(double) * nlat);
    int32_t *nlon = malloc(sizeof(int32_t) * nlat);
    CHECK(shtx_plan_nodes(p, mu, w));
    CHECK(shtx_plan_ring_lengths(p, nlon));

    /* spectra: field-major, interleaved complex, index(m, n) = m (2N + 3 - m) / 2 + n - m */
    double *a = calloc((size_t)nfld * nspec * 2, sizeof(double));
    const long i10 = 1, i11 = (2L * N + 2) / 2;
    a[2 * i10] = 1.0;
    a[2 * (nspec + i11)] = 0.5;
    a[2 * (nspec + i11) + 1] = 0.25;
    void *h_spec = malloc((size_t)nfld * nspec * 2 * el), *h_grid = malloc((size_t)nfld * npts * el);
    for (long i = 0; i < nfld * nspec * 2; ++i) {
        if (dbl)
            ((double *)h_spec)[i] = a[i];
        else
            ((float *)h_spec)[i] = (float)a[i];
    }
    void *d_spec = NULL, *d_grid = NULL, *d_back = NULL;
    HIPCHECK(hipMalloc(&d_spec, (size_t)nfld * nspec * 2 * el));
    HIPCHECK(hipMalloc(&d_back, (size_t)nfld * nspec * 2 * el));
    HIPCHECK(hipMalloc(&d_grid, (size_t)nfld * npts * el));
    HIPCHECK(hipMemcpy(d_spec, h_spec, (size_t)nfld * nspec * 2 * el, hipMemcpyHostToDevice));

    CHECK(shtx_inv_trans(p, d_spec, d_grid, NULL));
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipMemcpy(h_grid, d_grid, (size_t)nfld * npts * el, hipMemcpyDeviceToHost));
    double e_inv = 0.0;
    long off = 0;
    for (int j = 0; j < nlat; ++j) {
        const double s = sqrt((1.0 - mu[j]) * (1.0 + mu[j]));
        for (int k = 0; k < nlon[j]; ++k) {
            const double lam = 2.0 * kPi * k / nlon[j];
            const double g0 = sqrt(3.0) * mu[j];
            const double g1 = (cos(lam) - 0.5 * sin(lam)) * sqrt(1.5) * s;
            const double v0 = dbl ? ((double *)h_grid)[off + k] : ((float *)h_grid)[off + k];
            const double v1 = dbl ? ((double *)h_grid)[npts + off + k] : ((float *)h_grid)[npts + off + k];
            e_inv = fmax(e_inv, fmax(fabs(v0 - g0), fabs(v1 - g1)));
        }
        off += nlon[j];
    }

    CHECK(shtx_dir_trans(p, d_grid, d_back, NULL));
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipMemcpy(h_spec, d_back, (size_t)nfld * nspec * 2 * el, hipMemcpyDeviceToHost));
    double e_dir = 0.0;
    for (long i = 0; i < nfld * nspec * 2; ++i) {
        const double v = dbl ? ((double *)h_spec)[i] : ((float *)h_spec)[i];
        e_dir = fmax(e_dir, fabs(v - a[i]));
    }
    printf("C ABI %s: inverse max error %.3e, round trip max error %.3e (bound %.0e)\n", dbl ? "fp64" : "fp32", e_inv,
           e_dir, tol);
    CHECK(shtx_plan_destroy(p));
    (void)hipFree(d_spec);
    (void)hipFree(d_back);
    (void)hipFree(d_grid);
    free(mu);
    free(w);
    free(nlon);
    free(a);
    free(h_spec);
    free(h_grid);
    return e_inv <= tol && e_dir <= tol ? 0 : 1;
}
