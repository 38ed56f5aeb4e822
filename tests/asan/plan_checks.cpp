// Host-side plan logic under AddressSanitizer: every workload's geometry,
// ring blocking, FFT pass plans and GEMM work lists in every precision form
// (and, up to TCo639, every tile shape and FFT blocking the autotuner may
// pick), through the
// host-only dry runs of the C ABI (no GPU needed), plus the argument errors.
// Built by tests/asan/build.py with the library's sources instrumented on the
// host side only; exits 0 when every return code is the expected one (an
// AddressSanitizer report aborts with a non-zero status first).
#include <cstdio>

#include "shtx.h"

namespace {

struct Workload {
    int trunc, grid, nlat, nlon_full, nfld;
};

int failures = 0;

void expect(int rc, int want, const char *what, int a, int b)
{
    if (rc != want) {
        std::fprintf(stderr, "%s (%d, %d): got %d, expected %d\n", what, a, b, rc, want);
        ++failures;
    }
}

}  // namespace

int main()
{
    const Workload wl[] = {{79, SHTX_GRID_FULL, 160, 320, 1},        {255, SHTX_GRID_OCTAHEDRAL, 512, 0, 411},
                           {639, SHTX_GRID_OCTAHEDRAL, 1280, 0, 411}, {399, SHTX_GRID_OCTAHEDRAL, 800, 0, 137},
                           {1279, SHTX_GRID_OCTAHEDRAL, 2560, 0, 411}, {1999, SHTX_GRID_OCTAHEDRAL, 4000, 0, 411},
                           {0, SHTX_GRID_OCTAHEDRAL, 2, 0, 3},       {7, SHTX_GRID_FULL, 8, 16, 5}};
    const int precs[] = {SHTX_FP64, SHTX_FP32, SHTX_BF16X3, SHTX_FP16X3};
    // (inverse tile, direct tile) pairs per precision, as the autotuner's candidates
    const int f32[][2] = {{128, 128}, {64, 128}, {128, 64}};
    const int f64[][2] = {{64, 64}, {32, 64}, {64, 32}};
    const int b16[][2] = {{128, 128}, {64, 128}};
    for (const Workload &w : wl) {
        for (int prec : precs) {
            shtx_info info;
            int rc = shtx_plan_check(w.trunc, w.grid, w.nlat, w.nlon_full, w.nfld, prec, &info);
            expect(rc, SHTX_OK, "plan_check", w.trunc, prec);
            // the largest grids take the default shapes only (their layout
            // alone is seconds of instrumented host work)
            if (rc != SHTX_OK || w.trunc >= 1279) continue;
            const int(*t)[2] = prec == SHTX_FP64 ? f64 : prec == SHTX_FP32 ? f32 : b16;
            const int nt = prec == SHTX_FP64 || prec == SHTX_FP32 ? 3 : 2;
            for (int i = 0; i < nt; ++i) {
                const int j = (i + 1) % nt;
                for (int cap : {8192, 4096, 2730}) {
                    rc = shtx_plan_check_shapes(w.trunc, w.grid, w.nlat, w.nlon_full, w.nfld, prec, t[i][0], t[i][1],
                                                t[j][0], t[j][1], cap, &info);
                    expect(rc, SHTX_OK, "plan_check_shapes", w.trunc, cap);
                }
            }
        }
    }
    shtx_info info;
    expect(shtx_plan_check(-1, SHTX_GRID_OCTAHEDRAL, 64, 0, 1, SHTX_FP32, &info), SHTX_EINVAL, "negative trunc", -1, 0);
    expect(shtx_plan_check(31, SHTX_GRID_OCTAHEDRAL, 64, 0, 0, SHTX_FP32, &info), SHTX_EINVAL, "no fields", 31, 0);
    expect(shtx_plan_check(31, 7, 64, 0, 1, SHTX_FP32, &info), SHTX_EINVAL, "unknown grid", 31, 7);
    expect(shtx_plan_check(31, SHTX_GRID_OCTAHEDRAL, 63, 0, 1, SHTX_FP32, &info), SHTX_EUNSUPPORTED, "odd nlat", 31, 63);
    expect(shtx_plan_check_shapes(255, SHTX_GRID_OCTAHEDRAL, 512, 0, 7, SHTX_FP32, 96, 128, 128, 128, 6144, &info),
           SHTX_EUNSUPPORTED, "unknown tile", 96, 128);
    expect(shtx_plan_check_shapes(255, SHTX_GRID_OCTAHEDRAL, 512, 0, 7, SHTX_FP32, 128, 128, 128, 128, 0, &info),
           SHTX_EINVAL, "zero fft cap", 0, 0);
    std::printf("host plan checks under AddressSanitizer: %d failures\n", failures);
    return failures ? 1 : 0;
}
