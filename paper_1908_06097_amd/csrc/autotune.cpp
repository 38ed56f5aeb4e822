// Plan-time autotuner: times the candidate tile shapes of the two Legendre
// GEMM launches and the candidate FFT blockings on the plan's own workload
// (its truncation, grid, field count and precision) and keeps the fastest.
// Results can be kept in a JSON-lines cache named by SHTX_TUNE_CACHE, keyed by
// device architecture, plan shape and a hash of the kernel sources.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "shtx_internal.h"

#ifndef SHTX_BUILD_ID
#define SHTX_BUILD_ID "unversioned"
#endif

namespace shtx {

namespace {

struct TuneResult {
    int inv_bm = 0, inv_bn = 0, dir_bm = 0, dir_bn = 0, fft_cap = 0;
    double inv_ms = 0, dir_ms = 0, fft_ms = 0;
};

std::string tune_key(const Plan &p)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s|T%d|g%d|nlat%d|nlon%d|F%d|p%d|%s", arch.c_str(), p.trunc, p.grid, p.nlat,
                  p.nlon_full, p.nfld, p.prec, SHTX_BUILD_ID);
    return buf;
}

// Find the line for `key` in the cache file and parse its choices.
bool cache_lookup(const char *path, const std::string &key, TuneResult &r)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    const std::string needle = "\"key\": \"" + key + "\"";
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (!std::strstr(line, needle.c_str())) continue;
        const char *q = std::strstr(line, "\"inv\": [");
        const char *d = std::strstr(line, "\"dir\": [");
        const char *c = std::strstr(line, "\"fft_cap\": ");
        TuneResult t;
        if (q && d && c && std::sscanf(q, "\"inv\": [%d, %d]", &t.inv_bm, &t.inv_bn) == 2 &&
            std::sscanf(d, "\"dir\": [%d, %d]", &t.dir_bm, &t.dir_bn) == 2 &&
            std::sscanf(c, "\"fft_cap\": %d", &t.fft_cap) == 1) {
            r = t;
            found = true;  // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const TuneResult &r)
{
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"inv\": [%d, %d], \"dir\": [%d, %d], \"fft_cap\": %d, "
                 "\"inv_ms\": %.4f, \"dir_ms\": %.4f, \"fft_ms\": %.4f}\n",
                 key.c_str(), r.inv_bm, r.inv_bn, r.dir_bm, r.dir_bn, r.fft_cap, r.inv_ms, r.dir_ms, r.fft_ms);
    std::fclose(f);
}

// Median milliseconds of `reps` separately timed runs of `fn` after one
// untimed run.
template <class Fn>
double time_ms(hipStream_t s, hipEvent_t a, hipEvent_t b, int reps, Fn fn)
{
    if (fn() != hipSuccess) return -1.0;
    std::vector<double> t;
    for (int i = 0; i < reps; ++i) {
        if (hipEventRecord(a, s) != hipSuccess || fn() != hipSuccess || hipEventRecord(b, s) != hipSuccess ||
            hipEventSynchronize(b) != hipSuccess)
            return -1.0;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.0;
        t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

// Pseudo-random operands in [-1/2, 1/2) (a 32-bit integer hash of the
// index), so that the timed kernels see data like the transforms' own:
// constant or zero operands change the matrix cores' power draw and with it
// the clock, and timed the shapes in a different order than real data.
template <typename T>
__global__ void k_fill_noise(T *x, size_t n, unsigned seed)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        unsigned h = (unsigned)i * 0x9E3779B9u ^ seed;
        h ^= h >> 16;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        h *= 0xC2B2AE35u;
        h ^= h >> 16;
        x[i] = (T)((double)(h >> 8) * (1.0 / 16777216.0) - 0.5);
    }
}

hipError_t fill_noise(void *x, size_t bytes, bool dbl, unsigned seed, hipStream_t s)
{
    const size_t n = bytes / (dbl ? 8 : 4);
    if (dbl)
        k_fill_noise<double><<<1024, 256, 0, s>>>((double *)x, n, seed);
    else
        k_fill_noise<float><<<1024, 256, 0, s>>>((float *)x, n, seed);
    return hipGetLastError();
}

}  // namespace

int autotune_plan(Plan &p, hipStream_t s)
{
    const std::string key = tune_key(p);
    const char *cache = std::getenv("SHTX_TUNE_CACHE");
    TuneResult best;
    bool have = false;
    if (cache && *cache && cache_lookup(cache, key, best) && gemm_tile_supported(p.prec, best.inv_bm, best.inv_bn) &&
        gemm_tile_supported(p.prec, best.dir_bm, best.dir_bn) && best.fft_cap > 0)
        have = true;

    if (!have) {
        const bool dbl = p.prec == SHTX_FP64;
        const size_t cbytes = dbl ? 16 : 8, rbytes = dbl ? 8 : 4;
        void *spec = nullptr, *grid = nullptr;
        hipEvent_t ea = nullptr, eb = nullptr;
        int rc = SHTX_OK;
        const int reps = 5;
        auto fail = [&](int code) {
            rc = code;
            return code;
        };
        if (hipMalloc(&spec, cbytes * p.nfld * p.nspec) != hipSuccess ||
            hipMalloc(&grid, rbytes * p.nfld * p.npts) != hipSuccess || hipEventCreate(&ea) != hipSuccess ||
            hipEventCreate(&eb) != hipSuccess)
            fail(SHTX_ENOMEM);
        if (rc == SHTX_OK && (fill_noise(spec, cbytes * p.nfld * p.nspec, dbl, 1u, s) != hipSuccess ||
                              fill_noise(grid, rbytes * p.nfld * p.npts, dbl, 2u, s) != hipSuccess ||
                              fill_noise(p.d_four, cbytes * p.nfld * p.nfour, dbl, 3u, s) != hipSuccess))
            fail(SHTX_EHIP);

        int cbm[8], cbn[8];
        const int nc = gemm_tile_candidates(p.prec, cbm, cbn, 8);
        double bi = 1e300, bd = 1e300;
        // inverse-shaped and direct-shaped launches are tuned independently;
        // the candidates are timed twice, in forward then reverse order, and
        // each keeps its faster median (clock drift favours neither end)
        for (int cc = 0; cc < 2 * nc && rc == SHTX_OK; ++cc) {
            const int c = cc < nc ? cc : 2 * nc - 1 - cc;
            int arc = apply_shapes(p, cbm[c], cbn[c], cbm[c], cbn[c], p.fft_cap);
            if (arc == SHTX_EINVAL || arc == SHTX_EUNSUPPORTED) continue;
            if (arc != SHTX_OK) {
                fail(arc);
                break;
            }
            double ti = time_ms(s, ea, eb, reps, [&] { return launch_gemm_inverse(p, spec, p.d_four, p.d_fmax, s); });
            double td = time_ms(s, ea, eb, reps, [&] { return launch_gemm_direct(p, p.d_four, spec, false, p.d_fmax, s); });
            if (std::getenv("SHTX_DEBUG"))
                std::fprintf(stderr, "shtx tune: GEMM %dx%d inverse %.3f ms direct %.3f ms\n", cbm[c], cbn[c], ti, td);
            if (ti >= 0 && ti < bi) {
                bi = ti;
                best.inv_bm = cbm[c];
                best.inv_bn = cbn[c];
                best.inv_ms = ti;
            }
            if (td >= 0 && td < bd) {
                bd = td;
                best.dir_bm = cbm[c];
                best.dir_bn = cbn[c];
                best.dir_ms = td;
            }
        }
        const int maxcap = dbl ? kFftCapF64 : kFftCapF32;
        const int caps[] = {maxcap, maxcap / 2, maxcap / 3};
        double bf = 1e300;
        for (int cap : caps) {
            if (rc != SHTX_OK) break;
            int arc = apply_shapes(p, p.inv_bm, p.inv_bn, p.dir_bm, p.dir_bn, cap);
            if (arc == SHTX_EINVAL || arc == SHTX_EUNSUPPORTED) continue;
            if (arc != SHTX_OK) {
                fail(arc);
                break;
            }
            double tf = time_ms(s, ea, eb, reps, [&] {
                hipError_t e = launch_fft_c2r(p, p.d_four, grid, false, s);
                return e != hipSuccess ? e : launch_fft_r2c(p, grid, p.d_four, false, p.d_fmax, s);
            });
            if (std::getenv("SHTX_DEBUG")) std::fprintf(stderr, "shtx tune: FFT cap %d c2r+r2c %.3f ms\n", cap, tf);
            if (tf >= 0 && tf < bf) {
                bf = tf;
                best.fft_cap = cap;
                best.fft_ms = tf;
            }
        }
        if (hipStreamSynchronize(s) != hipSuccess) fail(SHTX_EHIP);
        if (spec) (void)hipFree(spec);
        if (grid) (void)hipFree(grid);
        if (ea) (void)hipEventDestroy(ea);
        if (eb) (void)hipEventDestroy(eb);
        if (rc != SHTX_OK) return rc;
        if (best.inv_bm == 0 || best.dir_bm == 0 || best.fft_cap == 0) return SHTX_EHIP;
        if (cache && *cache) cache_store(cache, key, best);
        p.tuned = 1;
    } else {
        p.tuned = 2;
    }

    const int tuned = p.tuned;
    int rc = apply_shapes(p, best.inv_bm, best.inv_bn, best.dir_bm, best.dir_bn, best.fft_cap);
    p.tuned = tuned;
    return rc;
}

namespace {

// The plan state that apply_shapes rebuilds, kept so that a failed call can
// put it back.
struct ShapeState {
    int inv_bm, inv_bn, dir_bm, dir_bn, inv_nmain, dir_nmain, inv_tail_bn, dir_tail_bn;
    int fft_lds_bytes, fft_lds_max, fft_cap;
    bool shapes_ok;
    std::vector<GemmItem> inv_items, dir_items;
    std::vector<FftItem> fft_items;
    std::vector<int> fb;
};

ShapeState save_shapes(const Plan &p)
{
    ShapeState s{p.inv_bm,      p.inv_bn,      p.dir_bm,      p.dir_bn,   p.inv_nmain, p.dir_nmain,
                 p.inv_tail_bn, p.dir_tail_bn, p.fft_lds_bytes, p.fft_lds_max, p.fft_cap, p.shapes_ok,
                 p.inv_items,   p.dir_items,   p.fft_items,   {}};
    for (const RingDesc &d : p.rings) s.fb.push_back(d.fb);
    return s;
}

void restore_shapes(Plan &p, ShapeState &s)
{
    p.inv_bm = s.inv_bm;
    p.inv_bn = s.inv_bn;
    p.dir_bm = s.dir_bm;
    p.dir_bn = s.dir_bn;
    p.inv_nmain = s.inv_nmain;
    p.dir_nmain = s.dir_nmain;
    p.inv_tail_bn = s.inv_tail_bn;
    p.dir_tail_bn = s.dir_tail_bn;
    p.fft_lds_bytes = s.fft_lds_bytes;
    p.fft_lds_max = s.fft_lds_max;
    p.fft_cap = s.fft_cap;
    p.shapes_ok = s.shapes_ok;
    p.inv_items.swap(s.inv_items);
    p.dir_items.swap(s.dir_items);
    p.fft_items.swap(s.fft_items);
    for (size_t j = 0; j < p.rings.size() && j < s.fb.size(); ++j) p.rings[j].fb = s.fb[j];
}

template <class T>
hipError_t upload_new(T **dst, const std::vector<T> &src)
{
    *dst = nullptr;
    if (src.empty()) return hipSuccess;
    hipError_t e = hipMalloc(dst, sizeof(T) * src.size());
    if (e != hipSuccess) {
        *dst = nullptr;
        return e;
    }
    e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(*dst);
        *dst = nullptr;
    }
    return e;
}

}  // namespace

int apply_shapes(Plan &p, int inv_bm, int inv_bn, int dir_bm, int dir_bn, int fft_cap)
{
    const int maxcap = p.prec == SHTX_FP64 ? kFftCapF64 : kFftCapF32;
    if (fft_cap < 1 || fft_cap > maxcap) return SHTX_EINVAL;
    if (!gemm_tile_supported(p.prec, inv_bm, inv_bn) || !gemm_tile_supported(p.prec, dir_bm, dir_bn))
        return SHTX_EUNSUPPORTED;
    ShapeState old = save_shapes(p);
    p.inv_bm = inv_bm;
    p.inv_bn = inv_bn;
    p.dir_bm = dir_bm;
    p.dir_bn = dir_bn;
    int rc = gemm_work_lists(p);
    if (rc == SHTX_OK) rc = fft_blocking(p, fft_cap);
    if (rc == SHTX_OK && (!gemm_shapes_ok(p) || !fft_shapes_ok(p))) rc = SHTX_EUNSUPPORTED;
    if (rc != SHTX_OK) {
        restore_shapes(p, old);
        return rc;
    }
    // new device lists first; the plan's are replaced only if all succeed
    GemmItem *di = nullptr, *dd = nullptr;
    FftItem *df = nullptr;
    hipError_t e = upload_new(&di, p.inv_items);
    if (e == hipSuccess) e = upload_new(&dd, p.dir_items);
    if (e == hipSuccess) e = upload_new(&df, p.fft_items);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (di) (void)hipFree(di);
        if (dd) (void)hipFree(dd);
        if (df) (void)hipFree(df);
        restore_shapes(p, old);
        return e == hipErrorOutOfMemory ? SHTX_ENOMEM : SHTX_EHIP;
    }
    if (p.d_inv_items) (void)hipFree(p.d_inv_items);
    if (p.d_dir_items) (void)hipFree(p.d_dir_items);
    if (p.d_fft_items) (void)hipFree(p.d_fft_items);
    p.d_inv_items = di;
    p.d_dir_items = dd;
    p.d_fft_items = df;
    p.shapes_ok = true;
    p.tuned = 0;
    return SHTX_OK;
}

}  // namespace shtx
