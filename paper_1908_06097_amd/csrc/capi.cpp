// C ABI of libshtx (declared in include/shtx.h).  Argument checking, the
// order of kernel launches per transform, optional hipGraph replay and the
// per-kernel timing events; the arithmetic lives in the kernels.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "shtx_internal.h"

namespace shtx {
int build_plan(Plan &p, int trunc, int grid, int nlat, int nlon_full, int nfld, int prec,
               unsigned flags, hipStream_t stream);
void free_plan(Plan &p);
}  // namespace shtx

using shtx::Plan;

namespace shtx {

namespace {

size_t spec_bytes(const Plan &p) { return (size_t)p.nfld * p.nspec * (p.prec == SHTX_FP64 ? 16 : 8); }
size_t grid_bytes(const Plan &p) { return (size_t)p.nfld * p.npts * (p.prec == SHTX_FP64 ? 8 : 4); }

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

bool aligned16(const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; }

// A transform's input and output must be device (or managed) memory on the
// plan's device: a host pointer handed to the kernels would fault the GPU
// instead of returning an error.
bool device_memory(const void *q, int device)
{
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, q) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (at.type == hipMemoryTypeManaged || at.isManaged) return true;
    return at.type == hipMemoryTypeDevice && at.device == device;
}

}  // namespace

// Remember the end of a transform's work on its stream, so that destroying
// the plan or changing its shapes waits for exactly that work.  A stream the
// caller is capturing records nothing here (the caller owns that graph).
hipError_t mark_done(Plan &p, hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return e;
    if (cs != hipStreamCaptureStatusNone) return hipSuccess;
    return hipEventRecord(p.done, s);
}

// Wait for the last recorded transform of the plan.
hipError_t wait_done(Plan &p) { return p.done ? hipEventSynchronize(p.done) : hipSuccess; }

// Argument checks shared by every transform entry point (in2: the wind
// transform's second input).
int check_args(const Plan &p, int kind, const void *in, const void *out, const void *in2)
{
    if (!in || !out || !p.shapes_ok) return SHTX_EINVAL;
    if (kind == kWind) {
        // vorticity and divergence at truncation trunc - 1, nfld / 2 fields each
        if (!in2 || !p.d_uvspec) return SHTX_EINVAL;
        const size_t nwin = (size_t)(p.nfld / 2) * p.trunc * (p.trunc + 1) / 2 * (p.prec == SHTX_FP64 ? 16 : 8);
        if (overlap(in, nwin, out, grid_bytes(p)) || overlap(in2, nwin, out, grid_bytes(p))) return SHTX_EINVAL;
        if (!aligned16(in) || !aligned16(in2) || !aligned16(out)) return SHTX_EINVAL;
        if (!device_memory(in, p.device) || !device_memory(in2, p.device) || !device_memory(out, p.device))
            return SHTX_EINVAL;
        return SHTX_OK;
    }
    bool spec_in = kind == kInverse || kind == kDirectAdj;
    size_t nin = spec_in ? spec_bytes(p) : grid_bytes(p);
    size_t nout = spec_in ? grid_bytes(p) : spec_bytes(p);
    if (overlap(in, nin, out, nout)) return SHTX_EINVAL;
    if (!aligned16(in) || !aligned16(out)) return SHTX_EINVAL;
    if (!device_memory(in, p.device) || !device_memory(out, p.device)) return SHTX_EINVAL;
    return SHTX_OK;
}

}  // namespace shtx

using shtx::check_args;
using shtx::mark_done;
using shtx::wait_done;

namespace {

int hip_status(hipError_t e)
{
    if (e == hipSuccess) return SHTX_OK;
    (void)hipGetLastError();
    if (std::getenv("SHTX_DEBUG")) std::fprintf(stderr, "shtx: HIP error %d: %s\n", (int)e, hipGetErrorString(e));
    return SHTX_EHIP;
}

// Launch the kernels of one transform kind on stream s.
hipError_t launch_kind(Plan &p, int kind, const void *in, void *out, hipStream_t s, bool timed,
                       const void *in2 = nullptr)
{
    hipError_t e = hipSuccess;
    auto timed_launch = [&](int tkind, auto &&fn) -> hipError_t {
        int slot = -1;
        if (timed && p.n_timed < Plan::kMaxTimed) {
            slot = p.n_timed++;
            p.ev_kind[slot] = tkind;
            hipError_t er = hipEventRecord(p.ev_start[slot], s);
            if (er != hipSuccess) return er;
        }
        hipError_t r = fn();
        if (r != hipSuccess) return r;
        if (slot >= 0) return hipEventRecord(p.ev_stop[slot], s);
        return hipSuccess;
    };
    switch (kind) {
    case shtx::kInverse:
        e = timed_launch(0, [&] { return shtx::launch_gemm_inverse(p, in, p.d_four, p.d_fmax, s); });
        if (e == hipSuccess) e = timed_launch(2, [&] { return shtx::launch_fft_c2r(p, p.d_four, out, false, s); });
        break;
    case shtx::kDirectAdj:
        e = timed_launch(0, [&] { return shtx::launch_gemm_inverse(p, in, p.d_four, p.d_fmax, s); });
        if (e == hipSuccess) e = timed_launch(2, [&] { return shtx::launch_fft_c2r(p, p.d_four, out, true, s); });
        break;
    case shtx::kDirect:
        e = timed_launch(3, [&] { return shtx::launch_fft_r2c(p, in, p.d_four, false, p.d_fmax, s); });
        if (e == hipSuccess) e = timed_launch(1, [&] { return shtx::launch_gemm_direct(p, p.d_four, out, false, p.d_fmax, s); });
        break;
    case shtx::kInverseAdj:
        e = timed_launch(3, [&] { return shtx::launch_fft_r2c(p, in, p.d_four, true, p.d_fmax, s); });
        if (e == hipSuccess) e = timed_launch(1, [&] { return shtx::launch_gemm_direct(p, p.d_four, out, true, p.d_fmax, s); });
        break;
    case shtx::kWind:
        // the wind step is timed with the inverse-shaped GEMM it feeds
        e = timed_launch(0, [&] {
            hipError_t r = shtx::launch_uv_spec(p, in, in2, p.d_uvspec, s);
            return r != hipSuccess ? r : shtx::launch_gemm_inverse(p, p.d_uvspec, p.d_four, p.d_fmax, s);
        });
        if (e == hipSuccess) e = timed_launch(2, [&] { return shtx::launch_fft_c2r(p, p.d_four, out, false, s); });
        break;
    default:
        e = hipErrorInvalidValue;
    }
    return e;
}


int run(shtx_plan h, int kind, const void *in, void *out, void *stream, const void *in2 = nullptr)
{
    if (!h) return SHTX_EINVAL;
    Plan &p = h->p;
    int rc = check_args(p, kind, in, out, in2);
    if (rc != SHTX_OK) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    bool timed = p.timing_on;
    bool graph = (p.flags & SHTX_FLAG_GRAPH) != 0 && !timed && s != nullptr;
    if (!graph) {
        hipError_t e = launch_kind(p, kind, in, out, s, timed, in2);
        if (e == hipSuccess) e = mark_done(p, s);
        return hip_status(e);
    }

    Plan::GraphEntry &g = p.graphs[kind];
    if (!(g.exec && g.in == in && g.in2 == in2 && g.out == out && g.stream == s)) {
        if (g.exec) {
            (void)hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
        }
        hipGraph_t graph_obj = nullptr;
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_status(e);
        hipError_t le = launch_kind(p, kind, in, out, s, false, in2);
        e = hipStreamEndCapture(s, &graph_obj);
        if (le != hipSuccess || e != hipSuccess) {
            if (graph_obj) (void)hipGraphDestroy(graph_obj);
            return hip_status(le != hipSuccess ? le : e);
        }
        e = hipGraphInstantiate(&g.exec, graph_obj, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph_obj);
        if (e != hipSuccess) {
            g.exec = nullptr;
            return hip_status(e);
        }
        g.in = in;
        g.in2 = in2;
        g.out = out;
        g.stream = s;
    }
    hipError_t e = hipGraphLaunch(g.exec, s);
    if (e == hipSuccess) e = mark_done(p, s);
    return hip_status(e);
}

// ---------------------------------------------------------------------------
// Static scratch of shtx_inv_trans_noalloc.  In host code `scratch` names a
// host-side stand-in, not device memory: kernels and copies get the address
// hipGetSymbolAddress returns for the device, found once per device.
// ---------------------------------------------------------------------------
__device__ __attribute__((aligned(256))) unsigned char scratch[SHTX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices];   // device address of `scratch` per device (null: not found)
bool scratch_tried[kMaxDevices];

// Find `scratch` on `device`, which must be the current device (plan creation).
void locate_scratch(int device)
{
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (device < 0 || device >= kMaxDevices || scratch_tried[device]) return;
    scratch_tried[device] = true;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess && ptr) {
        scratch_dev[device] = ptr;
    } else {
        (void)hipGetLastError();
        if (std::getenv("SHTX_DEBUG")) std::fprintf(stderr, "shtx: static scratch not found: %d\n", (int)e);
    }
}

void *scratch_on(int device)
{
    std::lock_guard<std::mutex> lock(scratch_mu);
    return device >= 0 && device < kMaxDevices ? scratch_dev[device] : nullptr;
}

}  // namespace

extern "C" {

int shtx_plan_create(shtx_plan *out, int trunc, int grid, int nlat, int nlon_full, int nfld,
                     int prec, unsigned flags, void *hip_stream)
{
    if (!out) return SHTX_EINVAL;
    *out = nullptr;
    shtx_plan h = new (std::nothrow) shtx_plan_s;
    if (!h) return SHTX_ENOMEM;
    int rc = shtx::build_plan(h->p, trunc, grid, nlat, nlon_full, nfld, prec, flags,
                              reinterpret_cast<hipStream_t>(hip_stream));
    if (rc != SHTX_OK) {
        shtx::free_plan(h->p);
        delete h;
        return rc;
    }
    locate_scratch(h->p.device);  // the plan's device is current here
    *out = h;
    return SHTX_OK;
}

static void fill_info(const Plan &p, shtx_info *o)
{
    std::memset(o, 0, sizeof(*o));
    o->trunc = p.trunc;
    o->nlat = p.nlat;
    o->nfld = p.nfld;
    o->prec = p.prec;
    o->grid = p.grid;
    o->max_nlon = p.max_nlon;
    o->nspec = p.nspec;
    o->npts = p.npts;
    o->nfour = p.nfour;
    o->table_bytes = p.table_bytes;
    o->workspace_bytes = p.workspace_bytes;
    o->legendre_flops = p.legendre_flops;
    o->plan_seconds = p.plan_seconds;
    o->inv_tile[0] = p.inv_bm;
    o->inv_tile[1] = p.inv_bn;
    o->dir_tile[0] = p.dir_bm;
    o->dir_tile[1] = p.dir_bn;
    o->fft_cap = p.fft_cap;
    o->tuned = p.tuned;
}

int shtx_plan_info(shtx_plan h, shtx_info *o)
{
    if (!h || !o) return SHTX_EINVAL;
    fill_info(h->p, o);
    return SHTX_OK;
}

int shtx_plan_check(int trunc, int grid, int nlat, int nlon_full, int nfld, int prec, shtx_info *out)
{
    Plan p;
    int rc = shtx::plan_layout(p, trunc, grid, nlat, nlon_full, nfld, prec, 0);
    if (rc != SHTX_OK) return rc;
    if (!shtx::gemm_shapes_ok(p) || !shtx::fft_shapes_ok(p)) return SHTX_EUNSUPPORTED;
    if (out) fill_info(p, out);
    return SHTX_OK;
}

int shtx_plan_check_shapes(int trunc, int grid, int nlat, int nlon_full, int nfld, int prec, int inv_bm, int inv_bn,
                           int dir_bm, int dir_bn, int fft_cap, shtx_info *out)
{
    Plan p;
    int rc = shtx::plan_layout(p, trunc, grid, nlat, nlon_full, nfld, prec, 0);
    if (rc != SHTX_OK) return rc;
    p.inv_bm = inv_bm;
    p.inv_bn = inv_bn;
    p.dir_bm = dir_bm;
    p.dir_bn = dir_bn;
    rc = shtx::gemm_work_lists(p);
    if (rc != SHTX_OK) return rc;
    rc = shtx::fft_blocking(p, fft_cap);
    if (rc != SHTX_OK) return rc;
    if (!shtx::gemm_shapes_ok(p) || !shtx::fft_shapes_ok(p)) return SHTX_EUNSUPPORTED;
    if (out) fill_info(p, out);
    return SHTX_OK;
}

int shtx_plan_ring_lengths(shtx_plan h, int32_t *nlon)
{
    if (!h || !nlon) return SHTX_EINVAL;
    std::memcpy(nlon, h->p.nlon.data(), sizeof(int32_t) * h->p.nlat);
    return SHTX_OK;
}

int shtx_plan_nodes(shtx_plan h, double *mu, double *w)
{
    if (!h) return SHTX_EINVAL;
    const Plan &p = h->p;
    hipError_t e = hipSuccess;
    if (mu) e = hipMemcpy(mu, p.d_mu, sizeof(double) * p.nlat, hipMemcpyDeviceToHost);
    if (e == hipSuccess && w) e = hipMemcpy(w, p.d_w, sizeof(double) * p.nlat, hipMemcpyDeviceToHost);
    return hip_status(e);
}

int shtx_plan_legendre(shtx_plan h, int m, double *out)
{
    if (!h) return SHTX_EINVAL;
    const Plan &p = h->p;
    if (m < 0 || m > p.trunc) return SHTX_EINVAL;
    const shtx::MBlock &b = p.mb[m];
    if (!out) return b.R;
    int K = p.trunc - m + 1;
    size_t el = p.prec == SHTX_FP64 ? 8 : p.prec == SHTX_FP32 ? 4 : 2;
    size_t cnt = 2 * (size_t)b.Rp * b.Kp;
    std::vector<unsigned char> hi(cnt * el), lo;
    hipError_t e = hipMemcpy(hi.data(), (const char *)p.d_tab_rk + b.off_rk * el, cnt * el,
                             hipMemcpyDeviceToHost);
    if (e == hipSuccess && shtx::split_form(p.prec)) {
        lo.resize(cnt * el);
        e = hipMemcpy(lo.data(), (const char *)p.d_tab_rk_lo + b.off_rk * el, cnt * el,
                      hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) return hip_status(e);
    auto val = [&](size_t idx) -> double {
        if (p.prec == SHTX_FP64) return reinterpret_cast<const double *>(hi.data())[idx];
        if (p.prec == SHTX_FP32) return reinterpret_cast<const float *>(hi.data())[idx];
        auto bf = [&](uint16_t u) {
            if (p.prec == SHTX_FP16X3) return (double)__builtin_bit_cast(_Float16, u);
            uint32_t x = (uint32_t)u << 16;
            float f;
            std::memcpy(&f, &x, 4);
            return (double)f;
        };
        double v = bf(reinterpret_cast<const uint16_t *>(hi.data())[idx]) +
                   bf(reinterpret_cast<const uint16_t *>(lo.data())[idx]);
        return std::ldexp(v, -b.e);
    };
    for (int r = 0; r < b.R; ++r)
        for (int t = 0; t < K; ++t) {
            int par = t & 1, k = t >> 1;
            size_t idx = (size_t)par * b.Rp * b.Kp + (size_t)r * b.Kp + k;
            out[(size_t)r * K + t] = val(idx);
        }
    return b.R;
}

int shtx_inv_trans(shtx_plan h, const void *spec, void *grid, void *stream)
{
    return run(h, shtx::kInverse, spec, grid, stream);
}

int shtx_uv_trans(shtx_plan h, const void *vor, const void *dvg, void *grid, void *stream)
{
    return run(h, shtx::kWind, vor, grid, stream, dvg);
}

int shtx_inv_trans_noalloc(shtx_plan h, const void *spec, void *grid, void *stream)
{
    if (!h) return SHTX_EINVAL;
    Plan &p = h->p;
    int rc = check_args(p, shtx::kInverse, spec, grid);
    if (rc != SHTX_OK) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p.device) return SHTX_EINVAL;
    const size_t celem = p.prec == SHTX_FP64 ? 16 : 8;
    const size_t four_bytes = (size_t)p.nfour * p.nfld * celem;
    const size_t fmax_off = (four_bytes + 255) / 256 * 256;
    const size_t need = p.prec == SHTX_FP16X3 ? fmax_off + sizeof(unsigned) * p.nfld : four_bytes;
    if (need > SHTX_NOALLOC_SCRATCH_BYTES) return SHTX_ESCRATCH;
    unsigned char *base = static_cast<unsigned char *>(scratch_on(p.device));
    if (!base) return SHTX_EHIP;
    unsigned *fmax = p.prec == SHTX_FP16X3 ? reinterpret_cast<unsigned *>(base + fmax_off) : nullptr;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the kernels overwrite every workspace entry the FFT reads, and the
    // maxima are rewritten before use: nothing needs clearing
    hipError_t e = shtx::launch_gemm_inverse(p, spec, base, fmax, s);
    if (e == hipSuccess) e = shtx::launch_fft_c2r(p, base, grid, false, s);
    if (e == hipSuccess) e = mark_done(p, s);
    return hip_status(e);
}

int shtx_dir_trans(shtx_plan h, const void *grid, void *spec, void *stream)
{
    return run(h, shtx::kDirect, grid, spec, stream);
}

int shtx_inv_trans_adj(shtx_plan h, const void *grid, void *spec, void *stream)
{
    return run(h, shtx::kInverseAdj, grid, spec, stream);
}

int shtx_dir_trans_adj(shtx_plan h, const void *spec, void *grid, void *stream)
{
    return run(h, shtx::kDirectAdj, spec, grid, stream);
}

int shtx_timing_reset(shtx_plan h)
{
    if (!h) return SHTX_EINVAL;
    h->p.n_timed = 0;
    return SHTX_OK;
}

int shtx_timing_enable(shtx_plan h, int on)
{
    if (!h || !(h->p.flags & SHTX_FLAG_TIMING)) return SHTX_EINVAL;
    h->p.timing_on = on != 0;
    return SHTX_OK;
}

int shtx_timing_read(shtx_plan h, double *ms_sum, int32_t *count)
{
    if (!h) return SHTX_EINVAL;
    Plan &p = h->p;
    double sum[4] = {0, 0, 0, 0};
    int32_t cnt[4] = {0, 0, 0, 0};
    for (int i = 0; i < p.n_timed; ++i) {
        hipError_t e = hipEventSynchronize(p.ev_stop[i]);
        if (e != hipSuccess) return hip_status(e);
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p.ev_start[i], p.ev_stop[i]);
        if (e != hipSuccess) return hip_status(e);
        sum[p.ev_kind[i]] += ms;
        cnt[p.ev_kind[i]] += 1;
    }
    for (int k = 0; k < 4; ++k) {
        if (ms_sum) ms_sum[k] = sum[k];
        if (count) count[k] = cnt[k];
    }
    return SHTX_OK;
}

int shtx_plan_set_shapes(shtx_plan h, int inv_bm, int inv_bn, int dir_bm, int dir_bn, int fft_cap)
{
    if (!h) return SHTX_EINVAL;
    Plan &p = h->p;
    // earlier transforms may still read the old work lists
    hipError_t e = wait_done(p);
    if (e != hipSuccess) return hip_status(e);
    for (auto &g : p.graphs)
        if (g.exec) {
            (void)hipGraphExecDestroy(g.exec);
            g = Plan::GraphEntry{};
        }
    return shtx::apply_shapes(p, inv_bm, inv_bn, dir_bm, dir_bn, fft_cap);
}

int shtx_plan_destroy(shtx_plan h)
{
    if (!h) return SHTX_EINVAL;
    (void)wait_done(h->p);
    shtx::free_plan(h->p);
    delete h;
    return SHTX_OK;
}

const char *shtx_strerror(int code)
{
    switch (code) {
    case SHTX_OK: return "success";
    case SHTX_EINVAL: return "invalid argument";
    case SHTX_ENOMEM: return "out of memory";
    case SHTX_EHIP: return "HIP runtime error";
    case SHTX_EUNSUPPORTED: return "unsupported configuration";
    case SHTX_ESCRATCH: return "transform needs more scratch than the static array of shtx_inv_trans_noalloc holds";
    default: return "unknown error";
    }
}

}  // extern "C"
