// Internal declarations shared by the plan code and the HIP kernels of libshtx.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "../../include/shtx.h"

namespace shtx {

// Legendre tables pad both the ring and the parity-k dimension of every m
// block to a multiple of this, so that GEMM tiles (whose sizes divide it)
// always read inside the block.
constexpr int kTablePad = 128;

// Ring-FFT kernels hold at most this many complex values of one block in LDS.
constexpr int kFftCapF32 = 8192;  // 64 KiB: two blocks per CU with the prime-pass roots
constexpr int kFftCapF64 = 8192;  // 128 KiB: one block per CU (the FP64 passes use 228 VGPRs)
constexpr int kFftThreads = 512;

// Butterflies per thread in a radix-R Stockham pass (rounds of kFftThreads):
// enough for a block's cap complex values for radices below 11; radices 11
// and up take one round, and the blocking keeps a block's fields within it
// (they only occur in rings whose whole FFT is a direct one).
__host__ __device__ constexpr int fft_rounds(int cap, int R)
{
    return R >= 11 ? 1 : (cap / R + kFftThreads - 1) / kFftThreads;
}

// General prime pass: a ring whose half-length has one prime factor p above
// the register radices, p <= kGpMaxPrime, runs it as the first pass on the
// matrix cores, reading the p-th roots of unity from p LDS entries after the
// field slots.  Its outputs come in units of 16 rows t (t = 0 .. (p-1)/2) by
// 16 columns (butterfly, real | imaginary part); each wave holds at most
// kGpUnits units (more would push the single-precision FFT kernels past the
// 128 VGPRs that keep two blocks per CU).
constexpr int kGpMaxPrime = 1021;
constexpr int kGpUnits = 4;
__host__ __device__ constexpr int gp_row_tiles(int p) { return ((p - 1) / 2 + 16) / 16; }
__host__ __device__ constexpr int gp_col_tiles(int nbutterflies) { return (2 * nbutterflies + 15) / 16; }
constexpr int kMaxRadices = 12;

// One m block of the Legendre tables.
struct MBlock {
    int R;          // northern rings carrying m (M_j >= m): j0 .. j0 + R - 1
    int j0;         // first such ring
    int K0, K1;     // number of n = m + p + 2k <= N for parity p = 0, 1
    int Rp, Kp;     // padded ring and parity-k extents
    int e;          // power-of-two exponent applied to the stored split table
    int pad_;
    int64_t off_kr; // element offset of the [p][Kp][Rp] block (parity 1 at + Kp*Rp)
    int64_t off_rk; // element offset of the [p][Rp][Kp] block (parity 1 at + Rp*Kp)
};

// One GEMM work item: wavenumber m, row tile, column tile (m < 0: no work).
struct GemmItem {
    int m, tr, tc, pad_;
};

// One ring of the grid (device copy of the FFT plan for that ring).
struct RingDesc {
    int n;        // ring length (even)
    int h;        // n / 2: length of the complex FFT
    int M;        // ring cutoff
    int L;        // executed FFT length (h, or the Bluestein length >= 2h - 1)
    int nrad;     // number of Stockham passes
    int blue;     // 1 if the length-h DFT goes through Bluestein's convolution
    int fb;       // fields per FFT block for this ring
    int lbuf;     // complex values per field slot: max(L, h + 1)
    int lbufp;    // LDS entries per field slot
    int pass_off; // first PassDesc of this ring length's Stockham passes
    unsigned long long radcode;  // radix of pass s in bits [5s, 5s + 5)
    int64_t tw_off;     // W_L[k] = exp(-2 pi i k / L), k < L
    int64_t post_off;   // exp(-2 pi i m / n), m <= h
    int64_t chirp_off;  // Bluestein chirp exp(-pi i k^2 / h), k < h
    int64_t bhat_off;   // Bluestein filter spectrum / L, L entries
    int64_t grid_off;   // first point of the ring inside one grid field
    int64_t four_off;   // first complex of the ring's [m][nfld] block
    double w;           // Gauss weight
};

// One Stockham pass of a ring length's FFT (shared by every ring of that
// length).  Divisions by nbf and Ns are done as mul_hi(a, magic) with
// magic = ceil(2^32 / d), exact for a * d < 2^32 (magic 0 stands for d = 1).
struct PassDesc {
    int R;          // radix
    int Ns;         // product of the radices of the earlier passes
    int nbf;        // butterflies per field: L / R
    int tstep;      // twiddle table stride of the butterfly index: L / (Ns R)
    unsigned mg_nbf, mg_ns;
};

__host__ __device__ inline unsigned div_magic(int d) { return d <= 1 ? 0u : 0xFFFFFFFFu / (unsigned)d + 1u; }

// Fourier-workspace offsets of a northern ring and its southern mirror, in
// units of nfld complex values (RingDesc::four_off / nfld).
struct __attribute__((aligned(8))) RingPair {
    int n, s;
};

// One FFT work item: a ring and a run of fields (ring < 0: no work).
struct FftItem {
    int ring, f0, nf, pad_;
};

enum TransformKind { kInverse = 0, kDirect = 1, kInverseAdj = 2, kDirectAdj = 3, kWind = 4 };
constexpr int kKinds = 5;

// The split-precision forms: hi + lo halves of bfloat16 or IEEE half.
inline bool split_form(int prec) { return prec == SHTX_BF16X3 || prec == SHTX_FP16X3; }

struct Plan {
    int trunc = 0, grid = 0, nlat = 0, nlon_full = 0, nfld = 0, prec = 0;
    unsigned flags = 0;
    int64_t nspec = 0, npts = 0, nfour = 0;
    std::vector<int32_t> nlon;
    std::vector<int> cutoff;
    std::vector<MBlock> mb;
    std::vector<RingDesc> rings;
    int max_nlon = 0;

    // GEMM tiling chosen at plan time (depends on precision).
    int inv_bm = 0, inv_bn = 0, dir_bm = 0, dir_bn = 0;
    // Each work list is its main part (tiles of bm x bn) followed, when the
    // last column tile would be less than half used, by a tail part whose
    // tiles are tail_bn columns wide; nmain counts the main part's items.
    std::vector<GemmItem> inv_items, dir_items;
    int inv_nmain = 0, dir_nmain = 0, inv_tail_bn = 0, dir_tail_bn = 0;
    std::vector<FftItem> fft_items;
    std::vector<PassDesc> passes;
    int fft_lds_bytes = 0;
    int fft_lds_max = 0;  // complex entries of LDS the largest FFT block may use
    int fft_cap = 0;      // LDS complex values per FFT block the blocking was made for
    int tuned = 0;        // 0 default tiles, 1 timed by the autotuner, 2 from the tune cache
    // True once every kernel's work list and launch shape has passed the host
    // checks and the device copies of the lists match them; launches check
    // only this flag, so the per-item checks run at plan time, not per call.
    bool shapes_ok = false;
    int device = -1;              // HIP device the plan's memory lives on
    hipEvent_t done = nullptr;    // recorded after each transform's launches
    bool timing_on = false;       // record kernel events (plans made with SHTX_FLAG_TIMING)

    // Device memory.
    double *d_mu = nullptr, *d_w = nullptr;  // nlat
    double *d_diag = nullptr;                // [NL][N+1] sectoral seeds q (plan time only) ...
    int *d_diag_e = nullptr;                 // ... and their exponents E: P̄_m^m = q 2^E
    void *d_tab_kr = nullptr, *d_tab_rk = nullptr;        // FP64/FP32 values or BF16 hi
    void *d_tab_kr_lo = nullptr, *d_tab_rk_lo = nullptr;  // BF16 lo
    unsigned long long *d_mmax = nullptr;                  // per-m max |P̄| bits (plan time)
    MBlock *d_mb = nullptr;
    GemmItem *d_inv_items = nullptr, *d_dir_items = nullptr;
    RingDesc *d_rings = nullptr;
    int64_t *d_ring_four_off = nullptr;  // per ring: RingDesc::four_off
    RingPair *d_ring_pair = nullptr;     // per northern ring
    void *d_ring_q = nullptr;            // per northern ring: w_j / 2 in grid precision
    FftItem *d_fft_items = nullptr;
    PassDesc *d_passes = nullptr;
    void *d_twid = nullptr;  // FFT twiddle pool (complex, grid precision)
    int64_t twid_elems = 0;  // complex entries in the pool
    std::vector<double> twid_host;  // pool (re, im) before upload
    void *d_four = nullptr;  // Fourier workspace [ring][m][nfld] complex
    // SHTX_FP16X3: per field, the largest magnitude (float bits) of the data
    // the next Legendre GEMM splits (spectral input or Fourier workspace)
    unsigned *d_fmax = nullptr;
    // SHTX_FLAG_UV: spectral wind images [nfld][nspec] (U then V) between the
    // wind step and the inverse transform
    void *d_uvspec = nullptr;
    double qmax = 0.0;  // max over northern rings of w_j / 2
    int64_t tab_elems = 0;   // elements per table layout
    size_t table_bytes = 0, workspace_bytes = 0;
    double legendre_flops = 0.0;
    double plan_seconds = 0.0;

    // Graph cache (one per transform kind, keyed on pointers and stream).
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        const void *in = nullptr, *in2 = nullptr;
        void *out = nullptr;
        hipStream_t stream = nullptr;
    } graphs[kKinds];

    // Kernel timing.
    static constexpr int kMaxTimed = 4096;
    std::vector<hipEvent_t> ev_start, ev_stop;
    std::vector<int> ev_kind;
    int n_timed = 0;
};

// Element sizes.
inline int grid_elem_bytes(int prec) { return prec == SHTX_FP64 ? 8 : 4; }

// Transform-call helpers of the C ABI (capi.cpp): argument checks (SHTX_OK or
// SHTX_EINVAL, nothing launched), and the per-plan completion event.
int check_args(const Plan &p, int kind, const void *in, const void *out, const void *in2 = nullptr);
hipError_t mark_done(Plan &p, hipStream_t s);
hipError_t wait_done(Plan &p);

// Kernel launchers (each checks its launch shape on the host first).
hipError_t launch_gauss_nodes(int nlat, double *mu, double *w, hipStream_t s);
hipError_t launch_legendre_tables(Plan &p, hipStream_t s);
// `fmax` is the per-field maxima buffer of a SHTX_FP16X3 plan (nfld words;
// ignored by the other forms): the plan's own, or a caller-provided one.
hipError_t launch_gemm_inverse(const Plan &p, const void *spec, void *four, unsigned *fmax, hipStream_t s);
hipError_t launch_gemm_direct(const Plan &p, const void *four, void *spec, bool adjoint, unsigned *fmax,
                              hipStream_t s);
hipError_t launch_fft_c2r(const Plan &p, const void *four, void *grid, bool adjoint,
                          hipStream_t s);
hipError_t launch_fft_r2c(const Plan &p, const void *grid, void *four, bool adjoint, unsigned *fmax,
                          hipStream_t s);
// Wind step of shtx_uv_trans: spectral vorticity and divergence of truncation
// trunc - 1 (nfld / 2 fields each) -> spectral U and V of truncation trunc.
hipError_t launch_uv_spec(const Plan &p, const void *vor, const void *dvg, void *out, hipStream_t s);
// Fields per ring-FFT block are at most this many when the r2c kernel also
// records each field's largest output magnitude (SHTX_FP16X3 plans).
constexpr int kFmaxFields = 1024;

// Host checks that every kernel's work list and launch shape stay inside the
// plan's arrays and the kernels' compile-time limits (no device access).
bool gemm_shapes_ok(const Plan &p);
bool fft_shapes_ok(const Plan &p);
int plan_layout(Plan &p, int trunc, int grid, int nlat, int nlon_full, int nfld, int prec, unsigned flags);

// GEMM tile sizes per precision (rows, columns) for each direction: the
// defaults, and whether a kernel instantiation exists for a shape.
void gemm_tiles(int prec, int *inv_bm, int *inv_bn, int *dir_bm, int *dir_bn);
bool gemm_tile_supported(int prec, int bm, int bn);
// Candidate shapes the autotuner times (count returned, shapes in bm[], bn[]).
int gemm_tile_candidates(int prec, int *bm, int *bn, int max);

// Rebuild the FFT blocking (fields per block within `cap` LDS complex
// values) and the GEMM work lists for the plan's current tile shapes.
int fft_blocking(Plan &p, int cap);
int gemm_work_lists(Plan &p);

// Time the candidate GEMM tile shapes and FFT blockings on this plan and keep
// the fastest (or take them from the tune cache); uploads the work lists.
int autotune_plan(Plan &p, hipStream_t s);
// Set the GEMM tile shapes and FFT blocking of a built plan: rebuilds the
// work lists, checks every launch shape, uploads the lists into new device
// buffers and only then replaces the plan's (the caller makes sure no
// transform is in flight).  On any error the plan is left as it was.
int apply_shapes(Plan &p, int inv_bm, int inv_bn, int dir_bm, int dir_bn, int fft_cap);
// Let the ring-FFT kernels of the plan's precision use the whole LDS of a
// workgroup as dynamic LDS (set per device at plan creation).
hipError_t fft_prepare(const Plan &p);

// Host-side Bluestein filter: out[k] = DFT_L(b)[k] / L in long double, b the
// conjugate chirp wrapped to length L.
void bluestein_filter(int h, int L, std::vector<long double> &re, std::vector<long double> &im);

// Work lists are laid out as 8 equal segments, one per XCD (the hardware
// deals workgroups to the 8 XCDs round-robin), padded with no-op items.
// xcd_remap maps the hardware block index to the item index so that segment x
// runs on XCD x in order: items that share data (the tiles of one m, the field
// runs of one ring) are put in the same segment and share that XCD's L2.
constexpr int kXcds = 8;

__device__ inline int xcd_remap(int bid, int grid)
{
    int per = grid / kXcds;
    return (bid % kXcds) * per + bid / kXcds;
}

// Host helper: place groups of items (each group kept on one XCD) into the 8
// segments, heaviest group first onto the least-loaded segment, and pad.
template <class Item>
std::vector<Item> layout_by_xcd(const std::vector<std::vector<Item>> &groups,
                                const std::vector<double> &cost, const Item &noop)
{
    std::vector<size_t> order(groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    std::vector<std::vector<Item>> seg(kXcds);
    double load[kXcds] = {0};
    for (size_t g : order) {
        int best = 0;
        for (int x = 1; x < kXcds; ++x)
            if (load[x] < load[best]) best = x;
        load[best] += cost[g];
        seg[best].insert(seg[best].end(), groups[g].begin(), groups[g].end());
    }
    size_t per = 0;
    for (auto &v : seg) per = std::max(per, v.size());
    if (per == 0) per = 1;
    std::vector<Item> out(per * kXcds, noop);
    for (int x = 0; x < kXcds; ++x)
        std::copy(seg[x].begin(), seg[x].end(), out.begin() + x * per);
    return out;
}

}  // namespace shtx

// The opaque handle of the C ABI.
struct shtx_plan_s {
    shtx::Plan p;
};
