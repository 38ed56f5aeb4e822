// Plan construction for libshtx: ring geometry, Legendre table layout, GEMM
// and ring-FFT work lists, FFT twiddle tables, device allocations, and the
// device-side generation of Gauss nodes and P̄_n^m tables.
//
// The paper (Section 3.1.1) keeps the transform's data resident on the GPU
// across time steps; here everything a transform needs (tables, twiddles,
// work lists, the Fourier workspace) is allocated once per plan so that the
// transform calls themselves never allocate.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>

#include "shtx_internal.h"

namespace shtx {

namespace {

int ring_cutoff(int trunc, int nlon)
{
    int m = (nlon - 1) / 2;
    return m < trunc ? m : trunc;
}

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// Radices the ring-FFT kernel implements directly (primes; 4, 8, 9 and 16
// are formed from the factors of 2 and 3).  FP64 plans stop at 17.
const int kPrimeRadices[] = {2, 3, 5, 7, 11, 13, 17, 19, 23};

// Factor n over the direct prime radices up to maxp; returns the unfactored
// remainder.
int smooth_factor(int n, std::vector<int> &f, int maxp = 23)
{
    f.clear();
    for (int p : kPrimeRadices)
        while (p <= maxp && n % p == 0) {
            f.push_back(p);
            n /= p;
        }
    return n;
}

bool is_prime(int n)
{
    if (n < 2) return false;
    for (int q = 2; q * q <= n; ++q)
        if (n % q == 0) return false;
    return true;
}

// Stockham radices for a smooth length: the odd factors first, largest
// first (the first pass needs no twiddles), with pairs of 3 merged into 9;
// then the power of two as radix-16 passes and one 8, 4 or 2.
std::vector<int> radices_for(int L)
{
    std::vector<int> f;
    smooth_factor(L, f);
    int twos = 0, threes = 0;
    std::vector<int> odd;
    for (int p : f) {
        if (p == 2)
            ++twos;
        else if (p == 3)
            ++threes;
        else
            odd.push_back(p);
    }
    for (; threes >= 2; threes -= 2) odd.push_back(9);
    if (threes) odd.push_back(3);
    std::sort(odd.rbegin(), odd.rend());
    std::vector<int> r(odd.begin(), odd.end());
    for (; twos >= 4; twos -= 4) r.push_back(16);
    if (twos == 3) r.push_back(8);
    if (twos == 2) r.push_back(4);
    if (twos == 1) r.push_back(2);
    return r;
}

template <class T>
hipError_t upload(T **dst, const std::vector<T> &src)
{
    if (src.empty()) {
        *dst = nullptr;
        return hipSuccess;
    }
    hipError_t e = hipMalloc(dst, sizeof(T) * src.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

}  // namespace

void gemm_tiles(int prec, int *inv_bm, int *inv_bn, int *dir_bm, int *dir_bn)
{
    if (prec == SHTX_FP64) {
        *inv_bm = 64; *inv_bn = 64; *dir_bm = 64; *dir_bn = 64;
    } else if (split_form(prec)) {
        // the autotuner's choices at TCo1279: 128 x 128 with eight waves in
        // both directions (64 x 128, four waves, wins on small workloads)
        *inv_bm = 128; *inv_bn = 128; *dir_bm = 128; *dir_bn = 128;
    } else {
        *inv_bm = 128; *inv_bn = 128; *dir_bm = 128; *dir_bn = 128;
    }
}

// Long-double mixed-radix DFT (forward) over a 2^a 3^b length, used once per
// ring length at plan time for the Bluestein filter spectrum.
static void dft_ld(std::complex<long double> *x, int n, int stride,
                   const std::vector<std::complex<long double>> &tw, int N,
                   std::vector<std::complex<long double>> &tmp)
{
    if (n == 1) return;
    int p = 2;
    for (int q : {2, 3, 5, 7, 11, 13, 17, 19, 23})
        if (n % q == 0) {
            p = q;
            break;
        }
    int m = n / p;
    // decimation in time: sub-sequence r holds x[k p + r]
    std::vector<std::complex<long double>> sub((size_t)n);
    for (int r = 0; r < p; ++r)
        for (int k = 0; k < m; ++k) sub[(size_t)r * m + k] = x[(size_t)(k * p + r) * stride];
    for (int r = 0; r < p; ++r) dft_ld(sub.data() + (size_t)r * m, m, 1, tw, N, tmp);
    int step = N / n;  // tw[t * step] = exp(-2 pi i t / n)
    for (int k = 0; k < m; ++k)
        for (int q = 0; q < p; ++q) {
            std::complex<long double> acc = 0;
            int kk = k + q * m;
            for (int r = 0; r < p; ++r) {
                int t = (int)(((int64_t)r * kk) % n);
                acc += sub[(size_t)r * m + k] * tw[(size_t)t * step];
            }
            x[(size_t)kk * stride] = acc;
        }
}

void bluestein_filter(int h, int L, std::vector<long double> &re, std::vector<long double> &im)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<std::complex<long double>> b((size_t)L, 0), tw((size_t)L), tmp;
    for (int k = 0; k < L; ++k) tw[k] = std::polar(1.0L, -2.0L * pi * k / L);
    for (int j = 0; j < h; ++j) {
        int64_t t = ((int64_t)j * j) % (2 * (int64_t)h);
        std::complex<long double> c = std::polar(1.0L, -pi * (long double)t / h);  // chirp
        b[j] = std::conj(c);
        if (j > 0) b[L - j] = std::conj(c);
    }
    dft_ld(b.data(), L, 1, tw, L, tmp);
    re.resize(L);
    im.resize(L);
    for (int k = 0; k < L; ++k) {
        re[k] = b[k].real() / L;
        im[k] = b[k].imag() / L;
    }
}

void free_plan(Plan &p)
{
    void *ptrs[] = {p.d_mu, p.d_w, p.d_diag, p.d_tab_kr, p.d_tab_rk, p.d_tab_kr_lo,
                    p.d_tab_rk_lo, p.d_mmax, p.d_mb, p.d_inv_items, p.d_dir_items,
                    p.d_rings, p.d_ring_four_off, p.d_ring_pair, p.d_ring_q, p.d_fft_items, p.d_passes,
                    p.d_twid, p.d_four, p.d_fmax, p.d_diag_e, p.d_uvspec};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    for (auto &g : p.graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (auto e : p.ev_start) (void)hipEventDestroy(e);
    for (auto e : p.ev_stop) (void)hipEventDestroy(e);
    if (p.done) (void)hipEventDestroy(p.done);
    p = Plan();
}

#define PLAN_TRY(expr)                                   \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) {                          \
            (void)hipGetLastError();                     \
            return e_ == hipErrorOutOfMemory ? SHTX_ENOMEM : SHTX_EHIP; \
        }                                                \
    } while (0)

// FFT blocking: fields per block (at most `cap` complex values of LDS per
// block), the XCD-segmented work list and the dynamic LDS size.
int fft_blocking(Plan &p, int cap)
{
    const int F = p.nfld, maxcap = p.prec == SHTX_FP64 ? kFftCapF64 : kFftCapF32;
    const size_t celem = p.prec == SHTX_FP64 ? 16 : 8;
    if (cap < 1 || cap > maxcap) return SHTX_EINVAL;
    int lds_elems = 0;
    std::vector<std::vector<FftItem>> fgroups;
    std::vector<double> fcost;
    for (int j = 0; j < p.nlat; ++j) {
        RingDesc &d = p.rings[j];
        if (d.lbuf > maxcap) return SHTX_EUNSUPPORTED;
        d.fb = std::max(1, std::min(F, cap / d.lbuf));
        // passes of radix 11 and up run one round of kFftThreads butterflies;
        // a general prime pass holds at most kGpUnits output units per wave
        int extra = 0;
        for (int s = 0; s < d.nrad; ++s) {
            const PassDesc &q = p.passes[d.pass_off + s];
            const int R = q.R;
            int lim;
            if (R > 23 || (p.prec == SHTX_FP64 && R > 17)) {
                // units = row tiles x ceil(2 fb nbf / 16)
                lim = 8 * (kGpUnits * (kFftThreads / 64) / gp_row_tiles(R)) / q.nbf;
                extra = R;
            } else {
                lim = fft_rounds(maxcap, R) * kFftThreads / q.nbf;
            }
            if (lim < 1) return SHTX_EUNSUPPORTED;
            d.fb = std::min(d.fb, lim);
        }
        lds_elems = std::max(lds_elems, d.fb * d.lbufp + extra);
        std::vector<FftItem> g;
        for (int f0 = 0; f0 < F; f0 += d.fb) g.push_back(FftItem{j, f0, std::min(d.fb, F - f0), 0});
        fgroups.push_back(g);
        fcost.push_back((double)F * d.L * (1 + d.blue) * std::log2((double)d.L + 1));
    }
    p.fft_lds_bytes = lds_elems * (int)celem;
    p.fft_lds_max = lds_elems;
    p.fft_cap = cap;
    if (p.fft_lds_bytes > 160 * 1024) return SHTX_EUNSUPPORTED;
    p.fft_items = layout_by_xcd(fgroups, fcost, FftItem{-1, 0, 0, 0});
    return SHTX_OK;
}

// GEMM work lists for the plan's current tile shapes: every (m, row tile,
// column tile), one XCD segment per group of tiles sharing an m.
int gemm_work_lists(Plan &p)
{
    if (!gemm_tile_supported(p.prec, p.inv_bm, p.inv_bn) || !gemm_tile_supported(p.prec, p.dir_bm, p.dir_bn))
        return SHTX_EUNSUPPORTED;
    if (kTablePad % p.inv_bm || kTablePad % p.dir_bm) return SHTX_EUNSUPPORTED;
    const int N = p.trunc, ncol = 2 * p.nfld;
    // a 128-column tile shape whose last column tile would hold at most 64
    // valid columns covers those with one 64-column tile (FP32 has a 128 x 64
    // kernel) in a second launch
    auto tail_of = [&](int bm, int bn) {
        return p.prec == SHTX_FP32 && bm == 128 && bn == 128 && ncol > 128 && ncol % 128 != 0 && ncol % 128 <= 64
                   ? 64
                   : 0;
    };
    p.inv_tail_bn = tail_of(p.inv_bm, p.inv_bn);
    p.dir_tail_bn = tail_of(p.dir_bm, p.dir_bn);
    std::vector<std::vector<GemmItem>> gi, gd, ti, td;
    std::vector<double> ci, cd, cti, ctd;
    for (int m = 0; m <= N; ++m) {
        const MBlock &b = p.mb[m];
        double cost = (double)std::max(b.R, 1) * (N - m + 1) * ncol;
        std::vector<GemmItem> a, c, at, ct;
        // main column tiles, then the tail tile's index in units of tail_bn
        int ntc_i = p.inv_tail_bn ? ncol / p.inv_bn : (ncol + p.inv_bn - 1) / p.inv_bn;
        int ntr_i = (b.R + p.inv_bm - 1) / p.inv_bm;
        for (int tr = 0; tr < ntr_i; ++tr) {
            for (int tc = 0; tc < ntc_i; ++tc) a.push_back(GemmItem{m, tr, tc, 0});
            if (p.inv_tail_bn) at.push_back(GemmItem{m, tr, ntc_i * p.inv_bn / p.inv_tail_bn, 0});
        }
        int ntc_d = p.dir_tail_bn ? ncol / p.dir_bn : (ncol + p.dir_bn - 1) / p.dir_bn;
        int ntk_d = (b.K0 + p.dir_bm - 1) / p.dir_bm;
        for (int tk = 0; tk < ntk_d; ++tk) {
            for (int tc = 0; tc < ntc_d; ++tc) c.push_back(GemmItem{m, tk, tc, 0});
            if (p.dir_tail_bn) ct.push_back(GemmItem{m, tk, ntc_d * p.dir_bn / p.dir_tail_bn, 0});
        }
        if (!a.empty()) {
            gi.push_back(a);
            ci.push_back(cost);
            if (!at.empty()) {
                ti.push_back(at);
                cti.push_back(cost);
            }
        }
        gd.push_back(c);
        cd.push_back(cost);
        if (!ct.empty()) {
            td.push_back(ct);
            ctd.push_back(cost);
        }
    }
    p.inv_items = layout_by_xcd(gi, ci, GemmItem{-1, 0, 0, 0});
    p.dir_items = layout_by_xcd(gd, cd, GemmItem{-1, 0, 0, 0});
    p.inv_nmain = (int)p.inv_items.size();
    p.dir_nmain = (int)p.dir_items.size();
    if (!ti.empty()) {
        std::vector<GemmItem> t = layout_by_xcd(ti, cti, GemmItem{-1, 0, 0, 0});
        p.inv_items.insert(p.inv_items.end(), t.begin(), t.end());
    }
    if (!td.empty()) {
        std::vector<GemmItem> t = layout_by_xcd(td, ctd, GemmItem{-1, 0, 0, 0});
        p.dir_items.insert(p.dir_items.end(), t.begin(), t.end());
    }
    return SHTX_OK;
}

// Host part of plan construction: geometry, table layout, FFT length plans
// and twiddle tables (kept on the host until uploaded), GEMM and FFT work
// lists.  Touches no device state, so it can be checked on any machine.
int plan_layout(Plan &p, int trunc, int grid, int nlat, int nlon_full, int nfld, int prec, unsigned flags)
{
    if (trunc < 0 || nfld < 1 || nlat < 2) return SHTX_EINVAL;
    if (grid != SHTX_GRID_FULL && grid != SHTX_GRID_OCTAHEDRAL) return SHTX_EINVAL;
    if (prec != SHTX_FP64 && prec != SHTX_FP32 && !split_form(prec)) return SHTX_EINVAL;
    if (nlat % 2) return SHTX_EUNSUPPORTED;
    if (grid == SHTX_GRID_FULL && (nlon_full < 2 || nlon_full % 2)) return nlon_full < 2 ? SHTX_EINVAL : SHTX_EUNSUPPORTED;
    if (trunc > 4095 || nlat > 16384 || nfld > (1 << 20)) return SHTX_EUNSUPPORTED;
    // wind images: truncation N + 1 >= 1 and fields U then V
    if ((flags & SHTX_FLAG_UV) && (trunc < 1 || nfld % 2)) return SHTX_EINVAL;

    p.trunc = trunc;
    p.grid = grid;
    p.nlat = nlat;
    p.nlon_full = nlon_full;
    p.nfld = nfld;
    p.prec = prec;
    p.flags = flags;
    const int N = trunc, NL = nlat / 2, F = nfld;

    // ---- ring geometry ----------------------------------------------------
    p.nlon.resize(nlat);
    p.cutoff.resize(nlat);
    for (int j = 0; j < nlat; ++j) {
        int i = j < NL ? j : nlat - 1 - j;
        p.nlon[j] = grid == SHTX_GRID_FULL ? nlon_full : 20 + 4 * i;
        p.cutoff[j] = ring_cutoff(N, p.nlon[j]);
        p.max_nlon = std::max(p.max_nlon, p.nlon[j]);
    }
    // The Legendre GEMM rows are the band of northern rings carrying m; it is
    // contiguous because the cutoff never decreases towards the equator.
    for (int j = 1; j < NL; ++j)
        if (p.cutoff[j] < p.cutoff[j - 1]) return SHTX_EUNSUPPORTED;
    p.nspec = (int64_t)(N + 1) * (N + 2) / 2;

    // ---- m blocks -----------------------------------------------------------
    p.mb.resize(N + 1);
    int64_t off = 0;
    double flops = 0.0;
    for (int m = 0; m <= N; ++m) {
        MBlock b{};
        int j0 = NL;
        for (int j = 0; j < NL; ++j)
            if (p.cutoff[j] >= m) {
                j0 = j;
                break;
            }
        b.R = NL - j0;
        b.j0 = j0;
        b.K0 = (N - m) / 2 + 1;
        b.K1 = (N - m + 1) / 2;
        b.Rp = (int)round_up(std::max(b.R, 1), kTablePad);
        b.Kp = (int)round_up(b.K0, kTablePad);
        b.off_kr = off;
        b.off_rk = off;
        off += 2 * (int64_t)b.Kp * b.Rp;
        p.mb[m] = b;
        flops += 4.0 * F * (double)b.R * (N - m + 1);
    }
    p.tab_elems = off;
    p.legendre_flops = flops;

    size_t tab_el = prec == SHTX_FP64 ? 8 : prec == SHTX_FP32 ? 4 : 2;
    p.table_bytes = (split_form(prec) ? 4 : 2) * tab_el * p.tab_elems;

    // ---- ring FFT plans and twiddle pool --------------------------------------
    const bool dbl = prec == SHTX_FP64;
    const int cap = dbl ? kFftCapF64 : kFftCapF32;
    struct LenPlan {
        int L, blue, pass_off;
        std::vector<int> rad;
        int64_t tw, post, chirp, bhat;
    };
    std::map<int, LenPlan> lens;
    std::vector<long double> pool;  // interleaved re, im
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < nlat; ++j) {
        int n = p.nlon[j];
        if (lens.count(n)) continue;
        int h = n / 2;
        LenPlan lp{};
        std::vector<int> f;
        const int maxp = dbl ? 17 : 23;
        const int rem = smooth_factor(h, f, maxp);
        // Bluestein length: the smallest 2^a 3^b >= 2h - 1 with 9 | L
        // (radix-16/9 passes; the leading radix-9 passes keep the power-of-two
        // passes' LDS writes off a single bank); if that exceeds the LDS cap
        // (rings of more than about 7776 points), the smallest such length
        // that may also hold factors 5 (radix-5 passes), e.g. 8100 for the
        // longest TCo1999 rings
        auto smallest = [](int lo, bool fives) {
            for (int x = lo;; ++x) {
                int y = x, threes = 0;
                while (y % 2 == 0) y /= 2;
                while (y % 3 == 0) y /= 3, ++threes;
                while (fives && y % 5 == 0) y /= 5;
                if (y == 1 && threes >= 2) return x;
            }
        };
        int Lb = smallest(2 * h - 1, false);
        if (Lb > cap) Lb = smallest(2 * h - 1, true);
        // one prime factor above the register radices, up to kGpMaxPrime, is
        // run as a general prime pass (first, at Ns = 1) instead of Bluestein
        // when one field's output units fit the block's waves and, above 191,
        // when the cost model of the two (fitted to single-precision ring
        // FFT timings on MI355X, in ps per grid point: prime pass
        // 3.2 + 0.0086 p, Bluestein 0.37 (L / h) log2 L) favours it; the same
        // choice measured faster in double precision too (C5 c2r 29.2 ->
        // 27.1 ms against the prime pass limited to 191)
        bool gp = rem > 1 && rem <= kGpMaxPrime && is_prime(rem) &&
                  gp_row_tiles(rem) * gp_col_tiles(h / rem) <= kGpUnits * (kFftThreads / 64);
        if (gp && rem > 191 && Lb <= cap) gp = 3.2 + 0.0086 * rem < 0.37 * Lb / h * std::log2((double)Lb);
        if (rem == 1 || gp) {
            lp.L = h;
            lp.blue = 0;
        } else {
            lp.L = Lb;
            lp.blue = 1;
        }
        if (std::max(lp.L, h + 1) > cap) return SHTX_EUNSUPPORTED;
        if (gp) {
            lp.rad = radices_for(lp.L / rem);
            lp.rad.insert(lp.rad.begin(), rem);
        } else {
            lp.rad = radices_for(lp.L);
        }
        if ((int)lp.rad.size() > kMaxRadices) return SHTX_EUNSUPPORTED;
        lp.pass_off = (int)p.passes.size();
        for (int s = 0, Ns = 1; s < (int)lp.rad.size(); Ns *= lp.rad[s], ++s) {
            PassDesc q{};
            q.R = lp.rad[s];
            q.Ns = Ns;
            q.nbf = lp.L / q.R;
            q.tstep = lp.L / (Ns * q.R);
            q.mg_nbf = div_magic(q.nbf);
            q.mg_ns = div_magic(Ns);
            p.passes.push_back(q);
        }
        auto push = [&](long double re, long double im) {
            pool.push_back(re);
            pool.push_back(im);
        };
        lp.tw = (int64_t)pool.size() / 2;
        for (int k = 0; k < lp.L; ++k) {
            long double a = 2.0L * pi * k / lp.L;
            push(cosl(a), -sinl(a));
        }
        lp.post = (int64_t)pool.size() / 2;
        for (int m = 0; m <= h; ++m) {
            long double a = 2.0L * pi * m / n;
            push(cosl(a), -sinl(a));
        }
        lp.chirp = lp.bhat = -1;
        if (lp.blue) {
            lp.chirp = (int64_t)pool.size() / 2;
            for (int k = 0; k < h; ++k) {
                int64_t t = ((int64_t)k * k) % (2 * (int64_t)h);
                long double a = pi * (long double)t / h;
                push(cosl(a), -sinl(a));
            }
            std::vector<long double> bre, bim;
            bluestein_filter(h, lp.L, bre, bim);
            lp.bhat = (int64_t)pool.size() / 2;
            for (int k = 0; k < lp.L; ++k) push(bre[k], bim[k]);
        }
        lens[n] = lp;
    }
    size_t celem = dbl ? 16 : 8;
    p.twid_elems = (int64_t)pool.size() / 2;
    p.twid_host.assign(pool.begin(), pool.end());
    p.workspace_bytes += (size_t)p.twid_elems * celem;

    p.rings.resize(nlat);
    int64_t goff = 0, foff = 0;
    for (int j = 0; j < nlat; ++j) {
        RingDesc d{};
        const LenPlan &lp = lens[p.nlon[j]];
        d.n = p.nlon[j];
        d.h = d.n / 2;
        d.M = p.cutoff[j];
        d.L = lp.L;
        d.blue = lp.blue;
        d.nrad = (int)lp.rad.size();
        d.pass_off = lp.pass_off;
        d.radcode = 0;
        // code 0 marks a general prime pass (its radix is in the pass descriptor)
        for (int r = 0; r < d.nrad; ++r) {
            const bool gp = lp.rad[r] > (prec == SHTX_FP64 ? 17 : 23);
            d.radcode |= (unsigned long long)(gp ? 0 : lp.rad[r]) << (5 * r);
        }
        d.lbuf = std::max(d.L, d.h + 1);
        d.lbufp = d.lbuf;
        d.tw_off = lp.tw;
        d.post_off = lp.post;
        d.chirp_off = lp.chirp;
        d.bhat_off = lp.bhat;
        d.grid_off = goff;
        d.four_off = foff;
        d.w = 0.0;  // filled in once the device has computed the weights
        goff += d.n;
        foff += (int64_t)(d.M + 1) * F;
        p.rings[j] = d;
    }
    p.npts = goff;
    p.nfour = foff / F;
    if (p.nfour > INT32_MAX) return SHTX_EUNSUPPORTED;  // ring offsets are stored as int32 / nfld
    int rc = fft_blocking(p, cap);
    if (rc != SHTX_OK) return rc;

    // ---- GEMM work lists ----------------------------------------------------------
    gemm_tiles(prec, &p.inv_bm, &p.inv_bn, &p.dir_bm, &p.dir_bn);
    rc = gemm_work_lists(p);
    if (rc != SHTX_OK) return rc;

    p.workspace_bytes += (size_t)p.nfour * F * celem;
    return SHTX_OK;
}

// Full plan: host layout, then the device work (nodes, weights, tables,
// uploads, workspace) on `stream`.
int build_plan(Plan &p, int trunc, int grid, int nlat, int nlon_full, int nfld, int prec,
               unsigned flags, hipStream_t stream)
{
    auto t0 = std::chrono::steady_clock::now();
    int rc = plan_layout(p, trunc, grid, nlat, nlon_full, nfld, prec, flags);
    if (rc != SHTX_OK) return rc;
    if (!gemm_shapes_ok(p) || !fft_shapes_ok(p)) return SHTX_EUNSUPPORTED;
    const int N = trunc, NL = nlat / 2;
    PLAN_TRY(hipGetDevice(&p.device));

    // ---- Gauss nodes and Legendre tables (device, FP64) ---------------------
    PLAN_TRY(hipMalloc(&p.d_mu, sizeof(double) * nlat));
    PLAN_TRY(hipMalloc(&p.d_w, sizeof(double) * nlat));
    PLAN_TRY(launch_gauss_nodes(nlat, p.d_mu, p.d_w, stream));

    size_t tab_el = prec == SHTX_FP64 ? 8 : prec == SHTX_FP32 ? 4 : 2;
    PLAN_TRY(hipMalloc(&p.d_tab_kr, tab_el * p.tab_elems));
    PLAN_TRY(hipMalloc(&p.d_tab_rk, tab_el * p.tab_elems));
    p.table_bytes = 2 * tab_el * p.tab_elems;
    if (split_form(prec)) {
        PLAN_TRY(hipMalloc(&p.d_tab_kr_lo, tab_el * p.tab_elems));
        PLAN_TRY(hipMalloc(&p.d_tab_rk_lo, tab_el * p.tab_elems));
        p.table_bytes *= 2;
    }
    PLAN_TRY(hipMalloc(&p.d_diag, sizeof(double) * (size_t)NL * (N + 1)));
    PLAN_TRY(hipMalloc(&p.d_diag_e, sizeof(int) * (size_t)NL * (N + 1)));
    PLAN_TRY(hipMalloc(&p.d_mmax, sizeof(unsigned long long) * (N + 1)));
    PLAN_TRY(upload(&p.d_mb, p.mb));
    PLAN_TRY(launch_legendre_tables(p, stream));
    PLAN_TRY(hipStreamSynchronize(stream));
    // exponents were decided on the device; refresh the host copy
    PLAN_TRY(hipMemcpy(p.mb.data(), p.d_mb, sizeof(MBlock) * p.mb.size(), hipMemcpyDeviceToHost));
    (void)hipFree(p.d_diag);
    p.d_diag = nullptr;
    (void)hipFree(p.d_diag_e);
    p.d_diag_e = nullptr;
    (void)hipFree(p.d_mmax);
    p.d_mmax = nullptr;


    std::vector<double> w(nlat);
    PLAN_TRY(hipMemcpy(w.data(), p.d_w, sizeof(double) * nlat, hipMemcpyDeviceToHost));
    for (int j = 0; j < nlat; ++j) p.rings[j].w = w[j];
    for (int j = 0; j < nlat / 2; ++j) p.qmax = std::max(p.qmax, 0.5 * w[j]);
    if (prec == SHTX_FP16X3) {
        // written by every transform before it is read; zero until then (the
        // autotuner times the GEMMs alone)
        PLAN_TRY(hipMalloc(&p.d_fmax, sizeof(unsigned) * nfld));
        PLAN_TRY(hipMemset(p.d_fmax, 0, sizeof(unsigned) * nfld));
    }

    const bool dbl = prec == SHTX_FP64;
    size_t celem = dbl ? 16 : 8;
    {
        size_t bytes = (size_t)p.twid_elems * celem;
        PLAN_TRY(hipMalloc(&p.d_twid, bytes));
        if (dbl) {
            PLAN_TRY(hipMemcpy(p.d_twid, p.twid_host.data(), bytes, hipMemcpyHostToDevice));
        } else {
            std::vector<float> host(p.twid_host.size());
            for (size_t i = 0; i < host.size(); ++i) host[i] = (float)p.twid_host[i];
            PLAN_TRY(hipMemcpy(p.d_twid, host.data(), bytes, hipMemcpyHostToDevice));
        }
        std::vector<double>().swap(p.twid_host);
    }
    PLAN_TRY(upload(&p.d_rings, p.rings));
    {
        std::vector<int64_t> fo(nlat);
        for (int j = 0; j < nlat; ++j) fo[j] = p.rings[j].four_off;
        PLAN_TRY(upload(&p.d_ring_four_off, fo));
        std::vector<RingPair> rp(nlat / 2);
        for (int j = 0; j < nlat / 2; ++j)
            rp[j] = RingPair{(int)(fo[j] / nfld), (int)(fo[nlat - 1 - j] / nfld)};
        PLAN_TRY(upload(&p.d_ring_pair, rp));
        if (dbl) {
            std::vector<double> q(nlat / 2);
            for (int j = 0; j < nlat / 2; ++j) q[j] = 0.5 * w[j];
            PLAN_TRY(upload(reinterpret_cast<double **>(&p.d_ring_q), q));
        } else {
            std::vector<float> q(nlat / 2);
            for (int j = 0; j < nlat / 2; ++j) q[j] = (float)(0.5 * w[j]);
            PLAN_TRY(upload(reinterpret_cast<float **>(&p.d_ring_q), q));
        }
    }
    PLAN_TRY(upload(&p.d_passes, p.passes));
    // checks every launch shape once more and uploads the work lists
    rc = apply_shapes(p, p.inv_bm, p.inv_bn, p.dir_bm, p.dir_bn, p.fft_cap);
    if (rc != SHTX_OK) return rc;
    PLAN_TRY(fft_prepare(p));
    PLAN_TRY(hipEventCreateWithFlags(&p.done, hipEventDisableTiming));

    PLAN_TRY(hipMalloc(&p.d_four, (size_t)p.nfour * nfld * celem));
    if (flags & SHTX_FLAG_UV) {
        PLAN_TRY(hipMalloc(&p.d_uvspec, (size_t)p.nspec * nfld * celem));
        p.workspace_bytes += (size_t)p.nspec * nfld * celem;
    }

    if (flags & SHTX_FLAG_AUTOTUNE) {
        int trc = autotune_plan(p, stream);
        if (trc != SHTX_OK) return trc;
    }

    if (flags & SHTX_FLAG_TIMING) {
        p.timing_on = true;
        p.ev_start.resize(Plan::kMaxTimed);
        p.ev_stop.resize(Plan::kMaxTimed);
        p.ev_kind.resize(Plan::kMaxTimed);
        for (int i = 0; i < Plan::kMaxTimed; ++i) {
            PLAN_TRY(hipEventCreate(&p.ev_start[i]));
            PLAN_TRY(hipEventCreate(&p.ev_stop[i]));
        }
    }
    PLAN_TRY(hipStreamSynchronize(stream));
    p.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return SHTX_OK;
}

}  // namespace shtx
