// Batched real FFTs along the latitude rings, one launch over every
// (ring, run of fields).
//
// A real ring of n = 2h points goes through one complex DFT of length h
// (even samples as real part, odd samples as imaginary part) with the usual
// split/merge step around it.  The length-h DFT is a Stockham autosort
// mixed-radix FFT (radices 16, 9, 8, 4, 2, 3 and the primes 5 to 23; 17 in
// FP64) held in LDS, run in place: each pass reads its butterflies into
// registers, synchronises, then writes.  One larger prime factor (up to 1021:
// always up to 191, above that where the plan's cost model prefers it to
// Bluestein) runs as a general prime pass on the matrix cores (below); other
// lengths go through Bluestein's chirp convolution at a length L = 2^a 3^b
// >= 2h - 1 (2^a 3^b 5^c when that exceeds the LDS cap), with the filter
// spectrum precomputed per ring length at plan time.  Only the kept
// wavenumbers m <= M_j are read or written; they live in the Fourier
// workspace laid out [ring][m][field], so a block's loads and stores are runs
// over fields.  For the split IEEE-half Legendre form the r2c kernel also
// records each field's largest output magnitude (the bound from which the
// direct GEMM scales its data operand).
//
// Inverse (c2r):  g_k = s_j * (Re Y_0 + 2 sum_{m=1}^{M} Re(Y_m e^{2 pi i m k / n}))
//   transform:            Y_m = F_m,                    s_j = 1
//   adjoint of direct:    Y_m = F_m / c_m,              s_j = w_j / (2 n)
// Direct (r2c):   G_m = s_j fac_m sum_k g_k e^{-2 pi i m k / n},  m <= M
//   transform:            fac_m = 1,    s_j = 1 / n
//   adjoint of inverse:   fac_m = c_m,  s_j = 1
//
// The paper (Section 3.1.1) keeps fields resident on the device and packs on
// the device; this kernel's layout and algorithm are this library's own.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "fft_roots.h"
#include "shtx_internal.h"

namespace shtx {

namespace {

template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) C2 {
    T x, y;
};

template <typename T>
__device__ inline C2<T> cmul(C2<T> a, C2<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ inline C2<T> cadd(C2<T> a, C2<T> b)
{
    return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ inline C2<T> csub(C2<T> a, C2<T> b)
{
    return {a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ inline C2<T> cconj(C2<T> a)
{
    return {a.x, -a.y};
}
// multiply by -i
template <typename T>
__device__ inline C2<T> cmi(C2<T> a)
{
    return {a.y, -a.x};
}

// Dynamic LDS of the FFT kernels, declared once at namespace scope so that the
// non-inlined pass functions address it as LDS (ds_* instructions) rather
// than through generic pointers.
extern __shared__ __attribute__((aligned(16))) unsigned char fft_smem[];

// Typed LDS pointers: address arithmetic on them stays 32-bit.
template <typename T>
using LdsC2 = __attribute__((address_space(3))) C2<T>;
template <typename T>
__device__ inline LdsC2<T> *lds_c2() { return (LdsC2<T> *)(__attribute__((address_space(3))) unsigned char *)fft_smem; }
// LDS byte addressing for the Stockham passes: element r of a butterfly sits
// at base + r * stride, formed with one 24-bit multiply-add per element.
typedef __attribute__((address_space(3))) unsigned char LdsByte;

// One complex value in or out of LDS as a single 2-element access.
template <typename T>
__device__ inline C2<T> ldc(const LdsC2<T> *p)
{
    typedef T V2 __attribute__((ext_vector_type(2)));
    V2 w = *(const __attribute__((address_space(3))) V2 *)p;
    return C2<T>{w.x, w.y};
}
template <typename T>
__device__ inline void stc(LdsC2<T> *p, C2<T> v)
{
    typedef T V2 __attribute__((ext_vector_type(2)));
    *(__attribute__((address_space(3))) V2 *)p = V2{v.x, v.y};
}
template <typename T>
__device__ inline C2<T> ldb(unsigned a)
{
    return ldc((const LdsC2<T> *)((LdsByte *)fft_smem + a));
}
template <typename T>
__device__ inline void stb(unsigned a, C2<T> v)
{
    stc((LdsC2<T> *)((LdsByte *)fft_smem + a), v);
}

struct FftArgs {
    const RingDesc *rings;
    const FftItem *items;
    const PassDesc *passes;
    const void *twid;
    const void *in;
    void *out;
    int nfld;
    int adjoint;
    int64_t npts;
    // r2c only, when not null: per field, the largest magnitude of the
    // Fourier values written (float bits, atomic max), collected per block in
    // nf words of LDS at byte offset fmax_lds
    unsigned *fmax;
    int fmax_lds;
};

// exp(-2 pi i t / R) for the odd prime radices (t taken mod R), as
// compile-time constants.
template <typename T, int R>
__device__ constexpr C2<T> root(int t)
{
    t %= R;
    const int u = t <= R / 2 ? t : R - t;
    const double sn = PrimeRoots<R>::s[u];
    return C2<T>{T(PrimeRoots<R>::c[u]), T(t <= R / 2 ? -sn : sn)};
}

// Forward radix-R DFT of v in registers.
template <typename T, int R>
__device__ inline void dft_reg(C2<T> *v)
{
    if constexpr (R == 2) {
        C2<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        // X_1,2 = v0 - (v1 + v2)/2 -+ i (sqrt3/2)(v1 - v2)
        const T r3 = T(0.86602540378443864676372317075293618347);
        C2<T> sm = cadd(v[1], v[2]), df = csub(v[1], v[2]);
        C2<T> t = {v[0].x - T(0.5) * sm.x, v[0].y - T(0.5) * sm.y};
        C2<T> u = {r3 * df.y, -r3 * df.x};  // -i (sqrt3/2) df
        v[0] = cadd(v[0], sm);
        v[1] = cadd(t, u);
        v[2] = csub(t, u);
    } else if constexpr (R == 9) {
        // 9 = 3 x 3: radix-3 over n1 for each n2 (x = v[3 n1 + n2]), twiddles
        // exp(-2 pi i n2 k1 / 9), radix-3 over n2 for each k1
        const C2<T> tw[5] = {{T(1), T(0)},
                             {T(0.76604444311897803520239265055541667394), T(-0.64278760968653932632264340990726343291)},
                             {T(0.17364817766693034885171662676931479600), T(-0.98480775301220805936674302458952301367)},
                             {T(0), T(0)},
                             {T(-0.93969262078590838405410927732473146993), T(-0.34202014332566873304409961468225958076)}};
        C2<T> y[3][3];
#pragma unroll
        for (int n2 = 0; n2 < 3; ++n2) {
            C2<T> t[3] = {v[n2], v[3 + n2], v[6 + n2]};
            dft_reg<T, 3>(t);
#pragma unroll
            for (int k1 = 0; k1 < 3; ++k1) y[n2][k1] = (n2 && k1) ? cmul(t[k1], tw[n2 * k1]) : t[k1];
        }
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) {
            C2<T> t[3] = {y[0][k1], y[1][k1], y[2][k1]};
            dft_reg<T, 3>(t);
#pragma unroll
            for (int k2 = 0; k2 < 3; ++k2) v[k1 + 3 * k2] = t[k2];
        }
    } else if constexpr (R == 4) {
        C2<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        C2<T> s13 = cadd(v[1], v[3]), d13 = cmi(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else if constexpr (R == 8) {
        // two radix-4 DFTs (even and odd samples) merged with exp(-2 pi i k / 8)
        C2<T> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        dft_reg<T, 4>(e);
        dft_reg<T, 4>(o);
        const T c = T(0.70710678118654752440084436210484903928);
        C2<T> o1 = {c * (o[1].x + o[1].y), c * (o[1].y - o[1].x)};   // * (1 - i)/sqrt2
        C2<T> o2 = cmi(o[2]);                                           // * -i
        C2<T> o3 = {c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y)};   // * (-1 - i)/sqrt2
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    } else if constexpr (R == 16) {
        // 16 = 4 x 4: radix-4 DFTs over n1 for each n2 (x = v[4 n1 + n2]),
        // twiddles exp(-2 pi i n2 k1 / 16), radix-4 DFTs over n2 for each k1
        const T c1 = T(0.92387953251128675612818318939678828682);  // cos(pi/8)
        const T s1 = T(0.38268343236508977172845998403039886676);  // sin(pi/8)
        const T h = T(0.70710678118654752440084436210484903928);
        const C2<T> tw[10] = {{T(1), T(0)}, {c1, -s1}, {h, -h}, {s1, -c1}, {T(0), T(-1)},
                              {-s1, -c1}, {-h, -h}, {-c1, -s1}, {T(-1), T(0)}, {-c1, s1}};
        C2<T> y[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            C2<T> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
            dft_reg<T, 4>(t);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = (n2 && k1) ? cmul(t[k1], tw[n2 * k1]) : t[k1];
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            C2<T> t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
            dft_reg<T, 4>(t);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
        }
    } else {
        // odd R: pair r with R - r
        constexpr int H = (R - 1) / 2;
        C2<T> sum[H], dif[H];
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            sum[r - 1] = cadd(v[r], v[R - r]);
            dif[r - 1] = csub(v[r], v[R - r]);
        }
        C2<T> x0 = v[0];
        C2<T> out0 = x0;
#pragma unroll
        for (int r = 0; r < H; ++r) out0 = cadd(out0, sum[r]);
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            C2<T> re = x0, im = {T(0), T(0)};
#pragma unroll
            for (int r = 1; r <= H; ++r) {
                const C2<T> w = root<T, R>(k * r);  // (cos, -sin) of 2 pi k r / R
                re.x += sum[r - 1].x * w.x;
                re.y += sum[r - 1].y * w.x;
                im.x += dif[r - 1].x * w.y;
                im.y += dif[r - 1].y * w.y;
            }
            // X_k = re + i*im', X_{R-k} = re - i*im' with im' = -sum dif sin
            v[k] = {re.x - im.y, re.y + im.x};
            v[R - k] = {re.x + im.y, re.y - im.x};
        }
        v[0] = out0;
    }
}

// Elements per thread whose global loads are issued together in the
// kernels' gather and scatter loops.
constexpr int kU = 4;

// floor(a / d) as mul_hi(a, magic), magic = ceil(2^32 / d) (PassDesc): exact
// for a * d < 2^32, which every caller keeps (a and d are at most a few
// times the LDS capacity).  magic 0 stands for d = 1.
__device__ inline int udiv(int a, unsigned magic) { return magic ? (int)__umulhi((unsigned)a, magic) : a; }

// Block-uniform values passed to the non-inlined pass functions arrive in
// vector registers; these move them to scalar registers.
__device__ inline int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline unsigned uni(unsigned x) { return (unsigned)__builtin_amdgcn_readfirstlane((int)x); }
__device__ inline PassDesc uniform(PassDesc d)
{
    d.R = uni(d.R);
    d.Ns = uni(d.Ns);
    d.nbf = uni(d.nbf);
    d.tstep = uni(d.tstep);
    d.mg_nbf = uni(d.mg_nbf);
    d.mg_ns = uni(d.mg_ns);
    return d;
}


// The table reads behind the twiddle powers of one butterfly: w = W[t1]
// (w = exp(-2 pi i k / (Ns R))) and, for radix 9 and 16, w^3 or w^4.
template <int R>
constexpr int twiddle_step2() { return R == 9 ? 3 : R == 16 ? 4 : 0; }

// Powers w^r (r = 1 .. R-1) from w and the second table value, by products
// at most three deep; tw[0] is unused.
template <typename T, int R>
__device__ inline void twiddle_powers(C2<T> *tw, C2<T> w1, C2<T> w2nd)
{
    tw[1] = w1;
    if constexpr (R == 9) {
        tw[2] = cmul(tw[1], tw[1]);
        tw[3] = w2nd;
        tw[6] = cmul(w2nd, w2nd);
#pragma unroll
        for (int a = 3; a <= 6; a += 3)
#pragma unroll
            for (int b = 1; b <= 2; ++b) tw[a + b] = cmul(tw[a], tw[b]);
    } else if constexpr (R == 16) {
        tw[2] = cmul(tw[1], tw[1]);
        tw[3] = cmul(tw[1], tw[2]);
        tw[4] = w2nd;
        tw[8] = cmul(w2nd, w2nd);
        tw[12] = cmul(w2nd, tw[8]);
#pragma unroll
        for (int a = 4; a <= 12; a += 4)
#pragma unroll
            for (int b = 1; b <= 3; ++b) tw[a + b] = cmul(tw[a], tw[b]);
    } else {
        if constexpr (R > 2) tw[2] = cmul(tw[1], tw[1]);
        if constexpr (R > 3) tw[3] = cmul(tw[1], tw[2]);
        if constexpr (R > 4) tw[4] = cmul(tw[2], tw[2]);
#pragma unroll
        for (int r = 5; r < R; ++r) tw[r] = cmul(tw[4], tw[r - 4]);
    }
}

// Radix-R DFT (R odd prime) of v, written to LDS as it is formed: output t
// goes to byte address a0 + t * stride.  Sums and differences of the pairs
// (r, R - r) replace the inputs in place, so only the inputs and two
// accumulators are live (the same arithmetic as dft_reg's odd radices).
template <typename T, int R>
__device__ inline void odd_butterfly_store(C2<T> *v, unsigned a0, unsigned stride)
{
    constexpr int H = (R - 1) / 2;
    const C2<T> x0 = v[0];
    C2<T> out0 = x0;
#pragma unroll
    for (int r = 1; r <= H; ++r) {
        const C2<T> sm = cadd(v[r], v[R - r]), df = csub(v[r], v[R - r]);
        v[r] = sm;
        v[R - r] = df;
        out0 = cadd(out0, sm);
    }
    stb<T>(a0, out0);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        C2<T> re = x0, im = {T(0), T(0)};
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            const C2<T> w = root<T, R>(k * r);  // (cos, -sin) of 2 pi k r / R
            re.x += v[r].x * w.x;
            re.y += v[r].y * w.x;
            im.x += v[R - r].x * w.y;
            im.y += v[R - r].y * w.y;
        }
        stb<T>(a0 + __umul24((unsigned)k, stride), C2<T>{re.x - im.y, re.y + im.x});
        stb<T>(a0 + __umul24((unsigned)(R - k), stride), C2<T>{re.x + im.y, re.y - im.x});
    }
}

// One in-place Stockham pass of radix R over nf fields of length L in LDS:
// every thread reads all of its butterflies into registers, the block
// synchronises, then each butterfly is twiddled, transformed and written.
// BHAT (the first pass of Bluestein's second FFT, where Ns = 1): each input
// X_i is first replaced by conj(X_i bhat_i), the pointwise step of the chirp
// convolution.
template <typename T>
using GlobalC2 = const __attribute__((address_space(1))) C2<T>;

template <typename T, int R, int CAP, bool BHAT, typename WPtr>
__device__ __attribute__((noinline)) void stockham_pass_impl(int buf_off, int lbufp, int nf, PassDesc pd, WPtr W,
                                                             GlobalC2<T> *bhat)
{
    constexpr int NB = fft_rounds(CAP, R);
    constexpr int C2ND = twiddle_step2<R>();
    constexpr unsigned CB = sizeof(C2<T>);
    pd = uniform(pd);
    buf_off = uni(buf_off);
    lbufp = uni(lbufp);
    nf = uni(nf);
    const int nbf = pd.nbf, total = nf * nbf, Ns = pd.Ns;
    const unsigned srd = nbf * CB, swr = Ns * CB;  // byte strides of a butterfly's reads and writes
    // radices above 19 run a streamed butterfly: twiddles by stepping from
    // table values read every 8 powers, outputs stored as they are formed
    constexpr bool STREAM = R > 19;
    constexpr int NRS = STREAM ? (R + 6) / 8 : 1;  // table restarts at powers 1, 9, 17, 25
    C2<T> v[NB][R];
    C2<T> w1[NB], w2[NB];  // twiddle table values, fetched before the barrier
    C2<T> wrs[NB][NRS];
    int fo[NB], qk[NB][2];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        int e = threadIdx.x + b * kFftThreads;
        if (e < total) {
            int f = udiv(e, pd.mg_nbf), j = e - f * nbf;
            int q = udiv(j, pd.mg_ns), k = j - q * Ns;
            fo[b] = buf_off + f * lbufp;
            qk[b][0] = q;
            qk[b][1] = k;
            if (Ns > 1) {
                const int t1 = k * pd.tstep;
                w1[b] = C2<T>{W[t1].x, W[t1].y};
                if constexpr (C2ND > 0) w2[b] = C2<T>{W[C2ND * t1].x, W[C2ND * t1].y};
                if constexpr (STREAM) {
#pragma unroll
                    for (int c = 0; c < NRS; ++c) wrs[b][c] = C2<T>{W[(8 * c + 1) * t1].x, W[(8 * c + 1) * t1].y};
                }
            }
            const unsigned a0 = (unsigned)(fo[b] + j) * CB;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = ldb<T>(a0 + __umul24((unsigned)r, srd));
            if constexpr (BHAT) {
                // first pass of Bluestein's second FFT (Ns = 1): its inputs
                // are conj(X_i bhat_i), X the first FFT's output
#pragma unroll
                for (int r = 0; r < R; ++r)
                    v[b][r] = cconj(cmul(v[b][r], C2<T>{bhat[j + r * nbf].x, bhat[j + r * nbf].y}));
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        int e = threadIdx.x + b * kFftThreads;
        if (e < total) {
            const int q = qk[b][0], k = qk[b][1];
            const int base = q * Ns * R + k;
            const unsigned a0 = (unsigned)(fo[b] + base) * CB;
            if constexpr (STREAM) {
                if (Ns > 1) {
                    C2<T> t = wrs[b][0];
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        if (r > 1) t = ((r - 1) % 8 == 0) ? wrs[b][(r - 1) / 8] : cmul(t, w1[b]);
                        v[b][r] = cmul(v[b][r], t);
                    }
                }
                odd_butterfly_store<T, R>(v[b], a0, swr);
            } else {
                if (Ns > 1) {
                    C2<T> tw[R];
                    twiddle_powers<T, R>(tw, w1[b], w2[b]);
#pragma unroll
                    for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], tw[r]);
                }
                dft_reg<T, R>(v[b]);
#pragma unroll
                for (int r = 0; r < R; ++r) stb<T>(a0 + __umul24((unsigned)r, swr), v[b][r]);
            }
        }
    }
    __syncthreads();
}

// Twiddles and filter from the global tables (L1/L2 resident), through
// global-address-space pointers so that the pass uses global_* loads.
template <typename T, int R, int CAP, bool BHAT>
__device__ inline void stockham_pass(int buf_off, int lbufp, int nf, const PassDesc &pd, const C2<T> *Wg,
                                     const C2<T> *bhat)
{
    stockham_pass_impl<T, R, CAP, BHAT>(buf_off, lbufp, nf, pd, (GlobalC2<T> *)Wg, (GlobalC2<T> *)bhat);
}

// Radices above the register butterflies run as the general prime pass.
template <typename T>
__host__ __device__ constexpr bool is_gp_radix(int R)
{
    return R > (sizeof(T) == 4 ? 23 : 17);
}

// General prime pass (radix p = pd.R, an odd prime, first pass so Ns = 1 and
// no input twiddles), as matrix products on the matrix cores.  With x_r the
// inputs of butterfly b, w = e^{-2 pi i / p}, H = (p - 1) / 2,
//   X_t = x_0 + P_t + i Q_t,   X_{p-t} = x_0 + P_t - i Q_t,   t = 0 .. H,
//   P_t = sum_{r=1}^{H} Re(w^{rt}) s_r,   Q_t = sum_{r=1}^{H} Im(w^{rt}) d_r,
// s_r = x_r + x_{p-r}, d_r = x_r - x_{p-r}: two real products of an H x H
// matrix (cosines, sines) with an H x (2 x butterflies) matrix whose columns
// are the real and imaginary parts of s or d.  A wave computes 16 x 16 output
// units (rows t, columns (butterfly, re|im)) with 16x16x4 MFMAs: the matrix
// operand is read from a table of the p-th roots in LDS at index r t mod p,
// the data operand forms s and d from the ring's LDS slots as it is read.
// The units' results stay in registers over a barrier (the pass is in place);
// X_t of butterfly j then goes to j p + t.
typedef float gp_f32x4 __attribute__((ext_vector_type(4)));
typedef double gp_f64x4 __attribute__((ext_vector_type(4)));
__device__ inline gp_f32x4 gp_mfma(float a, float b, gp_f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline gp_f64x4 gp_mfma(double a, double b, gp_f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Absolute LDS addresses (the dynamic LDS base already added), for loops that
// step addresses instead of re-adding the base at every access.
__device__ inline unsigned lds_base() { return (unsigned)(uintptr_t)(LdsByte *)fft_smem; }
template <typename T>
__device__ inline T lda(unsigned a)
{
    return *(const __attribute__((address_space(3))) T *)(uintptr_t)a;
}
// One real value to LDS at byte offset a of the dynamic LDS.
template <typename T>
__device__ inline void str(unsigned a, T v)
{
    *(__attribute__((address_space(3))) T *)((LdsByte *)fft_smem + a) = v;
}

// Geometry of a general prime pass shared by its units (block-uniform values
// and the lane's position in the 16 x 16 MFMA layout).
struct GpGeom {
    int p, H, mt, nb, nbf;
    unsigned mg_nbf;
    int buf_off, lbufp, ksteps;
    unsigned rb, rstr, rspan, rstep, lb;
    int lr, lk;
};

// K loop of NJ output units of a general prime pass, run together: for unit
// (row tile i, column tile g) the lane's matrix operand row is t = 16 i + lr
// with roots w^{r t}, r = 1 + lk + 4 k, addressed by (r t mod p) rstr and
// stepped by 4 t mod p with an unsigned min(x, x - span) wrap; its data
// operand column is c = 16 g + lr = 2 b + (re|im), forming s_r and d_r from
// x_r and x_{p-r}.  Operands of step k + 1 are read before the products of
// step k.  Rows r past H in the last step contribute 0.
template <typename T, int NJ, typename V4>
__device__ __attribute__((always_inline)) inline void gp_run(const GpGeom &g, const int (&unit)[NJ], V4 *P, V4 *Q,
                                                             T *x0)
{
    constexpr unsigned CB = sizeof(C2<T>), RB = sizeof(T);
    unsigned ur[NJ], du[NJ], ar[NJ], am[NJ];
    C2<T> w[NJ];
    T xr[NJ], xm[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        const int i = unit[q] % g.mt, gc = unit[q] / g.mt;
        const int t = 16 * i + g.lr;
        ur[q] = (unsigned)((t * (1 + g.lk)) % g.p) * g.rstr;
        du[q] = (unsigned)((4 * t) % g.p) * g.rstr;
        const int c = 16 * gc + g.lr;
        const int b = min(c >> 1, g.nb - 1);
        const int f = udiv(b, g.mg_nbf), j = b - f * g.nbf;
        const unsigned slot = g.lb + (unsigned)(g.buf_off + f * g.lbufp + j) * CB + (unsigned)(c & 1) * RB;
        ar[q] = slot + (unsigned)(1 + g.lk) * g.nbf * CB;
        am[q] = slot + (unsigned)(g.p - 1 - g.lk) * g.nbf * CB;
        x0[q] = lda<T>(slot);
        P[q] = V4{T(0), T(0), T(0), T(0)};
        Q[q] = V4{T(0), T(0), T(0), T(0)};
        w[q] = ldc<T>((const LdsC2<T> *)(uintptr_t)(g.rb + ur[q]));
        xr[q] = lda<T>(ar[q]);
        xm[q] = lda<T>(am[q]);
    }
    for (int k = 0; k < g.ksteps - 1; ++k) {
        C2<T> w1[NJ];
        T xr1[NJ], xm1[NJ];
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            const unsigned nx = ur[q] + du[q];
            ur[q] = min(nx, nx - g.rspan);
            ar[q] += g.rstep;
            am[q] -= g.rstep;
            w1[q] = ldc<T>((const LdsC2<T> *)(uintptr_t)(g.rb + ur[q]));
            xr1[q] = lda<T>(ar[q]);
            xm1[q] = lda<T>(am[q]);
        }
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            P[q] = gp_mfma(w[q].x, xr[q] + xm[q], P[q]);
            Q[q] = gp_mfma(w[q].y, xr[q] - xm[q], Q[q]);
            w[q] = w1[q];
            xr[q] = xr1[q];
            xm[q] = xm1[q];
        }
    }
    const bool live = 4 * (g.ksteps - 1) + 1 + g.lk <= g.H;
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        P[q] = gp_mfma(w[q].x, live ? xr[q] + xm[q] : T(0), P[q]);
        Q[q] = gp_mfma(w[q].y, live ? xr[q] - xm[q] : T(0), Q[q]);
    }
}

template <typename T>
__device__ __attribute__((noinline)) void gp_pass(int buf_off, int lbufp, int nf, PassDesc pd, GlobalC2<T> *Wg)
{
    using V4 = typename std::conditional<sizeof(T) == 4, gp_f32x4, gp_f64x4>::type;
    constexpr unsigned CB = sizeof(C2<T>), RB = sizeof(T);
    constexpr int NWV = kFftThreads / 64;
    pd = uniform(pd);
    buf_off = uni(buf_off);
    lbufp = uni(lbufp);
    nf = uni(nf);
    const int p = pd.R, H = (p - 1) / 2, nbf = pd.nbf, nb = nf * nbf;
    const int mt = gp_row_tiles(p), nunits = mt * gp_col_tiles(nb), ksteps = (H + 3) / 4;
    // 1. w^u = W_L[u nbf] (u < p) to a table of p roots after the field slots
    const int roots_off = buf_off + nf * lbufp;
    for (int u = threadIdx.x; u < p; u += kFftThreads)
        stb<T>((unsigned)(roots_off + u) * CB, C2<T>{Wg[u * nbf].x, Wg[u * nbf].y});
    __syncthreads();
    const unsigned rbase = (unsigned)roots_off * CB, rstr = CB;
    const unsigned rspan = (unsigned)p * rstr, rstep = 4u * nbf * CB;
    const unsigned lb = lds_base(), rb = lb + rbase;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, lr = lane & 15, lk = lane >> 4;
    constexpr int NU = kGpUnits;
    static_assert(NU % 2 == 0, "units run in pairs");
    V4 accp[NU], accq[NU];
    T x0[NU];
    // 2. units wave, wave + NWV, ...: rows t = 16 i + (0..15), columns
    //    c = 16 g + (0..15) = 2 b + (re|im); two units at a time run their
    //    K loops together (four independent MFMA chains per wave)
    const GpGeom gm{p, H, mt, nb, nbf, pd.mg_nbf, buf_off, lbufp, ksteps, rb, rstr, rspan, rstep, lb, lr, lk};
#pragma unroll
    for (int s = 0; s < NU; s += 2) {
        const int ua = wave + s * NWV, ub = wave + (s + 1) * NWV;
        if (ub < nunits) {
            const int u2[2] = {ua, ub};
            gp_run<T, 2>(gm, u2, accp + s, accq + s, x0 + s);
        } else if (ua < nunits) {
            const int u1[1] = {ua};
            gp_run<T, 1>(gm, u1, accp + s, accq + s, x0 + s);
        }
    }
    __syncthreads();
    // 3. lane (column c, four rows) holds P and Q of one real component; i Q
    //    takes the other component's Q from the neighbour lane.  Output rows of
    //    the 16x16x4 MFMA: 4 (lane / 16) + v in FP32, lane / 16 + 4 v in FP64.
#pragma unroll
    for (int s = 0; s < NU; ++s) {
        const int unit = wave + s * NWV;
        if (unit < nunits) {
            const int i = unit % mt, g = unit / mt;
            const int c = 16 * g + lr, b = c >> 1, im = c & 1;
            const int f = udiv(min(b, nb - 1), pd.mg_nbf), j = min(b, nb - 1) - f * nbf;
            const unsigned ob = (unsigned)(buf_off + f * lbufp + j * p) * CB + (unsigned)im * RB;
            const T sg = im ? T(1) : T(-1);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const T qo = __shfl_xor(accq[s][v], 1);
                const int t = 16 * i + (sizeof(T) == 8 ? lk + 4 * v : 4 * lk + v);
                if (b < nb && t <= H) {
                    str<T>(ob + (unsigned)t * CB, x0[s] + accp[s][v] + sg * qo);
                    if (t > 0) str<T>(ob + (unsigned)(p - t) * CB, x0[s] + accp[s][v] - sg * qo);
                }
            }
        }
    }
    __syncthreads();
}

template <typename T, int CAP, bool BHAT>
__device__ inline void pass_dispatch(int buf_off, int lbufp, int nf, const PassDesc &pd, const C2<T> *W,
                                     const C2<T> *bhat)
{
    if constexpr (BHAT) {
        // Bluestein lengths are 2^a 3^b with 9 | L and the radix-9 passes first
        // (checked on the host), so the filter pass is always radix 9
        stockham_pass<T, 9, CAP, true>(buf_off, lbufp, nf, pd, W, bhat);
        return;
    }
    if (is_gp_radix<T>(pd.R)) {
        gp_pass<T>(buf_off, lbufp, nf, pd, (GlobalC2<T> *)W);
        return;
    }
    switch (pd.R) {
    case 2: stockham_pass<T, 2, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    case 3: stockham_pass<T, 3, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    case 4: stockham_pass<T, 4, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    case 5: stockham_pass<T, 5, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    case 7: stockham_pass<T, 7, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    case 11: stockham_pass<T, 11, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    case 13: stockham_pass<T, 13, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    case 17: stockham_pass<T, 17, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    // FP64 plans stop at radix 17 (larger FP64 butterflies would not fit the
    // registers); the host never plans the radices below for them
    case 19:
        if constexpr (sizeof(T) == 4) stockham_pass<T, 19, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat);
        break;
    case 23:
        if constexpr (sizeof(T) == 4) stockham_pass<T, 23, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat);
        break;

    case 9: stockham_pass<T, 9, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    case 16: stockham_pass<T, 16, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    default: stockham_pass<T, 8, CAP, BHAT>(buf_off, lbufp, nf, pd, W, bhat); break;
    }
}

// Length-h forward DFT of the h values at the start of each field slot.
// Plain: a Stockham FFT of length h.  Bluestein: the input must already be
// multiplied by the chirp and zero-padded to L; the second FFT's first pass
// applies the filter (conj(X bhat)) to the first FFT's output, the second FFT
// leaves conj(conv), and the caller multiplies by the chirp when reading the
// first h outputs.
template <typename T, int CAP>
__device__ void dft_h(int buf_off, const RingDesc &d, const PassDesc *passes, int nf, const C2<T> *W,
                      const C2<T> *bhat)
{
    const PassDesc *ps = passes + d.pass_off;
    for (int s = 0; s < d.nrad; ++s) {
        const PassDesc pd = ps[s];
        pass_dispatch<T, CAP, false>(buf_off, d.lbufp, nf, pd, W, bhat);
    }
    if (d.blue)
        for (int s = 0; s < d.nrad; ++s) {
            const PassDesc pd = ps[s];
            if (s == 0)
                pass_dispatch<T, CAP, true>(buf_off, d.lbufp, nf, pd, W, bhat);
            else
                pass_dispatch<T, CAP, false>(buf_off, d.lbufp, nf, pd, W, bhat);
        }
}


// A ring's grid rows can be moved two complex values (four points) at a time
// with 16-byte accesses: no chirp, even h, and every field's row of the ring
// starting on a 16-byte boundary (the block's first row aligned, field stride
// a multiple of 4 points).
__device__ inline bool grid_pairs(const RingDesc &d, int h, unsigned npts, const void *row0)
{
    return !d.blue && (h & 1) == 0 && (npts & 3u) == 0 && (reinterpret_cast<uintptr_t>(row0) & 15) == 0;
}

template <typename T, int CAP>
__global__ __launch_bounds__(kFftThreads, 2) void k_fft_c2r(FftArgs a)
{
    LdsC2<T> *buf = lds_c2<T>();
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const FftItem it = a.items[item];
    if (it.ring < 0) return;
    const RingDesc d = a.rings[it.ring];
    const C2<T> *tw = (const C2<T> *)a.twid;
    const C2<T> *W = tw + d.tw_off;
    const C2<T> *post = tw + d.post_off;
    const C2<T> *chirp = tw + d.chirp_off, *bhat = tw + d.bhat_off;
    const int nf = it.nf, f0 = it.f0, h = d.h, M = d.M, lbufp = d.lbufp;
    const C2<T> *four = (const C2<T> *)a.in + d.four_off;
    const T facpos = a.adjoint ? T(0.5) : T(1);
    const unsigned mg_nf = div_magic(nf);
    const int buf_off = 0;

    // 1. read the kept coefficients Y_m, Y_{h-m} (m <= M) and merge them into
    //    the length-h sequence u = conj(Z'), Z'_m = (Y_m + conj Y_{h-m})
    //    + i e^{2 pi i m / n} (Y_m - conj Y_{h-m}); Bluestein: times the chirp
    //    and zero-padded to L.  Runs over fields are contiguous in memory.
    //    Each thread issues the loads of kU elements before using any.
    auto zprime = [&](C2<T> a1, C2<T> a2, C2<T> pst, C2<T> chp) {
        C2<T> A = cadd(a1, cconj(a2)), B = csub(a1, cconj(a2));
        C2<T> t = cmul(cconj(pst), B);
        C2<T> z = {A.x - t.y, A.y + t.x};
        C2<T> u = cconj(z);
        return d.blue ? cmul(u, chp) : u;
    };
    const int hp = h / 2 + 1, nmerge = nf * hp;
    const unsigned nfld = (unsigned)a.nfld;
    const C2<T> *fourb = four + f0;  // (m, f) at fourb[m nfld + f]
    for (int e0 = threadIdx.x; e0 < nmerge; e0 += kU * kFftThreads) {
        C2<T> ym[kU], yh[kU], pm[kU], ph[kU], cm[kU], ch[kU];
        int mm[kU], ff[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + u * kFftThreads;
            const bool ok = e < nmerge;
            int m = ok ? udiv(e, mg_nf) : 0;
            int f = ok ? e - m * nf : 0;
            mm[u] = ok ? m : -1;
            ff[u] = f;
            const C2<T> zero = {T(0), T(0)};
            ym[u] = zero;
            yh[u] = zero;
            // 32-bit unsigned element offsets from the block's base pointers
            if (ok && m <= M) ym[u] = fourb[(unsigned)m * nfld + (unsigned)f];
            if (ok && h - m <= M) yh[u] = fourb[(unsigned)(h - m) * nfld + (unsigned)f];
            // e^{-2 pi i (h - m) / n} = -conj(e^{-2 pi i m / n}); the chirp at h - m
            // is the chirp at m times (-1)^h (m > 0)
            pm[u] = post[(unsigned)m];
            ph[u] = C2<T>{-pm[u].x, pm[u].y};
            cm[u] = zero;
            ch[u] = zero;
            if (d.blue) {
                cm[u] = chirp[(unsigned)m];
                ch[u] = (m > 0 && (h & 1)) ? C2<T>{-cm[u].x, -cm[u].y} : cm[u];
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int m = mm[u];
            if (m < 0) continue;
            C2<T> y0 = ym[u], y1 = yh[u];
            if (m == 0)
                y0.y = T(0);
            else
                y0 = {y0.x * facpos, y0.y * facpos};
            y1 = {y1.x * facpos, y1.y * facpos};
            LdsC2<T> *sl = buf + ff[u] * lbufp;
            if (m != 0 && m != h - m) stc(sl + (h - m), zprime(y1, y0, ph[u], ch[u]));
            stc(sl + m, zprime(y0, y1, pm[u], cm[u]));
        }
    }
    if (d.blue) {
        const int zl = d.L - h;
        const unsigned mg_z = div_magic(zl);
        for (int e = threadIdx.x; e < nf * zl; e += kFftThreads) {
            int f = udiv(e, mg_z), k = h + e - f * zl;
            stc(buf + f * lbufp + k, C2<T>{T(0), T(0)});
        }
    }
    __syncthreads();
    // 2. forward DFT of length h
    dft_h<T, CAP>(buf_off, d, a.passes, nf, W, bhat);
    // 3. z = conj(DFT(u)): even samples Re z, odd samples Im z
    const T scale = a.adjoint ? T(d.w / (2.0 * d.n)) : T(1);
    const unsigned npts = (unsigned)a.npts;
    T *gridb = (T *)a.out + (uint64_t)f0 * npts + d.grid_off;  // field f at gridb + f npts
    // single precision, no chirp, even h and 16-byte aligned rows: two complex
    // values (four grid points) per element with one 16-byte store
    if (sizeof(T) == 4 && grid_pairs(d, h, npts, gridb)) {
        typedef T V4 __attribute__((ext_vector_type(4)));
        const int hh = h / 2;
        const unsigned mg_hh = div_magic(hh);
        for (int e0 = threadIdx.x; e0 < nf * hh; e0 += kU * kFftThreads) {
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int e = e0 + u * kFftThreads;
                if (e >= nf * hh) continue;
                const int f = udiv(e, mg_hh), kk = e - f * hh;
                const C2<T> x0 = ldc(buf + f * lbufp + 2 * kk), x1 = ldc(buf + f * lbufp + 2 * kk + 1);
                *reinterpret_cast<V4 *>(gridb + (uint64_t)(unsigned)f * npts + 4u * (unsigned)kk) =
                    V4{scale * x0.x, -scale * x0.y, scale * x1.x, -scale * x1.y};
            }
        }
        return;
    }
    const unsigned mg_h = div_magic(h);
    for (int e0 = threadIdx.x; e0 < nf * h; e0 += kU * kFftThreads) {
        C2<T> cp[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + u * kFftThreads;
            const int k = e < nf * h ? e - udiv(e, mg_h) * h : 0;
            cp[u] = d.blue ? chirp[(unsigned)k] : C2<T>{T(1), T(0)};
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + u * kFftThreads;
            if (e >= nf * h) continue;
            const int f = udiv(e, mg_h), k = e - f * h;
            const C2<T> x = ldc(buf + f * lbufp + k);
            const C2<T> r = d.blue ? cmul(cp[u], cconj(x)) : x;
            const C2<T> g = {scale * r.x, -scale * r.y};
            *reinterpret_cast<C2<T> *>(gridb + (uint64_t)(unsigned)f * npts + 2u * (unsigned)k) = g;
        }
    }
}

template <typename T, int CAP>
__global__ __launch_bounds__(kFftThreads, 2) void k_fft_r2c(FftArgs a)
{
    LdsC2<T> *buf = lds_c2<T>();
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const FftItem it = a.items[item];
    if (it.ring < 0) return;
    const RingDesc d = a.rings[it.ring];
    const C2<T> *tw = (const C2<T> *)a.twid;
    const C2<T> *W = tw + d.tw_off;
    const C2<T> *post = tw + d.post_off;
    const C2<T> *chirp = tw + d.chirp_off, *bhat = tw + d.bhat_off;
    const int nf = it.nf, f0 = it.f0, h = d.h, M = d.M, lbufp = d.lbufp;
    const unsigned npts = (unsigned)a.npts;
    const T *gridb = (const T *)a.in + (uint64_t)f0 * npts + d.grid_off;  // field f at gridb + f npts
    const int buf_off = 0;
    __attribute__((address_space(3))) unsigned *smax =
        (__attribute__((address_space(3))) unsigned *)((LdsByte *)fft_smem + a.fmax_lds);
    if (a.fmax)
        for (int f = threadIdx.x; f < nf; f += kFftThreads) smax[f] = 0u;  // ordered by the barrier below

    // 1. z_k = g_{2k} + i g_{2k+1}; Bluestein: times the chirp, zero-padded to L
    const int span = d.blue ? d.L : h;
    const unsigned mg_span = div_magic(span);
    // single precision, no chirp, even h and 16-byte aligned rows: four grid
    // points (two complex values) per element with one 16-byte load
    const bool pairs = sizeof(T) == 4 && grid_pairs(d, h, npts, gridb);
    if (pairs) {
        typedef T V4 __attribute__((ext_vector_type(4)));
        const int hh = h / 2;
        const unsigned mg_hh = div_magic(hh);
        for (int e0 = threadIdx.x; e0 < nf * hh; e0 += kU * kFftThreads) {
            V4 gv[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int e = e0 + u * kFftThreads;
                if (e < nf * hh) {
                    const int f = udiv(e, mg_hh), kk = e - f * hh;
                    gv[u] = *reinterpret_cast<const V4 *>(gridb + (uint64_t)(unsigned)f * npts + 4u * (unsigned)kk);
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int e = e0 + u * kFftThreads;
                if (e >= nf * hh) continue;
                const int f = udiv(e, mg_hh), kk = e - f * hh;
                stc(buf + f * lbufp + 2 * kk, C2<T>{gv[u].x, gv[u].y});
                stc(buf + f * lbufp + 2 * kk + 1, C2<T>{gv[u].z, gv[u].w});
            }
        }
    }
    for (int e0 = pairs ? nf * span : threadIdx.x; e0 < nf * span; e0 += kU * kFftThreads) {
        C2<T> z[kU], cp[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + u * kFftThreads;
            z[u] = C2<T>{T(0), T(0)};
            cp[u] = C2<T>{T(1), T(0)};
            if (e < nf * span) {
                const int f = udiv(e, mg_span), k = e - f * span;
                if (k < h) {
                    z[u] = *reinterpret_cast<const C2<T> *>(gridb + (uint64_t)(unsigned)f * npts + 2u * (unsigned)k);
                    if (d.blue) cp[u] = chirp[(unsigned)k];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + u * kFftThreads;
            if (e >= nf * span) continue;
            const int f = udiv(e, mg_span), k = e - f * span;
            stc(buf + f * lbufp + k, d.blue ? cmul(z[u], cp[u]) : z[u]);
        }
    }
    __syncthreads();
    dft_h<T, CAP>(buf_off, d, a.passes, nf, W, bhat);
    // 2. split: Y_m = (Z_m + conj Z_{h-m}) / 2 - (i/2) e^{-2 pi i m / n} (Z_m - conj Z_{h-m})
    const T scale = a.adjoint ? T(1) : T(1.0 / d.n);
    C2<T> *fourb = (C2<T> *)a.out + d.four_off + f0;  // (m, f) at fourb[m nfld + f]
    const unsigned nfld = (unsigned)a.nfld;
    const unsigned mg_nf = div_magic(nf);
    const int nout = nf * (M + 1);
    for (int e0 = threadIdx.x; e0 < nout; e0 += kU * kFftThreads) {
        C2<T> pm[kU], cm[kU], ch[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + u * kFftThreads;
            const int m = e < nout ? udiv(e, mg_nf) : 0;
            pm[u] = post[(unsigned)m];
            cm[u] = C2<T>{T(1), T(0)};
            ch[u] = C2<T>{T(1), T(0)};
            if (d.blue) {
                // the chirp at h - m is the chirp at m times (-1)^h (m > 0)
                cm[u] = chirp[(unsigned)m];
                ch[u] = (m > 0 && (h & 1)) ? C2<T>{-cm[u].x, -cm[u].y} : cm[u];
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + u * kFftThreads;
            if (e >= nout) continue;
            const int m = udiv(e, mg_nf), f = e - m * nf;
            const LdsC2<T> *sl = buf + f * lbufp;
            const C2<T> xm = ldc(sl + m), xc = ldc(sl + (m == 0 ? 0 : h - m));
            const C2<T> zm = d.blue ? cmul(cm[u], cconj(xm)) : xm;
            const C2<T> zc = cconj(d.blue ? cmul(ch[u], cconj(xc)) : xc);
            C2<T> A = cadd(zm, zc), B = csub(zm, zc);
            C2<T> t = cmul(pm[u], B);
            C2<T> y = {T(0.5) * (A.x + t.y), T(0.5) * (A.y - t.x)};
            T fac = (a.adjoint && m > 0) ? T(2) : T(1);
            y = {y.x * scale * fac, m == 0 ? T(0) : y.y * scale * fac};
            fourb[(unsigned)m * nfld + (unsigned)f] = y;
            if (a.fmax)
                __hip_atomic_fetch_max(smax + f, __float_as_uint((float)fmax(fabs(y.x), fabs(y.y))),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    if (a.fmax) {
        __syncthreads();
        for (int f = threadIdx.x; f < nf; f += kFftThreads) atomicMax(a.fmax + f0 + f, smax[f]);
    }
}

template <typename T>
bool check_fft(const Plan &p, int cap)
{
#define SHTX_FFT_FAIL                                                                    \
    do {                                                                                 \
        if (std::getenv("SHTX_DEBUG")) std::fprintf(stderr, "shtx: FFT check line %d\n", __LINE__); \
        return false;                                                                    \
    } while (0)
    if (p.fft_items.empty() || p.fft_items.size() % kXcds) SHTX_FFT_FAIL;
    size_t celem = 2 * sizeof(T);
    for (const RingDesc &d : p.rings) {
        if (d.lbuf > cap || d.L > d.lbuf || d.h + 1 > d.lbuf || d.M >= d.h) SHTX_FFT_FAIL;
        if (d.lbufp < d.lbuf) SHTX_FFT_FAIL;
        if (d.tw_off < 0 || d.tw_off + d.L > p.twid_elems) SHTX_FFT_FAIL;
        if (d.post_off < 0 || d.post_off + d.h + 1 > p.twid_elems) SHTX_FFT_FAIL;
        if (d.blue && (d.chirp_off < 0 || d.chirp_off + d.h > p.twid_elems || d.bhat_off < 0 ||
                       d.bhat_off + d.L > p.twid_elems))
            SHTX_FFT_FAIL;
        if (d.grid_off + d.n > p.npts || d.four_off + (int64_t)(d.M + 1) * p.nfld > p.nfour * p.nfld)
            SHTX_FFT_FAIL;
        // the kernels index a field's grid row and a ring's Fourier rows with
        // 32-bit unsigned element offsets
        if (p.npts >= (int64_t(1) << 32) || (int64_t)(d.M + 1) * p.nfld >= (int64_t(1) << 32)) SHTX_FFT_FAIL;
        if (d.pass_off < 0 || d.pass_off + d.nrad > (int)p.passes.size() || d.nrad < 1) SHTX_FFT_FAIL;
        // the second Bluestein FFT applies the filter in a radix-9 first pass
        if (d.blue && p.passes[d.pass_off].R != 9) SHTX_FFT_FAIL;
        int prod = 1, extra = 0;
        for (int s = 0; s < d.nrad; ++s) {
            const PassDesc &pd = p.passes[d.pass_off + s];
            const int R = pd.R;
            const int code = (int)((d.radcode >> (5 * s)) & 31u);
            if (R < 2 || d.L % R) SHTX_FFT_FAIL;
            if (is_gp_radix<T>(R)) {
                // a general prime pass: the first pass only, an odd prime up to
                // kGpMaxPrime, at most kGpUnits output units per wave
                if (s != 0 || code != 0 || R > kGpMaxPrime || R % 2 == 0 || d.blue) SHTX_FFT_FAIL;
                for (int q = 3; q * q <= R; q += 2)
                    if (R % q == 0) SHTX_FFT_FAIL;
                if ((int64_t)gp_row_tiles(R) * gp_col_tiles(d.fb * pd.nbf) >
                    (int64_t)kGpUnits * (kFftThreads / 64))
                    SHTX_FFT_FAIL;
                extra = R;
            } else {
                bool ok = R == 4 || R == 8;
                for (int q : {2, 3, 5, 7, 9, 11, 13, 16, 17}) ok = ok || R == q;
                ok = ok || ((R == 19 || R == 23) && sizeof(T) == 4);
                if (!ok || code != R) SHTX_FFT_FAIL;
                // every butterfly of a block's fields is covered by the pass's rounds
                if ((int64_t)d.fb * (d.L / R) > (int64_t)fft_rounds(cap, R) * kFftThreads) SHTX_FFT_FAIL;
            }
            // the pass descriptor must describe exactly this pass
            if (pd.Ns != prod || pd.nbf * R != d.L || pd.tstep * prod * R != d.L) SHTX_FFT_FAIL;
            if (pd.mg_nbf != div_magic(pd.nbf) || pd.mg_ns != div_magic(pd.Ns)) SHTX_FFT_FAIL;
            // twiddle reads W[c k tstep] (c = 1, and 3 or 4 for radix 9 or 16;
            // 1, 9, 17 for the streamed radix 23), k < Ns
            const int cmax = R == 16 ? 4 : R == 9 ? 3 : R > 19 ? 17 : 1;
            if (prod > 1 && (int64_t)cmax * (prod - 1) * pd.tstep >= d.L) SHTX_FFT_FAIL;
            prod *= R;
        }
        if ((size_t)(d.fb * d.lbufp + extra) * celem > (size_t)p.fft_lds_bytes)
            SHTX_FFT_FAIL;
        if (prod != d.L) SHTX_FFT_FAIL;
    }
    if (p.prec == SHTX_FP16X3) {
        // the r2c kernel's per-field maxima sit after the block's LDS
        for (const RingDesc &d : p.rings)
            if (d.fb > kFmaxFields) SHTX_FFT_FAIL;
        if (p.fft_lds_bytes + 4 * kFmaxFields > 160 * 1024) SHTX_FFT_FAIL;
    }
    for (const FftItem &it : p.fft_items) {
        if (it.ring < 0) continue;
        if (it.ring >= p.nlat || it.f0 < 0 || it.nf < 1 || it.f0 + it.nf > p.nfld) SHTX_FFT_FAIL;
        if (it.nf > p.rings[it.ring].fb) SHTX_FFT_FAIL;
    }
    return true;
#undef SHTX_FFT_FAIL
}

__global__ void k_zero_u32(unsigned *x, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0u;
}

// LDS words the r2c kernel adds for the per-field maxima: the largest
// fields-per-block of the plan.
int fmax_lds_bytes(const Plan &p)
{
    int fb = 0;
    for (const RingDesc &d : p.rings) fb = std::max(fb, d.fb);
    return 4 * fb;
}

template <typename T, int CAP, bool C2R>
hipError_t launch_fft(const Plan &p, const void *in, void *out, bool adjoint, unsigned *fmax, hipStream_t s)
{
    // the rings, passes and work list were checked against the kernels'
    // limits (check_fft) when the plan's blocking was built
    if (!p.shapes_ok || p.fft_items.empty()) return hipErrorInvalidValue;
    FftArgs a{p.d_rings, p.d_fft_items, p.d_passes, p.d_twid, in, out, p.nfld, adjoint ? 1 : 0, p.npts,
              nullptr, p.fft_lds_bytes};
    int lds = p.fft_lds_bytes;
    if (!C2R && p.prec == SHTX_FP16X3) {
        // per-field maxima of the Fourier workspace for the split-half GEMM:
        // cleared here (a kernel, not a memset, so that graph replays clear it)
        if (!fmax) return hipErrorInvalidValue;
        k_zero_u32<<<(p.nfld + 255) / 256, 256, 0, s>>>(fmax, p.nfld);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        a.fmax = fmax;
        lds += fmax_lds_bytes(p);
    }
    auto kern = C2R ? k_fft_c2r<T, CAP> : k_fft_r2c<T, CAP>;
    kern<<<(int)p.fft_items.size(), kFftThreads, lds, s>>>(a);
    return hipGetLastError();
}

// Dynamic LDS above 64 KiB must be allowed per kernel; allowing the whole
// workgroup LDS once (a limit, not a reservation: occupancy follows the
// LDS each launch asks for) keeps every plan's launches valid without
// per-launch attribute calls.
template <typename T, int CAP>
hipError_t fft_allow_lds()
{
    constexpr int kMaxLds = 160 * 1024;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_fft_c2r<T, CAP>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_fft_r2c<T, CAP>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    return e;
}

}  // namespace

hipError_t fft_prepare(const Plan &p)
{
    if (p.fft_lds_bytes > 160 * 1024) return hipErrorInvalidValue;
    return p.prec == SHTX_FP64 ? fft_allow_lds<double, kFftCapF64>() : fft_allow_lds<float, kFftCapF32>();
}

bool fft_shapes_ok(const Plan &p)
{
    bool ok = p.prec == SHTX_FP64 ? check_fft<double>(p, kFftCapF64) : check_fft<float>(p, kFftCapF32);
    if (!ok && std::getenv("SHTX_DEBUG")) std::fprintf(stderr, "shtx: ring-FFT launch shape check failed\n");
    return ok;
}

hipError_t launch_fft_c2r(const Plan &p, const void *four, void *grid, bool adjoint, hipStream_t s)
{
    if (p.prec == SHTX_FP64) return launch_fft<double, kFftCapF64, true>(p, four, grid, adjoint, nullptr, s);
    return launch_fft<float, kFftCapF32, true>(p, four, grid, adjoint, nullptr, s);
}

hipError_t launch_fft_r2c(const Plan &p, const void *grid, void *four, bool adjoint, unsigned *fmax, hipStream_t s)
{
    if (p.prec == SHTX_FP64) return launch_fft<double, kFftCapF64, false>(p, grid, four, adjoint, nullptr, s);
    return launch_fft<float, kFftCapF32, false>(p, grid, four, adjoint, fmax, s);
}

}  // namespace shtx
