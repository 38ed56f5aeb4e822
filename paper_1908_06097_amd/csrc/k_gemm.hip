// Legendre transforms as grouped, even/odd-split GEMMs on the CDNA4 matrix
// cores, one launch per direction covering every wavenumber m.
//
// For each m the n-range splits by the parity p of n - m, and the equatorial
// symmetry P̄_n^m(-mu) = (-1)^(n-m) P̄_n^m(mu) lets one product over the
// northern rings serve both hemispheres:
//
//   inverse:  S_p[r][c] = sum_k P_p[r][k] B_p[k][c],   B_p[k][c] = a^m_{m+p+2k}
//             F_m(north r) = S_0 + S_1,  F_m(south r) = S_0 - S_1
//   direct:   D_p[k][c] = sum_r P_p[r][k] A_p[r][c],
//             A_p[r][c] = q_r (G_m(north r) + (-1)^p G_m(south r))
//
// with c running over (field, re/im) pairs (the table is real), r over the
// R_m northern rings carrying m and q_r = w_r / 2 (direct transform) or 1
// (adjoint of the inverse).  The spectral operand is read from / written to
// the caller's [field][nspec] array directly (the pack and unpack steps are
// fused into the tile loads and the epilogue), and the Fourier operand lives
// in the [ring][m][field] workspace that the ring FFTs read and write.
//
// The paper treats this step only as part of the SH dwarf (Section 3.1.1);
// the design (grouped launch, XCD-aware work lists, LDS-staged tiles, MFMA)
// is this library's own.
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "shtx_internal.h"

namespace shtx {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Acc;
template <>
struct Acc<float> {
    typedef f32x4 type;
};
template <>
struct Acc<double> {
    typedef f64x4 type;
};

// 16x16x4 MFMA: lane l supplies A[l%16][l/16] and B[l/16][l%16].  It holds
// D[i][l%16] for v = 0..3 with i = 4(l/16) + v for the FP32 form and
// i = l/16 + 4v for the FP64 form (the two differ on CDNA).
__device__ inline f32x4 mfma16x16x4(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f64x4 mfma16x16x4(double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ inline int acc_row(int lane, int v)
{
    return sizeof(T) == 8 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
}

struct GemmArgs {
    const void *tab;     // table for the A operand
    const void *tab_lo;  // split-BF16 lo half of the table
    const MBlock *mb;
    const GemmItem *items;
    const RingPair *ring_pair;  // per northern ring: Fourier offsets of it and its mirror
    const void *ring_q;         // per northern ring: w_j / 2 (grid precision)
    const void *in;
    void *out;
    int trunc, nlat, nfld;
    int adjoint;
    int64_t nspec;
    // split IEEE-half form: per-field largest magnitude of the data source
    // (float bits) and the factor that turns it into a bound on the data
    // operand's entries
    const unsigned *fmax;
    float dbound;
};

__device__ inline int64_t spec_base(int trunc, int m) { return (int64_t)m * (2 * trunc + 3 - m) / 2; }

// ---------------------------------------------------------------------------
// FP64 / FP32.  NW (4 or 8) waves as 2 x (NW/2), each owning a (BM/2) x
// (2 BN/NW) tile per parity.  LDS tiles are K-major (As[buf][p][kappa][i],
// Bs[buf][p][kappa][j]) and double-buffered: the global loads of stage s+1
// are issued into registers before the MFMAs of stage s and written to the
// other buffer after them, with one barrier per stage.
//
// INV: rows i = northern rings of the m band, kappa = k, A = table [p][k][r],
//      B = spectral coefficients read straight from spec[f][index(m, n)].
// DIR: rows i = k, kappa = rings, A = table [p][r][k], B = hemispheric
//      fold of the Fourier workspace q_r (G_north +- G_south).
// ---------------------------------------------------------------------------
template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) Vec2 {
    T x, y;
};

// Inverse epilogue through LDS (single precision and the split forms): the
// tile's rows of one hemisphere at a time are staged as [row][column] floats
// (16-column groups swizzled by row so that the fragment writes spread over
// the banks) and written out as contiguous runs over the fields of each ring
// row, 16 bytes per lane, instead of 4-byte stores scattered over 64-byte
// pieces.  val(hs, i, j, v) is the fragment value of hemisphere hs (0 north,
// 1 south).  Called by every thread of the block after the K loop's final
// barrier; st must hold BM x BN floats.
typedef float f32x4s __attribute__((ext_vector_type(4)));
typedef float f32x4s8 __attribute__((ext_vector_type(4), aligned(8)));
template <int BM, int BN, int NT, int FM, int FN, typename ValFn>
__device__ inline void inv_epilogue_staged(const GemmArgs &a, const MBlock &b, int m, int row0, int col0, int wr,
                                           int wc, int lane, int tid, float *st, ValFn val)
{
    constexpr int TPR = BN / 4, RPP = NT / TPR, NPASS = BM / RPP;
    static_assert(BN >= 64 && NPASS * RPP == BM, "staged rows must split evenly over the block");
    const int ncol = 2 * a.nfld;
    // ring offsets of the rows this thread writes, fetched before the staging
    RingPair ro[NPASS];
#pragma unroll
    for (int k = 0; k < NPASS; ++k) {
        const int r = row0 + tid / TPR + k * RPP;
        ro[k] = RingPair{-1, -1};
        if (r < b.R) ro[k] = a.ring_pair[b.j0 + r];
    }
    float *four = (float *)a.out;
    const int cq = 4 * (tid % TPR);
#pragma unroll
    for (int hs = 0; hs < 2; ++hs) {
        if (hs) __syncthreads();  // the north half has been read out
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = wr + i * 16 + 4 * (lane >> 4) + v;
                    const int c = wc + j * 16 + (lane & 15);
                    st[r * BN + (c ^ ((r & 12) << 2))] = val(hs, i, j, v);
                }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPASS; ++k) {
            const RingPair o = ro[k];
            const int rl = tid / TPR + k * RPP;
            const int c = col0 + cq;
            if (o.n < 0 || c >= ncol) continue;
            const f32x4s x = *reinterpret_cast<const f32x4s *>(&st[rl * BN + (cq ^ ((rl & 12) << 2))]);
            float *dst = four + 2 * ((int64_t)(hs ? o.s : o.n) + m) * a.nfld + c;
            if (c + 3 < ncol) {
                *reinterpret_cast<f32x4s8 *>(dst) = x;
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (c + t < ncol) dst[t] = x[t];
            }
        }
    }
}

template <typename T, int BM, int BN, int BK, bool INV, int NW = 4>
__global__ __launch_bounds__(64 * NW, sizeof(T) == 4 ? 4 : 2) void k_leg_mfma(GemmArgs a)
{
    // NW waves as 2 x (NW / 2): rows split in two, columns in NW / 2
    constexpr int NT = 64 * NW, NWN = NW / 2;
    constexpr int WM = BM / 2, WN = BN / NWN, FM = WM / 16, FN = WN / 16;
    static_assert(NW == 4 || NW == 8, "4 or 8 waves per block");
    constexpr int LDA = BM + 16, LDB = BN + 16;
    constexpr int VEC = 16 / sizeof(T);                 // elements per 16-byte table load
    constexpr int NA = (2 * BK * BM) / (VEC * NT);      // table loads per thread per stage
    // complex operand loads per thread per stage: INV reads BN/2 fields x 2 BK
    // coefficients, DIR reads BK rings x BN/2 fields (north and south each)
    constexpr int NB = INV ? (BK * BN) / NT : (BK * BN) / (2 * NT);
    constexpr int NM = INV ? 1 : NB;  // ring metadata per thread (DIR)
    static_assert(NA * VEC * NT == 2 * BK * BM, "table tile must split evenly");
    static_assert(NB * (INV ? NT : 2 * NT) == BK * BN, "operand tile must split evenly");
    static_assert(BK == 16 && BN >= 32, "operand swizzle assumes 16-deep stages");
    typedef typename Acc<T>::type V;
    typedef T VecT __attribute__((ext_vector_type(VEC)));
    // operand tiles As[buf][p][kappa][i], Bs[buf][p][kappa][j]; the direct
    // GEMM reuses the same LDS to stage its output tile
    constexpr int NSMEM = 2 * 2 * BK * (LDA + LDB);
    __shared__ __attribute__((aligned(16))) T smem[NSMEM];
    auto As = reinterpret_cast<T(*)[2][BK][LDA]>(smem);
    auto Bs = reinterpret_cast<T(*)[2][BK][LDB]>(smem + 2 * 2 * BK * LDA);

    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const GemmItem it = a.items[item];
    if (it.m < 0) return;
    const int m = it.m;
    const MBlock b = a.mb[m];
    const int row0 = it.tr * BM, col0 = it.tc * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave / NWN) * WM, wc = (wave % NWN) * WN;
    const int ncol = 2 * a.nfld;
    const int64_t pstride = (int64_t)b.Kp * b.Rp;
    const T *A0 = (const T *)a.tab + (INV ? b.off_kr : b.off_rk);
    const int lda_g = INV ? b.Rp : b.Kp;  // global row stride of the table tile
    const int64_t sb = spec_base(a.trunc, m);
    const int kend = INV ? b.K0 : b.R;
    const int nstages = (kend + BK - 1) / BK;

    // INV stores the coefficient tile with the field index XOR-swizzled by
    // its (parity, k) slot, so that the column-strided stores of one wave
    // hit distinct LDS banks; the MFMA reads undo the swizzle.
    auto bswz = [](int p, int q) { return 2 * (((q >> 1) & 3) | (p << 2)); };

    VecT ra[NA];
    Vec2<T> rb0[NB], rb1[NB];
    // DIR: Fourier offsets and weights of each thread's rings, fetched one
    // stage ahead of the data so that no data load waits on them
    RingPair mp1[NM], mp2[NM];
    T mq1[NM], mq2[NM];

    auto meta = [&](int kk, RingPair *mp, T *mq) {
#pragma unroll
        for (int v = 0; v < NM; ++v) {
            int r = kk + (tid + v * NT) / (BN / 2);
            // with 64 fields per tile a wave's ring is uniform: scalar loads
            if constexpr (BN / 2 == 64) r = __builtin_amdgcn_readfirstlane(r);
            RingPair o = {-1, -1};
            T w = T(0);
            if (r < b.R) {
                o = a.ring_pair[b.j0 + r];
                w = a.adjoint ? T(1) : ((const T *)a.ring_q)[b.j0 + r];
            }
            mp[v] = o;
            mq[v] = w;
        }
    };
    // global -> registers (no arithmetic on the loaded values here, so that
    // nothing waits for the loads before the MFMAs of the current stage)
    auto load = [&](int kk) {
#pragma unroll
        for (int v = 0; v < NA; ++v) {
            int idx = tid + v * NT;
            int p = idx / (BK * BM / VEC), rem = idx - p * (BK * BM / VEC);
            int q = rem / (BM / VEC), i = (rem - q * (BM / VEC)) * VEC;
            ra[v] = *reinterpret_cast<const VecT *>(A0 + p * pstride + (int64_t)(kk + q) * lda_g + row0 + i);
        }
        if (INV) {
            const Vec2<T> *spec = (const Vec2<T> *)a.in;
#pragma unroll
            for (int v = 0; v < NB; ++v) {
                int idx = tid + v * NT;
                int fl = idx / (2 * BK), t = idx - fl * (2 * BK);
                int f = col0 / 2 + fl, nrel = 2 * kk + t;
                Vec2<T> z = {T(0), T(0)};
                if (f < a.nfld && m + nrel <= a.trunc) z = spec[(int64_t)f * a.nspec + sb + nrel];
                rb0[v] = z;
            }
        } else {
            const Vec2<T> *four = (const Vec2<T> *)a.in;
#pragma unroll
            for (int v = 0; v < NB; ++v) {
                int idx = tid + v * NT;
                int cp = idx % (BN / 2);
                int f = col0 / 2 + cp;
                Vec2<T> gn = {T(0), T(0)}, gs = {T(0), T(0)};
                if (mp1[v].n >= 0 && f < a.nfld) {
                    gn = four[((int64_t)mp1[v].n + m) * a.nfld + f];
                    gs = four[((int64_t)mp1[v].s + m) * a.nfld + f];
                }
                rb0[v] = gn;
                rb1[v] = gs;
            }
        }
    };
    // registers -> LDS: INV zeroes Im a^0_n, DIR folds the hemispheres
    auto store = [&](int buf) {
#pragma unroll
        for (int v = 0; v < NA; ++v) {
            int idx = tid + v * NT;
            int p = idx / (BK * BM / VEC), rem = idx - p * (BK * BM / VEC);
            int q = rem / (BM / VEC), i = (rem - q * (BM / VEC)) * VEC;
            *reinterpret_cast<VecT *>(&As[buf][p][q][i]) = ra[v];
        }
        if (INV) {
#pragma unroll
            for (int v = 0; v < NB; ++v) {
                int idx = tid + v * NT;
                int fl = idx / (2 * BK), t = idx - fl * (2 * BK);
                int p = t & 1, q = t >> 1;
                Vec2<T> z = rb0[v];
                if (m == 0) z.y = T(0);
                *reinterpret_cast<Vec2<T> *>(&Bs[buf][p][q][(2 * fl) ^ bswz(p, q)]) = z;
            }
        } else {
#pragma unroll
            for (int v = 0; v < NB; ++v) {
                int idx = tid + v * NT;
                int q = idx / (BN / 2), cp = idx - q * (BN / 2);
                const T w = mq1[v];
                const Vec2<T> gn = rb0[v], gs = rb1[v];
                Vec2<T> s0 = {w * (gn.x + gs.x), w * (gn.y + gs.y)};
                Vec2<T> s1 = {w * (gn.x - gs.x), w * (gn.y - gs.y)};
                *reinterpret_cast<Vec2<T> *>(&Bs[buf][0][q][2 * cp]) = s0;
                *reinterpret_cast<Vec2<T> *>(&Bs[buf][1][q][2 * cp]) = s1;
            }
        }
    };

    V acc[2][FM][FN];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[p][i][j] = V{};

    // per-lane column of the B reads for each k step and parity (INV swizzle)
    int bcol[BK / 4][2];
#pragma unroll
    for (int q = 0; q < BK; q += 4)
#pragma unroll
        for (int p = 0; p < 2; ++p)
            bcol[q / 4][p] = INV ? ((lane & 15) ^ bswz(p, q + (lane >> 4))) : (lane & 15);

    if (!INV) meta(0, mp1, mq1);
    load(0);
    store(0);
    if (!INV && nstages > 1) meta(BK, mp1, mq1);
    __syncthreads();
    // Row fragments of this wave's sub-tile that hold data: on the ragged
    // edge of an m block the fragments past the last valid row (and a wave
    // wholly past the valid rows or columns) skip their LDS reads and MFMAs,
    // still loading and storing their share of the operand tiles.  The K
    // loop is instantiated per count so that the accumulators stay in place.
    const int nfa = __builtin_amdgcn_readfirstlane(
        col0 + wc < ncol ? min(FM, max(0, ((INV ? b.R : b.K0) - row0 - wr + 15) / 16)) : 0);
    auto kloop = [&](auto nfa_c) __attribute__((always_inline)) {
        constexpr int NFA = decltype(nfa_c)::value;
        for (int s = 0; s < nstages; ++s) {
            const int cur = s & 1;
            const bool more = s + 1 < nstages;
            if (more) load((s + 1) * BK);
            if (!INV && s + 2 < nstages) meta((s + 2) * BK, mp2, mq2);
            if constexpr (NFA > 0) {
#pragma unroll
                for (int q = 0; q < BK; q += 4) {
                    const int qq = q + (lane >> 4);
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        T av[NFA], bv[FN];
#pragma unroll
                        for (int i = 0; i < NFA; ++i) av[i] = As[cur][p][qq][wr + i * 16 + (lane & 15)];
#pragma unroll
                        for (int j = 0; j < FN; ++j) bv[j] = Bs[cur][p][qq][wc + j * 16 + bcol[q / 4][p]];
#pragma unroll
                        for (int i = 0; i < NFA; ++i)
#pragma unroll
                            for (int j = 0; j < FN; ++j) acc[p][i][j] = mfma16x16x4(av[i], bv[j], acc[p][i][j]);
                    }
                }
            }
            if (more) store(cur ^ 1);
            if (!INV && s + 2 < nstages) {
#pragma unroll
                for (int v = 0; v < NM; ++v) {
                    mp1[v] = mp2[v];
                    mq1[v] = mq2[v];
                }
            }
            __syncthreads();
        }
    };
    static_assert(FM >= 1 && FM <= 4, "one to four row fragments per wave");
    // the inverse's ragged rows are few (2 % of its MFMAs against 6 % in the
    // direct): whole waves only, which keeps its registers within the two
    // blocks per CU
    if (nfa == FM || (INV && nfa > 0))
        kloop(std::integral_constant<int, FM>{});
    else if (!INV && FM >= 4 && nfa == 3)
        kloop(std::integral_constant<int, (FM >= 4 ? 3 : 0)>{});
    else if (!INV && FM >= 3 && nfa == 2)
        kloop(std::integral_constant<int, (FM >= 3 ? 2 : 0)>{});
    else if (!INV && FM >= 2 && nfa == 1)
        kloop(std::integral_constant<int, (FM >= 2 ? 1 : 0)>{});
    else
        kloop(std::integral_constant<int, 0>{});

    if constexpr (INV && sizeof(T) == 4) {
        static_assert(BM * BN <= NSMEM, "staged inverse tile must fit the operand LDS");
        inv_epilogue_staged<BM, BN, NT, FM, FN>(a, b, m, row0, col0, wr, wc, lane, tid, reinterpret_cast<float *>(smem),
                                                [&](int hs, int i, int j, int v) {
                                                    const float s0 = acc[0][i][j][v], s1 = acc[1][i][j][v];
                                                    return hs ? s0 - s1 : s0 + s1;
                                                });
    } else if constexpr (INV) {
        T *four = (T *)a.out;
        // all rows' ring offsets first, so that their loads overlap
        RingPair ro[FM][4];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int r = row0 + wr + i * 16 + acc_row<T>(lane, v);
                ro[i][v] = RingPair{-1, -1};
                if (r < b.R) ro[i][v] = a.ring_pair[b.j0 + r];
            }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const RingPair o = ro[i][v];
                if (o.n < 0) continue;
                T *fn = four + 2 * ((int64_t)o.n + m) * a.nfld;
                T *fs = four + 2 * ((int64_t)o.s + m) * a.nfld;
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    int c = col0 + wc + j * 16 + (lane & 15);
                    if (c < ncol) {
                        T s0 = acc[0][i][j][v], s1 = acc[1][i][j][v];
                        fn[c] = s0 + s1;
                        fs[c] = s0 - s1;
                    }
                }
            }
    } else if constexpr (sizeof(T) == 8) {
        // FP64: direct scattered stores (staging measured slower for the
        // smaller FP64 tiles)
        T *spec = (T *)a.out;
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        int k = row0 + wr + i * 16 + acc_row<T>(lane, v);
                        int c = col0 + wc + j * 16 + (lane & 15);
                        int nrel = p + 2 * k;
                        if (m + nrel <= a.trunc && c < ncol) {
                            T val = acc[p][i][j][v];
                            if (m == 0 && (c & 1)) val = 0;
                            spec[2 * ((int64_t)(c >> 1) * a.nspec + sb + nrel) + (c & 1)] = val;
                        }
                    }
    } else {
        // The tile covers n = m + 2 row0 + (0 .. 2 BM - 1) for BN/2 fields: each
        // column half (the fields of waves with the same wc) is staged in LDS
        // as [field][n] and written as contiguous runs of one field's spectrum.
        constexpr int FH = BN / 4;      // fields per column half
        constexpr int RS = 2 * BM + 1;  // staged complex values per field, padded
        static_assert(FH * RS * 2 <= NSMEM, "staged output half must fit the operand LDS");
        Vec2<T> *spec = (Vec2<T> *)a.out;
        const int nrel0 = 2 * row0;
        const int nvalid = min(2 * BM, a.trunc - m - nrel0 + 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            __syncthreads();  // the K loop's (or the previous half's) LDS reads are done
            if ((wave % NWN) / (NWN / 2) == h) {
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int k = wr + i * 16 + acc_row<T>(lane, v);
                                // column within the staged half
                                const int cl = wc - h * (BN / 2) + j * 16 + (lane & 15);
                                T val = acc[p][i][j][v];
                                if (m == 0 && (cl & 1)) val = 0;
                                smem[((cl >> 1) * RS + p + 2 * k) * 2 + (cl & 1)] = val;
                            }
            }
            __syncthreads();
            const int fbase = col0 / 2 + h * FH;
            for (int fl = wave; fl < FH; fl += NW) {
                const int f = fbase + fl;
                if (f >= a.nfld) break;
                Vec2<T> *dst = spec + (int64_t)f * a.nspec + sb + nrel0;
                for (int nr = lane; nr < nvalid; nr += 64)
                    dst[nr] = Vec2<T>{smem[(fl * RS + nr) * 2], smem[(fl * RS + nr) * 2 + 1]};
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Split half precision with FP32 accumulation: each operand is a sum hi + lo
// of two bfloat16 or two IEEE-half values, and a tile product is three MFMAs
// (hi*lo + lo*hi + hi*hi; lo*lo is dropped).  16x16x32 MFMA: lane l supplies
// A[l%16][8(l/16)..+7] and B[8(l/16)..+7][l%16]; LDS tiles are row-major
// with kappa contiguous: As[p][h][i][kappa], Bs[p][h][j][kappa] (h = hi, lo),
// unpadded, the 16-byte chunks of each row permuted by an XOR swizzle.
//
// The table is stored already split, scaled by 2^e_m per m.  The data
// operand is split here, once per block and stage, with the packed
// round-to-nearest-even conversions of gfx950.  IEEE half has a 5-bit
// exponent, so its data operand is also scaled per field by 2^E_f, chosen
// from a bound on the field's largest value; bfloat16 has the FP32 exponent
// range and needs no data scale.
// ---------------------------------------------------------------------------
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
// two complex values at an 8-byte aligned address, one 16-byte load (vector
// memory instructions need only 4-byte alignment)
typedef float f32x4a8 __attribute__((ext_vector_type(4), aligned(8)));

// lo = x - hi must be taken against the very hi that is stored.  Left to
// itself the compiler re-derives hi for that subtraction from the product
// that produced x, by another instruction (a mixed-precision FMA rounding the
// exact product to half once) whose result differs from the stored hi
// wherever the two roundings disagree; hi + lo is then off by a unit of hi.
// An empty asm statement makes the stored hi's bits opaque, so the residual
// is computed from them.
template <bool F16>
__device__ inline void split2(float x0, float x1, unsigned &hi, unsigned &lo)
{
    if constexpr (F16) {
        unsigned hb = __builtin_bit_cast(unsigned, f16x2{(_Float16)x0, (_Float16)x1});
        asm("" : "+v"(hb));
        const f16x2 h = __builtin_bit_cast(f16x2, hb);
        const f16x2 l = {(_Float16)(x0 - (float)h[0]), (_Float16)(x1 - (float)h[1])};
        hi = hb;
        lo = __builtin_bit_cast(unsigned, l);
    } else {
        unsigned hb = __builtin_bit_cast(unsigned, bf16x2{(__bf16)x0, (__bf16)x1});
        asm("" : "+v"(hb));
        const bf16x2 h = __builtin_bit_cast(bf16x2, hb);
        const bf16x2 l = {(__bf16)(x0 - (float)h[0]), (__bf16)(x1 - (float)h[1])};
        hi = hb;
        lo = __builtin_bit_cast(unsigned, l);
    }
}

// eight floats -> one 16-byte word of hi halves and one of lo halves
template <bool F16>
__device__ inline void split8(const float *x, u32x4 &hi, u32x4 &lo)
{
    unsigned h[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) split2<F16>(x[2 * i], x[2 * i + 1], h[i], l[i]);
    hi = u32x4{h[0], h[1], h[2], h[3]};
    lo = u32x4{l[0], l[1], l[2], l[3]};
}

template <bool F16>
__device__ inline f32x4 mfma_split(u32x4 a, u32x4 b, f32x4 c)
{
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
}

// Exponent E_f of field f's data operand in the half form: with the field's
// largest magnitude times `bound` (a bound on the operand's entries) equal to
// x 2^X, x in [1/2, 1), E_f = 14 - X puts the bound in [2^13, 2^14); 0 for an
// all-zero field.
__device__ inline int field_exp(const unsigned *fmax, int f, float bound)
{
    const float mx = __uint_as_float(fmax[f]) * bound;
    if (!(mx > 0.f)) return 0;
    int X;
    (void)frexpf(mx, &X);
    return 14 - X;
}

template <bool F16, int BM, int BN, int BK, bool INVERSE, int NW>
__global__ __launch_bounds__(64 * NW) void k_leg_split(GemmArgs a)
{
    // NW waves as 2 x (NW / 2): rows split in two, columns in NW / 2
    constexpr int NT = 64 * NW, NWN = NW / 2;
    constexpr int WM = BM / 2, WN = BN / NWN, FM = WM / 16, FN = WN / 16;
    static_assert(NW == 4 || NW == 8, "4 or 8 waves per block");
    constexpr int LDK = BK;     // unpadded rows; 16-byte chunks swizzled per row
    constexpr int CH = BK / 8;  // 16-byte chunks per tile row
    static_assert(CH == 4 || CH == 8, "the chunk swizzle permutes four or eight chunks");
    // physical chunk of logical chunk c in tile row r: c ^ sw(r), the bits
    // of r / PR (PR rows span 512 bytes) to the swizzle's upper bits and bit
    // 4 of r to bit 0.  Measured with an LDS probe: with four chunks (64-byte
    // rows) the fragment reads run at the rate of linear reads (unswizzled
    // 64- to 80-byte rows take twice as long); with eight chunks they still
    // take twice, off the critical path of these kernels
    constexpr int PR = 32 / CH;
    auto sw = [](int r) __attribute__((always_inline)) { return (((r / PR) & (CH / 2 - 1)) << 1) | ((r >> 4) & 1); };
    // LDS row of operand column (field fl, re/im ri): the inverse keeps them
    // interleaved, the direct places all real parts before all imaginary ones
    auto brow = [](int fl, int ri) __attribute__((always_inline)) {
        return INVERSE ? 2 * fl + ri : ri * (BN / 2) + fl;
    };
    constexpr int NA = (2 * 2 * BM * CH) / NT;  // table chunk loads per thread
    // DIR operand units: (field, 8 consecutive rings, north and south)
    constexpr int NUNIT = (BN / 2) * CH;
    constexpr int NU = (NUNIT + NT - 1) / NT;
    static_assert(NUNIT % 64 == 0, "direct operand units must fill whole waves");
    static_assert(NA * NT == 2 * 2 * BM * CH, "table tile must split evenly");
    // INV operand chunks: 4 consecutive n (two kappa of each parity) of one
    // field, 32 bytes; the JC chunks of a field's stage are taken by JC
    // consecutive lanes, so four lanes share each 128-byte line and one load
    // instruction of a wave touches 16 lines (one line per lane when each
    // lane read a whole run of 16 n)
    constexpr int JC = BK / 2;
    constexpr int NIU = (BN / 2) * JC / NT;
    static_assert(!INVERSE || (NIU * NT == (BN / 2) * JC && 4 * NIU <= 16 * NU),
                  "inverse operand chunks must split evenly");
    // operand tiles As[p][h][i][kappa], Bs[p][h][j][kappa]; the direct form
    // reuses the same LDS to stage its output tile
    constexpr int NOPER16 = 2 * 2 * (BM + BN) * LDK;
    // the direct form stages one half of its output columns (BN / 4 fields of
    // 2 BM + 1 complex values) in the same LDS
    constexpr int NSTAGE16 = INVERSE ? 0 : (BN / 4) * (2 * BM + 1) * 2 * 2;
    constexpr int NSMEM16 = NOPER16 > NSTAGE16 ? NOPER16 : NSTAGE16;
    __shared__ __attribute__((aligned(16))) unsigned short smem16[NSMEM16];
    auto As = reinterpret_cast<unsigned short(*)[2][BM][LDK]>(smem16);
    auto Bs = reinterpret_cast<unsigned short(*)[2][BN][LDK]>(smem16 + 2 * 2 * BM * LDK);

    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const GemmItem it = a.items[item];
    if (it.m < 0) return;
    const int m = it.m;
    const MBlock b = a.mb[m];
    const int row0 = it.tr * BM, col0 = it.tc * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave / NWN) * WM, wc = (wave % NWN) * WN;
    const int ncol = 2 * a.nfld;
    const int64_t sb = spec_base(a.trunc, m);
    // A operand rows are contiguous in kappa: inverse reads [p][r][k], direct [p][k][r]
    const int64_t off = INVERSE ? b.off_rk : b.off_kr;
    const int lda = INVERSE ? b.Kp : b.Rp;
    const int64_t pstride = (int64_t)b.Rp * b.Kp;
    const unsigned short *Th = (const unsigned short *)a.tab + off;
    const unsigned short *Tl = (const unsigned short *)a.tab_lo + off;
    const int kend = INVERSE ? b.K0 : b.R;
    const int nstages = (kend + BK - 1) / BK;

    // each thread's operand units keep their field over all stages
    int ufl[NU];
    bool uon[NU];
    float usc[NU];  // data scale 2^E_f (half form)
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int idx = tid + u * NT;
        ufl[u] = INVERSE ? idx / CH : idx % (BN / 2);
        uon[u] = idx < NUNIT;
        usc[u] = 1.f;
        if constexpr (F16) {
            const int f = col0 / 2 + ufl[u];
            if (uon[u] && f < a.nfld) usc[u] = ldexpf(1.f, field_exp(a.fmax, f, a.dbound));
        }
    }
    // INV: the fields of this thread's chunks and their data scales
    const int ij = tid % JC;
    float isc[NIU];
#pragma unroll
    for (int u = 0; u < NIU; ++u) {
        isc[u] = 1.f;
        if constexpr (F16 && INVERSE) {
            const int f = col0 / 2 + (u * NT + tid) / JC;
            if (f < a.nfld) isc[u] = ldexpf(1.f, field_exp(a.fmax, f, a.dbound));
        }
    }

    u32x4 ra[NA];
    float2 rv[NU][16];
    // DIR: Fourier offsets and weights of each unit's 8 rings, fetched one
    // stage ahead of the data so that no data load waits on them
    constexpr int NMU = INVERSE ? 1 : NU, NMQ = INVERSE ? 1 : 8;
    RingPair mp1[NMU][NMQ], mp2[NMU][NMQ];
    float mq1[NMU][NMQ], mq2[NMU][NMQ];
    auto meta = [&](int kk, RingPair (*mp)[NMQ], float (*mq)[NMQ]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NMU; ++u) {
            int rc = (tid + u * NT) / (BN / 2);
            // with 64 fields per tile a unit's rings are uniform over a wave:
            // scalar loads into scalar registers
            if constexpr (BN / 2 == 64) rc = __builtin_amdgcn_readfirstlane(rc);
#pragma unroll
            for (int q = 0; q < NMQ; ++q) {
                int r = kk + rc * 8 + q;
                RingPair o = {-1, -1};
                float w = 0.f;
                // units are whole waves (NUNIT is a multiple of 64), so uon is wave-uniform
                if ((NUNIT % NT == 0 || __builtin_amdgcn_readfirstlane(uon[u] ? 1 : 0)) && r < b.R) {
                    o = a.ring_pair[b.j0 + r];
                    w = a.adjoint ? 1.f : ((const float *)a.ring_q)[b.j0 + r];
                }
                mp[u][q] = o;
                mq[u][q] = w;
            }
        }
    };

    auto load = [&](int kk) __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < NA; ++v) {
            int idx = tid + v * NT;
            int p = idx / (2 * BM * CH), rem = idx - p * 2 * BM * CH;
            int hl = rem / (BM * CH);
            rem -= hl * BM * CH;
            int i = rem / CH, ch = rem - i * CH;
            ra[v] = *reinterpret_cast<const u32x4 *>((hl ? Tl : Th) + p * pstride + (int64_t)(row0 + i) * lda + kk +
                                                     ch * 8);
        }
        const float2 zero = {0.f, 0.f};
        if constexpr (INVERSE) {
#pragma unroll
            for (int u = 0; u < NIU; ++u) {
                const int f = col0 / 2 + (u * NT + tid) / JC;
                const int nrel = 2 * kk + 4 * ij;
                const float2 *src = (const float2 *)a.in + (int64_t)f * a.nspec + sb + nrel;
                if (f < a.nfld && m + nrel + 3 <= a.trunc) {
                    const f32x4a8 v0 = *reinterpret_cast<const f32x4a8 *>(src);
                    const f32x4a8 v1 = *reinterpret_cast<const f32x4a8 *>(src + 2);
                    rv[0][4 * u] = float2{v0[0], v0[1]};
                    rv[0][4 * u + 1] = float2{v0[2], v0[3]};
                    rv[0][4 * u + 2] = float2{v1[0], v1[1]};
                    rv[0][4 * u + 3] = float2{v1[2], v1[3]};
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        rv[0][4 * u + t] = (f < a.nfld && m + nrel + t <= a.trunc) ? src[t] : zero;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                // 8 consecutive rings of one field, north and south; the
                // rings' offsets come from the previous stage's meta fetch
                const int f = col0 / 2 + ufl[u];
                const float2 *four = (const float2 *)a.in;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    float2 gn = zero, gs = zero;
                    if (mp1[u][q].n >= 0 && f < a.nfld) {
                        gn = four[((int64_t)mp1[u][q].n + m) * a.nfld + f];
                        gs = four[((int64_t)mp1[u][q].s + m) * a.nfld + f];
                    }
                    rv[u][2 * q] = gn;
                    rv[u][2 * q + 1] = gs;
                }
            }
        }
    };
    auto store = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < NA; ++v) {
            int idx = tid + v * NT;
            int p = idx / (2 * BM * CH), rem = idx - p * 2 * BM * CH;
            int hl = rem / (BM * CH);
            rem -= hl * BM * CH;
            int i = rem / CH, ch = rem - i * CH;
            *reinterpret_cast<u32x4 *>(&As[p][hl][i][(ch ^ sw(i)) * 8]) = ra[v];
        }
        if constexpr (INVERSE) {
            // chunk u holds n = 4 ij + t (t = 0..3): kappa 2 ij + t / 2 of parity t & 1
#pragma unroll
            for (int u = 0; u < NIU; ++u) {
                const int fl = (u * NT + tid) / JC;
                const float sc = isc[u];
                unsigned hi, lo;
                const int r0 = brow(fl, 0), r1 = brow(fl, 1);
                const int k0 = ((ij >> 2) ^ sw(r0)) * 8 + 2 * (ij & 3), k1 = ((ij >> 2) ^ sw(r1)) * 8 + 2 * (ij & 3);
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    split2<F16>(rv[0][4 * u + p].x * sc, rv[0][4 * u + 2 + p].x * sc, hi, lo);
                    *reinterpret_cast<unsigned *>(&Bs[p][0][r0][k0]) = hi;
                    *reinterpret_cast<unsigned *>(&Bs[p][1][r0][k0]) = lo;
                    // Im a^0_n is ignored
                    const float y0 = m == 0 ? 0.f : rv[0][4 * u + p].y * sc;
                    const float y1 = m == 0 ? 0.f : rv[0][4 * u + 2 + p].y * sc;
                    split2<F16>(y0, y1, hi, lo);
                    *reinterpret_cast<unsigned *>(&Bs[p][0][r1][k1]) = hi;
                    *reinterpret_cast<unsigned *>(&Bs[p][1][r1][k1]) = lo;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                if (!uon[u]) continue;
                const int idx = tid + u * NT;
                const float sc = usc[u];
                float x[8];
                u32x4 hi, lo;
                // hemispheric fold: parity 0 takes q (north + south), parity 1 q (north - south)
                const int cp = ufl[u], rc = idx / (BN / 2);
                const int r0 = brow(cp, 0), r1 = brow(cp, 1);
                const int k0 = (rc ^ sw(r0)) * 8, k1 = (rc ^ sw(r1)) * 8;
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const float sg = p ? -1.f : 1.f;
#pragma unroll
                    for (int q = 0; q < 8; ++q) x[q] = (mq1[u][q] * sc) * (rv[u][2 * q].x + sg * rv[u][2 * q + 1].x);
                    split8<F16>(x, hi, lo);
                    *reinterpret_cast<u32x4 *>(&Bs[p][0][r0][k0]) = hi;
                    *reinterpret_cast<u32x4 *>(&Bs[p][1][r0][k0]) = lo;
#pragma unroll
                    for (int q = 0; q < 8; ++q) x[q] = (mq1[u][q] * sc) * (rv[u][2 * q].y + sg * rv[u][2 * q + 1].y);
                    split8<F16>(x, hi, lo);
                    *reinterpret_cast<u32x4 *>(&Bs[p][0][r1][k1]) = hi;
                    *reinterpret_cast<u32x4 *>(&Bs[p][1][r1][k1]) = lo;
                }
            }
        }
    };

    f32x4 acc[2][FM][FN];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[p][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // a wave whose whole sub-tile lies past the valid rows or columns (the
    // ragged edge of an m block or of the field range) still loads and
    // stores its share of the operand tiles but skips the MFMAs
    const bool mfma_on = __builtin_amdgcn_readfirstlane(
        (row0 + wr < (INVERSE ? b.R : b.K0) && (INVERSE ? col0 + wc < ncol : col0 / 2 + (wc & (BN / 2 - 1)) < a.nfld))
            ? 1
            : 0);

    // The K loop, in two copies: with MFMAs, and without them for a wave
    // whose sub-tile is wholly ragged (a wave-uniform branch outside the
    // loop keeps the accumulators in the MFMA accumulation registers).
    auto kloop = [&](auto with_mfma) __attribute__((always_inline)) {
        if (!INVERSE) meta(0, mp1, mq1);
        load(0);
        if (!INVERSE && nstages > 1) meta(BK, mp2, mq2);
        for (int s = 0; s < nstages; ++s) {
            store();  // uses the weights mq1 of stage s
            if (!INVERSE && s + 1 < nstages) {
#pragma unroll
                for (int u = 0; u < NMU; ++u)
#pragma unroll
                    for (int q = 0; q < NMQ; ++q) {
                        mp1[u][q] = mp2[u][q];
                        mq1[u][q] = mq2[u][q];
                    }
            }
            __syncthreads();
            if (s + 1 < nstages) load((s + 1) * BK);  // in flight during the MFMAs
            if (!INVERSE && s + 2 < nstages) meta((s + 2) * BK, mp2, mq2);
            if constexpr (decltype(with_mfma)::value) {
#pragma unroll
                for (int q = 0; q < BK; q += 32) {
                    const int kc = q / 8 + (lane >> 4);
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        u32x4 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
                        for (int i = 0; i < FM; ++i) {
                            const int ai = wr + i * 16 + (lane & 15);
                            const int ka = (kc ^ sw(ai)) * 8;
                            ah[i] = *reinterpret_cast<const u32x4 *>(&As[p][0][ai][ka]);
                            al[i] = *reinterpret_cast<const u32x4 *>(&As[p][1][ai][ka]);
                        }
#pragma unroll
                        for (int j = 0; j < FN; ++j) {
                            const int bj = wc + j * 16 + (lane & 15);
                            const int kb = (kc ^ sw(bj)) * 8;
                            bh[j] = *reinterpret_cast<const u32x4 *>(&Bs[p][0][bj][kb]);
                            bl[j] = *reinterpret_cast<const u32x4 *>(&Bs[p][1][bj][kb]);
                        }
#pragma unroll
                        for (int i = 0; i < FM; ++i)
#pragma unroll
                            for (int j = 0; j < FN; ++j) {
                                f32x4 c = acc[p][i][j];
                                c = mfma_split<F16>(ah[i], bl[j], c);
                                c = mfma_split<F16>(al[i], bh[j], c);
                                c = mfma_split<F16>(ah[i], bh[j], c);
                                acc[p][i][j] = c;
                            }
                    }
                }
            }
            __syncthreads();
        }
    };
    if (mfma_on)
        kloop(std::true_type{});
    else
        kloop(std::false_type{});

    // unscaling exponent of each of the lane's columns: e_m (+ E_f)
    int eu[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        eu[j] = b.e;
        if constexpr (F16) {
            const int bj = wc + j * 16 + (lane & 15);
            const int f = INVERSE ? (col0 + bj) >> 1 : col0 / 2 + (bj & (BN / 2 - 1));
            if (f < a.nfld) eu[j] += field_exp(a.fmax, f, a.dbound);
        }
    }
    if constexpr (INVERSE) {
        static_assert(BM * BN * 2 <= NSMEM16, "staged inverse tile must fit the operand LDS");
        inv_epilogue_staged<BM, BN, NT, FM, FN>(a, b, m, row0, col0, wr, wc, lane, tid, reinterpret_cast<float *>(smem16),
                                                [&](int hs, int i, int j, int v) {
                                                    const float s0 = acc[0][i][j][v], s1 = acc[1][i][j][v];
                                                    return ldexpf(hs ? s0 - s1 : s0 + s1, -eu[j]);
                                                });
    } else {
        // staged per column half as [field][n], written as contiguous runs
        // (as in k_leg_mfma)
        constexpr int FH = BN / 4, RS = 2 * BM + 1;
        static_assert(FH * RS * 2 * 2 <= NSMEM16, "staged output half must fit the operand LDS");
        float *st = reinterpret_cast<float *>(smem16);
        float2 *spec = (float2 *)a.out;
        const int nrel0 = 2 * row0;
        const int nvalid = min(2 * BM, a.trunc - m - nrel0 + 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            __syncthreads();
            // operand column bj is field bj % (BN / 2), real part for
            // bj < BN / 2; fragments of 16 columns never straddle a half
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int bj0 = wc + j * 16;
                if (((bj0 & (BN / 2 - 1)) / FH) != h) continue;
                const int ri = bj0 / (BN / 2);
                const int fl = (bj0 & (BN / 2 - 1)) - h * FH + (lane & 15);
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int k = wr + i * 16 + 4 * (lane >> 4) + v;
                            float val = ldexpf(acc[p][i][j][v], -eu[j]);
                            if (m == 0 && ri) val = 0.f;
                            st[(fl * RS + p + 2 * k) * 2 + ri] = val;
                        }
            }
            __syncthreads();
            const int fbase = col0 / 2 + h * FH;
            for (int fl = wave; fl < FH; fl += NW) {
                const int f = fbase + fl;
                if (f >= a.nfld) break;
                float2 *dst = spec + (int64_t)f * a.nspec + sb + nrel0;
                for (int nr = lane; nr < nvalid; nr += 64)
                    dst[nr] = float2{st[(fl * RS + nr) * 2], st[(fl * RS + nr) * 2 + 1]};
            }
        }
    }
}

GemmArgs make_args(const Plan &p, bool inverse_shape, const void *in, void *out, bool adjoint, unsigned *fmax)
{
    GemmArgs a{};
    a.mb = p.d_mb;
    a.items = inverse_shape ? p.d_inv_items : p.d_dir_items;
    a.ring_pair = p.d_ring_pair;
    a.ring_q = p.d_ring_q;
    a.in = in;
    a.out = out;
    a.trunc = p.trunc;
    a.nlat = p.nlat;
    a.nfld = p.nfld;
    a.adjoint = adjoint ? 1 : 0;
    a.nspec = p.nspec;
    if (split_form(p.prec)) {
        a.tab = inverse_shape ? p.d_tab_rk : p.d_tab_kr;
        a.tab_lo = inverse_shape ? p.d_tab_rk_lo : p.d_tab_kr_lo;
    } else {
        a.tab = inverse_shape ? p.d_tab_kr : p.d_tab_rk;
        a.tab_lo = nullptr;
    }
    // the inverse-shaped launch splits spectral coefficients (bounded by the
    // field maximum itself); the direct-shaped one splits q_r (G_north +-
    // G_south), bounded by 2 max_r q_r times the largest Fourier value
    a.fmax = fmax;
    a.dbound = inverse_shape ? 1.f : (float)(2.0 * (adjoint ? 1.0 : p.qmax));
    return a;
}

// Host check that every tile of items [first, first + count) of a work list
// reads and writes inside the table, Fourier and spectral arrays for the
// given tile sizes.  Run when a plan's work lists are built, not per launch.
bool check_items(const Plan &p, const std::vector<GemmItem> &items, size_t first, size_t count, bool inverse_shape,
                 int bm, int bn, int bk)
{
    if (count == 0 || count % kXcds || first + count > items.size()) return false;
    int ncol = 2 * p.nfld;
    for (size_t q = first; q < first + count; ++q) {
        const GemmItem &it = items[q];
        if (it.m < 0) continue;
        if (it.m > p.trunc) return false;
        const MBlock &b = p.mb[it.m];
        if (it.tc < 0 || it.tc * bn >= ncol) return false;
        if (inverse_shape) {
            if (it.tr < 0 || it.tr * bm >= b.R || (it.tr + 1) * bm > b.Rp) return false;
            if ((int64_t)((b.K0 + bk - 1) / bk) * bk > b.Kp) return false;
        } else {
            if (it.tr < 0 || it.tr * bm >= b.K0 || (it.tr + 1) * bm > b.Kp) return false;
            if ((int64_t)((b.R + bk - 1) / bk) * bk > b.Rp) return false;
        }
        if (b.j0 + b.R > p.nlat / 2) return false;
    }
    return true;
}

// A work list's main part with bm x bn tiles and its tail part (if any) with
// bm x tail_bn tiles.
bool check_work_list(const Plan &p, const std::vector<GemmItem> &items, int nmain, bool inverse_shape, int bm,
                     int bn, int tail_bn, int bk)
{
    bool ok = nmain >= 1 && nmain <= (int)items.size() &&
              check_items(p, items, 0, (size_t)nmain, inverse_shape, bm, bn, bk);
    if (ok && nmain < (int)items.size())
        ok = tail_bn > 0 && check_items(p, items, (size_t)nmain, items.size() - nmain, inverse_shape, bm, tail_bn, bk);
    if (!ok && std::getenv("SHTX_DEBUG"))
        std::fprintf(stderr, "shtx: Legendre GEMM work-list check failed (%s)\n", inverse_shape ? "inverse" : "direct");
    return ok;
}


// One launch over items [first, first + count) of a work list, tiles bm x bn.
template <typename T, int BK, bool INV>
hipError_t launch_mfma_part(const GemmArgs &args, int first, int count, int bm, int bn, hipStream_t s)
{
    GemmArgs a = args;
    a.items += first;
    const int grid = count;
#define SHTX_TILE(BM, BN, NW)                                              \
    if (bm == BM && bn == BN) {                                            \
        k_leg_mfma<T, BM, BN, BK, INV, NW><<<grid, 64 * NW, 0, s>>>(a);    \
        return hipGetLastError();                                          \
    }
    if constexpr (sizeof(T) == 4) {
        SHTX_TILE(128, 128, 8)
        SHTX_TILE(64, 128, 8)
        SHTX_TILE(128, 64, 8)
    } else {
        SHTX_TILE(64, 64, 8)
        SHTX_TILE(32, 64, 8)
        SHTX_TILE(64, 32, 4)
    }
#undef SHTX_TILE
    return hipErrorInvalidValue;
}

template <typename T, int BK, bool INV>
hipError_t launch_mfma(const Plan &p, const GemmArgs &a, int bm, int bn, hipStream_t s)
{
    // the work lists were checked against these shapes when they were built
    const std::vector<GemmItem> &items = INV ? p.inv_items : p.dir_items;
    const int nmain = INV ? p.inv_nmain : p.dir_nmain, tail_bn = INV ? p.inv_tail_bn : p.dir_tail_bn;
    if (!p.shapes_ok || nmain < 1) return hipErrorInvalidValue;
    hipError_t e = launch_mfma_part<T, BK, INV>(a, 0, nmain, bm, bn, s);
    if (e != hipSuccess || nmain == (int)items.size()) return e;
    return launch_mfma_part<T, BK, INV>(a, nmain, (int)items.size() - nmain, bm, tail_bn, s);
}

// Largest magnitude of each field's spectral coefficients (Re and Im of
// every a_n^m except Im a_n^0, which the transforms ignore), as float bits:
// the bound from which the half form scales the inverse-shaped GEMM's data
// operand.  Blocks (chunk, field) each take a contiguous chunk of one
// field's coefficients and fold their maximum into fmax[f] with an atomic
// max (non-negative floats order as their bits), after k_clear_u32 has
// zeroed it; the maximum does not depend on the order.
constexpr int kAbsmaxChunks = 8;

__global__ void k_clear_u32(unsigned *x, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0u;
}

__global__ __launch_bounds__(1024) void k_spec_absmax(const float2 *spec, int64_t nspec, int trunc, unsigned *fmax)
{
    __shared__ float red[16];
    const int f = blockIdx.y;
    const int64_t chunk = (nspec + kAbsmaxChunks - 1) / kAbsmaxChunks;
    const int64_t i0 = blockIdx.x * chunk, i1 = min(nspec, i0 + chunk);
    const float2 *row = spec + (int64_t)f * nspec;
    float mx = 0.f;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 1024) {
        const float2 z = row[i];
        mx = fmaxf(mx, fabsf(z.x));
        if (i > trunc) mx = fmaxf(mx, fabsf(z.y));  // index i <= N is m = 0
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int w = 0; w < 16; ++w) t = fmaxf(t, red[w]);
        atomicMax(fmax + f, __float_as_uint(t));
    }
}

// K-stage depth of the split kernels: 128 x 128 direct tiles take 64-deep
// stages (each tile row of a stage one whole 128-byte line of the table;
// measured 9.9 -> 8.8 ms at TCo1279), every other shape 32 (64 measured
// slower for the inverse)
constexpr int split_stage_depth(bool inverse, int bm) { return (!inverse && bm == 128) ? 64 : 32; }

template <bool F16, bool INV>
hipError_t launch_split(const Plan &p, const GemmArgs &a, int bm, int bn, hipStream_t s)
{
    const std::vector<GemmItem> &items = INV ? p.inv_items : p.dir_items;
    const int grid = (int)items.size();
    if (!p.shapes_ok || grid < 1) return hipErrorInvalidValue;
    if (bm == 128 && bn == 128)
        k_leg_split<F16, 128, 128, split_stage_depth(INV, 128), INV, 8><<<grid, 512, 0, s>>>(a);
    else if (bm == 64 && bn == 128)
        k_leg_split<F16, 64, 128, split_stage_depth(INV, 64), INV, 4><<<grid, 256, 0, s>>>(a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

// Tile shapes with a kernel instantiation (split forms: 128 x 128 with eight
// waves, 64 x 128 with four).
int gemm_tile_candidates(int prec, int *bm, int *bn, int max)
{
    static const int f32[][2] = {{128, 128}, {64, 128}, {128, 64}};
    static const int f64[][2] = {{64, 64}, {32, 64}, {64, 32}};
    static const int b16[][2] = {{64, 128}, {128, 128}};
    const int(*t)[2] = prec == SHTX_FP64 ? f64 : prec == SHTX_FP32 ? f32 : b16;
    int n = split_form(prec) ? 2 : 3;
    for (int i = 0; i < n && i < max; ++i) {
        bm[i] = t[i][0];
        bn[i] = t[i][1];
    }
    return n;
}

bool gemm_tile_supported(int prec, int bm, int bn)
{
    int cbm[8], cbn[8];
    int n = gemm_tile_candidates(prec, cbm, cbn, 8);
    for (int i = 0; i < n; ++i)
        if (cbm[i] == bm && cbn[i] == bn) return true;
    return false;
}

bool gemm_shapes_ok(const Plan &p)
{
    const bool split = split_form(p.prec);
    const int bk_inv = split ? split_stage_depth(true, p.inv_bm) : 16;
    const int bk_dir = split ? split_stage_depth(false, p.dir_bm) : 16;
    if (!gemm_tile_supported(p.prec, p.inv_bm, p.inv_bn) || !gemm_tile_supported(p.prec, p.dir_bm, p.dir_bn))
        return false;
    bool inv_ok = p.inv_items.empty() ||
                  check_work_list(p, p.inv_items, p.inv_nmain, true, p.inv_bm, p.inv_bn, p.inv_tail_bn, bk_inv);
    return inv_ok && check_work_list(p, p.dir_items, p.dir_nmain, false, p.dir_bm, p.dir_bn, p.dir_tail_bn, bk_dir);
}

hipError_t launch_gemm_inverse(const Plan &p, const void *spec, void *four, unsigned *fmax, hipStream_t s)
{
    GemmArgs a = make_args(p, true, spec, four, false, fmax);
    if (p.inv_items.empty()) return hipSuccess;
    if (p.prec == SHTX_FP64) return launch_mfma<double, 16, true>(p, a, p.inv_bm, p.inv_bn, s);
    if (p.prec == SHTX_FP32) return launch_mfma<float, 16, true>(p, a, p.inv_bm, p.inv_bn, s);
    if (p.prec == SHTX_FP16X3) {
        if (!fmax) return hipErrorInvalidValue;
        k_clear_u32<<<(p.nfld + 255) / 256, 256, 0, s>>>(fmax, p.nfld);
        k_spec_absmax<<<dim3(kAbsmaxChunks, p.nfld), 1024, 0, s>>>((const float2 *)spec, p.nspec, p.trunc, fmax);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_split<true, true>(p, a, p.inv_bm, p.inv_bn, s);
    }
    return launch_split<false, true>(p, a, p.inv_bm, p.inv_bn, s);
}

hipError_t launch_gemm_direct(const Plan &p, const void *four, void *spec, bool adjoint, unsigned *fmax,
                              hipStream_t s)
{
    GemmArgs a = make_args(p, false, four, spec, adjoint, fmax);
    if (p.prec == SHTX_FP64) return launch_mfma<double, 16, false>(p, a, p.dir_bm, p.dir_bn, s);
    if (p.prec == SHTX_FP32) return launch_mfma<float, 16, false>(p, a, p.dir_bm, p.dir_bn, s);
    if (p.prec == SHTX_FP16X3) {
        // the ring r2c FFT that wrote the workspace recorded each field's maximum
        if (!fmax) return hipErrorInvalidValue;
        return launch_split<true, false>(p, a, p.dir_bm, p.dir_bn, s);
    }
    return launch_split<false, false>(p, a, p.dir_bm, p.dir_bn, s);
}

}  // namespace shtx
