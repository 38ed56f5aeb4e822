/*
 * shtx — spherical-harmonic transforms of many scalar fields on one AMD
 * Instinct MI355X (gfx950).
 *
 * The operation is the spectral-transform workload of the IFS that the paper
 * optimises (Section 3, "Spectral Transform - Spherical Harmonics Dwarf";
 * Section 2.2.2 names it the most important challenge of the IFS).  The
 * paper gives no formula, so the definition implemented here is the
 * textbook one, fixed below and mirrored by an independent FP64 CPU oracle:
 *
 *   inverse   g_{j,k} = sum_{m=0}^{M_j} c_m Re(F_m(mu_j) e^{i m lambda_k}),
 *             F_m(mu_j) = sum_{n=m}^{N} a_n^m P̄_n^m(mu_j),
 *             c_0 = 1, c_m = 2 (m >= 1), lambda_k = 2 pi k / nlon_j;
 *   direct    a_n^m = (1/2) sum_{j: M_j >= m} w_j G_m(mu_j) P̄_n^m(mu_j),
 *             G_m(mu_j) = (1/nlon_j) sum_k g_{j,k} e^{-i m lambda_k},
 *             Im a_n^0 := 0;
 *   adjoints  the transposes of both under the Euclidean inner product on
 *             (Re, Im) of the stored triangle and on raw grid values.
 *
 * mu_j, w_j are the Gauss-Legendre nodes (descending, each the double nearest
 * to the true root) and weights on nlat latitudes; P̄_n^m is normalised to
 * (1/2) int_{-1}^{1} (P̄_n^m)^2 dmu = 1 with no Condon-Shortley phase;
 * M_j = min(N, floor((nlon_j - 1)/2)) is the ring cutoff.  The octahedral grid
 * O_{nlat/2} has 20 + 4 i points on the i-th ring from the nearer pole (the
 * TCo grids the paper runs, Sections 3.1.4.1 and 3.2.2).
 *
 * Layouts (device memory, caller-owned, contiguous, 16-byte aligned):
 *   spec  [nfld][nspec] interleaved complex, m-major, n ascending:
 *         index(m, n) = m (2N + 3 - m) / 2 + (n - m); nspec = (N+1)(N+2)/2.
 *         complex128 for SHTX_FP64 plans, complex64 otherwise.
 *   grid  [nfld][npts] real, rings concatenated north to south, each ring
 *         starting at lambda = 0.  float64 for SHTX_FP64 plans, float32
 *         otherwise.
 *
 * Precision forms (the Legendre arithmetic; the ring FFTs run in the grid
 * type): SHTX_FP64 plain double; SHTX_FP32 single precision on the matrix
 * cores with FP32 accumulation; SHTX_BF16X3 split bfloat16 hi+lo operands
 * (three products, lo*lo dropped) with per-m power-of-two scaling of the
 * Legendre table and FP32 accumulation; SHTX_FP16X3 the same split with IEEE
 * half hi+lo operands (11-bit halves, 5-bit exponent), the table block of
 * each m scaled so that its largest entry lies in [2^13, 2^14) and each
 * field's data operand scaled likewise from a bound on its largest value,
 * so that both halves stay in half's normal range; the scales are powers of
 * two and are undone exactly on the FP32 accumulators.
 *
 * Ownership and errors.  A plan owns its tables and workspace, allocated at
 * create time and freed at destroy; the transform calls allocate nothing.
 * Calls are asynchronous on the HIP stream passed (NULL = the default
 * stream); a plan may be used from one stream at a time because its
 * workspace is shared by every call.  Inputs are never modified; an output
 * that overlaps an input, a pointer that is not 16-byte aligned, and a
 * pointer that is not device (or managed) memory of the plan's device are
 * rejected with SHTX_EINVAL before anything is launched.  Functions return
 * SHTX_OK or a negative code; no C++ exception crosses this interface.
 * Device faults surface on the next synchronisation.  Destroying a plan or
 * changing its shapes waits for the plan's last transform call (not for the
 * rest of the device).
 */
#ifndef SHTX_H
#define SHTX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct shtx_plan_s *shtx_plan;

enum shtx_grid { SHTX_GRID_FULL = 0, SHTX_GRID_OCTAHEDRAL = 1 };
enum shtx_prec { SHTX_FP64 = 0, SHTX_FP32 = 1, SHTX_BF16X3 = 2, SHTX_FP16X3 = 3 };

enum shtx_status {
    SHTX_OK = 0,
    SHTX_EINVAL = -1,      /* bad argument, null or overlapping pointers */
    SHTX_ENOMEM = -2,      /* device or host allocation failed at plan time */
    SHTX_EHIP = -3,        /* a HIP runtime call or kernel launch failed */
    SHTX_EUNSUPPORTED = -4, /* valid but unsupported (odd nlat, odd ring length) */
    SHTX_ESCRATCH = -5      /* needs more scratch than shtx_inv_trans_noalloc's static array */
};

/* Flags for shtx_plan_create. */
#define SHTX_FLAG_GRAPH 1u /* replay each transform as a captured hipGraph */
/* Tile autotuning: plan creation times every candidate tile shape of the
 * two Legendre GEMM launches and every candidate ring-FFT blocking on the
 * plan's own shape (scratch operands filled with a pseudo-random integer hash
 * of the index: constant operands change the matrix cores' power draw and
 * clock) and keeps the fastest; the
 * choice is reported in shtx_info.  If the environment variable
 * SHTX_TUNE_CACHE names a file, choices are looked up there first and
 * appended after timing, one JSON object per line, keyed by GPU
 * architecture, truncation, grid, latitudes, fields, precision and a hash of
 * the kernel sources.  Without the flag each precision uses fixed shapes. */
#define SHTX_FLAG_AUTOTUNE 4u
/* Wind images: the plan also serves shtx_uv_trans (it then allocates one more
 * spectral array of its own shape at create time).  Such a plan has
 * truncation N + 1 and 2 F fields for F wind fields of truncation N; nfld
 * must be even and trunc >= 1 (else SHTX_EINVAL). */
#define SHTX_FLAG_UV 8u

typedef struct {
    int32_t trunc, nlat, nfld, prec, grid;
    int32_t max_nlon;
    int64_t nspec;          /* complex coefficients per field */
    int64_t npts;           /* grid points per field */
    int64_t nfour;          /* kept Fourier coefficients per field: sum_j (M_j + 1) */
    size_t table_bytes;     /* Legendre tables resident in HBM */
    size_t workspace_bytes; /* Fourier workspace and FFT tables */
    double legendre_flops;  /* algorithmic Legendre flops of one transform, all fields */
    double plan_seconds;    /* wall time of shtx_plan_create */
    int32_t inv_tile[2];    /* rows x columns of the inverse-shaped GEMM tiles */
    int32_t dir_tile[2];    /* rows x columns of the direct-shaped GEMM tiles */
    int32_t fft_cap;        /* LDS complex values per ring-FFT block (fields per block = cap / ring slot) */
    int32_t tuned;          /* 0 default shapes, 1 timed at plan creation, 2 read from the tune cache */
} shtx_info;

/* Create a plan for triangular truncation `trunc` on `nlat` Gaussian
 * latitudes (even).  grid = SHTX_GRID_FULL uses `nlon_full` (even) points on
 * every ring; SHTX_GRID_OCTAHEDRAL ignores it.  `nfld` fields per call.
 * Nodes, weights and P̄_n^m tables are generated on the device (FP64) on
 * `hip_stream`; the call returns after they are complete. */
int shtx_plan_create(shtx_plan *out, int trunc, int grid, int nlat, int nlon_full,
                     int nfld, int prec, unsigned flags, void *hip_stream);

int shtx_plan_info(shtx_plan p, shtx_info *out);

/* Host-only dry run of shtx_plan_create: builds the plan's geometry, table
 * layout, FFT length plans and work lists, checks every kernel's launch shape
 * against them, and fills `out` (may be NULL; plan_seconds is 0) without
 * touching any device.  Returns what shtx_plan_create would return for a
 * shape problem (SHTX_EINVAL / SHTX_EUNSUPPORTED) or SHTX_OK. */
int shtx_plan_check(int trunc, int grid, int nlat, int nlon_full, int nfld, int prec, shtx_info *out);

/* Like shtx_plan_check, with explicit GEMM tile shapes (rows x columns of
 * the inverse- and direct-shaped launches; one of the shapes the autotuner
 * considers for the precision) and ring-FFT blocking `fft_cap` (LDS complex
 * values per block, 1 .. 8192).  A shape without a kernel instantiation is
 * SHTX_EUNSUPPORTED; fft_cap out of range is SHTX_EINVAL. */
int shtx_plan_check_shapes(int trunc, int grid, int nlat, int nlon_full, int nfld, int prec, int inv_bm,
                           int inv_bn, int dir_bm, int dir_bn, int fft_cap, shtx_info *out);

/* Pin the GEMM tile shapes and ring-FFT blocking of an existing plan (for
 * example shapes chosen by an external tuner), with the same meaning and
 * checks as shtx_plan_check_shapes.  Waits for the plan's last transform
 * first; no transform of this plan may be issued concurrently from another
 * thread.  New work lists are checked and uploaded into new device buffers
 * before the plan's are replaced, so on any error (SHTX_EINVAL,
 * SHTX_EUNSUPPORTED, SHTX_ENOMEM, SHTX_EHIP) the plan is unchanged and keeps
 * working. */
int shtx_plan_set_shapes(shtx_plan p, int inv_bm, int inv_bn, int dir_bm, int dir_bn, int fft_cap);

/* Host copies of plan geometry: nlon[nlat] ring lengths. */
int shtx_plan_ring_lengths(shtx_plan p, int32_t *nlon_host);

/* Host copies of the device-generated Gauss nodes and weights, nlat each
 * (descending mu). */
int shtx_plan_nodes(shtx_plan p, double *mu_host, double *w_host);

/* Host copy of the stored Legendre table for wavenumber m, unscaled to
 * double: out[r][n - m] = P̄_n^m(mu_{j_m + r}) for the R_m northern rings
 * carrying m (j_m = first such ring), n = m..trunc.  Returns R_m (>= 0) or an
 * error.  out may be NULL to query R_m. */
int shtx_plan_legendre(shtx_plan p, int m, double *out_host);

/* Inverse transform spec -> grid. */
int shtx_inv_trans(shtx_plan p, const void *spec_d, void *grid_d, void *hip_stream);
/* Direct transform grid -> spec. */
int shtx_dir_trans(shtx_plan p, const void *grid_d, void *spec_d, void *hip_stream);
/* Adjoint of the inverse transform: grid -> spec. */
int shtx_inv_trans_adj(shtx_plan p, const void *grid_d, void *spec_d, void *hip_stream);
/* Adjoint of the direct transform: spec -> grid. */
int shtx_dir_trans_adj(shtx_plan p, const void *spec_d, void *grid_d, void *hip_stream);

/* Wind images from vorticity and divergence (the wind part of the IFS inverse
 * spectral transform, Section 2.2.2), for a plan made with SHTX_FLAG_UV:
 * truncation trunc = N + 1, nfld = 2 F.  On the unit sphere, with
 * streamfunction psi_n^m = -zeta_n^m / (n (n+1)) and velocity potential
 * chi_n^m = -D_n^m / (n (n+1)) (n >= 1),
 *   U = u cos(phi) = d chi / d lambda - (1 - mu^2) d psi / d mu,
 *   V = v cos(phi) = d psi / d lambda + (1 - mu^2) d chi / d mu,
 * fields of truncation N + 1, evaluated on the plan's grid (the same ring
 * cutoff and precision form as shtx_inv_trans).  vor_d, div_d: device
 * [F][(N+1)(N+2)/2] complex each (layout and dtype of the spectral arrays, at
 * truncation N; Im of the m = 0 coefficients ignored); uv_grid_d: device
 * [2F][npts] real, U of wind field f in row f and V in row F + f.  The
 * gradient (d s / d lambda, (1 - mu^2) d s / d mu) of a scalar s is this
 * transform with zeta = 0 and D_n^m = -n (n+1) s_n^m.  Same checks, errors,
 * stream semantics and graph replay as the other transforms. */
int shtx_uv_trans(shtx_plan p, const void *vor_d, const void *div_d, void *uv_grid_d, void *hip_stream);

/* For callers that cannot allocate device memory at transform time (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): shtx_inv_trans with the transform's scratch -- the Fourier
 * workspace [ring][m][nfld] and, for SHTX_FP16X3 plans, the per-field maxima
 * -- in a static device array of SHTX_NOALLOC_SCRATCH_BYTES bytes that the
 * library holds on each GPU it runs on until the process ends, instead of
 * the plan's workspace.  Same arguments, layouts, checks and result as
 * shtx_inv_trans (the same kernels; the output is bit-identical); it calls no
 * allocator.  A plan whose workspace needs more than the array holds
 * (nfour * nfld complex values, plus nfld words rounded to 256 bytes for
 * SHTX_FP16X3) gets SHTX_ESCRATCH and nothing is launched.  The array is
 * located once per device, when a plan is created with that device current;
 * the call must be made with the plan's device current (else SHTX_EINVAL).
 * Every call on one GPU shares that GPU's array, from any plan: calls that
 * overlap in time on one GPU (other streams, other threads) race and give
 * undefined results.  Runs eagerly (no graph replay, no kernel timing). */
#define SHTX_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int shtx_inv_trans_noalloc(shtx_plan p, const void *spec_d, void *grid_d, void *hip_stream);

/* Kernel timing.  With SHTX_FLAG_TIMING at plan creation every transform
 * call records HIP events around each of its kernels on the call's stream
 * (and runs eagerly, not as a graph) while timing is enabled, which it is
 * from creation; shtx_timing_enable(p, 0) turns it off (graph replay, if
 * the plan has SHTX_FLAG_GRAPH, resumes) and (p, 1) on again.  It returns
 * SHTX_EINVAL for a plan made without SHTX_FLAG_TIMING.
 * shtx_timing_read synchronises on the recorded events and returns, per
 * kernel kind, the summed duration in milliseconds and the launch count:
 * index 0 inverse-shaped Legendre GEMM (inv_trans, dir_trans_adj, and
 * uv_trans with its spectral wind step),
 * 1 direct-shaped Legendre GEMM (dir_trans, inv_trans_adj), 2 ring c2r FFT,
 * 3 ring r2c FFT.  Both arrays have 4 entries; either may be NULL.  At most
 * 4096 launches are recorded between resets; later ones are not timed. */
#define SHTX_FLAG_TIMING 2u
int shtx_timing_reset(shtx_plan p);
int shtx_timing_enable(shtx_plan p, int on);
int shtx_timing_read(shtx_plan p, double *ms_sum, int32_t *count);

int shtx_plan_destroy(shtx_plan p);

/* Peak probes (measurement only; no plan, no transform).  The roofline
 * fractions are set against the vendor peaks of MI355X; these probes measure
 * what this GPU sustains for the same units, as the measurement recipe asks
 * (a matrix-core loop and a copy kernel; the paper's roofline takes its
 * memory bandwidth from the STREAM benchmark, Section 4.1.2).
 *   SHTX_PROBE_MFMA_F64/F32  register-resident loop of 8 independent
 *                            16x16x4 MFMA chains per wave on every CU;
 *   SHTX_PROBE_MFMA_BF16/F16 the same with 16x16x32 MFMAs;
 *   SHTX_PROBE_VALU_F32      8 independent FP32 FMA chains per lane (packed
 *                            FP32 instructions are not used by this library);
 *   SHTX_PROBE_HBM_COPY      copies `bytes` from src_d to dst_d, 16 bytes per
 *                            lane, grid-stride (bytes read + bytes written);
 *   SHTX_PROBE_HBM_READ      reads `bytes` from src_d.
 * One warm-up launch, then three launches timed with HIP events on
 * hip_stream (the call synchronises on them).  *rate receives TFLOP/s
 * (compute kinds) or GB/s (memory kinds).  dst_d: device memory, 16-byte
 * aligned, at least 16 bytes for the compute kinds and the read probe (never
 * written at run time), `bytes` for the copy; src_d: device memory, 16-byte
 * aligned, for the memory kinds.  bytes: a multiple of 16, at least 1 MiB,
 * for the memory kinds (ignored otherwise).  Overlapping copy buffers, host
 * pointers, a NULL rate or an unknown kind give SHTX_EINVAL; a failed HIP
 * call SHTX_EHIP.  The probes take a few tens of milliseconds each. */
#define SHTX_PROBE_MFMA_F64 0
#define SHTX_PROBE_MFMA_F32 1
#define SHTX_PROBE_MFMA_BF16 2
#define SHTX_PROBE_MFMA_F16 3
#define SHTX_PROBE_VALU_F32 4
#define SHTX_PROBE_HBM_COPY 5
#define SHTX_PROBE_HBM_READ 6
int shtx_probe_peak(int kind, const void *src_d, void *dst_d, size_t bytes, double *rate, void *hip_stream);

const char *shtx_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SHTX_H */
