// Peak probes: the rates the roofline fractions are set against, measured on
// the GPU at hand (the measurement recipe asks for the vendor peaks to be
// re-measured with a matrix-core loop and a copy kernel, as the paper's
// roofline takes its bandwidth from the STREAM benchmark, Section 4.1.2).
// Nothing here is part of a transform.
//
// * matrix cores: every wave runs a loop of 8 independent MFMA chains on
//   register operands (FP64 16x16x4, FP32 16x16x4, BF16 and FP16 16x16x32);
// * vector ALU: 8 independent FP32 FMA chains per lane (packed FP32 is
//   disabled at build time, so this is the rate the ring FFTs can reach);
// * HBM: a 16-byte-per-lane grid-stride copy, and a read-only sweep.
// The sink argument is 0 at every call; the stores it guards keep the
// compiler from removing the work.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "shtx.h"

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocks = 256 * 8;  // 8 blocks per CU on 256 CUs
constexpr int kChains = 8;

template <int KIND>
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma(int iters, int sink, float *dst)
{
    const int t = blockIdx.x * kProbeThreads + threadIdx.x;
    float s = 0.f;
    if constexpr (KIND == SHTX_PROBE_MFMA_F64) {
        const double a = 1.0 + 1e-3 * (t & 7), b = 1.0 - 1e-3 * (t & 3);
        f64x4 c[kChains];
        for (int q = 0; q < kChains; ++q) c[q] = f64x4{0.0, 0.0, 0.0, 0.0};
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int q = 0; q < kChains; ++q) c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[q], 0, 0, 0);
        for (int q = 0; q < kChains; ++q) s += (float)c[q][0];
    } else if constexpr (KIND == SHTX_PROBE_MFMA_F32) {
        const float a = 1.f + 1e-3f * (t & 7), b = 1.f - 1e-3f * (t & 3);
        f32x4 c[kChains];
        for (int q = 0; q < kChains; ++q) c[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int q = 0; q < kChains; ++q) c[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[q], 0, 0, 0);
        for (int q = 0; q < kChains; ++q) s += c[q][0];
    } else {
        f32x4 c[kChains];
        for (int q = 0; q < kChains; ++q) c[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (KIND == SHTX_PROBE_MFMA_BF16) {
            bf16x8 a, b;
            for (int i = 0; i < 8; ++i) {
                a[i] = (__bf16)(1.f + 0.01f * ((t + i) & 7));
                b[i] = (__bf16)(1.f - 0.01f * ((t + i) & 3));
            }
            for (int it = 0; it < iters; ++it)
#pragma unroll
                for (int q = 0; q < kChains; ++q) c[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[q], 0, 0, 0);
        } else {
            f16x8 a, b;
            for (int i = 0; i < 8; ++i) {
                a[i] = (_Float16)(1.f + 0.01f * ((t + i) & 7));
                b[i] = (_Float16)(1.f - 0.01f * ((t + i) & 3));
            }
            for (int it = 0; it < iters; ++it)
#pragma unroll
                for (int q = 0; q < kChains; ++q) c[q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c[q], 0, 0, 0);
        }
        for (int q = 0; q < kChains; ++q) s += c[q][0];
    }
    if (sink) dst[t & 3] = s;
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_valu(int iters, int sink, float *dst)
{
    const int t = blockIdx.x * kProbeThreads + threadIdx.x;
    const float y = 1.f - 1e-7f * (t & 15), z = 1e-7f * (t & 7);
    float x[kChains];
    for (int q = 0; q < kChains; ++q) x[q] = 1.f + 1e-3f * q;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < kChains; ++q) x[q] = fmaf(x[q], y, z);
    float s = 0.f;
    for (int q = 0; q < kChains; ++q) s += x[q];
    if (sink) dst[t & 3] = s;
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const uint4 *src, uint4 *dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    for (int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const uint4 *src, int64_t n, int sink, unsigned *dst)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    unsigned acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x; i < n; i += stride) {
        const uint4 v = src[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (sink) dst[threadIdx.x & 3] = acc;
}

bool is_device_ptr(const void *p)
{
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

}  // namespace

extern "C" int shtx_probe_peak(int kind, const void *src_d, void *dst_d, size_t bytes, double *rate,
                               void *hip_stream)
{
    if (!rate || kind < SHTX_PROBE_MFMA_F64 || kind > SHTX_PROBE_HBM_READ) return SHTX_EINVAL;
    *rate = 0.0;
    const bool mem = kind == SHTX_PROBE_HBM_COPY || kind == SHTX_PROBE_HBM_READ;
    if (!is_device_ptr(dst_d) || reinterpret_cast<uintptr_t>(dst_d) % 16) return SHTX_EINVAL;
    if (mem) {
        if (!is_device_ptr(src_d) || reinterpret_cast<uintptr_t>(src_d) % 16) return SHTX_EINVAL;
        if (bytes < (size_t(1) << 20) || bytes % 16) return SHTX_EINVAL;
        if (kind == SHTX_PROBE_HBM_COPY) {
            const char *s = static_cast<const char *>(src_d), *d = static_cast<const char *>(dst_d);
            if (s < d + bytes && d < s + bytes) return SHTX_EINVAL;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // iterations per thread for about 15-25 ms per launch at the vendor peaks
    int iters = 0;
    double work = 0.0;  // flops or bytes per launch
    const double waves = (double)kProbeBlocks * kProbeThreads / 64;
    switch (kind) {
    case SHTX_PROBE_MFMA_F64: iters = 10000; work = waves * iters * kChains * 2.0 * 16 * 16 * 4; break;
    case SHTX_PROBE_MFMA_F32: iters = 20000; work = waves * iters * kChains * 2.0 * 16 * 16 * 4; break;
    case SHTX_PROBE_MFMA_BF16:
    case SHTX_PROBE_MFMA_F16: iters = 40000; work = waves * iters * kChains * 2.0 * 16 * 16 * 32; break;
    case SHTX_PROBE_VALU_F32: iters = 100000; work = (double)kProbeBlocks * kProbeThreads * iters * kChains * 2.0; break;
    case SHTX_PROBE_HBM_COPY: work = 2.0 * (double)bytes; break;
    default: work = (double)bytes; break;
    }
    const int64_t n16 = (int64_t)(bytes / 16);
    auto launch = [&]() -> hipError_t {
        switch (kind) {
        case SHTX_PROBE_MFMA_F64:
            k_probe_mfma<SHTX_PROBE_MFMA_F64><<<kProbeBlocks, kProbeThreads, 0, s>>>(iters, 0, (float *)dst_d);
            break;
        case SHTX_PROBE_MFMA_F32:
            k_probe_mfma<SHTX_PROBE_MFMA_F32><<<kProbeBlocks, kProbeThreads, 0, s>>>(iters, 0, (float *)dst_d);
            break;
        case SHTX_PROBE_MFMA_BF16:
            k_probe_mfma<SHTX_PROBE_MFMA_BF16><<<kProbeBlocks, kProbeThreads, 0, s>>>(iters, 0, (float *)dst_d);
            break;
        case SHTX_PROBE_MFMA_F16:
            k_probe_mfma<SHTX_PROBE_MFMA_F16><<<kProbeBlocks, kProbeThreads, 0, s>>>(iters, 0, (float *)dst_d);
            break;
        case SHTX_PROBE_VALU_F32: k_probe_valu<<<kProbeBlocks, kProbeThreads, 0, s>>>(iters, 0, (float *)dst_d); break;
        case SHTX_PROBE_HBM_COPY:
            k_probe_copy<<<kProbeBlocks * 2, kProbeThreads, 0, s>>>((const uint4 *)src_d, (uint4 *)dst_d, n16);
            break;
        default:
            k_probe_read<<<kProbeBlocks * 2, kProbeThreads, 0, s>>>((const uint4 *)src_d, n16, 0, (unsigned *)dst_d);
            break;
        }
        return hipGetLastError();
    };
    constexpr int kReps = 3;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = launch();  // warm-up (clocks, caches)
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < kReps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return SHTX_EHIP;
    if (!(ms > 0.f)) return SHTX_EHIP;
    const double sec = ms * 1e-3 / kReps;
    *rate = mem ? work / sec / 1e9 : work / sec / 1e12;
    return SHTX_OK;
}
