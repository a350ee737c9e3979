// Throughput probes (sht_probe.h; a benchmark-only library, libsht_probe.so,
// separate from the transform library): long runs of independent FP64 FMAs,
// FP32 16x16x4 and BF16 16x16x32 matrix instructions, and FP32 matrix
// instructions interleaved with FP64 FMAs (do the two overlap?), with no
// memory traffic in the loop.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sht_probe.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kProbeThreads = 256;
constexpr int kChains = 8;

__global__ __launch_bounds__(kProbeThreads) void k_probe_fma64(int iters, double *__restrict__ out) {
    const double x = 1.0 + 1e-9 * threadIdx.x, y = 1.0 - 1e-12;
    double a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = x + i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = fma(a[i], y, x);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

template <int KIND>
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma(int iters, double *__restrict__ out) {
    const float x = 1e-3f * threadIdx.x;
    floatx4 acc[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(x + e);
        b[e] = (__bf16)(x - e);
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) {
            if constexpr (KIND == SHT_PROBE_MFMA_F32)
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, x + i, acc[i], 0, 0, 0);
            else
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// kChains FP32 16x16x4 matrix instructions and kChains x kChains independent
// FP64 FMAs per iteration, interleaved (one matrix instruction, then kChains
// FMAs, as the compiler schedules them): its time against the sum of the two
// pure streams shows whether vector and matrix work overlap.
__global__ __launch_bounds__(kProbeThreads) void k_probe_mixed(int iters, double *__restrict__ out) {
    const float x = 1e-3f * threadIdx.x;
    const double dx = 1.0 + 1e-9 * threadIdx.x, y = 1.0 - 1e-12;
    floatx4 acc[kChains];
    double a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
        a[i] = dx + i;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) {
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, x + i, acc[i], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < kChains; ++j) a[j] = fma(a[j], y, dx);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i] + acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace

extern "C" {

double sht_probe_flops(int kind, int blocks, int iters) {
    if (blocks < 1 || iters < 1) return 0.0;
    const double threads = (double)blocks * kProbeThreads, waves = threads / 64.0;
    switch (kind) {
        case SHT_PROBE_FMA_F64: return threads * iters * kChains * 2.0;
        case SHT_PROBE_MFMA_F32: return waves * iters * kChains * (2.0 * 16 * 16 * 4);
        case SHT_PROBE_MFMA_BF16: return waves * iters * kChains * (2.0 * 16 * 16 * 32);
        case SHT_PROBE_MFMA_F32_FMA_F64:
            return waves * iters * kChains * (2.0 * 16 * 16 * 4) + threads * iters * kChains * kChains * 2.0;
        default: return 0.0;
    }
}

int sht_probe_run(int kind, int blocks, int iters, void *out, void *stream) {
    if (sht_probe_flops(kind, blocks, iters) == 0.0 || !out) return -1;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *o = static_cast<double *>(out);
    switch (kind) {
        case SHT_PROBE_FMA_F64:
            hipLaunchKernelGGL(k_probe_fma64, dim3((unsigned)blocks), dim3(kProbeThreads), 0, st, iters, o);
            break;
        case SHT_PROBE_MFMA_F32:
            hipLaunchKernelGGL(k_probe_mfma<SHT_PROBE_MFMA_F32>, dim3((unsigned)blocks), dim3(kProbeThreads), 0, st,
                               iters, o);
            break;
        case SHT_PROBE_MFMA_BF16:
            hipLaunchKernelGGL(k_probe_mfma<SHT_PROBE_MFMA_BF16>, dim3((unsigned)blocks), dim3(kProbeThreads), 0,
                               st, iters, o);
            break;
        default:
            hipLaunchKernelGGL(k_probe_mixed, dim3((unsigned)blocks), dim3(kProbeThreads), 0, st, iters, o);
            break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
