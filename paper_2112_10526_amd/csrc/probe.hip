// Throughput probes: the rates the hot-path kernels are measured against, taken
// on the device itself instead of the datasheet (which counts packed FP32 and
// structured sparsity that these kernels do not use).  Each probe keeps every
// lane busy with independent chains of one instruction kind and sums the
// chains into one store per thread, so nothing is optimised away.
#include "kernels.h"

namespace nqs {

constexpr int PR_ITERS = 4096;

// scalar FP32 FMA (v_fma_f32; packed FP32 is not used by this library)
__global__ __launch_bounds__(256) void k_probe_f32(float seed, float* out) {
    float a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = seed + (float)(threadIdx.x + c);
    const float m = 0.9999f, b = 1e-7f;
    for (int it = 0; it < PR_ITERS; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = __builtin_fmaf(a[c], m, b);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += a[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

// FP64 FMA (v_fma_f64)
__global__ __launch_bounds__(256) void k_probe_f64(double seed, double* out) {
    double a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = seed + (double)(threadIdx.x + c);
    const double m = 0.9999, b = 1e-7;
    for (int it = 0; it < PR_ITERS; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = __builtin_fma(a[c], m, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += a[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

// FP32 exponential (v_exp_f32, the transcendental unit behind tanh / exp)
__global__ __launch_bounds__(256) void k_probe_exp(float seed, float* out) {
    float a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = seed * 1e-3f * (float)(threadIdx.x + c);
    for (int it = 0; it < PR_ITERS / 4; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = __builtin_amdgcn_exp2f(-a[c]);  // (stays in (0, 1])
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += a[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

// FP64 matrix cores, v_mfma_f64_16x16x4f64 (2 * 16 * 16 * 4 flops each)
__global__ __launch_bounds__(256) void k_probe_mfma_f64(double seed, double* out) {
    v4d acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = v4d{0, 0, 0, 0};
    const double a = seed + 1e-3 * threadIdx.x, b = 1e-3;
    for (int it = 0; it < PR_ITERS / 16; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

// BF16 matrix cores, v_mfma_f32_16x16x32_bf16 (2 * 16 * 16 * 32 flops each)
__global__ __launch_bounds__(256) void k_probe_mfma_bf16(float seed, float* out) {
    typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
    v4f acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = v4f{0, 0, 0, 0};
    bf8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(seed + 1e-3f * (float)(threadIdx.x + e));
        b[e] = (__bf16)1e-3f;
    }
    for (int it = 0; it < PR_ITERS / 16; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

// ---------------------------------------------------------------------------
int probe_blocks() { return 256 * 4 * 8 / 4; }  // 8 waves per SIMD over 256 CUs
size_t probe_sink_bytes() { return (size_t)probe_blocks() * 256 * 8; }

double launch_probe(hipStream_t st, int kind, void* sink) {
    const int nb = probe_blocks();
    const double threads = (double)nb * 256, waves = threads / 64;
    switch (kind) {
        case 0:
            k_probe_f32<<<nb, 256, 0, st>>>(1.0f, (float*)sink);
            return threads * PR_ITERS * 8 * 2;             // flops
        case 1:
            k_probe_f64<<<nb, 256, 0, st>>>(1.0, (double*)sink);
            return threads * PR_ITERS * 8 * 2;
        case 2:
            k_probe_exp<<<nb, 256, 0, st>>>(1.0f, (float*)sink);
            return threads * (PR_ITERS / 4) * 8;            // exponentials
        case 3:
            k_probe_mfma_f64<<<nb, 256, 0, st>>>(1.0, (double*)sink);
            return waves * (PR_ITERS / 16) * 8 * 2.0 * 16 * 16 * 4;
        case 4:
            k_probe_mfma_bf16<<<nb, 256, 0, st>>>(1.0f, (float*)sink);
            return waves * (PR_ITERS / 16) * 8 * 2.0 * 16 * 16 * 32;
        default:
            return 0.0;
    }
}

}  // namespace nqs
