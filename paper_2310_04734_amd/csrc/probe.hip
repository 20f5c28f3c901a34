// Achievable-peak probes (measurement support for the rooflines, not part of the method): a
// streaming device-to-device copy and a loop of back-to-back MFMA instructions on every compute
// unit, each timed with HIP events on the context stream.
#include <algorithm>

#include "internal.h"
#include "util.cuh"

namespace cr {
namespace {

typedef double f64x4_p __attribute__((ext_vector_type(4)));
typedef float f32x4_p __attribute__((ext_vector_type(4)));

// dst[i] = src[i] for n 16-byte vectors, grid-stride
__global__ void __launch_bounds__(256) k_probe_copy(const int4* __restrict__ src, int4* __restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

// kChains independent 16x16x4 MFMA accumulators per wave, iters rounds; one value per lane
// written so that the loop is kept
constexpr int kChains = 8;
__global__ void __launch_bounds__(256) k_probe_mfma64(int iters, double seed, double* __restrict__ out) {
    f64x4_p acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f64x4_p{0, 0, 0, 0};
    const double a = seed * (1 + threadIdx.x), b = seed * (2 + blockIdx.x);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ void __launch_bounds__(256) k_probe_mfma32(int iters, float seed, double* __restrict__ out) {
    f32x4_p acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f32x4_p{0, 0, 0, 0};
    const float a = seed * (1 + threadIdx.x), b = seed * (2 + blockIdx.x);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    }
    float s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

template <typename Launch>
double time_ms(hipStream_t s, int reps, Launch launch) {
    hipEvent_t e0, e1;
    CR_HIP(hipEventCreate(&e0));
    CR_HIP(hipEventCreate(&e1));
    launch();   // warm-up
    CR_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) launch();
    CR_HIP(hipEventRecord(e1, s));
    CR_HIP(hipEventSynchronize(e1));
    float ms = 0;
    CR_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    CR_HIP(hipGetLastError());
    return ms;
}

}  // namespace
}  // namespace cr

using namespace cr;

extern "C" cr_status cr_probe_copy(cr_ctx ctx, int64_t bytes, int32_t reps, double* gbs) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        CR_REQUIRE(gbs && reps > 0 && bytes >= 16 && bytes % 16 == 0, CR_E_INVALID, "cr_probe_copy: bad arguments");
        const int64_t n = bytes / 16;
        DevBuf<int4> a(n), b(n);
        hipStream_t s = ctx->stream;
        fill_zero(reinterpret_cast<unsigned long long*>(a.p), n * 2, s);
        const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 256 * 64);
        const double ms = time_ms(s, reps, [&] { hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(256), 0, s, a.p, b.p, n); });
        *gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;   // read + write
    });
}

extern "C" cr_status cr_probe_mfma(cr_ctx ctx, cr_precision prec, int32_t reps, double* tflops) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        CR_REQUIRE(tflops && reps > 0 && (prec == CR_FP64 || prec == CR_MIXED), CR_E_INVALID,
                   "cr_probe_mfma: bad arguments");
        const int blocks = ctx->num_cu * 8, iters = 4096;   // 8 workgroups (32 waves) per compute unit
        DevBuf<double> out((size_t)blocks * 256);
        hipStream_t s = ctx->stream;
        const double ms = time_ms(s, reps, [&] {
            if (prec == CR_FP64)
                hipLaunchKernelGGL(k_probe_mfma64, dim3(blocks), dim3(256), 0, s, iters, 1e-3, out.p);
            else
                hipLaunchKernelGGL(k_probe_mfma32, dim3(blocks), dim3(256), 0, s, iters, 1e-3f, out.p);
        });
        const double flops = (double)blocks * 4 /* waves */ * iters * kChains * 2.0 * 16 * 16 * 4 * reps;
        *tflops = flops / (ms * 1e-3) / 1e12;
    });
}
