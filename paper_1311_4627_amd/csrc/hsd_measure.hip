// Calibration of the exponential's issue rate on the device: the heating
// rates need one single-precision exponential each, and the roofline of the
// solver quotes that rate next to the vector-ALU issue bound.
#include "hsd_internal.h"

namespace hsd {
namespace {

constexpr int kChains = 8;      // independent exponentials per lane and iteration
constexpr int kBlocks = 2048;   // 2048 x 256 lanes: eight waves per SIMD of the device
constexpr int kIters = 2048;

// Every lane runs kChains independent chains x <- 2^(-x) (the negation is a
// source modifier of the exponential instruction, so the loop body is
// exponentials only; the chains converge to the fixed point 0.64 and stay
// finite).  One float per lane is written so the work is not dropped.
__global__ void __launch_bounds__(256) k_exp2_rate(float* out, int iters) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = 0.01f * static_cast<float>(k + 1) + 1e-6f * static_cast<float>(t & 1023);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) x[k] = __builtin_amdgcn_exp2f(-x[k]);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[t] = s;
}

}  // namespace

hipError_t measure_exp2(double* per_s) {
    float* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = nullptr;
    hipError_t e = hipMalloc(&out, sizeof(float) * kBlocks * 256);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    constexpr int kRuns = 10;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_exp2_rate, dim3(kBlocks), dim3(256), 0, s, out, kIters);   // warm-up
        e = hipEventRecord(e0, s);
    }
    for (int r = 0; r < kRuns && e == hipSuccess; ++r) {
        hipLaunchKernelGGL(k_exp2_rate, dim3(kBlocks), dim3(256), 0, s, out, kIters);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess)
        *per_s = static_cast<double>(kRuns) * kBlocks * 256.0 * kIters * kChains / (static_cast<double>(ms) * 1e-3);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (out) (void)hipFree(out);
    return e;
}

}  // namespace hsd
