// Peak microbenchmarks of one gfx950 GPU (declared in include/qed_peaks.h): a 16-byte
// vector copy for the HBM bandwidth, and chains of fused multiply-adds for the
// non-packed FP32 and the FP64 vector issue rates.  Not part of the generator.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qed_peaks.h"

namespace {

constexpr int kBlock = 256;

// One 16-byte element per thread over a grid that covers the whole buffer (on
// gfx950 this streams faster than a grid-stride loop over fewer blocks).
__global__ __launch_bounds__(kBlock) void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                 uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_fma(T *__restrict__ sink, uint64_t iters, T a, T b) {
    T x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (T)(threadIdx.x + c) * (T)1e-3;
    for (uint64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
#pragma unroll
            for (int c = 0; c < 8; ++c) x[c] = fma(x[c], a, b);
        }
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c];
    sink[(uint64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Timer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
    bool init() { return hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess; }
};

}  // namespace

extern "C" {

int qed_peak_copy(const void *src, void *dst, uint64_t bytes, int reps, void *stream, float *ms) {
    if (!src || !dst || !ms || bytes == 0 || bytes % 16 || reps < 1) return -1;
    if (((uintptr_t)src | (uintptr_t)dst) % 16) return -1;
    const char *s = static_cast<const char *>(src);
    const char *d = static_cast<const char *>(dst);
    if (s < d + bytes && d < s + bytes) return -1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t n = bytes / 16;
    const uint64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 0x7FFFFFFFull) return -1;
    Timer t;
    if (!t.init()) return -4;
    // one untimed pass
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const float4 *)src, (float4 *)dst, n);
    if (hipGetLastError() != hipSuccess || hipEventRecord(t.e0, st) != hipSuccess) return -4;
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const float4 *)src, (float4 *)dst,
                           n);
    if (hipGetLastError() != hipSuccess || hipEventRecord(t.e1, st) != hipSuccess ||
        hipEventSynchronize(t.e1) != hipSuccess)
        return -4;
    float total = 0.0f;
    if (hipEventElapsedTime(&total, t.e0, t.e1) != hipSuccess) return -4;
    *ms = total / (float)reps;
    return 0;
}

int qed_peak_fma(int dtype, void *sink, int blocks, uint64_t iters, void *stream, float *ms, double *flops) {
    if (!sink || !ms || !flops || blocks < 1 || iters < 1 || (dtype != 0 && dtype != 1)) return -1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Timer t;
    if (!t.init()) return -4;
    auto launch = [&](uint64_t it) {
        if (dtype == 0)
            hipLaunchKernelGGL(k_fma<float>, dim3(blocks), dim3(kBlock), 0, st, (float *)sink, it, 0.999999f,
                               1e-7f);
        else
            hipLaunchKernelGGL(k_fma<double>, dim3(blocks), dim3(kBlock), 0, st, (double *)sink, it,
                               0.999999999999, 1e-13);
    };
    launch(1);  // warm-up
    if (hipGetLastError() != hipSuccess || hipEventRecord(t.e0, st) != hipSuccess) return -4;
    launch(iters);
    if (hipGetLastError() != hipSuccess || hipEventRecord(t.e1, st) != hipSuccess ||
        hipEventSynchronize(t.e1) != hipSuccess)
        return -4;
    if (hipEventElapsedTime(ms, t.e0, t.e1) != hipSuccess) return -4;
    *flops = 2.0 * 8.0 * 16.0 * (double)iters * (double)blocks * kBlock;
    return 0;
}

}  // extern "C"
