// Device-side checks of caller arrays that must be finite and >= 0
// (histograms, barycenter inputs, vertex weights).  They live in device
// memory, so the host cannot look at them before enqueueing work; one pass
// counts the non-finite and the negative entries into bad[0] and bad[1], and
// the driver reads the counts back at the call's synchronisation.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace gs {

namespace {

constexpr int kThreads = 256;
constexpr int64_t kMaxBlocks = 2048;

__global__ __launch_bounds__(kThreads) void count_invalid_kernel(const float* __restrict__ x, int64_t count,
                                                                 unsigned long long* __restrict__ bad) {
    unsigned long long nonfinite = 0, negative = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += stride) {
        const float v = x[i];
        if (!__builtin_isfinite(v))
            ++nonfinite;
        else if (v < 0.f)
            ++negative;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        nonfinite += __shfl_xor(nonfinite, o, 64);
        negative += __shfl_xor(negative, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (nonfinite) atomicAdd(bad, nonfinite);
        if (negative) atomicAdd(bad + 1, negative);
    }
}

}  // namespace

void launch_count_invalid(const float* x, int64_t count, unsigned long long* bad, hipStream_t st) {
    if (count <= 0) return;
    int64_t blocks = (count + kThreads - 1) / kThreads;
    if (blocks > kMaxBlocks) blocks = kMaxBlocks;
    hipLaunchKernelGGL(count_invalid_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, x, count, bad);
}

}  // namespace gs
