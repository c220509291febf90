// Measurement helper: the gather throughput that bounds the step kernel.
// One 8-lane group per run of 32 consecutive indices loads the 128-byte rows
// X[idx[e]] (32 floats, one float4 per lane, eight loads in flight) and
// writes their sum, so a pass moves m rows through the same gather path as
// the step kernel's neighbour loads, without its CSR stream, three-term update
// or accumulator.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace gs {

namespace {

constexpr int kRun = 32;      // indices per 8-lane group
constexpr int kInFlight = 8;  // row loads in flight per lane

__global__ __launch_bounds__(256) void gather_rows_kernel(const float4* __restrict__ X, int64_t n,
                                                          const int32_t* __restrict__ idx, int64_t m,
                                                          float4* __restrict__ out) {
    const int lane8 = threadIdx.x & 7;
    const int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 3;
    const int64_t e0 = grp * kRun;
    const int64_t e1 = e0 + kRun < m ? e0 + kRun : m;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t e = e0; e < e1; e += kInFlight) {
        float4 v[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            int64_t j = e + u < e1 ? idx[e + u] : 0;
            j = (j >= 0 && j < n) ? j : 0;
            v[u] = X[j * 8 + lane8];
        }
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            const float s = e + u < e1 ? 1.f : 0.f;
            acc.x = fmaf(s, v[u].x, acc.x);
            acc.y = fmaf(s, v[u].y, acc.y);
            acc.z = fmaf(s, v[u].z, acc.z);
            acc.w = fmaf(s, v[u].w, acc.w);
        }
    }
    if (e0 < m) out[grp * 8 + lane8] = acc;
}

}  // namespace

int64_t gather_out_floats(int64_t m) { return (m + kRun - 1) / kRun * 32; }

void launch_gather_rows(const float* X, int64_t n, const int32_t* idx, int64_t m, float* out, hipStream_t st) {
    const int64_t groups = (m + kRun - 1) / kRun;
    const int64_t blocks = (groups * 8 + 255) / 256;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                       reinterpret_cast<const float4*>(X), n, idx, m, reinterpret_cast<float4*>(out));
}

}  // namespace gs
