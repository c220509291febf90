// Moving columns between a set of m distributions and a batch of B pairs.
//
// Gather: a batch's mu (or nu) block takes column cols[b] of the node-major
// n x m distribution matrix H, out[i*B + b] = H[i*m + cols[b]]; one thread
// per output element, consecutive threads write consecutive elements.
//
// Per-distribution gradients from per-pair gradients.  When B pairs of a
// batch take their sources (or targets) from a set of m distributions, the
// gradient of a sum of the pairs' distances with respect to distribution c is
// the sum of the pair columns drawn from c (chain rule through the sum; a
// distribution paired with itself collects both its mu and its nu column).
//
// G is distribution-major (m x n: distribution c's gradient is the contiguous
// n-vector at G + c*n), so for a fixed column b the lanes of a wave update
// consecutive nodes of one row of G.  A block owns 256 consecutive nodes; it
// stages their src rows through LDS 32 columns at a time (coalesced loads of
// the node-major n x B block), then each thread adds its node's columns into
// G in the order b = 0, 1, ..., B-1.  One thread owns each node, so repeated
// indices in cols need no atomics and the sums are deterministic.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace gs {

namespace {

constexpr int kNodes = 256;  // nodes (threads) per block
constexpr int kCols = 32;    // columns staged per pass

__global__ __launch_bounds__(kNodes) void accumulate_columns_kernel(const float* __restrict__ src, int64_t n, int B,
                                                                    const int32_t* __restrict__ cols, int m,
                                                                    float* __restrict__ G) {
    __shared__ float tile[kNodes][kCols + 1];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kNodes;
    const int rows = n - r0 < kNodes ? (int)(n - r0) : kNodes;
    const int64_t node = r0 + tid;
    for (int b0 = 0; b0 < B; b0 += kCols) {
        const int w = B - b0 < kCols ? B - b0 : kCols;
        for (int e = tid; e < rows * w; e += kNodes) {
            const int r = e / w;
            const int cc = e - r * w;
            tile[r][cc] = src[(r0 + r) * B + b0 + cc];
        }
        __syncthreads();
        if (tid < rows) {
            for (int cc = 0; cc < w; ++cc) {
                const int c = cols[b0 + cc];
                if (c >= 0 && c < m) {
                    float* g = G + (size_t)c * (size_t)n + node;
                    *g = *g + tile[tid][cc];
                }
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void gather_columns_kernel(const float* __restrict__ H, int64_t n, int m,
                                                             const int32_t* __restrict__ cols, int B,
                                                             float* __restrict__ out) {
    const int64_t total = n * B;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / B;
        const int c = cols[e - i * B];
        out[e] = (c >= 0 && c < m) ? H[i * m + c] : 0.f;
    }
}

}  // namespace

void launch_gather_columns(const float* H, int64_t n, int m, const int32_t* cols, int B, float* out, hipStream_t st) {
    int64_t blocks = (n * B + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(gather_columns_kernel, dim3((unsigned)blocks), dim3(256), 0, st, H, n, m, cols, B, out);
}

void launch_accumulate_columns(const float* src, int64_t n, int B, const int32_t* cols, int m, float* G,
                               hipStream_t st) {
    const int64_t blocks = (n + kNodes - 1) / kNodes;
    hipLaunchKernelGGL(accumulate_columns_kernel, dim3((unsigned)blocks), dim3(kNodes), 0, st, src, n, B, cols, m,
                       G);
}

}  // namespace gs
