// Frontier levels of a support, set up before the first Chebyshev step.
//
// T_k = T_k(y) x is zero outside the k-hop neighbourhood of supp(x) (y couples
// a node only to itself and its graph neighbours), so step k can skip the rows
// more than k hops from the support.  Before step 1 the rows of the support
// hold level 0, their neighbours level 1 and every other row 255; step k < K
// then pushes level k + 1 to the neighbours of its level-k rows (in the step
// kernel, from the CSR it has staged), so at step k every row within k hops
// holds its exact distance and every other row a level above k.  Block levels
// (the minimum over a step block's rows) let whole blocks outside the
// frontier skip their CSR.  All writers of one launch store the same value,
// so the byte stores need no atomics.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace gs {

namespace {

constexpr int kBlk = 256;
constexpr uint8_t kFar = 255;

int blocks_for(int64_t count) {
    int64_t g = (count + kBlk - 1) / kBlk;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

__global__ __launch_bounds__(kBlk) void support_init_kernel(const float* h, int64_t n, int ldp, int B,
                                                            uint8_t* level) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        bool in = false;
        for (int c = 0; c < B; ++c) in = in || h[i * ldp + c] != 0.f;
        level[i] = in ? 0 : kFar;
    }
}

// Rows off the support with a neighbour on it move to level 1 (a row per
// thread, its nonzeros four at a time; it stops at the first such neighbour).
// Only 0 is read as "on the support" and only 1 is written, so rows lowered
// meanwhile by other threads are read correctly either way.
__global__ __launch_bounds__(kBlk) void support_neighbours_kernel(const int32_t* rowptr, const int32_t* col,
                                                                  int64_t n, uint8_t* level) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (level[i] == 0) continue;
        const int e1 = rowptr[i + 1];
        bool hit = false;
        for (int e = rowptr[i]; e < e1 && !hit; e += 4) {
            int j[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) j[u] = e + u < e1 ? col[e + u] : (int)i;
#pragma unroll
            for (int u = 0; u < 4; ++u) hit = hit || level[j[u]] == 0;
        }
        if (hit) level[i] = 1;
    }
}

__global__ __launch_bounds__(kBlk) void block_level_kernel(const uint8_t* level, int64_t n, int rpb,
                                                           uint8_t* blk_level) {
    const int64_t nb = (n + rpb - 1) / rpb;
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r1 = (b + 1) * rpb < n ? (b + 1) * rpb : n;
        int m = kFar;
        for (int64_t r = b * rpb; r < r1; ++r) m = level[r] < m ? level[r] : m;
        blk_level[b] = (uint8_t)m;
    }
}

}  // namespace

void launch_support_levels(const float* h, int64_t n, int ldp, int B, const int32_t* rowptr, const int32_t* col,
                           int rpb, uint8_t* level, uint8_t* blk_level, hipStream_t st) {
    if (rpb < 1) fail(GS_ERR_INVALID, "rows per block must be positive");
    if (n == 0) return;
    hipLaunchKernelGGL(support_init_kernel, dim3(blocks_for(n)), dim3(kBlk), 0, st, h, n, ldp, B, level);
    hipLaunchKernelGGL(support_neighbours_kernel, dim3(blocks_for(n)), dim3(kBlk), 0, st, rowptr, col, n, level);
    hipLaunchKernelGGL(block_level_kernel, dim3(blocks_for((n + rpb - 1) / rpb)), dim3(kBlk), 0, st, level, n, rpb,
                       blk_level);
}

}  // namespace gs
