// Hop levels of a support for the frontier-sparse Chebyshev steps.
//
// T_k = T_k(y) x is zero outside the k-hop neighbourhood of supp(x) (y couples
// a node only to itself and its graph neighbours), so step k can skip the rows
// more than k hops from the support.  The levels are the breadth-first hop
// distances from the support up to `depth` (kFarLevel beyond), found level by
// level: sweep s lowers the neighbours of the rows at level s - 1 that are
// still farther out to s.  Every writer of a sweep stores the same value s,
// and a row read as kFarLevel or s by another lane is handled alike, so the
// stores need no atomics.  A sweep after one that found no new row returns at
// once.  Block levels (the minimum over a step block's rows) let whole blocks
// outside the frontier skip their CSR.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace gs {

namespace {

constexpr int kBlk = 256;
constexpr int kLanesPerRow = 8;   // lanes sharing a frontier row's nonzeros in a sweep

int blocks_for(int64_t count) {
    int64_t g = (count + kBlk - 1) / kBlk;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

// Level 0 where any of the B columns of h is nonzero, kFarLevel elsewhere
// (h: n x ldp with zero padding columns, as the plan's buffers hold it);
// flags[s] (s = 0..depth) records whether sweep s found a new row (flags[0]:
// the support itself, taken as nonempty).
__global__ __launch_bounds__(kBlk) void support_init_kernel(const float* h, int64_t n, int ldp, int B,
                                                            uint32_t* level, int32_t* flags, int depth) {
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t0 <= depth) flags[t0] = t0 == 0 ? 1 : 0;
    for (int64_t i = t0; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float* hr = h + i * ldp;
        bool in = false;
        if (ldp % 4 == 0) {   // padded rows of float4 groups (padding columns hold zeros)
            const float4* h4 = reinterpret_cast<const float4*>(hr);
            for (int c = 0; c < ldp / 4 && !in; ++c) {
                const float4 v = h4[c];
                in = v.x != 0.f || v.y != 0.f || v.z != 0.f || v.w != 0.f;
            }
        } else {
            for (int c = 0; c < B && !in; ++c) in = hr[c] != 0.f;
        }
        level[i] = in ? 0u : kFarLevel;
    }
}

// Sweep s: a thread per row finds the rows at level s - 1 among its block's
// kBlk rows and lists them in LDS; then kLanesPerRow lanes per listed row walk
// its nonzeros (each every kLanesPerRow-th, four loads in flight) and lower
// neighbours still farther out to s.  The scan reads one level per row; only
// the frontier's rows read their nonzeros.
__global__ __launch_bounds__(kBlk) void level_sweep_kernel(const int32_t* rowptr, const int32_t* col, int64_t n,
                                                           uint32_t* level, int32_t* flags, int s) {
    if (flags[s - 1] == 0) return;   // the frontier is empty: every level is final
    __shared__ int32_t listed[kBlk];
    __shared__ int nlisted;
    const int sub = threadIdx.x % kLanesPerRow;
    const uint32_t prev = (uint32_t)(s - 1), cur = (uint32_t)s;
    bool found = false;
    for (int64_t base = blockIdx.x * (int64_t)kBlk; base < n; base += (int64_t)gridDim.x * kBlk) {
        if (threadIdx.x == 0) nlisted = 0;
        __syncthreads();
        const int64_t i = base + threadIdx.x;
        if (i < n && level[i] == prev) listed[atomicAdd(&nlisted, 1)] = (int32_t)i;
        __syncthreads();
        const int m = nlisted;
        for (int r = threadIdx.x / kLanesPerRow; r < m; r += kBlk / kLanesPerRow) {
            const int row = listed[r];
            const int e1 = rowptr[row + 1];
            for (int e = rowptr[row] + sub; e < e1; e += 4 * kLanesPerRow) {
                int j[4];
                uint32_t l[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) j[u] = e + u * kLanesPerRow < e1 ? col[e + u * kLanesPerRow] : -1;
#pragma unroll
                for (int u = 0; u < 4; ++u) l[u] = j[u] >= 0 ? level[j[u]] : 0u;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (l[u] > cur) {
                        level[j[u]] = cur;
                        found = true;
                    }
            }
        }
        __syncthreads();   // the list is rebuilt by the next pass
    }
    if (found) flags[s] = 1;
}

__global__ __launch_bounds__(kBlk) void block_level_kernel(const uint32_t* level, int64_t n, int rpb,
                                                           uint32_t* blk_level) {
    const int64_t nb = (n + rpb - 1) / rpb;
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r1 = (b + 1) * rpb < n ? (b + 1) * rpb : n;
        uint32_t m = kFarLevel;
        for (int64_t r = b * rpb; r < r1; ++r) m = level[r] < m ? level[r] : m;
        blk_level[b] = m;
    }
}

// Zeros in up to four float buffers of `count` elements each, one launch.
__global__ __launch_bounds__(kBlk) void zero_buffers_kernel(float* b0, float* b1, float* b2, float* b3,
                                                            int64_t count) {
    float* bufs[4] = {b0, b1, b2, b3};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (bufs[q]) bufs[q][i] = 0.f;
    }
}

}  // namespace

void launch_zero_buffers(float* b0, float* b1, float* b2, float* b3, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(zero_buffers_kernel, dim3(blocks_for(count)), dim3(kBlk), 0, st, b0, b1, b2, b3, count);
}

void launch_support_levels(const float* h, int64_t n, int ldp, int B, const int32_t* rowptr, const int32_t* col,
                           int depth, int rpb, uint32_t* level, uint32_t* blk_level, int32_t* flags, hipStream_t st) {
    if (rpb < 1 || depth < 1 || depth > GS_MAX_K) fail(GS_ERR_INVALID, "level depth or rows per block out of range");
    if (n == 0) return;
    // the flags are cleared by the first depth + 1 threads of the grid
    hipLaunchKernelGGL(support_init_kernel, dim3(blocks_for(n > depth + 1 ? n : depth + 1)), dim3(kBlk), 0, st, h,
                       n, ldp, B, level, flags, depth);
    for (int s = 1; s <= depth; ++s)
        hipLaunchKernelGGL(level_sweep_kernel, dim3(blocks_for(n)), dim3(kBlk), 0, st, rowptr, col, n, level, flags,
                           s);
    hipLaunchKernelGGL(block_level_kernel, dim3(blocks_for((n + rpb - 1) / rpb)), dim3(kBlk), 0, st, level, n, rpb,
                       blk_level);
}

}  // namespace gs
