// Candidate nearest neighbours for the common affinity graph (setup, not on
// the timed path).  Brute force over all pairs in 64 x 64 tiles: squared
// distances |q|^2 + |r|^2 - 2 q.r from float32 Gram tiles accumulated in
// registers out of LDS, then each query keeps its KK best candidates in a
// sorted register list.  The host re-ranks the candidates in float64 by exact
// squared distance, so float32 rounding only has to keep the true k nearest
// inside the KK = k + 8 candidates.
#include <cfloat>

#include "internal.h"

namespace gs {
namespace {

constexpr int QT = 64;   // queries per block
constexpr int RT = 64;   // references per tile
constexpr int DC = 32;   // coordinates per LDS chunk
constexpr int PAD = 4;

template <int KK>
__global__ __launch_bounds__(256) void knn_tile_kernel(const float* __restrict__ X, const float* __restrict__ norms,
                                                       int n, int d, int32_t* __restrict__ cand) {
    __shared__ __align__(16) float qs[DC][QT + PAD];
    __shared__ __align__(16) float rs[DC][RT + PAD];
    __shared__ float dt[QT][RT + 1];
    const int tid = threadIdx.x;
    const int ty = tid >> 4;   // queries 4ty .. 4ty+3
    const int tx = tid & 15;   // references 4tx .. 4tx+3
    const int q0 = blockIdx.x * QT;

    float bd[KK];
    int bi[KK];
#pragma unroll
    for (int p = 0; p < KK; ++p) {
        bd[p] = FLT_MAX;
        bi[p] = -1;
    }
    float qn[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = q0 + 4 * ty + i;
        qn[i] = q < n ? norms[q] : 0.f;
    }

    for (int r0 = 0; r0 < n; r0 += RT) {
        float acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;

        for (int d0 = 0; d0 < d; d0 += DC) {
            for (int e = tid; e < QT * DC; e += 256) {
                const int r = e / DC, dd = e % DC;
                const int gq = q0 + r, gr = r0 + r, gd = d0 + dd;
                qs[dd][r] = (gq < n && gd < d) ? X[(size_t)gq * d + gd] : 0.f;
                rs[dd][r] = (gr < n && gd < d) ? X[(size_t)gr * d + gd] : 0.f;
            }
            __syncthreads();
#pragma unroll 8
            for (int dd = 0; dd < DC; ++dd) {
                const float4 a = *reinterpret_cast<const float4*>(&qs[dd][4 * ty]);
                const float4 b = *reinterpret_cast<const float4*>(&rs[dd][4 * tx]);
                const float av[4] = {a.x, a.y, a.z, a.w};
                const float bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gr = r0 + 4 * tx + j;
            const float rn = gr < n ? norms[gr] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int gq = q0 + 4 * ty + i;
                float dist = qn[i] + rn - 2.f * acc[i][j];
                if (gr >= n || gr == gq) dist = FLT_MAX;
                dt[4 * ty + i][4 * tx + j] = dist;
            }
        }
        __syncthreads();
        if (tid < QT) {
            for (int r = 0; r < RT; ++r) {
                float cd = dt[tid][r];
                if (cd < bd[KK - 1]) {
                    int ci = r0 + r;
#pragma unroll
                    for (int p = 0; p < KK; ++p) {
                        const bool sw = cd < bd[p];
                        const float od = bd[p];
                        const int oi = bi[p];
                        bd[p] = sw ? cd : od;
                        bi[p] = sw ? ci : oi;
                        cd = sw ? od : cd;
                        ci = sw ? oi : ci;
                    }
                }
            }
        }
        __syncthreads();
    }
    if (tid < QT && q0 + tid < n) {
#pragma unroll
        for (int p = 0; p < KK; ++p) cand[(size_t)(q0 + tid) * KK + p] = bi[p];
    }
}

__global__ void row_norms_kernel(const float* X, int64_t n, int d, float* norms) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int j = 0; j < d; ++j) {
        const float x = X[i * d + j];
        s = fmaf(x, x, s);
    }
    norms[i] = s;
}

}  // namespace

void launch_knn_candidates(const float* Xc, const float* norms, int64_t n, int d, int kk, int32_t* cand,
                           hipStream_t st) {
    const int blocks = (int)((n + QT - 1) / QT);
    switch (kk) {
        case 16: hipLaunchKernelGGL(knn_tile_kernel<16>, dim3(blocks), dim3(256), 0, st, Xc, norms, (int)n, d, cand); break;
        case 24: hipLaunchKernelGGL(knn_tile_kernel<24>, dim3(blocks), dim3(256), 0, st, Xc, norms, (int)n, d, cand); break;
        case 32: hipLaunchKernelGGL(knn_tile_kernel<32>, dim3(blocks), dim3(256), 0, st, Xc, norms, (int)n, d, cand); break;
        case 40: hipLaunchKernelGGL(knn_tile_kernel<40>, dim3(blocks), dim3(256), 0, st, Xc, norms, (int)n, d, cand); break;
        default: fail(GS_ERR_INVALID, "unsupported candidate count");
    }
}

void launch_row_norms(const float* Xc, int64_t n, int d, float* norms, hipStream_t st) {
    hipLaunchKernelGGL(row_norms_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Xc, n, d, norms);
}

}  // namespace gs
