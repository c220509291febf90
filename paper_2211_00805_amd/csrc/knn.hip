// Candidate nearest neighbours for the common affinity graph (setup, not on
// the timed path).  Brute force over all pairs: squared distances
// |q|^2 + |r|^2 - 2 q.r from float32 Gram tiles computed on the matrix cores
// (the one dense contraction of the library), then each query keeps its KK
// best candidates in a sorted register list.  The host re-ranks the
// candidates in float64 by exact squared distance, so float32 rounding only
// has to keep the true k nearest inside the KK = k + 8 candidates.
#include <cfloat>

#include "internal.h"

namespace gs {
namespace {

// Block tile: T = 128 queries x T references; each of the 4 waves owns a
// 64 x 64 sub-tile as four 32 x 32 accumulators of v_mfma_f32_32x32x2f32
// (float32 products, float32 sums).  Operand layout of that instruction:
// lanes 0-31 carry k = 0 and lanes 32-63 k = 1 of A (row = lane % 32) and B
// (column = lane % 32); accumulator element i of lane l is
// C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].  Coordinates are staged DC at a
// time in LDS (odd row stride: the 32 rows a half-wave reads fall in distinct
// banks); after the coordinate loop the dot products go to an LDS tile that
// reuses the staging space; all threads mark, per query, the references that
// beat its current KK-th best distance (a 128-bit mask per query), and one
// thread per query inserts only those, in increasing order (the same result
// as a serial scan of the tile), into its sorted register list of the KK best
// (distance |q|^2 + |r|^2 - 2 q.r).
constexpr int T = 128;
constexpr int DC = 32;
constexpr int LDQ = DC + 1;
constexpr int LDD = T + 1;
static_assert(2 * T * LDQ <= T * LDD, "staging fits in the distance tile");

typedef float v16f __attribute__((ext_vector_type(16)));

template <int KK>
__global__ __launch_bounds__(256) void knn_mfma_kernel(const float* __restrict__ X, const float* __restrict__ norms,
                                                       int n, int d, int32_t* __restrict__ cand) {
    __shared__ float smem[T * LDD];   // {Q chunk, R chunk} while staging, then the dot-product tile
    __shared__ float rn_s[T];
    __shared__ float thr[T];                      // each query's current KK-th best distance
    __shared__ unsigned long long mask[T][2];     // references of the tile below that threshold
    float* qs = smem;
    float* rs = smem + T * LDQ;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int q0 = blockIdx.x * T;
    const bool vec4 = (d & 3) == 0;

    float bd[KK];
    int bi[KK];
#pragma unroll
    for (int p = 0; p < KK; ++p) {
        bd[p] = FLT_MAX;
        bi[p] = -1;
    }
    const float qn = (tid < T && q0 + tid < n) ? norms[q0 + tid] : 0.f;
    if (tid < T) thr[tid] = FLT_MAX;
    // prefilter roles: query fq, references fh*64 .. fh*64+63 of each tile
    const int fq = tid & (T - 1), fh = tid >> 7;
    const float fqn = q0 + fq < n ? norms[q0 + fq] : 0.f;

    for (int r0 = 0; r0 < n; r0 += T) {
        v16f acc00 = {0}, acc01 = {0}, acc10 = {0}, acc11 = {0};
        for (int d0 = 0; d0 < d; d0 += DC) {
            __syncthreads();   // the previous tile's readers of smem are done
            if (vec4) {
                for (int e = tid; e < T * (DC / 4); e += 256) {
                    const int r = e / (DC / 4), c = (e % (DC / 4)) * 4, gd = d0 + c;
                    const int gq = q0 + r, gr = r0 + r;
                    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
                    if (gq < n && gd < d) a = *reinterpret_cast<const float4*>(X + (size_t)gq * d + gd);
                    if (gr < n && gd < d) b = *reinterpret_cast<const float4*>(X + (size_t)gr * d + gd);
                    float* qd = qs + r * LDQ + c;
                    float* rd = rs + r * LDQ + c;
                    qd[0] = a.x; qd[1] = a.y; qd[2] = a.z; qd[3] = a.w;
                    rd[0] = b.x; rd[1] = b.y; rd[2] = b.z; rd[3] = b.w;
                }
            } else {
                for (int e = tid; e < T * DC; e += 256) {
                    const int r = e / DC, c = e % DC, gd = d0 + c;
                    const int gq = q0 + r, gr = r0 + r;
                    qs[r * LDQ + c] = (gq < n && gd < d) ? X[(size_t)gq * d + gd] : 0.f;
                    rs[r * LDQ + c] = (gr < n && gd < d) ? X[(size_t)gr * d + gd] : 0.f;
                }
            }
            __syncthreads();
            const int arow = (wm * 64 + (lane & 31)) * LDQ + (lane >> 5);
            const int brow = (wn * 64 + (lane & 31)) * LDQ + (lane >> 5);
            // the chunk's real width rounded up to even (staged zeros beyond d)
            const int kend = d - d0 < DC ? ((d - d0) + 1) & ~1 : DC;
#pragma unroll 4
            for (int k = 0; k < kend; k += 2) {
                const float a0 = qs[arow + k], a1 = qs[arow + 32 * LDQ + k];
                const float b0 = rs[brow + k], b1 = rs[brow + 32 * LDQ + k];
                acc00 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc00, 0, 0, 0);
                acc01 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc01, 0, 0, 0);
                acc10 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc10, 0, 0, 0);
                acc11 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc11, 0, 0, 0);
            }
        }
        __syncthreads();   // staging space becomes the dot-product tile
        {
            const int mb = wm * 64 + 4 * (lane >> 5), nb = wn * 64 + (lane & 31);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int m = mb + 8 * (v / 4) + (v % 4);
                smem[m * LDD + nb] = acc00[v];
                smem[m * LDD + nb + 32] = acc01[v];
                smem[(m + 32) * LDD + nb] = acc10[v];
                smem[(m + 32) * LDD + nb + 32] = acc11[v];
            }
        }
        if (tid < T) rn_s[tid] = r0 + tid < n ? norms[r0 + tid] : 0.f;
        __syncthreads();
        {
            // all threads: mark the references that beat the query's threshold
            const int rmax = n - r0 < T ? n - r0 : T;
            const float th = thr[fq];
            unsigned long long mk = 0;
            for (int j = 0; j < 64; ++j) {
                const int r = fh * 64 + j;
                const float cd = fqn + rn_s[r] - 2.f * smem[fq * LDD + r];
                if (r < rmax && r0 + r != q0 + fq && cd < th) mk |= 1ull << j;
            }
            mask[fq][fh] = mk;
        }
        __syncthreads();
        if (tid < T) {
            const int gq = q0 + tid;
            for (int h = 0; h < 2; ++h) {
                unsigned long long mk = mask[tid][h];
                while (mk) {
                    const int j = __ffsll((long long)mk) - 1;
                    mk &= mk - 1;
                    const int r = h * 64 + j;
                    float cd = qn + rn_s[r] - 2.f * smem[tid * LDD + r];
                    if (r0 + r == gq) cd = FLT_MAX;
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
            thr[tid] = bd[KK - 1];
        }
    }
    if (tid < T && q0 + tid < n) {
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
    const int blocks = (int)((n + T - 1) / T);
    switch (kk) {
        case 16: hipLaunchKernelGGL(knn_mfma_kernel<16>, dim3(blocks), dim3(256), 0, st, Xc, norms, (int)n, d, cand); break;
        case 24: hipLaunchKernelGGL(knn_mfma_kernel<24>, dim3(blocks), dim3(256), 0, st, Xc, norms, (int)n, d, cand); break;
        case 32: hipLaunchKernelGGL(knn_mfma_kernel<32>, dim3(blocks), dim3(256), 0, st, Xc, norms, (int)n, d, cand); break;
        case 40: hipLaunchKernelGGL(knn_mfma_kernel<40>, dim3(blocks), dim3(256), 0, st, Xc, norms, (int)n, d, cand); break;
        default: fail(GS_ERR_INVALID, "unsupported candidate count");
    }
}

void launch_row_norms(const float* Xc, int64_t n, int d, float* norms, hipStream_t st) {
    hipLaunchKernelGGL(row_norms_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Xc, n, d, norms);
}

}  // namespace gs
