// Backward-Euler heat kernel: conjugate-gradient kernels and the scaling
// epilogue used after a kernel application that is not a Chebyshev sum.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace gs {

namespace {

constexpr int kBlock = 256;

int grid_for(int64_t count) {
    int64_t g = (count + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// ------------------------------------------------------------------ backward-Euler kernel (CG)
// Conjugate gradients on (I + c L) x = b for every column at once, node-major
// n x ldp.  The product is one first-step launch of the step kernel with the
// operator scale -c, which yields qn = -(I + c L) p; the per-column scalars
// rr = r.r and pqn = p.qn are float64 device values from the column reduction,
// so no iteration waits on the host.  A column whose rr or pqn is zero (a
// zero right-hand side, padding) keeps alpha = beta = 0.

// r = b, p = b, x = 0 (x may alias b: each element is read before it is written).
__global__ void cg_init_kernel(const float* b, float* x, float* r, float* p, int64_t total) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const float v = b[e];
        r[e] = v;
        p[e] = v;
        x[e] = 0.f;
    }
}

// Column passes over the n x ldp arrays: a block owns rows_per_blk rows and
// up to 256 groups of VEC columns; RL = 256 / groups lanes walk the rows with
// four loads in flight, then the block sums its lanes through LDS into
// partials[block][column] (fixed order: results do not depend on timing).
//   CG_DOT:    partial of sum_i a[i, c] b[i, c]
//   CG_UPDATE: alpha_c = rr_c / (-pqn_c); x += alpha a; r += alpha b (a = p,
//              b = qn = -A p); partial of sum_i r_new[i, c]^2
enum CgPass { CG_DOT = 0, CG_UPDATE = 1 };

template <int VEC, int PASS>
__global__ __launch_bounds__(kBlock) void cg_pass_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                         float* __restrict__ x, float* __restrict__ r,
                                                         const double* rr, const double* pqn, int64_t n, int ldp,
                                                         int64_t rows_per_blk, double* partials) {
    __shared__ double sh[kBlock * VEC];
    const int ng = ldp / VEC;
    const int cw = ng < kBlock ? ng : kBlock;
    const int nrl = kBlock / cw;
    const int tid = threadIdx.x;
    const int g = blockIdx.y * cw + tid % cw;
    const int rl = tid / cw;
    const bool active = rl < nrl && g < ng;
    double acc[VEC];
    float alpha[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        acc[v] = 0.0;
        alpha[v] = 0.f;
        if (PASS == CG_UPDATE && active) {
            const int c = g * VEC + v;
            const double den = -pqn[c];
            alpha[v] = (rr[c] > 0.0 && den > 0.0) ? (float)(rr[c] / den) : 0.f;
        }
    }
    const int64_t r0 = blockIdx.x * rows_per_blk;
    const int64_t r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
    if (active) {
#pragma unroll 4
        for (int64_t i = r0 + rl; i < r1; i += nrl) {
            const size_t e = (size_t)i * ldp + (size_t)g * VEC;
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const float av = a[e + v], bv = b[e + v];
                if (PASS == CG_DOT) {
                    acc[v] += (double)av * (double)bv;
                } else {
                    x[e + v] = fmaf(alpha[v], av, x[e + v]);
                    const float rn = fmaf(alpha[v], bv, r[e + v]);
                    r[e + v] = rn;
                    acc[v] += (double)rn * (double)rn;
                }
            }
        }
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) sh[tid * VEC + v] = acc[v];
    __syncthreads();
    if (tid < cw && g < ng) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            double s = 0.0;
            for (int j = 0; j < nrl; ++j) s += sh[(tid + j * cw) * VEC + v];
            partials[(size_t)blockIdx.x * ldp + g * VEC + v] = s;
        }
    }
}

// out[c] = sum_b partials[b][c]: one block per column, a fixed-order tree sum.
__global__ __launch_bounds__(kBlock) void cg_final_kernel(const double* partials, int nblk, int ldp, double* out) {
    __shared__ double sh[kBlock];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) s += partials[(size_t)b * ldp + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
}

// beta = rr_new / rr_old; p = r + beta p.
__global__ void cg_dir_kernel(const float* r, float* p, const double* rr_old, const double* rr_new, int64_t total,
                              int ldp) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % ldp);
        const float beta = rr_old[c] > 0.0 ? (float)(rr_new[c] / rr_old[c]) : 0.f;
        p[e] = fmaf(beta, p[e], r[e]);
    }
}

// Algorithm 1's scaling after a kernel application held in acc, with the
// step epilogue's floor rule: d = acc if acc > phi else phi, out = num / d,
// out_a = a out, rec = d; floors counted where num > 0 when nfloor is given
// (one atomic per wave; the grid is capped so a thread walks several elements).
__global__ __launch_bounds__(kBlock) void scale_epilogue_kernel(const float* acc, const float* num, float* out,
                                                                float* out_a, const float* a, float* rec, float phi,
                                                                unsigned long long* nfloor, int64_t n, int ldp) {
    const int64_t total = n * (int64_t)ldp;
    unsigned cnt = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const float r = acc[e];
        const bool ok = r > phi;
        const float d = ok ? r : phi;
        const float nm = num[e];
        const float o = nm / d;
        out[e] = o;
        if (out_a) out_a[e] = a[e / ldp] * o;
        if (rec) rec[e] = d;
        cnt += (!ok && nm > 0.f) ? 1u : 0u;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (nfloor && (threadIdx.x & 63) == 0 && cnt) atomicAdd(nfloor, (unsigned long long)cnt);
}


}  // namespace

void launch_cg_init(const float* b, float* x, float* r, float* p, int64_t total, hipStream_t st) {
    hipLaunchKernelGGL(cg_init_kernel, dim3(grid_for(total)), dim3(kBlock), 0, st, b, x, r, p, total);
}

int cg_blocks(int64_t n) {
    int64_t nb = (n + 127) / 128;
    if (nb > kMaxCgBlocks) nb = kMaxCgBlocks;
    return nb < 1 ? 1 : (int)nb;
}

namespace {

template <int PASS>
void launch_cg_pass(const float* a, const float* b, float* x, float* r, const double* rr, const double* pqn,
                    int64_t n, int ldp, double* partials, double* out, hipStream_t st) {
    const int nblk = cg_blocks(n);
    const int64_t rows = (n + nblk - 1) / nblk;
    const int vec = (ldp % 4 == 0) ? 4 : 1;
    const int ng = ldp / vec;
    const int cw = ng < kBlock ? ng : kBlock;
    const dim3 grid(nblk, (ng + cw - 1) / cw);
    if (vec == 4)
        hipLaunchKernelGGL((cg_pass_kernel<4, PASS>), grid, dim3(kBlock), 0, st, a, b, x, r, rr, pqn, n, ldp, rows,
                           partials);
    else
        hipLaunchKernelGGL((cg_pass_kernel<1, PASS>), grid, dim3(kBlock), 0, st, a, b, x, r, rr, pqn, n, ldp, rows,
                           partials);
    hipLaunchKernelGGL(cg_final_kernel, dim3(ldp), dim3(kBlock), 0, st, partials, nblk, ldp, out);
}

}  // namespace

void launch_cg_dot(const float* a, const float* b, int64_t n, int ldp, double* partials, double* out,
                   hipStream_t st) {
    launch_cg_pass<CG_DOT>(a, b, nullptr, nullptr, nullptr, nullptr, n, ldp, partials, out, st);
}

void launch_cg_update(float* x, float* r, const float* p, const float* qn, const double* rr, const double* pqn,
                      int64_t n, int ldp, double* partials, double* rr_new, hipStream_t st) {
    launch_cg_pass<CG_UPDATE>(p, qn, x, r, rr, pqn, n, ldp, partials, rr_new, st);
}

void launch_cg_dir(const float* r, float* p, const double* rr_old, const double* rr_new, int64_t total, int ldp,
                   hipStream_t st) {
    hipLaunchKernelGGL(cg_dir_kernel, dim3(grid_for(total)), dim3(kBlock), 0, st, r, p, rr_old, rr_new, total, ldp);
}

void launch_scale_epilogue(const float* acc, const float* num, float* out, float* out_a, const float* a, float* rec,
                           float phi, unsigned long long* nfloor, int64_t n, int ldp, hipStream_t st) {
    const int grid = grid_for(n * (int64_t)ldp) < 1024 ? grid_for(n * (int64_t)ldp) : 1024;
    hipLaunchKernelGGL(scale_epilogue_kernel, dim3(grid), dim3(kBlock), 0, st, acc, num, out, out_a, a, rec, phi,
                       nfloor, n, ldp);
}

}  // namespace gs
