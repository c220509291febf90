// Device kernels of the Geodesic Sinkhorn hot path (gfx950, wave64).
//
// K1  cheb_step:   one Chebyshev step of p_K(L,t) X on n x B node-major signals,
//                  T_k = 2 y T_{k-1} - T_{k-2}, acc += b_k T_k (Sec. "Chebyshev
//                  Polynomials"), with y = (2/lambda_hat) L - I and
//                  (L x)_i = sum_j A_ij (x_i - x_j) (Sec. "Heat Diffusion on a
//                  Graph").  The sparse product, the three-term update and the
//                  coefficient accumulate are one pass over HBM.
// K2  epilogue of the last step: Algorithm 1's scaling out = num / floor(acc),
//                  out_a = a * out (the next application's input), floors counted.
// K3  colreduce:   per-column float64 reductions (distance, marginal error, dots)
//                  in two deterministic passes, no floating-point atomics.
// K4  bary_row:    barycenter update p = exp(sum alpha ln q), w = p / q.
// K5  bwd_*:       elementwise adjoints of Algorithm 1's updates.
//
// The step kernel is bound by its gathers (one row of T_{k-1} per nonzero);
// its launch shape (lanes splitting a row's nonzeros S, lanes across column
// groups C, float or float4 lanes) is a template parameter chosen per plan,
// lanes past a padded row stay idle, rows with very many nonzeros are taken
// by the first blocks of the same grid (one block per row), and the 1-D grid
// can be remapped (an autotuned choice) so that each of the 8 XCDs, which
// receive blocks round-robin, walks a contiguous range of rows.
#include <cfloat>
#include <cmath>

#include "internal.h"

namespace gs {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int xcd_remap(int b, int nb) {
    constexpr int nx = 8;
    const int q = nb / nx, r = nb % nx;
    const int x = b % nx, i = b / nx;
    return x * q + (x < r ? x : r) + i;
}

template <int VEC>
struct Vec {
    float v[VEC];
};

template <int VEC>
__device__ __forceinline__ Vec<VEC> vload(const float* p) {
    Vec<VEC> r;
    if constexpr (VEC == 4) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
    } else {
        r.v[0] = *p;
    }
    return r;
}

template <int VEC>
__device__ __forceinline__ void vstore(float* p, const Vec<VEC>& r) {
    if constexpr (VEC == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
    } else {
        *p = r.v[0];
    }
}

template <int VEC>
__device__ __forceinline__ Vec<VEC> vzero() {
    Vec<VEC> r;
#pragma unroll
    for (int i = 0; i < VEC; ++i) r.v[i] = 0.f;
    return r;
}

// Single-use streams (CSR pairs, T_{k-2}, accumulators, numerators) are read
// and written with non-temporal hints so they do not evict the gathered
// operand's rows from L2.
typedef float v4f __attribute__((ext_vector_type(4)));

template <int VEC>
__device__ __forceinline__ Vec<VEC> vload_nt(const float* p) {
    Vec<VEC> r;
    if constexpr (VEC == 4) {
        const v4f t = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
        r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
    } else {
        r.v[0] = __builtin_nontemporal_load(p);
    }
    return r;
}

template <int VEC>
__device__ __forceinline__ void vstore_nt(float* p, const Vec<VEC>& r) {
    if constexpr (VEC == 4) {
        v4f t = {r.v[0], r.v[1], r.v[2], r.v[3]};
        __builtin_nontemporal_store(t, reinterpret_cast<v4f*>(p));
    } else {
        __builtin_nontemporal_store(r.v[0], p);
    }
}

// sum += w * (own - x)
template <int VEC>
__device__ __forceinline__ void vacc(Vec<VEC>& sum, float w, const Vec<VEC>& own, const Vec<VEC>& x) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) sum.v[i] = fmaf(w, own.v[i] - x.v[i], sum.v[i]);
}

// ------------------------------------------------------------------ K1 + K2
// One block owns RPB consecutive rows and one column tile.  Its CSR range is
// staged through LDS with coalesced loads; every row's own T_{k-1}, T_{k-2}
// and accumulator loads are issued before the gathers, and the gathers are
// issued kUnroll at a time (branch-free: padding entries re-read the row's
// own value with weight 0), so each row costs three dependent memory round
// trips.  (L x)_i = d_i x_i - sum_j A_ij x_j with d_i = sum_j A_ij formed in
// the same loop.  The accumulator is touched only on flush steps (every third
// step and the last), each adding up to three terms b_{k-2} T_{k-2},
// b_{k-1} T_{k-1}, b_k T_k that the step already holds.
//
// MODE selects the accumulating form, the adjoint form with a second
// accumulator, or Clenshaw's recurrence (each its own symbol, so profiles
// separate them).
constexpr int kChunk = 2048;   // staged (col, weight) pairs per block and pass
// Gathers in flight per lane: 5 is the deepest unroll whose registers fit in
// 64 VGPRs, i.e. 8 waves per SIMD; measured on the 1M-node graph at B = 32,
// 8 in flight at 6 waves/SIMD was 10% slower, 4 or 3 at 8 waves 3% and 8%.
constexpr int kUnroll = 5;

__device__ __forceinline__ float coef_at(const float* b, int idx) { return idx == 0 ? 0.5f * b[0] : b[idx]; }

// Step forms: the accumulating recurrence, its adjoint form with a second
// accumulator, and Clenshaw's backward recurrence (no accumulator).
constexpr int kModeFwd = 0, kModeDual = 1, kModeClen = 2;

// Step epilogue for one row and one group of VEC columns: the three-term
// update, the accumulator flush and (last step) Algorithm 1's scaling.
//
// Clenshaw form (MODE == kModeClen), product j = A.k of K for
// p_K X = b_0/2 X + sum_k b_k T_k(y) X: with u_{K+1} = u_{K+2} = 0,
// u_k = 2 y u_{k+1} - u_{k+2} + b_k X (k = K-1..1) and the result
// y u_1 - u_2 + (b_0/2) X.  Product j gathers G = u_{K-j+1} (X standing
// for u_K = b_K X when j = 1) and writes u_{K-j}, or the result when j = K:
//   out = c_y (y G) - [u_{K-j+2}, read when j >= 3] + c_x X,
//   c_y = (j < K ? 2 : 1) * (j == 1 ? b_K : 1),  c_x = b_{K-j} (b_0 halved)
//   minus b_K when j == 2 (u_K = b_K X folded in).
template <int VEC, int MODE>
__device__ __forceinline__ void step_epilogue(const StepArgs& A, int row, size_t off, const Vec<VEC>& own,
                                              const Vec<VEC>& p2, const Vec<VEC>& ac, const Vec<VEC>& ac2,
                                              const Vec<VEC>& sx, float sw) {
    const int flags = A.flags;
    const int k = A.k;
    const float alpha = A.coef[0];
    const float* b = A.coef + 1;
    Vec<VEC> t, accn, acc2n;
    if constexpr (MODE == kModeClen) {
        const int K = A.K;
        const float cy = (k < K ? 2.f : 1.f) * (k == 1 ? b[K] : 1.f);
        const float cx = coef_at(b, K - k) - (k == 2 ? b[K] : 0.f);
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            const float yx = fmaf(alpha, fmaf(sw, own.v[i], -sx.v[i]), -own.v[i]);   // (y G)_i
            // ac holds X; adding +0 turns a -0 into +0 and changes no other value, so
            // rows beyond the frontier hold +0 here as in the accumulating forms
            t.v[i] = fmaf(cy, yx, fmaf(cx, ac.v[i], -p2.v[i])) + 0.f;
            accn.v[i] = t.v[i];
        }
    } else {
        const float* db = A.coef + 2 + A.K;
        const int m = A.cmask;
        const float c2 = (m & 1) ? coef_at(b, k - 2) : 0.f;
        const float c1 = (m & 2) ? coef_at(b, k - 1) : 0.f;
        const float c0 = (m & 4) ? coef_at(b, k) : 0.f;
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            const float yx = fmaf(alpha, fmaf(sw, own.v[i], -sx.v[i]), -own.v[i]);   // (y T_{k-1})_i
            t.v[i] = (flags & STEP_FIRST) ? yx : fmaf(2.f, yx, -p2.v[i]);
            accn.v[i] = fmaf(c0, t.v[i], fmaf(c1, own.v[i], fmaf(c2, p2.v[i], ac.v[i])));
        }
        if constexpr (MODE == kModeDual) {
            const float d2 = (m & 1) ? coef_at(db, k - 2) : 0.f;
            const float d1 = (m & 2) ? coef_at(db, k - 1) : 0.f;
            const float d0 = (m & 4) ? coef_at(db, k) : 0.f;
#pragma unroll
            for (int i = 0; i < VEC; ++i)
                acc2n.v[i] = fmaf(d0, t.v[i], fmaf(d1, own.v[i], fmaf(d2, p2.v[i], ac2.v[i])));
        }
    }
    if (flags & STEP_WRITE_T) vstore<VEC>(A.tout + off, t);
    if (flags & STEP_EPI_SCALE) {
        const Vec<VEC> nm = vload_nt<VEC>(A.num + off);
        const float ai = A.a ? A.a[row] : 1.f;
        const float phi = A.phi;
        Vec<VEC> dd, o, oa;
        bool fl[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            const float r = accn.v[i];
            const bool ok = r > phi;
            dd.v[i] = ok ? r : phi;
            o.v[i] = nm.v[i] / dd.v[i];
            oa.v[i] = ai * o.v[i];
            fl[i] = !ok && nm.v[i] > 0.f;
        }
        vstore<VEC>(A.out + off, o);
        if (A.out_a) vstore<VEC>(A.out_a + off, oa);
        if (A.rec) vstore<VEC>(A.rec + off, dd);
        if (A.nfloor) {
            // floors on the numerator's support, one atomic per wave (the
            // lanes here can be any subset of the wave: ballots count them)
            unsigned long long cnt = 0;
#pragma unroll
            for (int i = 0; i < VEC; ++i) cnt += __popcll(__ballot(fl[i]));
            const int leader = __ffsll((long long)__ballot(1)) - 1;
            if (cnt && (int)(threadIdx.x & 63) == leader) atomicAdd(A.nfloor, cnt);
        }
    } else if (flags & STEP_ACC_WRITE) {
        vstore_nt<VEC>(A.acc + off, accn);
        if constexpr (MODE == kModeDual) vstore_nt<VEC>(A.acc2 + off, acc2n);
    }
}

template <int VEC, int MODE>
__device__ __forceinline__ void load_row_operands(const StepArgs& A, size_t off, Vec<VEC>& own, Vec<VEC>& p2,
                                                  Vec<VEC>& ac, Vec<VEC>& ac2) {
    own = vload<VEC>(A.tprev + off);
    if constexpr (MODE == kModeClen) {
        if (A.flags & STEP_CLEN_P2) p2 = vload_nt<VEC>(A.tprev2 + off);
        ac = vload_nt<VEC>(A.xin + off);
        return;
    }
    if (!(A.flags & STEP_FIRST)) p2 = vload_nt<VEC>(A.tprev2 + off);
    if (A.flags & STEP_ACC_READ) {
        ac = vload_nt<VEC>(A.acc + off);
        if constexpr (MODE == kModeDual) ac2 = vload_nt<VEC>(A.acc2 + off);
    }
}

// Frontier rows (level above the step index) have all-zero operands: they
// skip their gathers, whole blocks of them their CSR, and they still load
// their own operands (issued before any row level is known, which keeps the
// level loads off the blocks' critical path).  The epilogue then computes
// from the same operands as the dense kernel with zero neighbour sums, which
// gives the dense kernel's bits, signs of zeros included.  Those bits are
// +0 for T_k (u_k in Clenshaw's form, whose update adds +0 to turn -0 into
// +0) and the accumulator, so when the application has zeroed its buffers
// beforehand (A.skip_dead, never on the last step, whose epilogue writes
// every row) a whole block beyond the frontier returns before loading
// anything.

// Rows with more than A.long_thr nonzeros: one block per row and column tile,
// 256/C lanes splitting the nonzeros, a block reduction through LDS.  FR: the
// frontier form (A.level set).
template <int VEC, int C, int MODE, bool FR>
__device__ __forceinline__ void long_row_block(const StepArgs& A, int item, int ncoltiles, float* red_lds) {
    constexpr int SL = kBlock / C;   // lanes over the nonzeros
    float (*red)[C][VEC + 1] = reinterpret_cast<float (*)[C][VEC + 1]>(red_lds);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int s = tid / C;
    const int c = tid - s * C;
    const int li = item / ncoltiles;
    const int row = A.long_rows[li];
    const int colofs = (item - li * ncoltiles) * (VEC * C) + c * VEC;
    const bool colok = colofs < A.ldp;   // lanes past the padded row stay idle
    const size_t off = (size_t)row * A.ldp + (colok ? colofs : 0);
    Vec<VEC> own = vzero<VEC>(), p2 = vzero<VEC>(), ac = vzero<VEC>(), ac2 = vzero<VEC>();
    if (s == 0 && colok) load_row_operands<VEC, MODE>(A, off, own, p2, ac, ac2);
    const bool dead = FR && A.level[row] > (uint32_t)A.k;   // block-uniform
    if (FR && A.skip_dead && dead) return;
    const int rs = A.rowptr[row], re = (colok && !dead) ? A.rowptr[row + 1] : rs;
    const float* __restrict__ xcol = A.tprev + colofs;
    Vec<VEC> sx = vzero<VEC>();
    float sw = 0.f;
    for (int e = rs + s; e < re; e += kUnroll * SL) {
        Vec<VEC> xv[kUnroll];
        float w[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int eu = e + u * SL;
            const bool ok = eu < re;
            const int j = ok ? (A.csr_nt ? __builtin_nontemporal_load(A.col + eu) : A.col[eu]) : row;
            w[u] = ok ? (A.csr_nt ? __builtin_nontemporal_load(A.val + eu) : A.val[eu]) : 0.f;
            xv[u] = vload<VEC>(xcol + (size_t)j * A.ldp);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            sw += w[u];
#pragma unroll
            for (int i = 0; i < VEC; ++i) sx.v[i] = fmaf(w[u], xv[u].v[i], sx.v[i]);
        }
    }
#pragma unroll
    for (int o = C; o < 64; o <<= 1) {
        sw += __shfl_xor(sw, o, 64);
#pragma unroll
        for (int i = 0; i < VEC; ++i) sx.v[i] += __shfl_xor(sx.v[i], o, 64);
    }
    if (lane < C) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) red[wave][c][i] = sx.v[i];
        red[wave][c][VEC] = sw;
    }
    __syncthreads();
    if (tid < C && colok) {
#pragma unroll
        for (int wv = 1; wv < 4; ++wv) {
#pragma unroll
            for (int i = 0; i < VEC; ++i) sx.v[i] += red[wv][c][i];
            sw += red[wv][c][VEC];
        }
        step_epilogue<VEC, MODE>(A, row, off, own, p2, ac, ac2, sx, sw);
    }
}

template <int VEC, int S, int C, int MODE, bool FR>
__global__ __launch_bounds__(kBlock) void cheb_step_kernel(StepArgs A) {
    constexpr int LPR = S * C;       // lanes per row
    constexpr int RPW = 64 / LPR;    // rows per wave
    constexpr int RPB = 4 * RPW;     // rows per block
    __shared__ int2 stage[kChunk];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ldp = A.ldp;
    const int ncoltiles = (ldp + VEC * C - 1) / (VEC * C);
    // the first blocks take the long rows (dispatched first, they overlap the tiles)
    const int nlb = A.nlong * ncoltiles;
    if ((int)blockIdx.x < nlb) {
        long_row_block<VEC, C, MODE, FR>(A, blockIdx.x, ncoltiles, reinterpret_cast<float*>(stage));
        return;
    }
    const int bt = (int)blockIdx.x - nlb;
    const int L = A.remap ? xcd_remap(bt, (int)gridDim.x - nlb) : bt;
    const int rt = L / ncoltiles;
    const int ct = L - rt * ncoltiles;
    if constexpr (FR) {
        if (A.skip_dead && A.blk_level[rt] > (uint32_t)A.k) return;   // zeros already in place
    }
    const int lr = lane % LPR;
    const int s = lr / C;
    const int c = lr - s * C;
    const int r0 = rt * RPB;
    const int r1 = r0 + RPB < A.n ? r0 + RPB : A.n;
    const int row = r0 + wave * RPW + lane / LPR;
    const int colofs = ct * (VEC * C) + c * VEC;
    // lanes past the last row or the padded row stay idle but join the shuffles
    const bool valid = row < A.n && colofs < ldp;
    const size_t off = (size_t)(valid ? row : r0) * ldp + (colofs < ldp ? colofs : 0);

    const int eb = A.rowptr[r0];
    int ee = A.rowptr[r1];
    // frontier: the block's and the row's levels load beside the row
    // pointers and are consulted only once every load is issued
    const uint32_t blv = FR ? A.blk_level[rt] : 0u;
    int rs = 0, re = 0;
    uint32_t lv = 0u;   // first used after the CSR loads are issued
    Vec<VEC> own = vzero<VEC>(), p2 = vzero<VEC>(), ac = vzero<VEC>(), ac2 = vzero<VEC>();
    bool longrow = false;
    if (valid) {
        if (FR) lv = A.level[row];
        rs = A.rowptr[row];
        re = A.rowptr[row + 1];
        longrow = A.long_thr > 0 && re - rs > A.long_thr;
        if (longrow) {
            re = rs;   // taken by a long-row block at the head of the grid
        } else {
            load_row_operands<VEC, MODE>(A, off, own, p2, ac, ac2);
        }
    }
    if (FR && blv > (uint32_t)A.k) ee = eb;   // a block beyond step k's reach reads no CSR

    Vec<VEC> sx = vzero<VEC>();
    float sw = 0.f;
    const float* __restrict__ xrow = A.tprev + (colofs < ldp ? colofs : 0);
    const int self = valid ? row : r0;
    for (int cb = eb; cb < ee; cb += kChunk) {
        const int cend = cb + kChunk < ee ? cb + kChunk : ee;
        if (A.csr_nt) {   // streamed CSR: keep L2 for the gathered rows
            for (int e = cb + (int)threadIdx.x; e < cend; e += kBlock)
                stage[e - cb] = make_int2(__builtin_nontemporal_load(A.col + e),
                                          __float_as_int(__builtin_nontemporal_load(A.val + e)));
        } else {          // a CSR that fits the caches stays there across steps
            for (int e = cb + (int)threadIdx.x; e < cend; e += kBlock)
                stage[e - cb] = make_int2(A.col[e], __float_as_int(A.val[e]));
        }
        __syncthreads();
        const int lo = rs > cb ? rs : cb;
        const int hi = re < cend ? re : cend;
        // the level is read here, past the barrier: an empty asm keeps the
        // compiler from hoisting the comparisons (and the wait for the level
        // load) above the CSR loads
        uint32_t lvk = lv;
        if constexpr (FR) asm volatile("" : "+v"(lvk));
        if (valid && lo < hi && (!FR || lvk <= (uint32_t)A.k)) {
            // first e >= lo with (e - rs) % S == s
            const int e0 = lo + (((s - (lo - rs)) % S) + S) % S;
            for (int e = e0; e < hi; e += kUnroll * S) {
                Vec<VEC> x[kUnroll];
                float w[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int eu = e + u * S;
                    const bool ok = eu < hi;
                    const int2 pr = stage[ok ? eu - cb : 0];
                    const int j = ok ? pr.x : self;
                    w[u] = ok ? __int_as_float(pr.y) : 0.f;
                    x[u] = vload<VEC>(xrow + (size_t)j * ldp);
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    sw += w[u];
#pragma unroll
                    for (int i = 0; i < VEC; ++i) sx.v[i] = fmaf(w[u], x[u].v[i], sx.v[i]);
                }
            }
        }
        __syncthreads();
    }
    // combine the S partial sums of a row (lanes lr, lr ^ C, lr ^ 2C, ...)
#pragma unroll
    for (int o = C; o < LPR; o <<= 1) {
        sw += __shfl_xor(sw, o, 64);
#pragma unroll
        for (int i = 0; i < VEC; ++i) sx.v[i] += __shfl_xor(sx.v[i], o, 64);
    }
    if (!valid || s != 0 || longrow) return;
    step_epilogue<VEC, MODE>(A, row, off, own, p2, ac, ac2, sx, sw);
}

template <int VEC, int S, int C, bool FR>
void launch_mode(const StepArgs& a, int grid, hipStream_t st) {
    if (a.flags & STEP_CLENSHAW)
        hipLaunchKernelGGL((cheb_step_kernel<VEC, S, C, kModeClen, FR>), dim3(grid), dim3(kBlock), 0, st, a);
    else if (a.flags & STEP_DUAL)
        hipLaunchKernelGGL((cheb_step_kernel<VEC, S, C, kModeDual, FR>), dim3(grid), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((cheb_step_kernel<VEC, S, C, kModeFwd, FR>), dim3(grid), dim3(kBlock), 0, st, a);
}

template <int VEC, int S, int C>
void launch_shape(const StepArgs& a, hipStream_t st) {
    constexpr int RPB = 4 * (64 / (S * C));
    const int nrt = (a.n + RPB - 1) / RPB;
    const int nct = (a.ldp + VEC * C - 1) / (VEC * C);
    const int grid = nrt * nct + a.nlong * nct;
    if (a.level)
        launch_mode<VEC, S, C, true>(a, grid, st);
    else
        launch_mode<VEC, S, C, false>(a, grid, st);
}

// ------------------------------------------------------------------ small kernels
__global__ void fill_kernel(float* p, float v, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void copy_ld_kernel(const float* src, int lds, float* dst, int ldd, int64_t n, int B) {
    const int64_t total = n * (int64_t)ldd;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ldd;
        const int c = (int)(e - i * ldd);
        dst[e] = c < B ? src[i * lds + c] : 0.f;
    }
}

struct CoefPack {
    float v[2 * (GS_MAX_K + 1) + 1];
};

__global__ void set_coef_kernel(float* dcoef, CoefPack pk, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) dcoef[i] = pk.v[i];
}

// Bandwidth reference: each thread moves kCopyUnroll float4 (loads issued
// before the stores, non-temporal), block-strided so every load instruction
// is coalesced; one pass over the array (grid = n4 / (256 kCopyUnroll)).
// Measured on 1 GiB: 6.27 TB/s read + write against 5.44 TB/s for one float4
// per thread in a grid-stride loop.
constexpr int kCopyUnroll = 4;

__global__ __launch_bounds__(kBlock) void stream_copy_kernel(const float4* src, float4* dst, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * kCopyUnroll;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x * kCopyUnroll + threadIdx.x; i < n4; i += stride) {
        v4f v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const int64_t j = i + (int64_t)u * blockDim.x;
            if (j < n4) v[u] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(src) + j);
        }
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const int64_t j = i + (int64_t)u * blockDim.x;
            if (j < n4) __builtin_nontemporal_store(v[u], reinterpret_cast<v4f*>(dst) + j);
        }
    }
}

__global__ void stream_copy_tail_kernel(const float* src, float* dst, int64_t from, int64_t count) {
    const int64_t i = from + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < count) dst[i] = src[i];
}

int grid_for(int64_t count, int per_block = kBlock) {
    int64_t g = (count + per_block - 1) / per_block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// ------------------------------------------------------------------ K3
__device__ __forceinline__ double red_term(const ReduceArgs& R, int64_t i, int c) {
    const size_t e = (size_t)i * R.ldp + c;
    const double ai = R.a ? (double)R.a[i] : 1.0;
    switch (R.op) {
        case RED_DIST: {
            double s = 0.0;
            const double mu = R.x0[e], nu = R.x2[e];
            if (mu > 0.0) s += mu * log((double)R.x1[e]);
            if (nu > 0.0) s += nu * log((double)R.x3[e]);
            return ai * s;
        }
        case RED_MARG: {
            const double v = R.x0[e], r = R.x1[e], mu = R.x2[e];
            return fabs(ai * v * r - ai * mu);
        }
        case RED_DOT: {
            const double y = R.x1 ? (double)R.x1[e] : 1.0;
            return ai * (double)R.x0[e] * y;
        }
        default: {  // RED_DOT_QUOT
            return ai * (double)R.x0[e] * ((double)R.x1[e] / (double)R.x2[e]);
        }
    }
}

__global__ __launch_bounds__(kBlock) void colreduce_kernel(ReduceArgs R, double* partials, int64_t rows_per_blk) {
    __shared__ double sh[kBlock];
    const int CW = R.B < kBlock ? R.B : kBlock;
    const int nrl = kBlock / CW;
    const int tid = threadIdx.x;
    const int ct = blockIdx.y;
    const int c = ct * CW + tid % CW;
    const int rl = tid / CW;
    double acc = 0.0;
    const int64_t r0 = blockIdx.x * rows_per_blk;
    int64_t r1 = r0 + rows_per_blk;
    if (r1 > R.n) r1 = R.n;
    if (rl < nrl && c < R.B) {
        for (int64_t i = r0 + rl; i < r1; i += nrl) acc += red_term(R, i, c);
    }
    sh[tid] = acc;
    __syncthreads();
    if (tid < CW && c < R.B) {
        double s = 0.0;
        for (int j = 0; j < nrl; ++j) s += sh[tid + j * CW];
        partials[(size_t)blockIdx.x * R.B + c] = s;
    }
}

__global__ void colreduce_final_kernel(const double* partials, int nblk, int B, double* out, int accumulate,
                                       double scale) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= B) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partials[(size_t)b * B + c];
    out[c] = (accumulate ? out[c] : 0.0) + scale * s;
}

// ------------------------------------------------------------------ K4
__global__ __launch_bounds__(kBlock) void bary_row_kernel(const float* acc, const float* alpha, int64_t n, int ldp,
                                                          int m, float phi, float* bary, float* w, float* xw,
                                                          const float* a, unsigned long long* nfloor) {
    const int lane = threadIdx.x & 63;
    const int64_t row = blockIdx.x * (int64_t)(kBlock / 64) + (threadIdx.x >> 6);
    if (row >= n) return;
    const size_t base = (size_t)row * ldp;
    double ls = 0.0;
    unsigned cnt = 0;
    for (int s = lane; s < m; s += 64) {
        const float r = acc[base + s];
        const float q = r > phi ? r : phi;
        cnt += r > phi ? 0u : 1u;
        ls += (double)alpha[s] * log((double)q);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        ls += __shfl_xor(ls, o, 64);
        cnt += __shfl_xor(cnt, o, 64);
    }
    const double p = exp(ls);
    const float ai = a ? a[row] : 1.f;
    for (int s = lane; s < m; s += 64) {
        const float r = acc[base + s];
        const float q = r > phi ? r : phi;
        const float wv = (float)(p / (double)q);
        w[base + s] = wv;
        if (xw) xw[base + s] = ai * wv;
    }
    if (lane == 0) {
        bary[row] = (float)p;
        if (nfloor && cnt) atomicAdd(nfloor, (unsigned long long)cnt);
    }
}

// ------------------------------------------------------------------ K5
// Seeds of the reverse sweep from D = 4t sum a (mu ln v + nu ln w):
// dmu = 4t a ln v, dnu = 4t a ln w, vbar = 4t a mu / v, wbar = 4t a nu / w
// (on the supports; g4t carries 4t times the upstream gradient per column).
__global__ void bwd_seed_kernel(const float* mu, const float* nu, const float* v, const float* w, const float* a,
                                const float* g4t, int64_t n, int ldp, float* dmu, float* dnu, float* vbar,
                                float* wbar) {
    const int64_t total = n * (int64_t)ldp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ldp;
        const int c = (int)(e - i * ldp);
        const float s = g4t[c] * (a ? a[i] : 1.f);
        const float m = mu[e], u = nu[e];
        dmu[e] = m > 0.f ? s * logf(v[e]) : 0.f;
        dnu[e] = u > 0.f ? s * logf(w[e]) : 0.f;
        vbar[e] = m > 0.f ? s * (m / v[e]) : 0.f;
        wbar[e] = u > 0.f ? s * (u / w[e]) : 0.f;
    }
}

// w_j = nu / e_j:  dnu += wbar / e_j;  ebar = -wbar * w_j / e_j * 1[e_j > phi]
__global__ void bwd_e_kernel(const float* wbar, const float* e_, const float* nu, int64_t total, float phi, float* dnu,
                             float* ebar) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const float ev = e_[e], wb = wbar[e];
        const float wj = nu[e] / ev;
        dnu[e] += wb / ev;
        ebar[e] = ev > phi ? -(wb * wj) / ev : 0.f;
    }
}

// v_j = mu / d_j:  vbar = seed + a z;  dmu += vbar / d_j;  dbar = -vbar * v_j / d_j * 1[d_j > phi]
__global__ void bwd_d_kernel(const float* z, float* vseed, const float* d_, const float* mu, const float* a, int64_t n,
                             int ldp, float phi, float* dmu, float* dbar) {
    const int64_t total = n * (int64_t)ldp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ldp;
        const float ai = a ? a[i] : 1.f;
        const float vb = fmaf(ai, z[e], vseed[e]);
        vseed[e] = 0.f;
        const float dv = d_[e];
        const float vj = mu[e] / dv;
        dmu[e] += vb / dv;
        dbar[e] = dv > phi ? -(vb * vj) / dv : 0.f;
    }
}

__global__ void bwd_w_kernel(const float* z, const float* a, int64_t n, int ldp, float* wbar) {
    const int64_t total = n * (int64_t)ldp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ldp;
        wbar[e] = (a ? a[i] : 1.f) * z[e];
    }
}

__global__ void mask_support_kernel(const float* h, int64_t total, float* g) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        if (!(h[e] > 0.f)) g[e] = 0.f;
}

__global__ void mul_a_kernel(const float* x, const float* a, int64_t n, int ldp, float* out) {
    const int64_t total = n * (int64_t)ldp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = a[e / ldp] * x[e];
}

// ------------------------------------------------------------------ Lanczos helpers (B = 1)
__global__ void lap_spmv_kernel(const int32_t* rowptr, const int32_t* col, const float* val, int32_t n,
                                const float* x, float* y) {
    const int lane = threadIdx.x & 15;
    const int row = blockIdx.x * (kBlock / 16) + (threadIdx.x >> 4);
    float s = 0.f;
    float xi = 0.f;
    if (row < n) {
        xi = x[row];
        for (int e = rowptr[row] + lane; e < rowptr[row + 1]; e += 16) s = fmaf(val[e], xi - x[col[e]], s);
    }
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o, 16);
    if (row < n && lane == 0) y[row] = s;
}

__global__ void lanczos_update_kernel(float* z, const float* q, const float* qprev, float alpha, float beta, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = z[i] - alpha * q[i] - beta * qprev[i];
}

__global__ void scale_kernel(float* dst, const float* src, float s, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = s * src[i];
}

}  // namespace

// ================================================================== launchers
bool shape_supported(const LaunchShape& s) {
    if (s.vec == 1) return s.C == 1 && (s.S == 2 || s.S == 4 || s.S == 8 || s.S == 16 || s.S == 32 || s.S == 64);
    if (s.vec != 4) return false;
    const int lpr = s.S * s.C;
    const bool pow2S = s.S == 1 || s.S == 2 || s.S == 4 || s.S == 8 || s.S == 16;
    const bool pow2C = s.C == 1 || s.C == 2 || s.C == 4 || s.C == 8 || s.C == 16 || s.C == 32 || s.C == 64;
    return pow2S && pow2C && lpr <= 64;
}

bool column_lanes_ok(int ldp, int vec, int C) {
    if (vec == 1) return C == 1;
    return C == 1 || C / 2 < ldp / 4;   // some tile keeps more than half its column lanes busy
}

int long_row_threshold(const LaunchShape& s) {
    const int t = 32 * kUnroll * s.S;   // rows needing more than 32 gather batches per lane
    return t < 256 ? 256 : t;
}

std::vector<LaunchShape> candidate_shapes(int ldp) {
    std::vector<LaunchShape> out;
    for (int nt : {1, 0})
        for (int remap : {1, 0}) {
            if (ldp == 1) {
                for (int S : {2, 4, 8, 16, 32, 64}) out.push_back({1, S, 1, remap, nt});
                continue;
            }
            for (int C : {1, 2, 4, 8, 16, 32, 64}) {
                if (!column_lanes_ok(ldp, 4, C)) continue;
                for (int S : {1, 2, 4, 8, 16}) {
                    LaunchShape s{4, S, C, remap, nt};
                    if (shape_supported(s)) out.push_back(s);
                }
            }
        }
    return out;
}

#define GS_SHAPE_CASE(V, S_, C_)                       \
    if (shape.vec == V && shape.S == S_ && shape.C == C_) { \
        launch_shape<V, S_, C_>(a, st);                \
        return;                                        \
    }

void launch_step(const LaunchShape& shape, const StepArgs& a_in, hipStream_t st) {
    StepArgs a = a_in;
    a.remap = shape.remap;
    a.csr_nt = shape.csr_nt;
    GS_SHAPE_CASE(1, 2, 1) GS_SHAPE_CASE(1, 4, 1) GS_SHAPE_CASE(1, 8, 1) GS_SHAPE_CASE(1, 16, 1)
    GS_SHAPE_CASE(1, 32, 1) GS_SHAPE_CASE(1, 64, 1)
    GS_SHAPE_CASE(4, 1, 1) GS_SHAPE_CASE(4, 2, 1) GS_SHAPE_CASE(4, 4, 1) GS_SHAPE_CASE(4, 8, 1) GS_SHAPE_CASE(4, 16, 1)
    GS_SHAPE_CASE(4, 1, 2) GS_SHAPE_CASE(4, 2, 2) GS_SHAPE_CASE(4, 4, 2) GS_SHAPE_CASE(4, 8, 2) GS_SHAPE_CASE(4, 16, 2)
    GS_SHAPE_CASE(4, 1, 4) GS_SHAPE_CASE(4, 2, 4) GS_SHAPE_CASE(4, 4, 4) GS_SHAPE_CASE(4, 8, 4) GS_SHAPE_CASE(4, 16, 4)
    GS_SHAPE_CASE(4, 1, 8) GS_SHAPE_CASE(4, 2, 8) GS_SHAPE_CASE(4, 4, 8) GS_SHAPE_CASE(4, 8, 8)
    GS_SHAPE_CASE(4, 1, 16) GS_SHAPE_CASE(4, 2, 16) GS_SHAPE_CASE(4, 4, 16)
    GS_SHAPE_CASE(4, 1, 32) GS_SHAPE_CASE(4, 2, 32)
    GS_SHAPE_CASE(4, 1, 64)
    fail(GS_ERR_INVALID, "unsupported launch shape");
}
#undef GS_SHAPE_CASE

void launch_fill(float* p, float v, size_t count, hipStream_t st) {
    if (count == 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for((int64_t)count)), dim3(kBlock), 0, st, p, v, count);
}

void launch_copy_ld(const float* src, int lds, float* dst, int ldd, int64_t n, int B, hipStream_t st) {
    hipLaunchKernelGGL(copy_ld_kernel, dim3(grid_for(n * ldd)), dim3(kBlock), 0, st, src, lds, dst, ldd, n, B);
}

void launch_set_coef(float* dcoef, double alpha, const double* b, const double* db, int K, hipStream_t st) {
    CoefPack pk{};
    pk.v[0] = (float)alpha;
    for (int k = 0; k <= K; ++k) {
        pk.v[1 + k] = (float)b[k];
        pk.v[2 + K + k] = db ? (float)db[k] : 0.f;
    }
    hipLaunchKernelGGL(set_coef_kernel, dim3(1), dim3(kBlock), 0, st, dcoef, pk, 2 * (K + 1) + 1);
}

void launch_stream_copy(const float* src, float* dst, int64_t count, hipStream_t st) {
    const int64_t n4 = count / 4;
    if (n4 > 0) {
        int64_t blocks = (n4 + (int64_t)kBlock * kCopyUnroll - 1) / ((int64_t)kBlock * kCopyUnroll);
        if (blocks > (1 << 30)) blocks = 1 << 30;   // the loop covers the rest
        hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st,
                           reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n4);
    }
    if (count > n4 * 4)
        hipLaunchKernelGGL(stream_copy_tail_kernel, dim3(1), dim3(kBlock), 0, st, src, dst, n4 * 4, count);
}

int reduce_blocks(int64_t n) {
    int64_t nb = (n + 2047) / 2048;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    return (int)nb;
}

void launch_reduce(const ReduceArgs& r, double* partials, int nblk, double* out, int accumulate, double scale,
                   hipStream_t st) {
    const int CW = r.B < kBlock ? r.B : kBlock;
    const int nct = (r.B + CW - 1) / CW;
    const int64_t rows = (r.n + nblk - 1) / nblk;
    hipLaunchKernelGGL(colreduce_kernel, dim3(nblk, nct), dim3(kBlock), 0, st, r, partials, rows);
    hipLaunchKernelGGL(colreduce_final_kernel, dim3((r.B + 63) / 64), dim3(64), 0, st, partials, nblk, r.B, out,
                       accumulate, scale);
}

void launch_bary_row(const float* acc, const float* alpha, int64_t n, int ldp, int m, float phi, float* bary, float* w,
                     float* xw, const float* a, unsigned long long* nfloor, hipStream_t st) {
    const int64_t blocks = (n + 3) / 4;
    hipLaunchKernelGGL(bary_row_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, acc, alpha, n, ldp, m, phi, bary,
                       w, xw, a, nfloor);
}

void launch_bwd_seed(const float* mu, const float* nu, const float* v, const float* w, const float* a,
                     const float* g4t, int64_t n, int ldp, float* dmu, float* dnu, float* vbar_seed, float* wbar,
                     hipStream_t st) {
    hipLaunchKernelGGL(bwd_seed_kernel, dim3(grid_for(n * ldp)), dim3(kBlock), 0, st, mu, nu, v, w, a, g4t, n, ldp,
                       dmu, dnu, vbar_seed, wbar);
}

void launch_bwd_e(const float* wbar, const float* e, const float* nu, int64_t n, int ldp, float phi, float* dnu,
                  float* ebar, hipStream_t st) {
    hipLaunchKernelGGL(bwd_e_kernel, dim3(grid_for(n * ldp)), dim3(kBlock), 0, st, wbar, e, nu, n * (int64_t)ldp, phi,
                       dnu, ebar);
}

void launch_bwd_d(const float* z, float* vbar_seed, const float* d, const float* mu, const float* a, int64_t n,
                  int ldp, float phi, float* dmu, float* dbar, hipStream_t st) {
    hipLaunchKernelGGL(bwd_d_kernel, dim3(grid_for(n * ldp)), dim3(kBlock), 0, st, z, vbar_seed, d, mu, a, n, ldp, phi,
                       dmu, dbar);
}

void launch_bwd_w(const float* z, const float* a, int64_t n, int ldp, float* wbar, hipStream_t st) {
    hipLaunchKernelGGL(bwd_w_kernel, dim3(grid_for(n * ldp)), dim3(kBlock), 0, st, z, a, n, ldp, wbar);
}

void launch_mask_support(const float* h, int64_t n, int ldp, float* g, hipStream_t st) {
    hipLaunchKernelGGL(mask_support_kernel, dim3(grid_for(n * ldp)), dim3(kBlock), 0, st, h, n * (int64_t)ldp, g);
}

void launch_mul_a(const float* x, const float* a, int64_t n, int ldp, float* out, hipStream_t st) {
    hipLaunchKernelGGL(mul_a_kernel, dim3(grid_for(n * ldp)), dim3(kBlock), 0, st, x, a, n, ldp, out);
}

void launch_lap_spmv(const int32_t* rowptr, const int32_t* col, const float* val, int32_t n, const float* x, float* y,
                     hipStream_t st) {
    const int blocks = (n + (kBlock / 16) - 1) / (kBlock / 16);
    hipLaunchKernelGGL(lap_spmv_kernel, dim3(blocks), dim3(kBlock), 0, st, rowptr, col, val, n, x, y);
}

void launch_lanczos_update(float* z, const float* q, const float* qprev, double alpha, double beta, int64_t n,
                           hipStream_t st) {
    hipLaunchKernelGGL(lanczos_update_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, z, q, qprev, (float)alpha,
                       (float)beta, n);
}

void launch_scale(float* dst, const float* src, double s, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, dst, src, (float)s, n);
}

}  // namespace gs
