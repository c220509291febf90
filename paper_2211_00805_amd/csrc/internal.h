// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/geosink.h"

namespace gs {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
void clear_error();

struct Fail {
    gs_status code;
};

[[noreturn]] void fail(gs_status code, const std::string& msg);

#define GS_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            ::gs::fail(GS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define GS_REQUIRE(cond, msg)                                  \
    do {                                                       \
        if (!(cond)) ::gs::fail(GS_ERR_INVALID, (msg));        \
    } while (0)

// Device allocation owned by RAII.
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t count = 0;
    DevBuf() = default;
    explicit DevBuf(size_t c) { alloc(c); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void alloc(size_t c) {
        release();
        if (c == 0) return;
        void* q = nullptr;
        if (hipMalloc(&q, c * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            fail(GS_ERR_OOM, "hipMalloc of " + std::to_string(c * sizeof(T)) + " bytes failed");
        }
        p = static_cast<T*>(q);
        count = c;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        count = 0;
    }
};

// ---------------------------------------------------------------- coefficients
// e^{-t} I_k(t) for k = 0..kmax by Miller's backward recurrence.
void bessel_ive_table(double t, int kmax, std::vector<double>& out);
void cheby_coeffs(double t, int K, double* b, double* db);
double cheby_tail(double t, int K);

// ---------------------------------------------------------------- kernels (kernels.hip)
enum StepFlags : int32_t {
    STEP_FIRST = 1,      // k == 1: T_1 = y X (no T_{k-2})
    STEP_WRITE_T = 2,    // store T_k
    STEP_DUAL = 4,       // second accumulator with the d/dt coefficients
    STEP_ACC_WRITE = 8,  // store the accumulator(s)
    STEP_EPI_SCALE = 16, // last step: out = num / floor(acc); out_a = a * out; record floors
    STEP_ACC_READ = 32,  // accumulator(s) hold earlier terms (else they start at 0)
    STEP_CLENSHAW = 64,  // Clenshaw form: out = c_y (y G) - u_{k+2} + c_x X, G gathered (tprev)
    STEP_CLEN_P2 = 128   // Clenshaw step reads u_{k+2} from tprev2 (products 3..K)
};

struct StepArgs {
    const int32_t* rowptr;
    const int32_t* col;
    const float* val;
    int32_t n;
    int32_t ldp;          // leading dimension (padded B)
    const float* tprev;   // T_{k-1} (T_0 = X when k == 1): gathered
    const float* tprev2;  // T_{k-2} (k >= 2)
    float* tout;          // T_k (may alias tprev2)
    float* acc;
    float* acc2;
    const float* coef;    // [alpha, b_0..b_K, db_0..db_K] (float)
    int32_t k;
    int32_t K;
    int32_t flags;
    int32_t cmask;        // terms added to the accumulator: 1 T_{k-2}, 2 T_{k-1}, 4 T_k
    int32_t remap;        // 1: give each XCD a contiguous range of row tiles
    int32_t csr_nt;       // 1: CSR loads with non-temporal hints; 0: cached
    int32_t long_thr;     // rows with more nonzeros go to the long-row blocks (0: none)
    int32_t nlong;        // number of such rows
    const int32_t* long_rows;
    // scaling epilogue
    const float* num;
    float* out;
    float* out_a;
    const float* a;
    float* rec;
    float phi;
    unsigned long long* nfloor;
    const float* xin;     // Clenshaw: the applied signal X (read on every product)
    // frontier (nullptr: every row computed): level[i] is the hop distance of
    // row i from the applied vector's support (above K where farther), and
    // blk_level[b] the lowest level of row block b (the shape's rows per
    // block).  At step k the rows above k have all-zero operands: they skip
    // their gathers, and a block of them its CSR; the epilogue runs on the
    // dense kernel's operands.
    const uint32_t* level;
    const uint32_t* blk_level;
    // frontier: the application zeroed its T (u) and accumulator buffers
    // before step 1, and this step is not the last; a block beyond the
    // frontier then leaves at once (the dense kernel would write +0 there,
    // which the buffers already hold)
    int32_t skip_dead;
};

struct LaunchShape {
    int vec;         // 1 (float) or 4 (float4)
    int S;           // lanes splitting a row's nonzeros
    int C;           // lanes over column groups of `vec` floats
    int remap = 1;   // XCD-contiguous block order
    int csr_nt = 1;  // CSR read with non-temporal hints (streamed) or cached (graphs that fit the caches)
    bool operator==(const LaunchShape& o) const {
        return vec == o.vec && S == o.S && C == o.C && remap == o.remap && csr_nt == o.csr_nt;
    }
};

bool shape_supported(const LaunchShape& s);
// C column lanes of vec floats over a padded row of ldp floats: a row takes
// ceil(ldp / (vec C)) column tiles; lanes past the row stay idle
bool column_lanes_ok(int ldp, int vec, int C);
int long_row_threshold(const LaunchShape& s);
std::vector<LaunchShape> candidate_shapes(int ldp);
void launch_step(const LaunchShape& shape, const StepArgs& a, hipStream_t st);

void launch_fill(float* p, float v, size_t count, hipStream_t st);
void launch_copy_ld(const float* src, int lds, float* dst, int ldd, int64_t n, int B, hipStream_t st);
void launch_set_coef(float* dcoef, double alpha, const double* b, const double* db, int K, hipStream_t st);
void launch_stream_copy(const float* src, float* dst, int64_t count, hipStream_t st);

// column reductions (fp64, deterministic two-pass)
enum ReduceOp : int32_t {
    RED_DIST = 0,   // sum a (mu ln v + nu ln w) over supports
    RED_MARG = 1,   // sum |a v r - a mu|
    RED_DOT = 2,    // sum a x y (y NULL: ones)
    RED_DOT_QUOT = 3,  // sum a x0 x1 / x2
};
struct ReduceArgs {
    int32_t op;
    int64_t n;
    int32_t ldp;
    int32_t B;
    const float* x0;   // DIST: mu   MARG: v   DOT: x   DOT_QUOT: x
    const float* x1;   // DIST: v    MARG: r   DOT: y   DOT_QUOT: numerator
    const float* x2;   // DIST: nu   MARG: mu           DOT_QUOT: denominator
    const float* x3;   // DIST: w
    const float* a;    // nullable
};
int reduce_blocks(int64_t n);
void launch_reduce(const ReduceArgs& r, double* partials, int nblk, double* out, int accumulate,
                   double scale_from, hipStream_t st);

// barycenter row kernel: q = floor(acc); p = exp(sum alpha ln q); w = p / q; xw = a w
void launch_bary_row(const float* acc, const float* alpha, int64_t n, int ldp, int m, float phi,
                     float* bary, float* w, float* xw, const float* a, unsigned long long* nfloor,
                     hipStream_t st);

// backward elementwise kernels
void launch_bwd_seed(const float* mu, const float* nu, const float* v, const float* w, const float* a,
                     const float* g4t, int64_t n, int ldp, float* dmu, float* dnu, float* vbar_seed,
                     float* wbar, hipStream_t st);
void launch_bwd_e(const float* wbar, const float* e, const float* nu, int64_t n, int ldp, float phi,
                  float* dnu, float* ebar, hipStream_t st);
void launch_bwd_d(const float* z, float* vbar_seed, const float* d, const float* mu, const float* a,
                  int64_t n, int ldp, float phi, float* dmu, float* dbar, hipStream_t st);
void launch_bwd_w(const float* z, const float* a, int64_t n, int ldp, float* wbar, hipStream_t st);
void launch_mul_a(const float* x, const float* a, int64_t n, int ldp, float* out, hipStream_t st);
void launch_mask_support(const float* h, int64_t n, int ldp, float* g, hipStream_t st);

// Laplacian mat-vec and Lanczos helpers (B = 1)
void launch_lap_spmv(const int32_t* rowptr, const int32_t* col, const float* val, int32_t n,
                     const float* x, float* y, hipStream_t st);
void launch_lanczos_update(float* z, const float* q, const float* qprev, double alpha, double beta,
                           int64_t n, hipStream_t st);
void launch_scale(float* dst, const float* src, double s, int64_t n, hipStream_t st);

// backward-Euler kernel by conjugate gradients (per-column float64 scalars on the device)
constexpr int kMaxCgBlocks = 1024;    // row blocks of a CG column pass (partials: kMaxCgBlocks x ldp)
int cg_blocks(int64_t n);
void launch_cg_init(const float* b, float* x, float* r, float* p, int64_t total, hipStream_t st);
// out[c] = sum_i a[i, c] b[i, c] (float64)
void launch_cg_dot(const float* a, const float* b, int64_t n, int ldp, double* partials, double* out,
                   hipStream_t st);
// alpha = rr / (-pqn); x += alpha p; r += alpha qn; rr_new[c] = sum_i r[i, c]^2 (float64)
void launch_cg_update(float* x, float* r, const float* p, const float* qn, const double* rr, const double* pqn,
                      int64_t n, int ldp, double* partials, double* rr_new, hipStream_t st);
void launch_cg_dir(const float* r, float* p, const double* rr_old, const double* rr_new, int64_t total, int ldp,
                   hipStream_t st);
// out = num / floor(acc) (+ a out, recorded denominators, floor count), as the step epilogue
void launch_scale_epilogue(const float* acc, const float* num, float* out, float* out_a, const float* a, float* rec,
                           float phi, unsigned long long* nfloor, int64_t n, int ldp, hipStream_t st);

// hop levels of a support (frontier.hip): level[i] = breadth-first distance
// of row i from the rows where any of the B columns of h (n x ldp) is nonzero,
// exact up to `depth`, kFarLevel beyond; blk_level[b] = min level over rows
// [b rpb, (b + 1) rpb); flags: depth + 1 ints of scratch
constexpr uint32_t kFarLevel = 1u << 30;
// zeros in up to four float buffers (nullptr: none) of count elements each
void launch_zero_buffers(float* b0, float* b1, float* b2, float* b3, int64_t count, hipStream_t st);
void launch_support_levels(const float* h, int64_t n, int ldp, int B, const int32_t* rowptr, const int32_t* col,
                           int depth, int rpb, uint32_t* level, uint32_t* blk_level, int32_t* flags, hipStream_t st);

// gather-throughput helper (measure.hip): out holds gather_out_floats(m) floats
int64_t gather_out_floats(int64_t m);
void launch_gather_rows(const float* X, int64_t n, const int32_t* idx, int64_t m, float* out, hipStream_t st);

// bad[0] += non-finite entries of x[0, count), bad[1] += negative ones (validate.hip)
void launch_count_invalid(const float* x, int64_t count, unsigned long long* bad, hipStream_t st);

// out[i*B + b] = H[i*m + cols[b]] (0 for cols[b] outside [0, m)) (accumulate.hip)
void launch_gather_columns(const float* H, int64_t n, int m, const int32_t* cols, int B, float* out, hipStream_t st);

// G[cols[b]*n + i] += src[i*B + b] for cols[b] in [0, m), b = 0..B-1 in order (accumulate.hip)
void launch_accumulate_columns(const float* src, int64_t n, int B, const int32_t* cols, int m, float* G,
                               hipStream_t st);

// kNN candidates (knn.hip): cand (n x kk) int32, candidate ids sorted by fp32 Gram distance
void launch_knn_candidates(const float* Xc, const float* norms, int64_t n, int d, int kk, int32_t* cand,
                           hipStream_t st);
void launch_row_norms(const float* Xc, int64_t n, int d, float* norms, hipStream_t st);

}  // namespace gs

// ---------------------------------------------------------------- handles
struct gs_graph_s {
    int64_t n = 0;
    int64_t nnz = 0;
    int device = 0;
    gs::DevBuf<int32_t> rowptr, col;
    gs::DevBuf<float> val;
    std::vector<int32_t> h_rowptr, h_col;
    std::vector<float> h_val, h_deg;
    int32_t n_components = 0;
    double deg_max = 0.0, edge_bound = 0.0, median = 0.0;
    // plans the graph-level calls create for (K, B) when given none; freed
    // with the graph
    std::mutex plans_mu;
    std::map<std::pair<int32_t, int32_t>, gs_plan_s*> plans;
};
