// Plan: device workspace, launch shape and captured hipGraphs for one (graph, K, B).
#pragma once

#include <map>
#include <string>
#include <tuple>

#include "internal.h"

namespace gs {

enum class ApplyMode { Store, Dual, Scale };

constexpr int kRecordChunk = 8;   // iterations per captured graph in record mode

struct StepSched {
    int flags;
    int cmask;
};

// Hop levels of one support (rows, row blocks of the plan's shape);
// row == nullptr: dense steps.
struct Levels {
    uint32_t* row = nullptr;
    uint32_t* blk = nullptr;
};

struct ScaleEpi {
    const float* num = nullptr;
    float* out = nullptr;
    float* out_a = nullptr;
    const float* a = nullptr;
    float* rec = nullptr;
};

}  // namespace gs

struct gs_plan_s {
    gs_graph g = nullptr;
    int K = 0, B = 0, ldp = 0, flags = 0;
    int64_t n = 0;
    gs::LaunchShape shape{4, 1, 1};
    std::string shape_origin;  // "default", "autotuned", "cache"
    hipStream_t cap = nullptr; // private stream used only for graph capture

    // Chebyshev buffers (n x ldp)
    gs::DevBuf<float> X, U, V, ACC, ACC2;
    // Sinkhorn state (n x ldp) and vertex weights (n)
    gs::DevBuf<float> mu, nu, v, w, xv, xw, a;
    gs::DevBuf<float> coef;
    gs::DevBuf<int32_t> long_rows;  // rows handled by the long-row blocks for the current shape
    int nlong = 0, long_thr = 0;
    gs::DevBuf<double> partials, red;
    gs::DevBuf<unsigned long long> nfloor;
    gs::DevBuf<unsigned long long> badin;   // non-finite / negative input entries of the current call
    bool count_floors = false;  // this call reports floored denominators (kernels skip the count otherwise)
    gs::DevBuf<float> alpha;   // barycenter weights (m)
    gs::DevBuf<float> bary;    // barycenter (n)
    // backward workspace (allocated on first use)
    int seg_cap = 0;
    const float* rec_buf = nullptr;   // record buffer whose addresses the captured graphs hold
    gs::DevBuf<float> segd, sege, dmu, dnu, vseed, wbar, wck, g4t;
    gs::DevBuf<double> tbar;

    // kernel selection: GS_KERNEL_CHEBYSHEV, GS_KERNEL_CLENSHAW (the same
    // polynomial by Clenshaw's recurrence) or GS_KERNEL_EULER (N solves of
    // cg_m conjugate-gradient iterations; cg_iters == 0 picks cg_m per call)
    int kernel = GS_KERNEL_CHEBYSHEV;
    int euler_N = 0, cg_iters = 0, cg_m = 0;
    gs::DevBuf<float> er, ep, eq, ecoef;   // CG residual, direction, product; operator scale
    gs::DevBuf<double> ers;                // per-column rr (two slots), p.qn, then column-pass partials

    // frontier-sparse steps (opt-in): per-row hop levels of the supports the
    // applications start from (mu's also serves gs_heat_apply's X)
    int frontier = 0;
    gs::DevBuf<uint32_t> lev_mu, lev_nu, blk_mu, blk_nu;
    gs::DevBuf<int32_t> lev_flags;   // per-sweep flags of the level computation

    std::map<std::string, hipGraphExec_t> graphs;
    std::map<std::string, hipGraph_t> graph_defs;

    ~gs_plan_s();
    size_t sz() const { return (size_t)n * ldp; }
};

namespace gs {

gs_plan_s* plan_create(gs_graph g, int K, int B, int flags, const char* tune_cache);
void set_coefs(gs_plan_s& P, double lambda_hat, double t, hipStream_t st);
void enqueue_apply(gs_plan_s& P, const float* X, ApplyMode mode, const ScaleEpi& epi, float phi, hipStream_t st,
                   Levels lev = Levels{});
void set_frontier(gs_plan_s& P, int enable);
void set_kernel(gs_plan_s& P, int kernel, int N, int cg_iters);
int euler_cg_iterations(double t, int N);
void heat_apply(gs_plan_s& P, double lam, double t, const float* X, float* Y, float* Ydt, hipStream_t st);
void sinkhorn(gs_plan_s& P, double lam, double t, const float* a, const float* mu, const float* nu, int J, float phi,
              int C, float* ckpt, float* v, float* w, double* dist, double* marg, int64_t* nfl, hipStream_t st);
void sinkhorn_backward(gs_plan_s& P, double lam, double t, const float* a, const float* mu, const float* nu, int J,
                       float phi, int C, const float* ckpt, const double* gd, float* gmu, float* gnu, double* gt,
                       hipStream_t st);
void barycenter(gs_plan_s& P, double lam, double t, const float* a, const float* mus, const double* alpha, int J,
                float phi, float* bary, float* v, float* w, double* marg, int64_t* nfl, hipStream_t st);
void drop_graphs(gs_plan_s& P);
void update_long_rows(gs_plan_s& P);
double time_step(gs_plan_s& P, const LaunchShape& shape, int reps, hipStream_t st, double* bytes_per_launch);
std::vector<StepSched> step_schedule(int K, ApplyMode mode);
StepSched step_sched_at(int K, int k, ApplyMode mode);
std::vector<StepSched> clenshaw_schedule(int K, ApplyMode mode);
LaunchShape default_shape(int ldp, double nnz_per_row);
void heat_apply_noalloc(gs_graph_s& g, double lam, double t, int K, const float* X, float* Y, int B, hipStream_t st);
double step_bytes(const gs_plan_s& P, const StepSched& sc, bool has_out_a, bool has_rec);
double lambda_max(gs_graph_s& g, int iters, uint64_t seed, double safety, hipStream_t st);

void build_graph_from_points(const float* X, int64_t n, int d, int k, hipStream_t st, gs_graph_s& g);
void build_graph_from_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const float* w,
                          gs_graph_s& g);
void upload_graph(gs_graph_s& g, hipStream_t st);

}  // namespace gs
