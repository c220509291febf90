// extern "C" entry points: argument validation (before any HIP call), error
// capture into a thread-local message, and dispatch into the drivers.
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <new>

#include "plan.h"

namespace gs {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

void fail(gs_status code, const std::string& msg) {
    set_error(msg);
    throw Fail{code};
}

namespace {

template <class F>
gs_status guarded(F&& f) {
    clear_error();
    try {
        f();
        return GS_OK;
    } catch (const Fail& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return GS_ERR_OOM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return GS_ERR_INVALID;
    } catch (...) {
        set_error("unknown failure");
        return GS_ERR_INVALID;
    }
}

void require_device() {
    int count = 0;
    const hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) {
        (void)hipGetLastError();
        fail(GS_ERR_NO_DEVICE, std::string("no HIP device is visible (hipGetDeviceCount: ") + hipGetErrorString(e) +
                                   ", count " + std::to_string(count) + ")");
    }
    int dev = 0;
    GS_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    GS_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        fail(GS_ERR_NO_DEVICE, std::string("library is built for gfx950, device is ") + prop.gcnArchName);
}

// The plan a graph-level call runs on: the caller's, which must belong to
// (g, K, B), or the one the graph keeps for (K, B), created on first use
// with default flags (default launch shape, captured graphs).
gs_plan resolve_plan(gs_graph g, int32_t K, int32_t B, gs_plan plan) {
    GS_REQUIRE(g != nullptr, "graph is NULL");
    GS_REQUIRE(K >= 1 && K <= GS_MAX_K, "K must be in [1, GS_MAX_K]");
    GS_REQUIRE(B >= 1 && B <= 4096, "B must be in [1, 4096]");
    if (plan) {
        GS_REQUIRE(plan->g == g && plan->K == K && plan->B == B, "plan was created for another graph, K or B");
        return plan;
    }
    std::lock_guard<std::mutex> lk(g->plans_mu);
    gs_plan& slot = g->plans[{K, B}];
    if (!slot) {
        require_device();
        slot = plan_create(g, K, B, 0, nullptr);
    }
    return slot;
}

void check_plan_args(gs_plan p, double lam, double t) {
    GS_REQUIRE(p != nullptr, "plan is NULL");
    GS_REQUIRE(std::isfinite(lam) && lam > 0.0, "lambda_hat must be finite and > 0");
    GS_REQUIRE(std::isfinite(t) && t >= 0.0, "t must be finite and >= 0");
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

const char* gs_last_error(void) { return g_last_error.c_str(); }

int32_t gs_abi_version(void) { return GS_ABI_VERSION; }

gs_status gs_graph_from_points(const float* X, int64_t n, int32_t d, int32_t k, int32_t require_connected,
                               hipStream_t stream, gs_graph* out) {
    return guarded([&] {
        GS_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        GS_REQUIRE(X != nullptr, "X is NULL");
        GS_REQUIRE(n >= 2 && n < (int64_t)1 << 31, "n must be in [2, 2^31)");
        GS_REQUIRE(d >= 1 && d <= 4096, "d must be in [1, 4096]");
        GS_REQUIRE(k >= 1 && k <= 32 && k < n, "k must be in [1, 32] and < n");
        for (int64_t i = 0; i < n * (int64_t)d; ++i)
            if (!std::isfinite(X[i])) fail(GS_ERR_NONFINITE, "X holds a non-finite value");
        require_device();
        auto g = std::make_unique<gs_graph_s>();
        build_graph_from_points(X, n, d, k, stream, *g);
        if (require_connected && g->n_components != 1)
            fail(GS_ERR_NOT_CONNECTED, "graph has " + std::to_string(g->n_components) + " connected components");
        *out = g.release();
    });
}

gs_status gs_graph_from_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const float* w,
                            hipStream_t stream, gs_graph* out) {
    return guarded([&] {
        GS_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        GS_REQUIRE(n >= 1 && n < (int64_t)1 << 31, "n must be in [1, 2^31)");
        GS_REQUIRE(nnz >= 0 && nnz < (int64_t)1 << 31, "nnz must be in [0, 2^31)");
        GS_REQUIRE(rowptr != nullptr, "rowptr is NULL");
        GS_REQUIRE(nnz == 0 || (col != nullptr && w != nullptr), "col / w is NULL");
        auto g = std::make_unique<gs_graph_s>();
        build_graph_from_csr(n, nnz, rowptr, col, w, *g);  // validates on the host
        require_device();
        upload_graph(*g, stream);
        *out = g.release();
    });
}

gs_status gs_graph_info(gs_graph g, int64_t* n, int64_t* nnz, int32_t* n_components, double* deg_max,
                        double* edge_bound, double* median_dist) {
    return guarded([&] {
        GS_REQUIRE(g != nullptr, "graph is NULL");
        if (n) *n = g->n;
        if (nnz) *nnz = g->nnz;
        if (n_components) *n_components = g->n_components;
        if (deg_max) *deg_max = g->deg_max;
        if (edge_bound) *edge_bound = g->edge_bound;
        if (median_dist) *median_dist = g->median;
    });
}

gs_status gs_graph_export(gs_graph g, int32_t* rowptr, int32_t* col, float* w, float* deg) {
    return guarded([&] {
        GS_REQUIRE(g != nullptr, "graph is NULL");
        if (rowptr) std::memcpy(rowptr, g->h_rowptr.data(), (g->n + 1) * sizeof(int32_t));
        if (col && g->nnz) std::memcpy(col, g->h_col.data(), g->nnz * sizeof(int32_t));
        if (w && g->nnz) std::memcpy(w, g->h_val.data(), g->nnz * sizeof(float));
        if (deg) std::memcpy(deg, g->h_deg.data(), g->n * sizeof(float));
    });
}

void gs_graph_destroy(gs_graph g) {
    if (g)
        for (auto& kv : g->plans) delete kv.second;
    delete g;
}

gs_status gs_lambda_max(gs_graph g, int32_t iters, uint64_t seed, double safety, hipStream_t stream,
                        double* lambda_hat) {
    return guarded([&] {
        GS_REQUIRE(g != nullptr, "graph is NULL");
        GS_REQUIRE(lambda_hat != nullptr, "lambda_hat is NULL");
        GS_REQUIRE(iters >= 2 && iters <= 10000, "iters must be in [2, 10000]");
        GS_REQUIRE(std::isfinite(safety) && safety >= 1.0, "safety must be >= 1");
        GS_REQUIRE(g->nnz > 0, "graph has no edges");
        *lambda_hat = lambda_max(*g, iters, seed, safety, stream);
    });
}

gs_status gs_cheby_coeffs(double t, int32_t K, double* b, double* db_dt) {
    return guarded([&] {
        GS_REQUIRE(b != nullptr, "b is NULL");
        GS_REQUIRE(std::isfinite(t) && t >= 0.0, "t must be finite and >= 0");
        GS_REQUIRE(K >= 0 && K <= GS_MAX_K, "K must be in [0, GS_MAX_K]");
        cheby_coeffs(t, K, b, db_dt);
    });
}

gs_status gs_cheby_tail_bound(double t, int32_t K, double* bound) {
    return guarded([&] {
        GS_REQUIRE(bound != nullptr, "bound is NULL");
        GS_REQUIRE(std::isfinite(t) && t >= 0.0, "t must be finite and >= 0");
        GS_REQUIRE(K >= 0 && K <= GS_MAX_K, "K must be in [0, GS_MAX_K]");
        *bound = cheby_tail(t, K);
    });
}

gs_status gs_plan_create(gs_graph g, int32_t K, int32_t B, int32_t flags, const char* tune_cache, gs_plan* out) {
    return guarded([&] {
        GS_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        GS_REQUIRE(g != nullptr, "graph is NULL");
        GS_REQUIRE(K >= 1 && K <= GS_MAX_K, "K must be in [1, GS_MAX_K]");
        GS_REQUIRE(B >= 1 && B <= 4096, "B must be in [1, 4096]");
        GS_REQUIRE((flags & ~(GS_PLAN_AUTOTUNE | GS_PLAN_NO_GRAPH)) == 0, "unknown plan flags");
        require_device();
        *out = plan_create(g, K, B, flags, tune_cache);
    });
}

gs_status gs_plan_set_shape(gs_plan p, int32_t vec, int32_t S, int32_t C) {
    return guarded([&] {
        GS_REQUIRE(p != nullptr, "plan is NULL");
        const LaunchShape s{vec, S, C, p->shape.remap, p->shape.csr_nt};
        GS_REQUIRE(shape_supported(s), "unsupported launch shape");
        GS_REQUIRE((vec == 1) == (p->ldp == 1), "vec must be 1 exactly when B == 1");
        GS_REQUIRE(column_lanes_ok(p->ldp, vec, C), "C must be 1 or below twice the padded B's float4 groups");
        GS_HIP(hipDeviceSynchronize());
        drop_graphs(*p);
        p->shape = s;
        p->shape_origin = "set";
        update_long_rows(*p);
    });
}

gs_status gs_plan_set_csr_hint(gs_plan p, int32_t streamed) {
    return guarded([&] {
        GS_REQUIRE(p != nullptr, "plan is NULL");
        GS_REQUIRE(streamed == 0 || streamed == 1, "streamed must be 0 or 1");
        GS_HIP(hipDeviceSynchronize());
        drop_graphs(*p);
        p->shape.csr_nt = streamed;
        p->shape_origin = "set";
    });
}

gs_status gs_plan_set_frontier(gs_plan p, int32_t enable) {
    return guarded([&] {
        GS_REQUIRE(p != nullptr, "plan is NULL");
        GS_REQUIRE(enable == 0 || enable == 1, "enable must be 0 or 1");
        GS_HIP(hipDeviceSynchronize());
        drop_graphs(*p);
        set_frontier(*p, enable);
    });
}

gs_status gs_plan_set_kernel(gs_plan p, int32_t kernel, int32_t N, int32_t cg_iters) {
    return guarded([&] {
        GS_REQUIRE(p != nullptr, "plan is NULL");
        GS_REQUIRE(kernel == GS_KERNEL_CHEBYSHEV || kernel == GS_KERNEL_CLENSHAW || kernel == GS_KERNEL_EULER,
                   "unknown kernel");
        if (kernel == GS_KERNEL_EULER) {
            GS_REQUIRE(N >= 1 && N <= 1024, "N must be in [1, 1024]");
            GS_REQUIRE(cg_iters >= 0 && cg_iters <= 1000, "cg_iters must be in [0, 1000]");
        }
        GS_HIP(hipDeviceSynchronize());
        set_kernel(*p, kernel, N, cg_iters);
    });
}

gs_status gs_plan_describe(gs_plan p, char* buf, int32_t len) {
    return guarded([&] {
        GS_REQUIRE(p != nullptr && buf != nullptr && len > 0, "bad arguments");
        const std::string s = "vec=" + std::to_string(p->shape.vec) + " S=" + std::to_string(p->shape.S) +
                              " C=" + std::to_string(p->shape.C) + " xcd=" + std::to_string(p->shape.remap) +
                              (p->shape.csr_nt ? " csr=nt" : " csr=t") +
                              " ldp=" + std::to_string(p->ldp) + (p->frontier ? " frontier=on" : "") +
                              " origin=" + p->shape_origin + ((p->flags & GS_PLAN_NO_GRAPH) ? " graphs=off" : " graphs=on") +
                              (p->kernel == GS_KERNEL_EULER
                                   ? " kernel=euler N=" + std::to_string(p->euler_N) + " cg=" +
                                         (p->cg_iters > 0 ? std::to_string(p->cg_iters) : std::string("auto"))
                                   : std::string(p->kernel == GS_KERNEL_CLENSHAW ? " kernel=clenshaw"
                                                                                 : " kernel=chebyshev"));
        std::strncpy(buf, s.c_str(), len - 1);
        buf[len - 1] = 0;
    });
}

void gs_plan_destroy(gs_plan p) { delete p; }

gs_status gs_heat_apply(gs_plan p, double lambda_hat, double t, const float* X, float* Y, float* Ydt,
                        hipStream_t stream) {
    return guarded([&] {
        check_plan_args(p, lambda_hat, t);
        GS_REQUIRE(X != nullptr && Y != nullptr, "X / Y is NULL");
        GS_REQUIRE(X != Y && (const float*)Ydt != X && Ydt != Y, "X, Y and Ydt must be distinct");
        GS_REQUIRE(Ydt == nullptr || p->kernel != GS_KERNEL_EULER,
                   "the time derivative needs a Chebyshev kernel");
        heat_apply(*p, lambda_hat, t, X, Y, Ydt, stream);
    });
}

gs_status gs_heat_apply_noalloc(gs_graph g, double lambda_hat, double t, int32_t K, const float* X, float* Y,
                                int32_t B, hipStream_t stream) {
    return guarded([&] {
        GS_REQUIRE(g != nullptr, "graph is NULL");
        GS_REQUIRE(std::isfinite(lambda_hat) && lambda_hat > 0.0, "lambda_hat must be finite and > 0");
        GS_REQUIRE(std::isfinite(t) && t >= 0.0, "t must be finite and >= 0");
        GS_REQUIRE(K >= 1 && K <= GS_MAX_K, "K must be in [1, GS_MAX_K]");
        GS_REQUIRE(B == 1 || (B >= 4 && B % 4 == 0), "B must be 1 or a multiple of 4");
        GS_REQUIRE(g->n * (int64_t)B <= (int64_t)GS_NOALLOC_MAX_NB,
                   "n * B exceeds GS_NOALLOC_MAX_NB (the fixed scratch array of the no-allocation entry point)");
        GS_REQUIRE(X != nullptr && Y != nullptr, "X / Y is NULL");
        GS_REQUIRE((const float*)Y != X, "X and Y must be distinct");
        heat_apply_noalloc(*g, lambda_hat, t, K, X, Y, B, stream);
    });
}

gs_status gs_sinkhorn(gs_plan p, double lambda_hat, double t, const float* a, const float* mu, const float* nu,
                      int32_t iters, float phi, int32_t ckpt_every, float* ckpt, float* v, float* w, double* dist,
                      double* marg_err, int64_t* n_floored, hipStream_t stream) {
    return guarded([&] {
        check_plan_args(p, lambda_hat, t);
        GS_REQUIRE(mu != nullptr && nu != nullptr, "mu / nu is NULL");
        GS_REQUIRE(iters >= 1, "iters must be >= 1");
        GS_REQUIRE(std::isfinite(phi) && phi > 0.f, "phi must be finite and > 0");
        GS_REQUIRE(ckpt == nullptr || ckpt_every >= 1 || ckpt_every == GS_RECORD_ALL,
                   "ckpt_every must be >= 1 or GS_RECORD_ALL when ckpt is given");
        sinkhorn(*p, lambda_hat, t, a, mu, nu, iters, phi, ckpt ? ckpt_every : 1, ckpt, v, w, dist, marg_err,
                 n_floored, stream);
    });
}

gs_status gs_sinkhorn_backward(gs_plan p, double lambda_hat, double t, const float* a, const float* mu,
                               const float* nu, int32_t iters, float phi, int32_t ckpt_every, const float* ckpt,
                               const double* grad_dist, float* grad_mu, float* grad_nu, double* grad_t,
                               hipStream_t stream) {
    return guarded([&] {
        check_plan_args(p, lambda_hat, t);
        GS_REQUIRE(p->kernel != GS_KERNEL_EULER, "the reverse sweep needs a Chebyshev kernel");
        GS_REQUIRE(t > 0.0, "t must be > 0 for the backward");
        GS_REQUIRE(mu != nullptr && nu != nullptr && ckpt != nullptr && grad_dist != nullptr,
                   "mu / nu / ckpt / grad_dist is NULL");
        GS_REQUIRE(iters >= 1 && (ckpt_every >= 1 || ckpt_every == GS_RECORD_ALL),
                   "iters must be >= 1 and ckpt_every >= 1 or GS_RECORD_ALL");
        GS_REQUIRE(std::isfinite(phi) && phi > 0.f, "phi must be finite and > 0");
        for (int b = 0; b < p->B; ++b) GS_REQUIRE(std::isfinite(grad_dist[b]), "grad_dist must be finite");
        sinkhorn_backward(*p, lambda_hat, t, a, mu, nu, iters, phi, ckpt_every, ckpt, grad_dist, grad_mu, grad_nu,
                          grad_t, stream);
    });
}

gs_status gs_barycenter(gs_plan p, double lambda_hat, double t, const float* a, const float* mus,
                        const double* alpha, int32_t iters, float phi, float* bary, float* v, float* w,
                        double* marg_err, int64_t* n_floored, hipStream_t stream) {
    return guarded([&] {
        check_plan_args(p, lambda_hat, t);
        GS_REQUIRE(mus != nullptr && alpha != nullptr && bary != nullptr, "mus / alpha / bary is NULL");
        GS_REQUIRE(iters >= 1, "iters must be >= 1");
        GS_REQUIRE(std::isfinite(phi) && phi > 0.f, "phi must be finite and > 0");
        for (int i = 0; i < p->B; ++i) GS_REQUIRE(std::isfinite(alpha[i]) && alpha[i] >= 0.0, "alpha must be >= 0");
        barycenter(*p, lambda_hat, t, a, mus, alpha, iters, phi, bary, v, w, marg_err, n_floored, stream);
    });
}

gs_status gs_graph_heat_apply(gs_graph g, double lambda_hat, double t, int32_t K, const float* X, float* Y,
                              float* Ydt, int32_t B, gs_plan plan, hipStream_t stream) {
    gs_plan p = nullptr;
    const gs_status s = guarded([&] { p = resolve_plan(g, K, B, plan); });
    return s != GS_OK ? s : gs_heat_apply(p, lambda_hat, t, X, Y, Ydt, stream);
}

gs_status gs_graph_sinkhorn(gs_graph g, double lambda_hat, double t, int32_t K, const float* a, const float* mu,
                            const float* nu, int32_t B, int32_t iters, float phi, int32_t ckpt_every, float* ckpt,
                            float* v, float* w, double* dist, double* marg_err, int64_t* n_floored, gs_plan plan,
                            hipStream_t stream) {
    gs_plan p = nullptr;
    const gs_status s = guarded([&] { p = resolve_plan(g, K, B, plan); });
    return s != GS_OK ? s
                      : gs_sinkhorn(p, lambda_hat, t, a, mu, nu, iters, phi, ckpt_every, ckpt, v, w, dist, marg_err,
                                    n_floored, stream);
}

gs_status gs_graph_sinkhorn_backward(gs_graph g, double lambda_hat, double t, int32_t K, const float* a,
                                     const float* mu, const float* nu, int32_t B, int32_t iters, float phi,
                                     int32_t ckpt_every, const float* ckpt, const double* grad_dist, float* grad_mu,
                                     float* grad_nu, double* grad_t, gs_plan plan, hipStream_t stream) {
    gs_plan p = nullptr;
    const gs_status s = guarded([&] { p = resolve_plan(g, K, B, plan); });
    return s != GS_OK ? s
                      : gs_sinkhorn_backward(p, lambda_hat, t, a, mu, nu, iters, phi, ckpt_every, ckpt, grad_dist,
                                             grad_mu, grad_nu, grad_t, stream);
}

gs_status gs_graph_barycenter(gs_graph g, double lambda_hat, double t, int32_t K, const float* a, const float* mus,
                              const double* alpha, int32_t m, int32_t iters, float phi, float* bary, float* v,
                              float* w, double* marg_err, int64_t* n_floored, gs_plan plan, hipStream_t stream) {
    gs_plan p = nullptr;
    const gs_status s = guarded([&] { p = resolve_plan(g, K, m, plan); });
    return s != GS_OK ? s
                      : gs_barycenter(p, lambda_hat, t, a, mus, alpha, iters, phi, bary, v, w, marg_err, n_floored,
                                      stream);
}

gs_status gs_expectation(const float* p, const float* Y, int64_t n, int32_t d, hipStream_t stream, double* out) {
    return guarded([&] {
        GS_REQUIRE(p != nullptr && Y != nullptr && out != nullptr, "p / Y / out is NULL");
        GS_REQUIRE(n >= 1, "n must be >= 1");
        GS_REQUIRE(d >= 1 && d <= 4096, "d must be in [1, 4096]");
        require_device();
        const int nblk = reduce_blocks(n);
        DevBuf<double> part((size_t)nblk * d), red((size_t)d + 1);
        ReduceArgs r{};
        r.op = RED_DOT;      // sum_i p_i Y[i, c]  (p as the row weight)
        r.n = n;
        r.ldp = d;
        r.B = d;
        r.x0 = Y;
        r.a = p;
        launch_reduce(r, part.p, nblk, red.p, 0, 1.0, stream);
        ReduceArgs mass{};
        mass.op = RED_DOT;   // sum_i p_i
        mass.n = n;
        mass.ldp = 1;
        mass.B = 1;
        mass.x0 = p;
        launch_reduce(mass, part.p, nblk, red.p + d, 0, 1.0, stream);
        std::vector<double> h((size_t)d + 1);
        GS_HIP(hipMemcpyAsync(h.data(), red.p, (d + 1) * sizeof(double), hipMemcpyDeviceToHost, stream));
        GS_HIP(hipStreamSynchronize(stream));
        GS_HIP(hipGetLastError());
        if (!(h[d] != 0.0) || !std::isfinite(h[d])) fail(GS_ERR_NONFINITE, "signal has zero or non-finite mass");
        for (int c = 0; c < d; ++c) out[c] = h[c] / h[d];
    });
}

gs_status gs_plan_time_step(gs_plan p, int32_t reps, hipStream_t stream, double* avg_ms, double* bytes_per_launch) {
    return guarded([&] {
        GS_REQUIRE(p != nullptr && avg_ms != nullptr, "plan / avg_ms is NULL");
        GS_REQUIRE(reps >= 1 && reps <= 100000, "reps must be in [1, 100000]");
        *avg_ms = time_step(*p, p->shape, reps, stream, bytes_per_launch);
    });
}

gs_status gs_stream_copy(const float* src, float* dst, int64_t count, hipStream_t stream) {
    return guarded([&] {
        GS_REQUIRE(src != nullptr && dst != nullptr && count >= 0, "bad arguments");
        launch_stream_copy(src, dst, count, stream);
        GS_HIP(hipGetLastError());
    });
}

gs_status gs_gather_columns(const float* H, int64_t n, int32_t m, const int32_t* cols, int32_t B, float* out,
                            hipStream_t stream) {
    return guarded([&] {
        GS_REQUIRE(H != nullptr && cols != nullptr && out != nullptr, "H / cols / out is NULL");
        GS_REQUIRE(n >= 1 && n < (int64_t)1 << 31, "n must be in [1, 2^31)");
        GS_REQUIRE(m >= 1, "m must be >= 1");
        GS_REQUIRE(B >= 1 && B <= 4096, "B must be in [1, 4096]");
        GS_REQUIRE((const float*)out != H, "H and out must not overlap");
        launch_gather_columns(H, n, m, cols, B, out, stream);
        GS_HIP(hipGetLastError());
    });
}

gs_status gs_accumulate_columns(const float* src, int64_t n, int32_t B, const int32_t* cols, int32_t m, float* G,
                                hipStream_t stream) {
    return guarded([&] {
        GS_REQUIRE(src != nullptr && cols != nullptr && G != nullptr, "src / cols / G is NULL");
        GS_REQUIRE(n >= 1 && n < (int64_t)1 << 31, "n must be in [1, 2^31)");
        GS_REQUIRE(B >= 1 && B <= 4096, "B must be in [1, 4096]");
        GS_REQUIRE(m >= 1, "m must be >= 1");
        GS_REQUIRE((const float*)G != src, "src and G must not overlap");
        launch_accumulate_columns(src, n, B, cols, m, G, stream);
        GS_HIP(hipGetLastError());
    });
}

gs_status gs_stream_gather(const float* X, int64_t n, const int32_t* idx, int64_t m, float* out,
                           hipStream_t stream) {
    return guarded([&] {
        GS_REQUIRE(X != nullptr && idx != nullptr && out != nullptr, "X / idx / out is NULL");
        GS_REQUIRE(n >= 1 && m >= 0 && m < ((int64_t)1 << 40), "bad sizes");
        if (m == 0) return;
        launch_gather_rows(X, n, idx, m, out, stream);
        GS_HIP(hipGetLastError());
    });
}

}  // extern "C"
