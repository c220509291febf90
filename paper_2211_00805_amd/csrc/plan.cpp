// Plans and the host drivers of the hot path: heat application, Algorithm 1,
// its checkpointed reverse sweep, the barycenter iteration, the step-shape
// autotuner and hipGraph capture of whole iterations.
#include "plan.h"

#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <fstream>
#include <initializer_list>
#include <memory>
#include <sstream>
#include <thread>
#include <utility>

namespace gs {

namespace {

std::string phi_tag(float phi) {
    char b[32];
    std::snprintf(b, sizeof(b), ":%a", (double)phi);
    return b;
}

int pad_ld(int B) { return B == 1 ? 1 : ((B + 3) / 4) * 4; }

float* T(gs_plan_s& P, int j) { return (j % 2) ? P.U.p : P.V.p; }

StepArgs base_args(gs_plan_s& P) {
    StepArgs a{};
    a.rowptr = P.g->rowptr.p;
    a.col = P.g->col.p;
    a.val = P.g->val.p;
    a.n = (int32_t)P.n;
    a.ldp = P.ldp;
    a.coef = P.coef.p;
    a.K = P.K;
    a.acc = P.ACC.p;
    a.acc2 = P.ACC2.p;
    a.nfloor = P.count_floors ? P.nfloor.p : nullptr;
    a.long_thr = P.nlong > 0 ? P.long_thr : 0;
    a.nlong = P.nlong;
    a.long_rows = P.long_rows.p;
    return a;
}

// Run `body` on `st` directly, or capture it once into a hipGraph (on the
// plan's private stream) and replay the graph on `st`.
template <class F>
void run_graph(gs_plan_s& P, const std::string& key, hipStream_t st, F&& body) {
    if (P.flags & GS_PLAN_NO_GRAPH) {
        body(st);
        GS_HIP(hipGetLastError());
        return;
    }
    const std::string full = (P.kernel == GS_KERNEL_EULER
                                  ? key + ":E" + std::to_string(P.euler_N) + "." + std::to_string(P.cg_m)
                                  : key) +
                             (P.count_floors ? ":F" : "") + (P.frontier ? ":R" : "");
    auto it = P.graphs.find(full);
    if (it == P.graphs.end()) {
        GS_HIP(hipStreamBeginCapture(P.cap, hipStreamCaptureModeThreadLocal));
        try {
            body(P.cap);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(P.cap, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        hipGraph_t g = nullptr;
        GS_HIP(hipStreamEndCapture(P.cap, &g));
        GS_HIP(hipGetLastError());
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            fail(GS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        P.graph_defs[full] = g;
        it = P.graphs.emplace(full, ex).first;
    }
    GS_HIP(hipGraphLaunch(it->second, st));
}

std::string arch_name() {
    int dev = 0;
    GS_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    GS_HIP(hipGetDeviceProperties(&prop, dev));
    std::string a = prop.gcnArchName;
    const auto c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// --------------------------------------------------------------- tune cache (flat JSON object)
std::map<std::string, std::string> read_cache(const std::string& path) {
    std::map<std::string, std::string> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    while (true) {
        const size_t k0 = s.find('"', pos);
        if (k0 == std::string::npos) break;
        const size_t k1 = s.find('"', k0 + 1);
        const size_t v0 = s.find('"', k1 + 1);
        const size_t v1 = v0 == std::string::npos ? v0 : s.find('"', v0 + 1);
        if (k1 == std::string::npos || v1 == std::string::npos) break;
        m[s.substr(k0 + 1, k1 - k0 - 1)] = s.substr(v0 + 1, v1 - v0 - 1);
        pos = v1 + 1;
    }
    return m;
}

// Written to a private temporary file and renamed over the cache, so that
// processes or threads tuning at the same time never leave a mixed file
// (the last rename wins; a cache that cannot be written is not an error).
void write_cache(const std::string& path, const std::map<std::string, std::string>& m) {
    const std::string tmp = path + ".tmp." + std::to_string((long long)getpid()) + "." +
                            std::to_string(std::hash<std::thread::id>{}(std::this_thread::get_id()));
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return;
        f << "{\n";
        size_t i = 0;
        for (const auto& kv : m)
            f << "  \"" << kv.first << "\": \"" << kv.second << "\"" << (++i < m.size() ? ",\n" : "\n");
        f << "}\n";
        if (!f) {
            f.close();
            std::remove(tmp.c_str());
            return;
        }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

double tridiag_max_eig(const std::vector<double>& al, const std::vector<double>& be) {
    const int m = (int)al.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(be[i]) : 0.0);
        lo = std::min(lo, al[i] - r);
        hi = std::max(hi, al[i] + r);
    }
    auto count_below = [&](double x) {  // Sturm count of eigenvalues < x
        int c = 0;
        double d = 1.0;
        for (int i = 0; i < m; ++i) {
            d = al[i] - x - (i > 0 ? be[i - 1] * be[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++c;
        }
        return c;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_below(mid) >= m) hi = mid; else lo = mid;
    }
    return hi;
}

// Last component of the unit eigenvector of the tridiagonal T (diagonal al,
// off-diagonal be) for its largest eigenvalue theta, by inverse iteration with
// the shift sigma slightly above theta: T - sigma I is negative definite, so
// its LU factorisation without pivoting is stable.
double tridiag_last_component(const std::vector<double>& al, const std::vector<double>& be, double theta) {
    const int m = (int)al.size();
    if (m == 1) return 1.0;
    const double sigma = theta + 1e-12 * std::max(1.0, std::fabs(theta));
    std::vector<double> x(m, 1.0), d(m), c(m);
    for (int it = 0; it < 3; ++it) {
        // solve (T - sigma I) y = x (Thomas algorithm), then normalise
        d[0] = al[0] - sigma;
        c[0] = x[0];
        for (int i = 1; i < m; ++i) {
            const double l = be[i - 1] / d[i - 1];
            d[i] = al[i] - sigma - l * be[i - 1];
            c[i] = x[i] - l * c[i - 1];
        }
        x[m - 1] = c[m - 1] / d[m - 1];
        for (int i = m - 2; i >= 0; --i) x[i] = (c[i] - be[i] * x[i + 1]) / d[i];
        double nrm = 0.0;
        for (double v : x) nrm += v * v;
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) return 1.0;   // no estimate: the caller keeps safety * theta
        for (double& v : x) v /= nrm;
    }
    return x[m - 1];
}

}  // namespace

// Column lanes: the smallest power of two covering the row's float4 groups
// (at most 16; a short last tile or idle lanes when the groups are not a
// power of two), and S = 8 / C lanes over a row's nonzeros.
LaunchShape default_shape(int ldp, double nnz_per_row) {
    if (ldp == 1) return {1, nnz_per_row > 12.0 ? 16 : 8, 1, 1, 1};
    int C = 1;
    while (C < 16 && C < ldp / 4) C *= 2;
    int S = std::max(1, 8 / C);
    return {4, S, C, 1, 1};
}

}  // namespace gs

gs_plan_s::~gs_plan_s() {
    gs::drop_graphs(*this);
    if (cap) (void)hipStreamDestroy(cap);
}

namespace gs {

// Rows whose nonzeros exceed the shape's threshold are processed one block per
// row by the long-row blocks at the head of the step grid (a single row group
// would serialise them).
void update_long_rows(gs_plan_s& P) {
    const int thr = long_row_threshold(P.shape);
    std::vector<int32_t> rows;
    const auto& rp = P.g->h_rowptr;
    for (int64_t i = 0; i < P.n; ++i)
        if (rp[i + 1] - rp[i] > thr) rows.push_back((int32_t)i);
    P.long_thr = thr;
    P.nlong = (int)rows.size();
    if (P.nlong) {
        if (P.long_rows.count < rows.size()) P.long_rows.alloc(rows.size());
        GS_HIP(hipMemcpy(P.long_rows.p, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
}

void drop_graphs(gs_plan_s& P) {
    for (auto& kv : P.graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : P.graph_defs) (void)hipGraphDestroy(kv.second);
    P.graphs.clear();
    P.graph_defs.clear();
}

void set_coefs(gs_plan_s& P, double lambda_hat, double t, hipStream_t st) {
    std::vector<double> b(P.K + 1), db(P.K + 1);
    cheby_coeffs(t, P.K, b.data(), db.data());
    launch_set_coef(P.coef.p, 2.0 / lambda_hat, b.data(), db.data(), P.K, st);
    if (P.kernel == GS_KERNEL_EULER) {
        // operator scale -c, c = (t/N)(2/lambda_hat): one first step yields -(I + c L) p
        launch_fill(P.ecoef.p, (float)(-(t / P.euler_N) * (2.0 / lambda_hat)), 1, st);
        P.cg_m = P.cg_iters > 0 ? P.cg_iters : euler_cg_iterations(t, P.euler_N);
    }
}

// Conjugate-gradient iterations per backward-Euler solve: with L_op's
// spectrum in [0, 2], (I + (t/N) L_op) has condition number kappa <= 1 + 2t/N,
// and after m iterations from x = 0 the error is at most
// 2 sqrt(kappa) ((sqrt(kappa) - 1)/(sqrt(kappa) + 1))^m ||b||_2.  CG from zero
// is a degree-m polynomial in the system matrix, so a solve reaches m hops;
// the exact kernel is positive on every node, and Algorithm 1 takes logarithms
// of its small entries, so m is the smallest count that brings the bound below
// 2^-52 (well under float32 resolution), not merely below float32 resolution.
int euler_cg_iterations(double t, int N) {
    const double sk = std::sqrt(1.0 + 2.0 * t / N);
    const double rho = (sk - 1.0) / (sk + 1.0);
    if (!(rho > 0.0)) return 1;
    const double m = std::log(2.0 * sk / 0x1p-52) / std::log(1.0 / rho);
    return std::max(1, (int)std::ceil(m));
}

void set_kernel(gs_plan_s& P, int kernel, int N, int cg_iters) {
    drop_graphs(P);
    P.kernel = kernel;
    P.euler_N = kernel == GS_KERNEL_EULER ? N : 0;
    P.cg_iters = kernel == GS_KERNEL_EULER ? cg_iters : 0;
    P.cg_m = P.cg_iters;
    if (kernel == GS_KERNEL_EULER && !P.er.p) {
        for (auto* b : {&P.er, &P.ep, &P.eq}) b->alloc(P.sz());
        P.ecoef.alloc(2 * (GS_MAX_K + 1) + 1);
        P.ers.alloc((3 + (size_t)kMaxCgBlocks) * P.ldp);
        for (auto* b : {&P.er, &P.ep, &P.eq}) launch_fill(b->p, 0.f, P.sz(), P.cap);
        launch_fill(P.ecoef.p, 0.f, P.ecoef.count, P.cap);
        GS_HIP(hipStreamSynchronize(P.cap));
    }
}

// Flush the accumulator on steps 2, 5, 8, ... and on the last step; a flush
// adds every term since the previous flush (at most T_{k-2}, T_{k-1}, T_k, all
// of which the step holds).
StepSched step_sched_at(int K, int k, ApplyMode mode) {
    auto flushes = [K](int j) { return j == K || (j >= 2 && (j - 2) % 3 == 0); };
    int f = 0, m = 0;
    if (k == 1) f |= STEP_FIRST;
    if (mode == ApplyMode::Dual) f |= STEP_DUAL;
    const bool final = k == K;
    if (flushes(k)) {
        int last = -1;  // highest term index already in the accumulator
        for (int j = 2; j < k; ++j)
            if (flushes(j)) last = j;
        for (int idx = last + 1; idx <= k; ++idx) m |= idx == k - 2 ? 1 : idx == k - 1 ? 2 : 4;
        if (last >= 0) f |= STEP_ACC_READ;
        f |= (final && mode == ApplyMode::Scale) ? STEP_EPI_SCALE : STEP_ACC_WRITE;
    }
    if (!final) f |= STEP_WRITE_T;
    return {f, m};
}

std::vector<StepSched> step_schedule(int K, ApplyMode mode) {
    std::vector<StepSched> out(K);
    for (int k = 1; k <= K; ++k) out[k - 1] = step_sched_at(K, k, mode);
    return out;
}

std::vector<StepSched> clenshaw_schedule(int K, ApplyMode mode) {
    // Product j = 1..K of Clenshaw's recurrence: j = 1 gathers X itself, u_{K-j+2}
    // is read from memory from j = 3 on (j = 2 folds u_K = b_K X into its X
    // coefficient), and the last product writes the result (or scales).
    std::vector<StepSched> out(K);
    for (int j = 1; j <= K; ++j) {
        int f = STEP_CLENSHAW;
        if (j == 1) f |= STEP_FIRST;
        if (j >= 3) f |= STEP_CLEN_P2;
        if (j < K) f |= STEP_WRITE_T;
        else f |= mode == ApplyMode::Scale ? STEP_EPI_SCALE : STEP_ACC_WRITE;
        out[j - 1] = {f, 0};
    }
    return out;
}

double step_bytes(const gs_plan_s& P, const StepSched& sc, bool has_out_a, bool has_rec) {
    const double nb = 4.0 * (double)P.n * P.B;
    const double acc = (sc.flags & STEP_DUAL) ? 2.0 : 1.0;
    double b = 4.0 * (P.n + 1) + 8.0 * P.g->nnz + nb;  // CSR once, T_{k-1} once
    if (sc.flags & STEP_CLENSHAW) {
        b += nb;                                      // X
        if (sc.flags & STEP_CLEN_P2) b += nb;         // u_{k+2}
        if (sc.flags & STEP_WRITE_T) b += nb;         // u_k
        if (sc.flags & STEP_ACC_WRITE) b += nb;       // result
        if (sc.flags & STEP_EPI_SCALE) b += 2.0 * nb + (has_out_a ? nb : 0.0) + (has_rec ? nb : 0.0);
        return b;
    }
    if (!(sc.flags & STEP_FIRST)) b += nb;
    if (sc.flags & STEP_WRITE_T) b += nb;
    if (sc.flags & STEP_ACC_READ) b += acc * nb;
    if (sc.flags & STEP_ACC_WRITE) b += acc * nb;
    if (sc.flags & STEP_EPI_SCALE) b += 2.0 * nb + (has_out_a ? nb : 0.0) + (has_rec ? nb : 0.0);
    return b;
}

namespace {

void enqueue_cheb_apply(gs_plan_s& P, const float* X, ApplyMode mode, const ScaleEpi& epi, float phi,
                        hipStream_t st, Levels lev = Levels{}) {
    StepArgs base = base_args(P);
    base.level = lev.row;
    base.blk_level = lev.blk;
    if (lev.row) {
        // frontier: zeros in the T and accumulator buffers let blocks beyond
        // the frontier leave at once on every step but the last
        launch_zero_buffers(P.U.p, P.V.p, P.ACC.p, mode == ApplyMode::Dual ? P.ACC2.p : nullptr, (int64_t)P.sz(),
                            st);
    }
    const std::vector<StepSched> sched = step_schedule(P.K, mode);
    for (int k = 1; k <= P.K; ++k) {
        StepArgs a = base;
        a.k = k;
        a.skip_dead = lev.row && k < P.K && !(sched[k - 1].flags & STEP_EPI_SCALE) ? 1 : 0;
        a.tprev = k == 1 ? X : T(P, k - 1);
        a.tprev2 = k >= 2 ? (k == 2 ? X : T(P, k - 2)) : nullptr;
        a.tout = T(P, k);
        a.phi = phi;
        a.flags = sched[k - 1].flags;
        a.cmask = sched[k - 1].cmask;
        if (a.flags & STEP_EPI_SCALE) {
            a.num = epi.num;
            a.out = epi.out;
            a.out_a = epi.out_a;
            a.a = epi.a;
            a.rec = epi.rec;
        }
        launch_step(P.shape, a, st);
    }
}

// p_K X by Clenshaw's recurrence into ACC (or scaled into epi.out); u_k
// rotates through U and V like T_k, written over u_{k+2} in place.
void enqueue_clenshaw_apply(gs_plan_s& P, const float* X, ApplyMode mode, const ScaleEpi& epi, float phi,
                            hipStream_t st, Levels lev = Levels{}) {
    StepArgs base = base_args(P);
    base.level = lev.row;
    base.blk_level = lev.blk;
    if (lev.row) launch_zero_buffers(P.U.p, P.V.p, P.ACC.p, nullptr, (int64_t)P.sz(), st);   // as above
    const std::vector<StepSched> sched = clenshaw_schedule(P.K, mode);
    for (int j = 1; j <= P.K; ++j) {
        StepArgs a = base;
        a.k = j;
        a.skip_dead = lev.row && j < P.K && !(sched[j - 1].flags & STEP_EPI_SCALE) ? 1 : 0;
        a.tprev = j == 1 ? X : T(P, j - 1);
        a.tprev2 = j >= 3 ? T(P, j - 2) : nullptr;
        a.tout = T(P, j);
        a.xin = X;
        a.phi = phi;
        a.flags = sched[j - 1].flags;
        a.cmask = 0;
        if (a.flags & STEP_EPI_SCALE) {
            a.num = epi.num;
            a.out = epi.out;
            a.out_a = epi.out_a;
            a.a = epi.a;
            a.rec = epi.rec;
        }
        launch_step(P.shape, a, st);
    }
}

// (I + c L)^{-N} X into ACC: N solves, each cg_m CG iterations from x = 0 on
// all columns; the right-hand side of a solve is the previous solution.
void enqueue_euler_apply(gs_plan_s& P, const float* X, ApplyMode mode, const ScaleEpi& epi, float phi,
                         hipStream_t st) {
    if (mode == ApplyMode::Dual) fail(GS_ERR_INVALID, "the backward-Euler kernel has no time-derivative form");
    StepArgs mv = base_args(P);
    mv.coef = P.ecoef.p;
    mv.k = 1;
    mv.flags = STEP_FIRST | STEP_WRITE_T;
    mv.cmask = 0;
    mv.tprev = P.ep.p;
    mv.tprev2 = nullptr;
    mv.tout = P.eq.p;
    const int64_t total = P.n * (int64_t)P.ldp;
    double* rr[2] = {P.ers.p, P.ers.p + P.ldp};
    double* pq = P.ers.p + 2 * P.ldp;
    double* part = P.ers.p + 3 * P.ldp;
    const float* rhs = X;
    for (int s = 0; s < P.euler_N; ++s) {
        launch_cg_init(rhs, P.ACC.p, P.er.p, P.ep.p, total, st);
        launch_cg_dot(P.er.p, P.er.p, P.n, P.ldp, part, rr[0], st);
        int cur = 0;
        for (int it = 0; it < P.cg_m; ++it) {
            launch_step(P.shape, mv, st);
            launch_cg_dot(P.ep.p, P.eq.p, P.n, P.ldp, part, pq, st);
            launch_cg_update(P.ACC.p, P.er.p, P.ep.p, P.eq.p, rr[cur], pq, P.n, P.ldp, part, rr[1 - cur], st);
            if (it + 1 < P.cg_m) {
                launch_cg_dir(P.er.p, P.ep.p, rr[cur], rr[1 - cur], total, P.ldp, st);
                cur = 1 - cur;
            }
        }
        rhs = P.ACC.p;
    }
    if (mode == ApplyMode::Scale)
        launch_scale_epilogue(P.ACC.p, epi.num, epi.out, epi.out_a, epi.a, epi.rec, phi,
                              P.count_floors ? P.nfloor.p : nullptr, P.n, P.ldp, st);
}

}  // namespace

// `lev`: frontier levels of a superset of supp(X), set up by enqueue_levels
// (row == nullptr: dense steps); the results are the dense ones bit for bit.
void enqueue_apply(gs_plan_s& P, const float* X, ApplyMode mode, const ScaleEpi& epi, float phi, hipStream_t st,
                   Levels lev) {
    if (P.kernel == GS_KERNEL_EULER)
        enqueue_euler_apply(P, X, mode, epi, phi, st);
    else if (P.kernel == GS_KERNEL_CLENSHAW && mode != ApplyMode::Dual)
        enqueue_clenshaw_apply(P, X, mode, epi, phi, st, lev);   // the dual form needs the accumulators
    else
        enqueue_cheb_apply(P, X, mode, epi, phi, st, lev);
}

void set_frontier(gs_plan_s& P, int enable) {
    // the buffers first: a failed allocation leaves the option off
    if (enable && !P.lev_flags.p) {
        const size_t nr = P.n ? (size_t)P.n : 1;
        const size_t nb = nr / 4 + 1;   // row blocks of the smallest shape (4 rows)
        P.lev_mu.alloc(nr);
        P.lev_nu.alloc(nr);
        P.blk_mu.alloc(nb);
        P.blk_nu.alloc(nb);
        P.lev_flags.alloc(GS_MAX_K + 1);
    }
    P.frontier = enable;
}

namespace {

// Frontier steps apply to the polynomial kernels (the conjugate-gradient
// solves of the Euler kernel have no step index to compare a level with).
bool frontier_on(const gs_plan_s& P) { return P.frontier && P.kernel != GS_KERNEL_EULER; }

// Hop levels of supp(h) (rows where any of the B columns is nonzero), exact up
// to K hops, with row blocks of the plan's launch shape.
void enqueue_levels(gs_plan_s& P, const float* h, Levels lev, hipStream_t st) {
    const int rpb = 4 * (64 / (P.shape.S * P.shape.C));
    launch_support_levels(h, P.n, P.ldp, P.B, P.g->rowptr.p, P.g->col.p, P.K, rpb, lev.row, lev.blk,
                          P.lev_flags.p, st);
}

Levels levels_mu(gs_plan_s& P) { return {P.lev_mu.p, P.blk_mu.p}; }
Levels levels_nu(gs_plan_s& P) { return {P.lev_nu.p, P.blk_nu.p}; }

}  // namespace

// Average duration (ms) of one step launch over `reps` whole applications of
// p_K (the accumulator form, or Clenshaw's when the plan selects it), and
// the average algorithmic bytes of a launch.
double time_step(gs_plan_s& P, const LaunchShape& shape, int reps, hipStream_t st, double* bytes_per_launch) {
    const LaunchShape saved = P.shape;
    P.shape = shape;
    if (!(shape == saved) || P.long_thr == 0) update_long_rows(P);
    const bool clen = P.kernel == GS_KERNEL_CLENSHAW;
    auto apply = [&] {
        if (clen)
            enqueue_clenshaw_apply(P, P.X.p, ApplyMode::Store, ScaleEpi{}, 0.f, st);
        else
            enqueue_cheb_apply(P, P.X.p, ApplyMode::Store, ScaleEpi{}, 0.f, st);
    };
    apply();
    hipEvent_t e0, e1;
    GS_HIP(hipEventCreate(&e0));
    GS_HIP(hipEventCreate(&e1));
    GS_HIP(hipEventRecord(e0, st));
    for (int i = 0; i < reps; ++i) apply();
    GS_HIP(hipEventRecord(e1, st));
    GS_HIP(hipEventSynchronize(e1));
    if (!(shape == saved)) {
        P.shape = saved;
        update_long_rows(P);
    }
    float ms = 0.f;
    GS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    GS_HIP(hipGetLastError());
    if (bytes_per_launch) {
        double tot = 0.0;
        for (const auto& sc : clen ? clenshaw_schedule(P.K, ApplyMode::Store) : step_schedule(P.K, ApplyMode::Store))
            tot += step_bytes(P, sc, false, false);
        *bytes_per_launch = tot / P.K;
    }
    return (double)ms / ((double)reps * P.K);
}

gs_plan_s* plan_create(gs_graph g, int K, int B, int flags, const char* tune_cache) {
    auto P = std::make_unique<gs_plan_s>();
    P->g = g;
    P->K = K;
    P->B = B;
    P->ldp = pad_ld(B);
    P->n = g->n;
    P->flags = flags;
    const size_t sz = P->sz();
    for (auto* b : {&P->X, &P->U, &P->V, &P->ACC, &P->mu, &P->nu, &P->v, &P->w}) b->alloc(sz);
    P->coef.alloc(2 * (GS_MAX_K + 1) + 1);
    P->partials.alloc((size_t)reduce_blocks(P->n) * P->ldp);
    P->red.alloc(P->ldp);
    P->nfloor.alloc(1);
    P->badin.alloc(2);
    GS_HIP(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
    for (auto* b : {&P->X, &P->U, &P->V, &P->ACC, &P->mu, &P->nu, &P->v, &P->w}) launch_fill(b->p, 0.f, sz, P->cap);
    {
        std::vector<double> b0(K + 1, 0.0);
        launch_set_coef(P->coef.p, 1.0, b0.data(), b0.data(), K, P->cap);
    }
    GS_HIP(hipStreamSynchronize(P->cap));

    const double npr = g->n ? (double)g->nnz / (double)g->n : 0.0;
    P->shape = default_shape(P->ldp, npr);
    P->shape_origin = "default";
    if (flags & GS_PLAN_AUTOTUNE) {
        const std::string key = arch_name() + ":n=" + std::to_string(P->n) + ":nnz=" + std::to_string(g->nnz) +
                                ":B=" + std::to_string(B);
        std::map<std::string, std::string> cache;
        if (tune_cache) cache = read_cache(tune_cache);
        const auto hit = cache.find(key);
        int vv = 0, ss = 0, cc = 0, rr = 1, nt = 1;   // entries without the fifth field: streamed CSR
        const int got = hit != cache.end()
                            ? std::sscanf(hit->second.c_str(), "%d,%d,%d,%d,%d", &vv, &ss, &cc, &rr, &nt) : 0;
        if (got >= 4 && shape_supported({vv, ss, cc, rr, nt}) && column_lanes_ok(P->ldp, vv, cc) &&
            (vv == 1) == (P->ldp == 1) && (nt == 0 || nt == 1)) {
            P->shape = {vv, ss, cc, rr, nt};
            P->shape_origin = "cache";
        } else {
            hipStream_t st = P->cap;
            launch_fill(P->U.p, 0.5f, sz, st);
            launch_fill(P->V.p, 0.25f, sz, st);
            launch_fill(P->ACC.p, 0.f, sz, st);
            std::vector<double> b(K + 1, 0.01), db(K + 1, 0.0);
            launch_set_coef(P->coef.p, 0.1, b.data(), db.data(), K, st);
            double best = 1e300;
            for (const auto& s : candidate_shapes(P->ldp)) {
                const double ms = time_step(*P, s, 2, st, nullptr);
                if (ms < best) {
                    best = ms;
                    P->shape = s;
                }
            }
            P->shape_origin = "autotuned";
            if (tune_cache) {
                cache[key] = std::to_string(P->shape.vec) + "," + std::to_string(P->shape.S) + "," +
                             std::to_string(P->shape.C) + "," + std::to_string(P->shape.remap) + "," +
                             std::to_string(P->shape.csr_nt);
                write_cache(tune_cache, cache);
            }
        }
    }
    update_long_rows(*P);
    return P.release();
}

// ------------------------------------------------------------------ heat apply
void heat_apply(gs_plan_s& P, double lam, double t, const float* X, float* Y, float* Ydt, hipStream_t st) {
    const bool dual = Ydt != nullptr;
    P.count_floors = false;
    if (dual && !P.ACC2.p) P.ACC2.alloc(P.sz());
    set_coefs(P, lam, t, st);
    launch_copy_ld(X, P.B, P.X.p, P.ldp, P.n, P.B, st);
    const bool fr = frontier_on(P);
    run_graph(P, dual ? "heat:dual" : "heat", st, [&](hipStream_t s) {
        if (fr) enqueue_levels(P, P.X.p, levels_mu(P), s);
        enqueue_apply(P, P.X.p, dual ? ApplyMode::Dual : ApplyMode::Store, ScaleEpi{}, 0.f, s,
                      fr ? levels_mu(P) : Levels{});
    });
    launch_copy_ld(P.ACC.p, P.ldp, Y, P.B, P.n, P.B, st);
    if (dual) launch_copy_ld(P.ACC2.p, P.ldp, Ydt, P.B, P.n, P.B, st);
    GS_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ Algorithm 1
namespace {

void load_inputs(gs_plan_s& P, const float* a, const float* mu, const float* nu, hipStream_t st) {
    launch_copy_ld(mu, P.B, P.mu.p, P.ldp, P.n, P.B, st);
    if (nu) launch_copy_ld(nu, P.B, P.nu.p, P.ldp, P.n, P.B, st);
    if (a) {
        if (!P.a.p) {
            P.a.alloc(P.n);
            P.xv.alloc(P.sz());
            P.xw.alloc(P.sz());
        }
        GS_HIP(hipMemcpyAsync(P.a.p, a, P.n * sizeof(float), hipMemcpyDeviceToDevice, st));
    }
}

// One Sinkhorn iteration: v = mu / floor(p_K(a w)), w = nu / floor(p_K(a v)).
// lev_w, lev_v: hop levels of supersets of supp(a w) and supp(a v) for
// frontier steps, or nullptr.
void enqueue_iteration(gs_plan_s& P, bool has_a, float phi, float* rec_d, float* rec_e, hipStream_t s,
                       Levels lev_w = Levels{}, Levels lev_v = Levels{}) {
    ScaleEpi e1{P.mu.p, P.v.p, has_a ? P.xv.p : nullptr, has_a ? P.a.p : nullptr, rec_d};
    enqueue_apply(P, has_a ? P.xw.p : P.w.p, ApplyMode::Scale, e1, phi, s, lev_w);
    ScaleEpi e2{P.nu.p, P.w.p, has_a ? P.xw.p : nullptr, has_a ? P.a.p : nullptr, rec_e};
    enqueue_apply(P, has_a ? P.xv.p : P.v.p, ApplyMode::Scale, e2, phi, s, lev_v);
}

void reduce_to_host(gs_plan_s& P, const ReduceArgs& r, double scale, double* host, hipStream_t st) {
    launch_reduce(r, P.partials.p, reduce_blocks(P.n), P.red.p, 0, scale, st);
    GS_HIP(hipMemcpyAsync(host, P.red.p, P.B * sizeof(double), hipMemcpyDeviceToHost, st));
}

ReduceArgs red_args(gs_plan_s& P, int op, const float* x0, const float* x1, const float* x2, const float* x3,
                    const float* a) {
    ReduceArgs r{};
    r.op = op;
    r.n = P.n;
    r.ldp = P.ldp;
    r.B = P.B;
    r.x0 = x0;
    r.x1 = x1;
    r.x2 = x2;
    r.x3 = x3;
    r.a = a;
    return r;
}

}  // namespace

namespace {

// Captured record-mode graphs hold the record buffer's slot addresses: a call
// with another buffer drops them.
void use_record_buffer(gs_plan_s& P, const float* rec) {
    if (P.rec_buf != rec) {
        drop_graphs(P);
        P.rec_buf = rec;
    }
}

// Inputs that must be finite and >= 0 are counted on the device when the call
// starts; the counts are read back where the call synchronises.
void count_invalid_inputs(gs_plan_s& P, std::initializer_list<std::pair<const float*, size_t>> arrays,
                          hipStream_t st) {
    GS_HIP(hipMemsetAsync(P.badin.p, 0, 2 * sizeof(unsigned long long), st));
    for (const auto& a : arrays)
        if (a.first) launch_count_invalid(a.first, (int64_t)a.second, P.badin.p, st);
}

// Host results of a call: a non-finite entry fails the call (after the
// input checks, which explain most of them).
void require_finite(const double* x, int count, const char* what) {
    for (int b = 0; b < count; ++b)
        if (!std::isfinite(x[b]))
            fail(GS_ERR_NONFINITE, std::string(what) + " of column " + std::to_string(b) + " is not finite");
}

void report_invalid_inputs(const unsigned long long* bad, const char* what) {
    if (bad[0]) fail(GS_ERR_NONFINITE, std::string(what) + " hold " + std::to_string(bad[0]) + " non-finite entries");
    if (bad[1]) fail(GS_ERR_INVALID, std::string(what) + " hold " + std::to_string(bad[1]) + " negative entries");
}

}  // namespace

void sinkhorn(gs_plan_s& P, double lam, double t, const float* a, const float* mu, const float* nu, int J, float phi,
              int C, float* ckpt, float* v, float* w, double* dist, double* marg, int64_t* nfl, hipStream_t st) {
    const bool has_a = a != nullptr;
    P.count_floors = nfl != nullptr;
    set_coefs(P, lam, t, st);
    const size_t nB = (size_t)P.n * P.B;
    count_invalid_inputs(P, {{mu, nB}, {nu, nB}, {a, (size_t)P.n}}, st);
    load_inputs(P, a, mu, nu, st);
    launch_fill(P.w.p, 1.f, P.sz(), st);
    if (has_a) launch_mul_a(P.w.p, P.a.p, P.n, P.ldp, P.xw.p, st);
    GS_HIP(hipMemsetAsync(P.nfloor.p, 0, sizeof(unsigned long long), st));
    // frontier steps: a v lies on supp(mu), and a w on supp(nu) once the first
    // iteration has replaced w = 1 (the quotients vanish with their numerators)
    const bool fr = frontier_on(P);
    if (fr) {
        enqueue_levels(P, P.mu.p, levels_mu(P), st);
        enqueue_levels(P, P.nu.p, levels_nu(P), st);
    }
    const Levels lev_v = fr ? levels_mu(P) : Levels{};
    auto lev_w = [&](int j) { return fr && j > 0 ? levels_nu(P) : Levels{}; };
    const std::string key = std::string("fwd:") + (has_a ? "a" : "1") + phi_tag(phi);
    if (ckpt && C == GS_RECORD_ALL) {
        // every iteration's floored denominators d_j, e_j into slots 2j, 2j+1
        // (graphs per chunk of iterations: the slot addresses are baked in)
        use_record_buffer(P, ckpt);
        const size_t sz = P.sz();
        for (int j0 = 0; j0 < J; j0 += kRecordChunk) {
            const int ns = std::min(kRecordChunk, J - j0);
            run_graph(P, "fwdrec:" + std::to_string(j0) + ":" + std::to_string(ns) + ":" + key, st,
                      [&](hipStream_t s) {
                          for (int j = j0; j < j0 + ns; ++j)
                              enqueue_iteration(P, has_a, phi, ckpt + 2 * (size_t)j * sz,
                                                ckpt + (2 * (size_t)j + 1) * sz, s, lev_w(j), lev_v);
                      });
        }
    } else {
        for (int j = 0; j < J; ++j) {
            if (ckpt && j % C == 0)
                launch_copy_ld(P.w.p, P.ldp, ckpt + (size_t)(j / C) * P.n * P.B, P.B, P.n, P.B, st);
            run_graph(P, fr && j == 0 ? key + ":first" : key, st, [&](hipStream_t s) {
                enqueue_iteration(P, has_a, phi, nullptr, nullptr, s, lev_w(j), lev_v);
            });
        }
    }
    const float* ap = has_a ? P.a.p : nullptr;
    if (dist) reduce_to_host(P, red_args(P, RED_DIST, P.mu.p, P.v.p, P.nu.p, P.w.p, ap), 4.0 * t, dist, st);
    if (marg) {
        const std::string mkey = std::string("marg:") + (has_a ? "a" : "1") + phi_tag(phi);
        run_graph(P, mkey, st, [&](hipStream_t s) {
            enqueue_apply(P, has_a ? P.xw.p : P.w.p, ApplyMode::Store, ScaleEpi{}, phi, s, lev_w(J));
        });
        reduce_to_host(P, red_args(P, RED_MARG, P.v.p, P.ACC.p, P.mu.p, nullptr, ap), 1.0, marg, st);
    }
    if (v) launch_copy_ld(P.v.p, P.ldp, v, P.B, P.n, P.B, st);
    if (w) launch_copy_ld(P.w.p, P.ldp, w, P.B, P.n, P.B, st);
    unsigned long long nf = 0, bad[2] = {0, 0};
    if (nfl) GS_HIP(hipMemcpyAsync(&nf, P.nfloor.p, sizeof(nf), hipMemcpyDeviceToHost, st));
    GS_HIP(hipGetLastError());
    if (dist || marg || nfl) {
        GS_HIP(hipMemcpyAsync(bad, P.badin.p, sizeof(bad), hipMemcpyDeviceToHost, st));
        GS_HIP(hipStreamSynchronize(st));
        report_invalid_inputs(bad, "mu / nu / a");
        if (nfl) *nfl = (int64_t)nf;
        if (dist) require_finite(dist, P.B, "distance");
        if (marg) require_finite(marg, P.B, "marginal error");
    }
}

// ------------------------------------------------------------------ reverse sweep
void sinkhorn_backward(gs_plan_s& P, double lam, double t, const float* a, const float* mu, const float* nu, int J,
                       float phi, int C, const float* ckpt, const double* gd, float* gmu, float* gnu, double* gt,
                       hipStream_t st) {
    const bool has_a = a != nullptr;
    P.count_floors = false;
    const size_t sz = P.sz();
    if (!P.ACC2.p) P.ACC2.alloc(sz);
    if (P.seg_cap < C) {
        // captured segment graphs hold the old slot addresses: drop them
        // before the buffers move
        drop_graphs(P);
        P.segd.alloc(sz * C);
        P.sege.alloc(sz * C);
        P.seg_cap = C;
    }
    if (!P.dmu.p) {
        for (auto* b : {&P.dmu, &P.dnu, &P.vseed, &P.wbar, &P.wck}) b->alloc(sz);
        P.g4t.alloc(P.ldp);
        P.tbar.alloc(P.ldp);
    }
    set_coefs(P, lam, t, st);
    count_invalid_inputs(P, {{mu, (size_t)P.n * P.B}, {nu, (size_t)P.n * P.B}, {a, (size_t)P.n}}, st);
    load_inputs(P, a, mu, nu, st);
    std::vector<float> g4(P.ldp, 0.f);
    for (int b = 0; b < P.B; ++b) g4[b] = (float)(4.0 * t * gd[b]);
    GS_HIP(hipMemcpyAsync(P.g4t.p, g4.data(), P.ldp * sizeof(float), hipMemcpyHostToDevice, st));
    GS_HIP(hipMemsetAsync(P.tbar.p, 0, P.ldp * sizeof(double), st));
    GS_HIP(hipMemsetAsync(P.nfloor.p, 0, sizeof(unsigned long long), st));
    const float* ap = has_a ? P.a.p : nullptr;
    const int nblk = reduce_blocks(P.n);
    std::vector<double> D(P.B, 0.0);

    // The derivative in t needs the second accumulator (dual steps) and two
    // reductions per iteration; without grad_t the adjoint applications are
    // plain ones, whose first accumulator is bitwise the dual form's.
    const bool want_t = gt != nullptr;
    const ApplyMode adj_mode = want_t ? ApplyMode::Dual : ApplyMode::Store;
    const std::string ttag = want_t ? ":t" : ":nt";

    // One reverse iteration j from its denominators d_j, e_j (w_j = nu / e_j,
    // v_j = mu / d_j); e_prev = e_{j-1} or NULL for j = 0 (w^0 = 1), w_prev =
    // the stored w^j instead of nu / e_{j-1} when given.
    auto reverse_iteration = [&](const float* dj, const float* ej, const float* e_prev, const float* w_prev,
                                 hipStream_t q) {
        launch_bwd_e(P.wbar.p, ej, P.nu.p, P.n, P.ldp, phi, P.dnu.p, P.X.p, q);
        enqueue_apply(P, P.X.p, adj_mode, ScaleEpi{}, phi, q);
        if (want_t)
            launch_reduce(red_args(P, RED_DOT_QUOT, P.ACC2.p, P.mu.p, dj, nullptr, ap), P.partials.p, nblk, P.tbar.p,
                          1, 1.0, q);
        launch_bwd_d(P.ACC.p, P.vseed.p, dj, P.mu.p, ap, P.n, P.ldp, phi, P.dmu.p, P.X.p, q);
        enqueue_apply(P, P.X.p, adj_mode, ScaleEpi{}, phi, q);
        if (want_t && e_prev)
            launch_reduce(red_args(P, RED_DOT_QUOT, P.ACC2.p, P.nu.p, e_prev, nullptr, ap), P.partials.p, nblk,
                          P.tbar.p, 1, 1.0, q);
        else if (want_t)
            launch_reduce(red_args(P, RED_DOT, P.ACC2.p, w_prev, nullptr, nullptr, ap), P.partials.p, nblk, P.tbar.p,
                          1, 1.0, q);
        launch_bwd_w(P.ACC.p, ap, P.n, P.ldp, P.wbar.p, q);
    };

    if (C == GS_RECORD_ALL) {
        // no recomputation: the forward recorded every d_j, e_j; the final
        // v = mu / d_{J-1}, w = nu / e_{J-1} are rebuilt bitwise from them
        use_record_buffer(P, ckpt);
        const float* rec = ckpt;
        launch_scale_epilogue(rec + 2 * (size_t)(J - 1) * sz, P.mu.p, P.v.p, nullptr, nullptr, nullptr, phi,
                              nullptr, P.n, P.ldp, st);
        launch_scale_epilogue(rec + (2 * (size_t)(J - 1) + 1) * sz, P.nu.p, P.w.p, nullptr, nullptr, nullptr, phi,
                              nullptr, P.n, P.ldp, st);
        if (want_t)
            reduce_to_host(P, red_args(P, RED_DIST, P.mu.p, P.v.p, P.nu.p, P.w.p, ap), 4.0 * t, D.data(), st);
        launch_bwd_seed(P.mu.p, P.nu.p, P.v.p, P.w.p, ap, P.g4t.p, P.n, P.ldp, P.dmu.p, P.dnu.p, P.vseed.p, P.wbar.p,
                        st);
        const std::string tag = std::string(has_a ? ":a" : ":1") + phi_tag(phi) + ttag;
        for (int j0 = ((J - 1) / kRecordChunk) * kRecordChunk; j0 >= 0; j0 -= kRecordChunk) {
            const int ns = std::min(kRecordChunk, J - j0);
            run_graph(P, "adjrec:" + std::to_string(j0) + ":" + std::to_string(ns) + tag, st, [&](hipStream_t q) {
                for (int j = j0 + ns - 1; j >= j0; --j) {
                    const float* dj = rec + 2 * (size_t)j * sz;
                    reverse_iteration(dj, dj + sz, j > 0 ? dj - sz : nullptr, nullptr, q);
                }
            });
        }
    }
    const int nseg = C == GS_RECORD_ALL ? 0 : (J + C - 1) / C;
    for (int s = nseg - 1; s >= 0; --s) {
        const int j0 = s * C;
        const int ns = std::min(J, j0 + C) - j0;
        launch_copy_ld(ckpt + (size_t)s * P.n * P.B, P.B, P.wck.p, P.ldp, P.n, P.B, st);
        GS_HIP(hipMemcpyAsync(P.w.p, P.wck.p, sz * sizeof(float), hipMemcpyDeviceToDevice, st));
        if (has_a) launch_mul_a(P.w.p, P.a.p, P.n, P.ldp, P.xw.p, st);
        const std::string tag = std::to_string(ns) + (has_a ? ":a" : ":1") + phi_tag(phi);
        run_graph(P, "rec:" + tag, st, [&](hipStream_t q) {
            for (int slot = 0; slot < ns; ++slot)
                enqueue_iteration(P, has_a, phi, P.segd.p + slot * sz, P.sege.p + slot * sz, q);
        });
        if (s == nseg - 1) {
            if (want_t)
                reduce_to_host(P, red_args(P, RED_DIST, P.mu.p, P.v.p, P.nu.p, P.w.p, ap), 4.0 * t, D.data(), st);
            launch_bwd_seed(P.mu.p, P.nu.p, P.v.p, P.w.p, ap, P.g4t.p, P.n, P.ldp, P.dmu.p, P.dnu.p, P.vseed.p,
                            P.wbar.p, st);
        }
        run_graph(P, "adj:" + tag + ttag, st, [&](hipStream_t q) {
            for (int slot = ns - 1; slot >= 0; --slot) {
                const float* dj = P.segd.p + slot * sz;
                const float* ej = P.sege.p + slot * sz;
                reverse_iteration(dj, ej, slot > 0 ? ej - sz : nullptr, P.wck.p, q);
            }
        });
    }
    launch_mask_support(P.mu.p, P.n, P.ldp, P.dmu.p, st);
    launch_mask_support(P.nu.p, P.n, P.ldp, P.dnu.p, st);
    if (gmu) launch_copy_ld(P.dmu.p, P.ldp, gmu, P.B, P.n, P.B, st);
    if (gnu) launch_copy_ld(P.dnu.p, P.ldp, gnu, P.B, P.n, P.B, st);
    std::vector<double> tb(P.ldp, 0.0);
    if (gt) GS_HIP(hipMemcpyAsync(tb.data(), P.tbar.p, P.ldp * sizeof(double), hipMemcpyDeviceToHost, st));
    unsigned long long bad[2] = {0, 0};
    GS_HIP(hipMemcpyAsync(bad, P.badin.p, sizeof(bad), hipMemcpyDeviceToHost, st));
    GS_HIP(hipGetLastError());
    GS_HIP(hipStreamSynchronize(st));
    report_invalid_inputs(bad, "mu / nu / a");
    if (gt) {
        for (int b = 0; b < P.B; ++b) gt[b] = tb[b] + gd[b] * D[b] / t;
        require_finite(gt, P.B, "gradient in t");
    }
}

// ------------------------------------------------------------------ barycenter
void barycenter(gs_plan_s& P, double lam, double t, const float* a, const float* mus, const double* alpha, int J,
                float phi, float* bary, float* v, float* w, double* marg, int64_t* nfl, hipStream_t st) {
    const bool has_a = a != nullptr;
    P.count_floors = nfl != nullptr;
    if (!P.alpha.p) P.alpha.alloc(P.ldp);
    if (!P.bary.p) P.bary.alloc(P.n);
    set_coefs(P, lam, t, st);
    count_invalid_inputs(P, {{mus, (size_t)P.n * P.B}, {a, (size_t)P.n}}, st);
    load_inputs(P, a, mus, nullptr, st);
    std::vector<float> al(P.ldp, 0.f);
    for (int i = 0; i < P.B; ++i) al[i] = (float)alpha[i];
    GS_HIP(hipMemcpyAsync(P.alpha.p, al.data(), P.ldp * sizeof(float), hipMemcpyHostToDevice, st));
    launch_fill(P.w.p, 1.f, P.sz(), st);
    if (has_a) launch_mul_a(P.w.p, P.a.p, P.n, P.ldp, P.xw.p, st);
    GS_HIP(hipMemsetAsync(P.nfloor.p, 0, sizeof(unsigned long long), st));
    const float* ap = has_a ? P.a.p : nullptr;
    const std::string key = std::string("bary:") + (has_a ? "a" : "1") + phi_tag(phi);
    for (int j = 0; j < J; ++j) {
        run_graph(P, key, st, [&](hipStream_t s) {
            ScaleEpi e1{P.mu.p, P.v.p, has_a ? P.xv.p : nullptr, ap, nullptr};
            enqueue_apply(P, has_a ? P.xw.p : P.w.p, ApplyMode::Scale, e1, phi, s);
            enqueue_apply(P, has_a ? P.xv.p : P.v.p, ApplyMode::Store, ScaleEpi{}, phi, s);
            launch_bary_row(P.ACC.p, P.alpha.p, P.n, P.ldp, P.B, phi, P.bary.p, P.w.p, has_a ? P.xw.p : nullptr, ap,
                            P.count_floors ? P.nfloor.p : nullptr, s);
        });
    }
    GS_HIP(hipMemcpyAsync(bary, P.bary.p, P.n * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (v) launch_copy_ld(P.v.p, P.ldp, v, P.B, P.n, P.B, st);
    if (w) launch_copy_ld(P.w.p, P.ldp, w, P.B, P.n, P.B, st);
    if (marg) {
        run_graph(P, std::string("bmarg:") + (has_a ? "a" : "1") + phi_tag(phi), st, [&](hipStream_t s) {
            enqueue_apply(P, has_a ? P.xw.p : P.w.p, ApplyMode::Store, ScaleEpi{}, phi, s);
        });
        reduce_to_host(P, red_args(P, RED_MARG, P.v.p, P.ACC.p, P.mu.p, nullptr, ap), 1.0, marg, st);
    }
    unsigned long long nf = 0, bad[2] = {0, 0};
    if (nfl) GS_HIP(hipMemcpyAsync(&nf, P.nfloor.p, sizeof(nf), hipMemcpyDeviceToHost, st));
    GS_HIP(hipGetLastError());
    if (marg || nfl) {
        GS_HIP(hipMemcpyAsync(bad, P.badin.p, sizeof(bad), hipMemcpyDeviceToHost, st));
        GS_HIP(hipStreamSynchronize(st));
        report_invalid_inputs(bad, "mus / a");
        if (nfl) *nfl = (int64_t)nf;
        if (marg) require_finite(marg, P.B, "marginal error");
    }
}

// ------------------------------------------------------------------ Lanczos estimate of lambda_max
double lambda_max(gs_graph_s& g, int iters, uint64_t seed, double safety, hipStream_t st) {
    const int64_t n = g.n;
    DevBuf<float> q(n), qp(n), z(n);
    const int nblk = reduce_blocks(n);
    DevBuf<double> part((size_t)nblk), red(1);
    std::vector<float> h(n);
    uint64_t x = seed ? seed : 0x9E3779B97F4A7C15ull;
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i) {  // splitmix64 -> uniform(-1, 1)
        x += 0x9E3779B97F4A7C15ull;
        uint64_t y = x;
        y = (y ^ (y >> 30)) * 0xBF58476D1CE4E5B9ull;
        y = (y ^ (y >> 27)) * 0x94D049BB133111EBull;
        y ^= y >> 31;
        const double u = 2.0 * ((double)(y >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
        h[i] = (float)u;
        nrm += (double)h[i] * h[i];
    }
    const double inv = 1.0 / std::sqrt(nrm);
    for (auto& e : h) e = (float)(e * inv);
    GS_HIP(hipMemcpyAsync(q.p, h.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
    launch_fill(qp.p, 0.f, n, st);
    auto dot = [&](const float* u, const float* v) {
        ReduceArgs r{};
        r.op = RED_DOT;
        r.n = n;
        r.ldp = 1;
        r.B = 1;
        r.x0 = u;
        r.x1 = v;
        launch_reduce(r, part.p, nblk, red.p, 0, 1.0, st);
        double out = 0.0;
        GS_HIP(hipMemcpyAsync(&out, red.p, sizeof(double), hipMemcpyDeviceToHost, st));
        GS_HIP(hipStreamSynchronize(st));
        return out;
    };
    std::vector<double> al, be;
    double beta_prev = 0.0, beta_last = 0.0;
    for (int j = 0; j < iters; ++j) {
        launch_lap_spmv(g.rowptr.p, g.col.p, g.val.p, (int32_t)n, q.p, z.p, st);
        const double aj = dot(q.p, z.p);
        launch_lanczos_update(z.p, q.p, qp.p, aj, beta_prev, n, st);
        const double bj = std::sqrt(std::max(0.0, dot(z.p, z.p)));
        al.push_back(aj);
        beta_last = bj;
        if (j == iters - 1 || bj <= 1e-10 * std::max(1.0, std::fabs(aj))) break;
        be.push_back(bj);
        launch_scale(qp.p, z.p, 1.0 / bj, n, st);
        std::swap(q.p, qp.p);
        beta_prev = bj;
    }
    GS_HIP(hipGetLastError());
    const double theta = tridiag_max_eig(al, be);
    if (!(theta > 0.0) || !std::isfinite(theta))
        fail(GS_ERR_SPECTRUM, "Lanczos produced no positive Ritz value (graph without edges?)");
    // ||L y - theta y|| = beta_m |s_m| for the Ritz vector y = Q s: an eigenvalue
    // of L lies within it of theta, so theta + residual covers lambda_max once
    // theta approximates it, when the safety factor alone would not
    const double resid = beta_last * std::fabs(tridiag_last_component(al, be, theta));
    return std::min(std::max(safety * theta, theta + resid), g.edge_bound);
}

}  // namespace gs
