/*
 * geosink.h -- C ABI of the MI355X (gfx950) Geodesic Sinkhorn hot path.
 *
 * Geodesic Sinkhorn (Huguet, Tong et al., "Geodesic Sinkhorn for Fast and
 * Accurate Optimal Transport on Manifolds") computes entropic optimal transport
 * between signals on a graph whose kernel is the graph heat kernel
 * H_t = exp(-t L).  The kernel is never formed: every application is an
 * order-K Chebyshev recurrence of sparse products with the graph Laplacian
 * (Sec. "Chebyshev Polynomials"), and Algorithm 1 alternates two such
 * applications per Sinkhorn iteration.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns a gs_status; GS_OK is 0, errors are negative.  No call
 *    aborts, throws or prints.  gs_last_error() returns a thread-local message
 *    describing the last failure on the calling thread.
 *  - Argument validation happens before any HIP call; a call that fails
 *    validation has no effect.  The contents of device arrays that must be
 *    finite and >= 0 (histograms, vertex weights) can only be checked on the
 *    device: they are counted while the call runs and reported when it
 *    synchronises (gs_sinkhorn, gs_sinkhorn_backward, gs_barycenter).
 *  - Ownership: gs_graph and gs_plan handles are created and freed by the
 *    library.  Every array argument is owned by the caller and only borrowed
 *    for the duration of the call (device work reading or writing it is
 *    enqueued on `stream` and may still be pending when the call returns,
 *    unless the call returns host results, see below).
 *  - Device signals are float32, node-major: an n x B block stores the B
 *    values of node i contiguously at [i*B, i*B+B) (leading dimension B).
 *  - Device work is enqueued on `stream` (0 = the null stream).  Calls that
 *    write host outputs (distances, errors, counters, lambda_hat, gradients
 *    in t) synchronise `stream` before returning.
 *  - A gs_plan is not thread-safe: calls on one plan must not overlap (they
 *    share the plan's device workspace).  Different plans are independent.
 *  - Readings of the paper that the library fixes (all documented with the
 *    oracle):  the operator is rescaled as L_op = (2/lambda_hat) L and t is
 *    the diffusion time on L_op (H_t = exp(-t L_op), y = L_op - I); degree K
 *    means coefficients b_0..b_K with b_0 halved (K sparse products); the
 *    regularisation of Algorithm 1 is 4t; denominators are floored at phi.
 */
#ifndef GEOSINK_H
#define GEOSINK_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_ABI_VERSION 2
#define GS_MAX_K 256          /* largest Chebyshev degree a plan accepts */

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID = -1,        /* bad argument (null pointer, size, value)   */
    GS_ERR_OOM = -2,            /* device or host allocation failed           */
    GS_ERR_HIP = -3,            /* a HIP runtime call failed                  */
    GS_ERR_NOT_CONNECTED = -4,  /* graph has > 1 component and that was refused */
    GS_ERR_SPECTRUM = -5,       /* lambda_max estimate could not be formed    */
    GS_ERR_NONFINITE = -6,      /* non-finite value in an input or a result   */
    GS_ERR_NO_DEVICE = -7       /* no usable gfx950 device                    */
} gs_status;

typedef struct gs_graph_s* gs_graph;
typedef struct gs_plan_s* gs_plan;

/* Thread-local text of the last error on this thread ("" if none). */
const char* gs_last_error(void);

/* GS_ABI_VERSION of the loaded library. */
int32_t gs_abi_version(void);

/* ------------------------------------------------------------------------ */
/* Common graph (Sec. "Geodesic Sinkhorn Distances": one affinity graph over  */
/* all datasets; Sec. "Heat Diffusion on a Graph": A, D, L = D - A).          */
/* ------------------------------------------------------------------------ */

/* Build the symmetrised kNN graph of n points in R^d.
 *   X      host float32 (n x d), row-major (point i at X[i*d .. i*d+d)).
 *   k      neighbours per point, 1 <= k <= 32 and k < n.
 *   require_connected  nonzero: return GS_ERR_NOT_CONNECTED (and no graph)
 *          when the graph has more than one connected component.
 * Edges are the union of the directed k-nearest-neighbour relations (self
 * excluded, equal distances broken towards the lower node id); the weight of
 * edge {i,j} is exp(-|x_i - x_j|^2 / m^2) with m the median of the n*k
 * directed neighbour distances (GS_ERR_INVALID when m = 0, i.e. more than
 * half of the directed pairs are duplicate points; duplicates below that get
 * weight 1).  Candidate neighbours are found on the GPU
 * (float32 Gram tiles, k+8 candidates per point) and ranked on the host in
 * float64 by exact squared distance.  Device CSR (int32 row pointers and
 * column ids, float32 weights) stays resident in the returned handle.
 * Uses the current HIP device; work runs on `stream` and is complete when
 * the call returns. */
gs_status gs_graph_from_points(const float* X, int64_t n, int32_t d, int32_t k,
                               int32_t require_connected, hipStream_t stream, gs_graph* out);

/* Wrap a caller-built symmetric adjacency (host CSR arrays, copied).
 *   rowptr int32 (n+1), col int32 (nnz), w float32 (nnz): A_ij = w for each
 *   (i, col) entry.  Requirements (else GS_ERR_INVALID): rowptr[0] = 0,
 *   non-decreasing, rowptr[n] = nnz < 2^31; col in [0, n); no self loops; no
 *   duplicate entries in a row; w finite and >= 0; A symmetric in pattern
 *   and bitwise in value.  Rows are stored sorted by column id. */
gs_status gs_graph_from_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                            const float* w, hipStream_t stream, gs_graph* out);

/* Scalars of a graph; any out pointer may be NULL.
 *   edge_bound = max over edges of (d_i + d_j) >= lambda_max(L);
 *   median_dist = m of the Gaussian weights (0 for gs_graph_from_csr). */
gs_status gs_graph_info(gs_graph g, int64_t* n, int64_t* nnz, int32_t* n_components,
                        double* deg_max, double* edge_bound, double* median_dist);

/* Copy the graph to caller host arrays (any may be NULL): rowptr (n+1),
 * col (nnz), w (nnz), deg (n; float32 of the float64 row sums of w). */
gs_status gs_graph_export(gs_graph g, int32_t* rowptr, int32_t* col, float* w, float* deg);

void gs_graph_destroy(gs_graph g);

/* ------------------------------------------------------------------------ */
/* Spectral rescaling and coefficients (Sec. "Chebyshev Polynomials")         */
/* ------------------------------------------------------------------------ */

/* Estimate lambda_hat >= lambda_max(L) for the rescaling L_op = (2/lambda_hat) L.
 * Runs `iters` (>= 2) Lanczos steps on the GPU from a start vector drawn with
 * `seed`, takes the largest Ritz value theta with its residual norm
 * r = ||L y - theta y|| (= beta_m |s_m|: L has an eigenvalue within r of theta)
 * and returns min(max(safety * theta, theta + r), edge_bound); safety >= 1.
 * The paper only assumes the spectrum is bounded; the residual covers a Ritz
 * value that has not converged to within the safety factor, and the edge bound
 * max_E(d_i + d_j) >= lambda_max caps a generous factor.  Synchronises `stream`. */
gs_status gs_lambda_max(gs_graph g, int32_t iters, uint64_t seed, double safety,
                        hipStream_t stream, double* lambda_hat);

/* Chebyshev coefficients of exp(-t(y+1)) on [-1,1]:
 *   b[k] = 2 (-1)^k e^{-t} I_k(t), k = 0..K (b[0] NOT halved), and
 *   db_dt[k] = d b[k] / dt (NULL to skip).  Host arrays of K+1 doubles.
 * I_k is evaluated by Miller's backward recurrence normalised with
 * e^t = I_0 + 2 sum_k I_k.  t >= 0, 0 <= K <= GS_MAX_K.  Pure host code. */
gs_status gs_cheby_coeffs(double t, int32_t K, double* b, double* db_dt);

/* sum_{k>K} |b_k|: bound on the truncation error of the degree-K series. */
gs_status gs_cheby_tail_bound(double t, int32_t K, double* bound);

/* ------------------------------------------------------------------------ */
/* Plans: device workspace + tuned launch shape for (graph, K, B)            */
/* ------------------------------------------------------------------------ */

#define GS_PLAN_AUTOTUNE 1   /* time the candidate launch shapes at creation */
#define GS_PLAN_NO_GRAPH 2   /* launch kernels directly instead of replaying  */
                             /* captured hipGraphs                            */

/* Create a plan for degree K (1..GS_MAX_K) and B (>= 1) right-hand sides.
 * tune_cache: path of a JSON file caching autotuned shapes (NULL: no cache);
 * read and updated only with GS_PLAN_AUTOTUNE.  Allocates device workspace
 * (about 9*n*B floats, more on the first backward call). */
gs_status gs_plan_create(gs_graph g, int32_t K, int32_t B, int32_t flags, const char* tune_cache,
                         gs_plan* out);

/* Override the launch shape of the fused Chebyshev step (tuning studies,
 * tests).  vec = 1 (float lanes, only when B == 1) or 4 (float4 lanes);
 * S lanes split each row's nonzeros (power of two), C lanes span column
 * groups of vec floats (power of two), S*C <= 64; a row takes
 * ceil(padded B / (vec*C)) column tiles, lanes past the padded row idle, and
 * C must be 1 or below twice the number of float4 groups (padded B / 4).
 * Cached hipGraphs of the plan are dropped. */
gs_status gs_plan_set_shape(gs_plan p, int32_t vec, int32_t S, int32_t C);

/* How the step kernel reads the graph's CSR arrays: streamed = 1 with
 * non-temporal hints (a CSR larger than the caches passes once per step and
 * leaves L2 to the gathered rows), 0 with ordinary cached loads (a CSR that
 * fits the caches stays there across the K steps).  The autotuner chooses it
 * with the launch shape (GS_PLAN_AUTOTUNE); this call overrides it (tuning
 * studies, tests).  Results are bitwise the same either way.  Cached hipGraphs
 * of the plan are dropped; synchronises the device. */
gs_status gs_plan_set_csr_hint(gs_plan p, int32_t streamed);

/* Frontier-sparse steps (enable = 1; 0, the default, computes every row).
 * T_k(y) x vanishes beyond k hops of supp(x), since y = (2/lambda_hat) L - I
 * couples a node only to its graph neighbours (Sec. "Chebyshev Polynomials").
 * With the option on, each call first finds the breadth-first hop distances
 * (up to K) from the supports its applications start from, on the device, a
 * sweep per hop that returns at once after the frontier empties:
 * gs_heat_apply from the rows where any column of X is nonzero; gs_sinkhorn
 * from supp(mu) for the applications to a v and from supp(nu) for those to
 * a w after the first iteration (which applies to w = 1 densely).  Step k
 * then skips the gathers of rows more than k hops away, and a block of such
 * rows skips its CSR (on every step but the last it skips everything: each
 * application zeroes its T and accumulator buffers first).  Results are bitwise those of the dense steps.  The
 * option pays where supports stay localised for many hops (a few nodes on
 * a large sparse graph) and costs the distance sweeps and about a
 * microsecond per step where they cover the graph within a few hops (kNN
 * graphs).  gs_barycenter and the reverse sweep of gs_sinkhorn_backward stay
 * dense; the backward-Euler kernel ignores the option.  Allocates about
 * 10 n bytes on first use; cached hipGraphs of the plan are dropped;
 * synchronises the device.  GS_ERR_INVALID unless enable is 0 or 1. */
gs_status gs_plan_set_frontier(gs_plan p, int32_t enable);

/* Kernel a plan applies in gs_heat_apply, gs_sinkhorn and gs_barycenter. */
#define GS_KERNEL_CHEBYSHEV 0 /* p_K(L, t): degree-K Chebyshev sum (default) */
#define GS_KERNEL_EULER 1     /* backward-Euler (I + (t/N) L_op)^{-N}       */
#define GS_KERNEL_CLENSHAW 2  /* the same p_K(L, t) by Clenshaw's recurrence */

/* Select the heat-kernel approximation (paper, Sec. "Related work": the heat
 * kernel applied by solving the linear systems of an implicit discretisation
 * of the heat equation, N solves per application; the ground cost of that
 * discretisation is stated next to Proposition "ground cost", whose sign typo
 * is read as (I + (t/N) L_op)^{-N}, eps = 4t).  L_op = (2/lambda_hat) L as for
 * the Chebyshev kernel, so each system I + (t/N) L_op has condition number at
 * most 1 + 2t/N when lambda_hat >= lambda_max.
 *   kernel   GS_KERNEL_CHEBYSHEV (N, cg_iters ignored) or GS_KERNEL_EULER.
 *   N        1..1024 implicit steps per application.
 *   cg_iters 1..1000 conjugate-gradient iterations per solve (from x = 0, all
 *            columns at once), or 0: per call, the smallest count whose CG
 *            bound 2 sqrt(kappa) ((sqrt(kappa)-1)/(sqrt(kappa)+1))^m with
 *            kappa = 1 + 2t/N is below 2^-52 (relative 2-norm error per
 *            solve).  m iterations reach m hops, and Algorithm 1's logarithms
 *            depend on small kernel entries far from a support: a bound at
 *            float32 resolution (1e-7) leaves distances off by ~1e-3.
 * With GS_KERNEL_EULER, gs_heat_apply's Ydt and gs_sinkhorn_backward fail with
 * GS_ERR_INVALID (no time derivative or reverse sweep for this kernel);
 * allocates 3 n x B float buffers on first use; drops cached hipGraphs and
 * synchronises the device. */
gs_status gs_plan_set_kernel(gs_plan p, int32_t kernel, int32_t N, int32_t cg_iters);

/* Human-readable description of the chosen launch shape and kernel into buf. */
gs_status gs_plan_describe(gs_plan p, char* buf, int32_t len);

void gs_plan_destroy(gs_plan p);

/* ------------------------------------------------------------------------ */
/* Hot path                                                                   */
/* ------------------------------------------------------------------------ */

/* Y = p_K(L, t) X (Sec. "Chebyshev Polynomials"): b_0/2 X + sum_{k=1..K} b_k T_k(y) X
 * with T_0 = X, T_1 = y X, T_k = 2 y T_{k-1} - T_{k-2}, y = (2/lambda_hat) L - I.
 *   X, Y   device n x B.  Ydt: device n x B receiving (d/dt) p_K(L,t) X, or NULL.
 *   lambda_hat > 0, t >= 0.  Y and X must not overlap. */
gs_status gs_heat_apply(gs_plan p, double lambda_hat, double t, const float* X, float* Y,
                        float* Ydt, hipStream_t stream);

/* ckpt_every value of gs_sinkhorn / gs_sinkhorn_backward: record every
 * iteration's denominators instead of checkpointing w. */
#define GS_RECORD_ALL (-1)

/* Algorithm 1 (Geodesic Sinkhorn) for B independent pairs (column b of mu, nu).
 *   a        device n vertex weights (finite, >= 0), or NULL for all ones.
 *   mu, nu   device n x B, finite, >= 0 (not renormalised).  Being device
 *            data, these are checked on the device while the call runs: when
 *            the call synchronises (any host output requested) it fails with
 *            GS_ERR_NONFINITE for a non-finite entry of mu, nu or a, else
 *            GS_ERR_INVALID for a negative one (outputs then unspecified); a
 *            call with no host output does not report them.
 *   iters    J >= 1 Sinkhorn iterations, w^0 = 1, v updated before w.
 *   phi      denominator floor (> 0, e.g. 1e-30): d = r if r > phi else phi.
 *   ckpt_every, ckpt   if ckpt != NULL, w^{s*C} (C = ckpt_every >= 1) is
 *            stored at ckpt + s*n*B for s = 0..ceil(J/C)-1 (device, caller
 *            sized ceil(J/C)*n*B floats), for gs_sinkhorn_backward.  With
 *            ckpt_every = GS_RECORD_ALL, ckpt instead receives every
 *            iteration's floored denominators d_j = floor(p_K(a w^j)) and
 *            e_j = floor(p_K(a v^{j+1})) (slots 2j and 2j+1, each n x ldp with
 *            ldp = B rounded up to a multiple of 4, 1 when B = 1; caller sized
 *            2*J*n*ldp floats: 51 GB at n = 1M, B = 32, J = 200), so that the
 *            reverse sweep recomputes nothing.  Captured graphs hold the
 *            record buffer's address; a call with another buffer recaptures.
 *   v, w     device n x B outputs v^J, w^J (either may be NULL).
 *   dist     host B doubles: D = 4t sum_i a_i (mu_i ln v_i + nu_i ln w_i)
 *            (0 ln 0 = 0), the value on Algorithm 1's return line; NULL ok.
 *   marg_err host B doubles or NULL: ||a v p_K(a w) - a mu||_1 (one extra
 *            heat application per call).
 *   n_floored host int64 or NULL: count of floored denominators on the
 *            numerators' supports over all iterations (NULL: not counted,
 *            which saves the atomic updates when floors are frequent).  A
 *            lambda_hat below the largest Laplacian eigenvalue voids the
 *            truncation bound and, far enough below, overflows the float32
 *            recurrence: its NaN / inf denominators are floored (r > phi
 *            fails) and show up here, not as a non-finite distance.
 * A non-finite dist or marg_err entry (e.g. float32 overflow of v from
 * histogram entries near FLT_MAX) fails the call with GS_ERR_NONFINITE.
 * Synchronises `stream` when any host output is requested. */
gs_status gs_sinkhorn(gs_plan p, double lambda_hat, double t, const float* a, const float* mu,
                      const float* nu, int32_t iters, float phi, int32_t ckpt_every, float* ckpt,
                      float* v, float* w, double* dist, double* marg_err, int64_t* n_floored,
                      hipStream_t stream);

/* Gradient of sum_b grad_dist[b] * D_b with respect to mu, nu and t, through
 * exactly `iters` unrolled iterations of Algorithm 1 (d floor(r)/dr = 1[r>phi],
 * lambda_hat held fixed).  Iterates are recomputed segment by segment from
 * the checkpoints written by gs_sinkhorn with the same arguments (or, with
 * ckpt_every = GS_RECORD_ALL, read from its records without recomputation;
 * grad_mu and grad_nu are then bitwise those of the checkpointed sweep); p_K is
 * symmetric, so every adjoint is another Chebyshev application, with a second
 * accumulator (db_k/dt) for the gradient in t.
 *   grad_dist  host B doubles (the upstream gradient of each D_b).
 *   grad_mu, grad_nu  device n x B outputs (either may be NULL); entries off
 *              the support of mu (resp. nu) are set to 0 (the derivative is
 *              -infinity there).
 *   grad_t     host B doubles or NULL (per-pair dD_b/dt times grad_dist[b]);
 *              NULL skips the second accumulator and the reductions in t
 *              (grad_mu and grad_nu are bitwise the same either way).
 * mu, nu and a are checked on the device as in gs_sinkhorn and reported
 * (GS_ERR_NONFINITE, GS_ERR_INVALID) at the end of every call.
 * Synchronises `stream`. */
gs_status gs_sinkhorn_backward(gs_plan p, double lambda_hat, double t, const float* a,
                               const float* mu, const float* nu, int32_t iters, float phi,
                               int32_t ckpt_every, const float* ckpt, const double* grad_dist,
                               float* grad_mu, float* grad_nu, double* grad_t, hipStream_t stream);

/* Fixed-support barycenter of the plan's B = m inputs (Sec. "Interpolation
 * with discrete support"; the paper gives no algorithm: iterative Bregman
 * projections, v_i = mu_i / p_K(a w_i), q_i = floor(p_K(a v_i)),
 * p = exp(sum_i alpha_i ln q_i), w_i = p / q_i, from w_i = 1).
 *   mus      device n x m inputs (finite, >= 0; checked on the device and
 *            reported as in gs_sinkhorn, with a, when marg_err or n_floored
 *            is requested); alpha host m doubles (>= 0).
 *   bary     device n output p.  v, w: device n x m outputs or NULL.
 *   marg_err host m doubles or NULL: ||a v_i p_K(a w_i) - a mu_i||_1.
 *   n_floored host int64 or NULL: floored denominators (on mu_i's support
 *            for the v update, everywhere for q; NULL: not counted). */
gs_status gs_barycenter(gs_plan p, double lambda_hat, double t, const float* a, const float* mus,
                        const double* alpha, int32_t iters, float phi, float* bary, float* v,
                        float* w, double* marg_err, int64_t* n_floored, hipStream_t stream);

/* Graph-level forms of the four calls above (the heat application of Sec.
 * "Chebyshev Polynomials", Algorithm 1, its reverse sweep and the barycenter
 * problem of Sec. "Interpolation with discrete support"), taking the graph, K and
 * the number of columns (B pairs, or m input distributions) directly.  The
 * arguments that follow mean what they mean for the plan-bound call, which
 * runs them and whose validation and errors apply.  plan: NULL uses a plan
 * the graph keeps for (K, B), created on the first such call with default
 * flags (default launch shape, captured hipGraphs; no autotuning) and freed
 * by gs_graph_destroy; or a plan created for this graph, K and B
 * (GS_ERR_INVALID otherwise).  Calls sharing a plan share its workspace:
 * calls on one graph with the same K and B and plan NULL must not overlap
 * (another host thread or stream); give each its own plan instead. */
gs_status gs_graph_heat_apply(gs_graph g, double lambda_hat, double t, int32_t K, const float* X,
                              float* Y, float* Ydt, int32_t B, gs_plan plan, hipStream_t stream);
gs_status gs_graph_sinkhorn(gs_graph g, double lambda_hat, double t, int32_t K, const float* a,
                            const float* mu, const float* nu, int32_t B, int32_t iters, float phi,
                            int32_t ckpt_every, float* ckpt, float* v, float* w, double* dist,
                            double* marg_err, int64_t* n_floored, gs_plan plan, hipStream_t stream);
gs_status gs_graph_sinkhorn_backward(gs_graph g, double lambda_hat, double t, int32_t K,
                                     const float* a, const float* mu, const float* nu, int32_t B,
                                     int32_t iters, float phi, int32_t ckpt_every, const float* ckpt,
                                     const double* grad_dist, float* grad_mu, float* grad_nu,
                                     double* grad_t, gs_plan plan, hipStream_t stream);
gs_status gs_graph_barycenter(gs_graph g, double lambda_hat, double t, int32_t K, const float* a,
                              const float* mus, const double* alpha, int32_t m, int32_t iters,
                              float phi, float* bary, float* v, float* w, double* marg_err,
                              int64_t* n_floored, gs_plan plan, hipStream_t stream);

/* Expectation of node features under a (not necessarily normalised) signal:
 * out[c] = sum_i p_i Y[i*d + c] / sum_i p_i, c < d (float64 sums, two
 * deterministic passes).  The Expected Barycenter Effect (Sec. "Geodesic
 * Sinkhorn Distances", definition of the barycentric distance and the
 * Expected Barycenter Effect) is the difference of two such expectations
 * under two barycenters.
 *   p  device n floats; Y device n x d float32 (node-major, 1 <= d <= 4096);
 *   out host d doubles.
 * Allocates temporary device memory; synchronises `stream`.  Fails with
 * GS_ERR_NONFINITE when sum_i p_i is zero or not finite. */
gs_status gs_expectation(const float* p, const float* Y, int64_t n, int32_t d, hipStream_t stream,
                         double* out);

/* A batch's mu (or nu) block from a set of m distributions (the pairs of the
 * Sec. "Nearest-Wasserstein-neighbor distributions" experiment):
 * out[i*B + b] = H[i*m + cols[b]].
 *   H     device n x m float32, node-major (distribution c is column c).
 *   cols  device B int32: the distribution of each batch column; entries
 *         outside [0, m) give a zero column.
 *   out   device n x B float32 (a gs_sinkhorn input), must not overlap H.
 *   1 <= n < 2^31, m >= 1, 1 <= B <= 4096.  Asynchronous; allocates nothing. */
gs_status gs_gather_columns(const float* H, int64_t n, int32_t m, const int32_t* cols, int32_t B, float* out,
                            hipStream_t stream);

/* Per-distribution gradients from a batch's per-pair gradients.  When the B
 * pairs of a gs_sinkhorn batch draw their columns from m distributions (all
 * pairs of the Sec. "Nearest-Wasserstein-neighbor distributions" experiment),
 * the gradient of the sum of their distances with respect to distribution c
 * is, by the chain rule, the sum of the gradient columns drawn from c; call
 * once with grad_mu and the pairs' source indices and once with grad_nu and
 * their target indices (a pair (c, c) then collects both columns).
 *   src   device n x B float32, node-major (grad_mu or grad_nu of
 *         gs_sinkhorn_backward).
 *   cols  device B int32: the distribution of each column; entries outside
 *         [0, m) are skipped (e.g. -1 for a batch's padding columns).
 *   G     device m x n float32, distribution-major (distribution c's
 *         gradient is the n-vector at G + c*n), read and updated:
 *         G[c*n + i] += src[i*B + b] for every b with cols[b] = c, in the
 *         order b = 0, 1, ..., B-1 (one thread per node i: deterministic,
 *         also when cols repeats an index).  G must not overlap src.
 *   1 <= n < 2^31, 1 <= B <= 4096, m >= 1.  Asynchronous; allocates nothing. */
gs_status gs_accumulate_columns(const float* src, int64_t n, int32_t B, const int32_t* cols, int32_t m,
                                float* G, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Measurement helpers                                                        */
/* ------------------------------------------------------------------------ */

/* Average duration (ms, HIP events on `stream`) of one launch of the fused
 * Chebyshev step kernel over `reps` whole applications of p_K (K launches
 * each) in the plan's launch shape, and the average algorithmic bytes of one
 * launch: per step the CSR once (4(n+1) + 8 nnz), T_{k-1} once (4nB, the
 * gathered operand), T_{k-2} (4nB, all steps but the first), T_k (4nB, all
 * steps but the last) and the accumulator (4nB read and/or written on every
 * third step and on the last).  1 <= reps <= 100000.  Synchronises `stream`. */
gs_status gs_plan_time_step(gs_plan p, int32_t reps, hipStream_t stream, double* avg_ms,
                            double* bytes_per_launch);

/* ------------------------------------------------------------------------ */
/* Entry point that allocates nothing                                         */
/* ------------------------------------------------------------------------ */

#define GS_NOALLOC_MAX_NB (4 << 20) /* largest n * B of gs_heat_apply_noalloc */

/* For callers that cannot allocate device memory: code under hipGraph stream
 * capture, serving loops and harnesses that forbid hipMalloc.
 * Y = p_K(L, t) X as gs_heat_apply computes it (the same accumulating
 * Chebyshev steps and kernel), without a plan: the two n x B Chebyshev buffers
 * and the coefficient table live in a file-scope device array of
 * 2 * GS_NOALLOC_MAX_NB + 1024 floats (32 MiB) that each GPU the library runs
 * on holds until the process ends; X is read in place and Y is the
 * accumulator.  No hipMalloc, hipFree, memset, host synchronisation or
 * allocating library call is made, so the call can be captured into a
 * hipGraph; its first call on a device resolves the array's address there
 * (make one call outside capture first).
 *   g          graph on the current device;
 *   lambda_hat > 0 (finite), t >= 0 (finite), 1 <= K <= GS_MAX_K;
 *   X, Y       device n x B float32, node-major (ld = B), distinct;
 *   B          1 or a multiple of 4, with n * B <= GS_NOALLOC_MAX_NB
 *              (GS_ERR_INVALID beyond it, checked before any device work).
 * Default launch shape, every row in the row-group kernel (no long-row
 * blocks).  Every call on one GPU shares that GPU's array and keeps the last
 * call's contents (each call writes all it reads): calls that overlap on one
 * device (two streams, two host threads) race on it and must be ordered by
 * the caller.  Asynchronous on `stream`. */
gs_status gs_heat_apply_noalloc(gs_graph g, double lambda_hat, double t, int32_t K, const float* X, float* Y,
                                int32_t B, hipStream_t stream);

/* dst[i] = src[i] for i < count (device float32) with a plain streaming copy
 * kernel; a bandwidth reference for the step kernel. */
gs_status gs_stream_copy(const float* src, float* dst, int64_t count, hipStream_t stream);

/* Gather reference for the step kernel: for each run of 32 consecutive
 * entries of idx (m entries), the sum of the 128-byte rows X[idx[e]] (X device
 * n x 32 float32, node-major; an entry outside [0, n) reads row 0) is written
 * to out (device, 32 * ceil(m / 32) floats).  With idx = a graph's CSR column
 * array, one pass moves exactly the rows the step kernel gathers at B = 32,
 * through the same load path, without the rest of the step.  Asynchronous. */
gs_status gs_stream_gather(const float* X, int64_t n, const int32_t* idx, int64_t m, float* out,
                           hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GEOSINK_H */
