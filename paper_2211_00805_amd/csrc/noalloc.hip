// Heat application that allocates nothing: for callers that cannot call
// hipMalloc (code under hipGraph stream capture, serving loops that forbid
// allocation).  The two rotating Chebyshev buffers and the coefficient table
// live in a file-scope device array (`scratch`) of fixed size; the caller
// brings the graph, the input X and the output Y, which also serves as the
// accumulator.  Every call on a GPU shares that GPU's array: calls that
// overlap on one device (two streams, two host threads) race on it.  Nothing
// in the array needs to start at zero: each call writes the coefficients and
// every T_k before reading them.
#include <mutex>

#include "plan.h"

namespace gs {

namespace {

constexpr int64_t kCoefFloats = 1024;   // >= 2 (GS_MAX_K + 1) + 1, padded
static_assert(kCoefFloats >= 2 * (GS_MAX_K + 1) + 1, "coefficient table does not fit");

static __device__ __align__(256) float scratch[2 * GS_NOALLOC_MAX_NB + kCoefFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (each GPU holds its own copy),
// resolved once per device with that device current.
float* scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) fail(GS_ERR_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            fail(GS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

// Y = p_K(L, t) X by the accumulating Chebyshev recurrence (the plan form's
// schedule and step kernel, default launch shape, rows of every length in the
// row groups), T_k rotating through the two halves of `scratch`, X read in
// place (T_0), Y the accumulator.  B == 1 or a multiple of 4, so that the
// caller's n x B arrays are the kernel's padded layout.
void heat_apply_noalloc(gs_graph_s& g, double lam, double t, int K, const float* X, float* Y, int B,
                        hipStream_t st) {
    int dev = 0;
    GS_HIP(hipGetDevice(&dev));
    if (dev != g.device) fail(GS_ERR_INVALID, "the current device is not the graph's device");
    float* base = scratch_on(dev);
    float* buf[2] = {base, base + GS_NOALLOC_MAX_NB};
    float* coef = base + 2 * GS_NOALLOC_MAX_NB;
    double b[GS_MAX_K + 1], db[GS_MAX_K + 1];   // host stack: no heap or device allocation
    cheby_coeffs(t, K, b, db);
    launch_set_coef(coef, 2.0 / lam, b, db, K, st);

    const double npr = g.n ? (double)g.nnz / (double)g.n : 0.0;
    const LaunchShape shape = default_shape(B, npr);
    StepArgs base_args{};
    base_args.rowptr = g.rowptr.p;
    base_args.col = g.col.p;
    base_args.val = g.val.p;
    base_args.n = (int32_t)g.n;
    base_args.ldp = B;
    base_args.coef = coef;
    base_args.K = K;
    base_args.acc = Y;
    auto T = [&](int k) { return buf[k % 2]; };
    for (int k = 1; k <= K; ++k) {
        const StepSched sc = step_sched_at(K, k, ApplyMode::Store);
        StepArgs a = base_args;
        a.k = k;
        a.tprev = k == 1 ? X : T(k - 1);
        a.tprev2 = k >= 2 ? (k == 2 ? X : T(k - 2)) : nullptr;
        a.tout = T(k);
        a.flags = sc.flags;
        a.cmask = sc.cmask;
        launch_step(shape, a, st);
    }
    GS_HIP(hipGetLastError());
}

}  // namespace gs
