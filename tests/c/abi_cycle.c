/* The C ABI used from plain C (no Python, no torch): device buffers from the
 * HIP runtime, a graph from a CSR array, a plan, a heat application and
 * Algorithm 1, checked against closed forms of the cycle graph C_n.
 *
 * Cycle: eigenvalues lam_k = 2 - 2 cos(2 pi k / n) with Fourier vectors, so
 * exp(-t (2/lambda_hat) L) x is a discrete Fourier transform away; p_K differs
 * from it by at most the Chebyshev tail bound per eigenvalue (2-norm).  Two
 * adjacent Diracs: the only coupling moves the unit mass along one edge, and
 * after one w-update Algorithm 1 returns D = -4t ln H_01.  Also: a negative
 * histogram entry reported by status, the reverse sweep from recorded
 * denominators, and two columns summed into one distribution by
 * gs_accumulate_columns.
 * Exit status 0 on success, 1 on a failed check, 77 without a device. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "geosink.h"

static const double kPi = 3.14159265358979323846;

#define FAIL(...)                         \
    do {                                  \
        fprintf(stderr, __VA_ARGS__);     \
        fprintf(stderr, "\n");            \
        exit(1);                          \
    } while (0)
#define GS(call)                                                                   \
    do {                                                                           \
        gs_status s_ = (call);                                                     \
        if (s_ != GS_OK) FAIL("%s -> %d: %s", #call, (int)s_, gs_last_error());    \
    } while (0)
#define HIPCK(call)                                                                 \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) FAIL("%s -> %s", #call, hipGetErrorString(e_));       \
    } while (0)

/* exp(-t (2/lam_hat) L) applied to x on C_n, by a direct DFT in double. */
static void cycle_exact(int n, double lam_hat, double t, const double* x, double* y) {
    const double tw = 2.0 * kPi / n;
    double* re = malloc(sizeof(double) * n);
    double* im = malloc(sizeof(double) * n);
    for (int k = 0; k < n; ++k) {
        double a = 0.0, b = 0.0;
        for (int j = 0; j < n; ++j) {
            a += x[j] * cos(tw * k * j);
            b -= x[j] * sin(tw * k * j);
        }
        const double g = exp(-t * (2.0 / lam_hat) * (2.0 - 2.0 * cos(tw * k)));
        re[k] = a * g;
        im[k] = b * g;
    }
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += re[k] * cos(tw * k * j) - im[k] * sin(tw * k * j);
        y[j] = s / n;
    }
    free(re);
    free(im);
}

int main(void) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        printf("abi_cycle: no device\n");
        return 77;
    }
    /* errors come back as status codes with a message */
    gs_plan bad = NULL;
    if (gs_plan_create(NULL, 10, 1, 0, NULL, &bad) != GS_ERR_INVALID || strlen(gs_last_error()) == 0)
        FAIL("NULL graph not rejected");

    const int n = 1000, B = 2, K = 40;
    const double lam_hat = 4.0, t = 2.0;
    int32_t* rowptr = malloc(sizeof(int32_t) * (n + 1));
    int32_t* col = malloc(sizeof(int32_t) * 2 * n);
    float* w = malloc(sizeof(float) * 2 * n);
    for (int i = 0; i < n; ++i) {
        const int a = (i + n - 1) % n, b = (i + 1) % n;
        rowptr[i] = 2 * i;
        col[2 * i] = a < b ? a : b;
        col[2 * i + 1] = a < b ? b : a;
        w[2 * i] = w[2 * i + 1] = 1.0f;
    }
    rowptr[n] = 2 * n;
    gs_graph g = NULL;
    GS(gs_graph_from_csr(n, 2 * n, rowptr, col, w, 0, &g));
    gs_plan p = NULL;
    GS(gs_plan_create(g, K, B, 0, NULL, &p));

    /* column 0: a Dirac at node 0; column 1: deterministic values in [0, 1) */
    float* hx = malloc(sizeof(float) * n * B);
    uint32_t st = 12345u;
    for (int i = 0; i < n; ++i) {
        st = st * 1664525u + 1013904223u;
        hx[i * B] = i == 0 ? 1.0f : 0.0f;
        hx[i * B + 1] = (float)(st >> 8) / 16777216.0f;
    }
    float *dx = NULL, *dy = NULL;
    HIPCK(hipMalloc((void**)&dx, sizeof(float) * n * B));
    HIPCK(hipMalloc((void**)&dy, sizeof(float) * n * B));
    HIPCK(hipMemcpy(dx, hx, sizeof(float) * n * B, hipMemcpyHostToDevice));
    GS(gs_heat_apply(p, lam_hat, t, dx, dy, NULL, 0));
    float* hy = malloc(sizeof(float) * n * B);
    HIPCK(hipMemcpy(hy, dy, sizeof(float) * n * B, hipMemcpyDeviceToHost));
    double tail = 0.0;
    GS(gs_cheby_tail_bound(t, K, &tail));
    double* xc = malloc(sizeof(double) * n);
    double* yc = malloc(sizeof(double) * n);
    double h01 = 0.0;
    for (int c = 0; c < B; ++c) {
        double nx = 0.0, mx = 0.0, err = 0.0;
        for (int i = 0; i < n; ++i) {
            xc[i] = hx[i * B + c];
            nx += xc[i] * xc[i];
            if (fabs(xc[i]) > mx) mx = fabs(xc[i]);
        }
        cycle_exact(n, lam_hat, t, xc, yc);
        if (c == 0) h01 = yc[1];
        for (int i = 0; i < n; ++i) {
            const double d = fabs(hy[i * B + c] - yc[i]);
            if (d > err) err = d;
        }
        const double tol = tail * sqrt(nx) + 8.0 * K * ldexp(1.0, -24) * mx;
        if (!(err <= tol)) FAIL("heat apply column %d: max error %g > %g", c, err, tol);
    }

    /* Algorithm 1 on two adjacent Diracs (column 0) and the same pair reversed (column 1) */
    float* hmu = calloc(n * B, sizeof(float));
    float* hnu = calloc(n * B, sizeof(float));
    hmu[0 * B + 0] = 1.0f;
    hnu[1 * B + 0] = 1.0f;
    hmu[1 * B + 1] = 1.0f;
    hnu[0 * B + 1] = 1.0f;
    float *dmu = NULL, *dnu = NULL;
    HIPCK(hipMalloc((void**)&dmu, sizeof(float) * n * B));
    HIPCK(hipMalloc((void**)&dnu, sizeof(float) * n * B));
    HIPCK(hipMemcpy(dmu, hmu, sizeof(float) * n * B, hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(dnu, hnu, sizeof(float) * n * B, hipMemcpyHostToDevice));
    double dist[2] = {0.0, 0.0};
    int64_t nfl = -1;
    GS(gs_sinkhorn(p, lam_hat, t, NULL, dmu, dnu, 5, 1e-30f, 0, NULL, NULL, NULL, dist, NULL, &nfl, 0));
    const double dref = -4.0 * t * log(h01);
    for (int c = 0; c < B; ++c) {
        const double tol = 1e-5 * fmax(fabs(dref), 4.0 * t) + 4.0 * t * tail / h01;
        if (!(fabs(dist[c] - dref) <= tol)) FAIL("distance %d: %.9g vs %.9g", c, dist[c], dref);
    }
    if (nfl != 0) FAIL("unexpected floors: %lld", (long long)nfl);

    /* a negative histogram entry is reported at the call's synchronisation */
    hmu[7 * B + 1] = -0.25f;
    HIPCK(hipMemcpy(dmu, hmu, sizeof(float) * n * B, hipMemcpyHostToDevice));
    double dbad[2];
    if (gs_sinkhorn(p, lam_hat, t, NULL, dmu, dnu, 5, 1e-30f, 0, NULL, NULL, NULL, dbad, NULL, NULL, 0) !=
            GS_ERR_INVALID || strstr(gs_last_error(), "negative") == NULL)
        FAIL("negative histogram entry not reported: %s", gs_last_error());
    hmu[7 * B + 1] = 0.0f;
    HIPCK(hipMemcpy(dmu, hmu, sizeof(float) * n * B, hipMemcpyHostToDevice));

    /* reverse sweep from recorded denominators (finite gradients), and the
     * accumulation of both columns of a known n x 2 block (the heat test's
     * input) into distribution 0 of a 2 x n gradient, in column order */
    const int J = 5, ldp = 4;   /* B = 2 rounds up to a padded row of 4 floats */
    float *drec = NULL, *dgmu = NULL, *dG = NULL;
    int32_t* dcols = NULL;
    HIPCK(hipMalloc((void**)&drec, sizeof(float) * 2 * J * (size_t)n * ldp));
    HIPCK(hipMalloc((void**)&dgmu, sizeof(float) * n * B));
    HIPCK(hipMalloc((void**)&dG, sizeof(float) * 2 * n));
    HIPCK(hipMalloc((void**)&dcols, sizeof(int32_t) * B));
    HIPCK(hipMemset(dG, 0, sizeof(float) * 2 * n));
    const int32_t hcols[2] = {0, 0};
    HIPCK(hipMemcpy(dcols, hcols, sizeof(hcols), hipMemcpyHostToDevice));
    GS(gs_sinkhorn(p, lam_hat, t, NULL, dmu, dnu, J, 1e-30f, GS_RECORD_ALL, drec, NULL, NULL, dist, NULL, NULL, 0));
    const double ones[2] = {1.0, 1.0};
    double gt[2] = {0.0, 0.0};
    GS(gs_sinkhorn_backward(p, lam_hat, t, NULL, dmu, dnu, J, 1e-30f, GS_RECORD_ALL, drec, ones, dgmu, NULL, gt, 0));
    GS(gs_accumulate_columns(dx, n, B, dcols, 2, dG, 0));
    HIPCK(hipDeviceSynchronize());
    float* hg = malloc(sizeof(float) * n * B);
    float* hG = malloc(sizeof(float) * 2 * n);
    HIPCK(hipMemcpy(hg, dgmu, sizeof(float) * n * B, hipMemcpyDeviceToHost));
    HIPCK(hipMemcpy(hG, dG, sizeof(float) * 2 * n, hipMemcpyDeviceToHost));
    for (int i = 0; i < n * B; ++i)
        if (!isfinite(hg[i])) FAIL("non-finite gradient at %d", i);
    if (!isfinite(gt[0]) || !isfinite(gt[1])) FAIL("non-finite gradient in t");
    for (int i = 0; i < n; ++i) {
        const float want = (0.0f + hx[i * B]) + hx[i * B + 1];
        if (hG[i] != want || hG[n + i] != 0.0f) FAIL("accumulated column at node %d: %g vs %g", i, hG[i], want);
    }
    HIPCK(hipFree(drec));
    HIPCK(hipFree(dgmu));
    HIPCK(hipFree(dG));
    HIPCK(hipFree(dcols));
    free(hg);
    free(hG);

    gs_plan_destroy(p);
    gs_graph_destroy(g);
    HIPCK(hipFree(dx));
    HIPCK(hipFree(dy));
    HIPCK(hipFree(dmu));
    HIPCK(hipFree(dnu));
    free(rowptr); free(col); free(w); free(hx); free(hy); free(xc); free(yc); free(hmu); free(hnu);
    printf("abi_cycle ok: D = %.9f (closed form %.9f), tail bound %.3g\n", dist[0], dref, tail);
    return 0;
}
