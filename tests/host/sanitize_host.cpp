// Host-only parts of the library under AddressSanitizer and UBSan (built with
// g++, no GPU code, run without a device): the Chebyshev coefficients, their
// t-derivatives and tail bounds over a grid of (t, K), and the validation of
// caller-built CSR graphs on a valid cycle and on every kind of malformed
// input the C ABI documents.  Exit status 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <functional>
#include <string>
#include <vector>

#include "internal.h"

namespace gs {
// Stand-ins for the pieces this program does not link: the error plumbing of
// the C ABI (a failure is a Fail exception carrying the status) and the kNN
// kernels (graph building from points is not exercised here).
void set_error(const std::string&) {}
void clear_error() {}
void fail(gs_status code, const std::string&) { throw Fail{code}; }
void launch_knn_candidates(const float*, const float*, int64_t, int, int, int32_t*, hipStream_t) {}
void launch_row_norms(const float*, int64_t, int, float*, hipStream_t) {}
void build_graph_from_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const float* w,
                          gs_graph_s& g);
}  // namespace gs

namespace {

int failures = 0;

void check(bool ok, const std::string& what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what.c_str());
        ++failures;
    }
}

struct Csr {
    std::vector<int32_t> rowptr, col;
    std::vector<float> w;
};

Csr cycle(int n) {
    Csr c;
    for (int i = 0; i < n; ++i) {
        c.rowptr.push_back(2 * i);
        const int a = (i + n - 1) % n, b = (i + 1) % n;
        c.col.push_back(a < b ? a : b);
        c.col.push_back(a < b ? b : a);
        c.w.push_back(0.5f + 0.01f * (float)((a < b ? a : b) + (a < b ? b : a)));
        c.w.push_back(0.0f);
    }
    c.rowptr.push_back(2 * n);
    // weight of edge {i, j} depends on the unordered pair only: symmetric
    for (int i = 0; i < n; ++i)
        for (int e = 2 * i; e < 2 * i + 2; ++e) c.w[e] = 0.5f + 0.01f * (float)((i + c.col[e]) % 97);
    return c;
}

gs_status build(const Csr& c, int64_t n) {
    gs_graph_s g;
    try {
        gs::build_graph_from_csr(n, (int64_t)c.col.size(), c.rowptr.data(), c.col.data(), c.w.data(), g);
    } catch (const gs::Fail& f) {
        return f.code;
    }
    return GS_OK;
}

}  // namespace

int main() {
    // coefficients
    const double ts[] = {0.0, 1e-3, 0.5, 1.0, 2.0, 8.0, 50.0, 200.0, 1000.0};
    const int Ks[] = {0, 1, 5, 30, 50, GS_MAX_K};
    for (double t : ts)
        for (int K : Ks) {
            std::vector<double> b(K + 1), db(K + 1);
            gs::cheby_coeffs(t, K, b.data(), db.data());
            double p0 = 0.5 * b[0];
            bool finite = true;
            for (int k = 0; k <= K; ++k) {
                finite = finite && std::isfinite(b[k]) && std::isfinite(db[k]);
                if (k) p0 += (k % 2 ? -b[k] : b[k]);
            }
            const double tail = gs::cheby_tail(t, K);
            check(finite && std::isfinite(tail) && tail >= 0.0, "finite coefficients t=" + std::to_string(t));
            check(std::fabs(p0 - 1.0) <= tail + 1e-12 || tail > 1e-3, "p_K(0) = 1 within the tail, t=" +
                                                                           std::to_string(t) + " K=" + std::to_string(K));
        }
    std::vector<double> table;
    gs::bessel_ive_table(3.0, 400, table);
    check(table.size() >= 401 && std::isfinite(table[400]), "Bessel table");

    // CSR validation
    const int n = 50;
    const Csr ok = cycle(n);
    check(build(ok, n) == GS_OK, "valid cycle accepted");
    Csr one;
    one.rowptr = {0, 0};
    check(build(one, 1) == GS_OK, "single node without edges accepted");
    const std::vector<std::pair<std::string, std::function<void(Csr&)>>> bad = {
        {"rowptr[0] != 0", [](Csr& c) { c.rowptr[0] = 1; }},
        {"decreasing rowptr", [](Csr& c) { c.rowptr[3] = c.rowptr[2] - 1; }},
        {"rowptr[n] != nnz", [](Csr& c) { c.rowptr.back() -= 1; }},
        {"negative column", [](Csr& c) { c.col[4] = -1; }},
        {"column past n", [](Csr& c) { c.col[4] = n; }},
        {"self loop", [](Csr& c) { c.col[2 * 7] = 7; }},
        {"NaN weight", [](Csr& c) { c.w[9] = std::nanf(""); }},
        {"infinite weight", [](Csr& c) { c.w[9] = INFINITY; }},
        {"negative weight", [](Csr& c) { c.w[9] = -1.0f; }},
        {"duplicate entry", [](Csr& c) { c.col[2 * 10 + 1] = c.col[2 * 10]; }},
        {"asymmetric pattern", [](Csr& c) { c.col[2 * 20 + 1] = (c.col[2 * 20 + 1] + 5) % n; }},
        {"asymmetric value", [](Csr& c) { c.w[2 * 30] *= 1.5f; }},
    };
    for (const auto& [name, mutate] : bad) {
        Csr c = ok;
        mutate(c);
        check(build(c, n) == GS_ERR_INVALID, "rejected: " + name);
    }
    if (failures) return 1;
    std::printf("host checks ok\n");
    return 0;
}
