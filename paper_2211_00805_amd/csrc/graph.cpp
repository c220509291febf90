// Common affinity graph: kNN candidates on the GPU, exact ranking, union
// symmetrisation, Gaussian-median weights and CSR assembly on the host.
//
// Paper: Sec. "Geodesic Sinkhorn Distances" (one common graph over all
// datasets built with an affinity kernel) and Sec. "Heat Diffusion on a
// Graph" (weighted adjacency A, degrees D_ii = sum_k A_ik, L = D - A).
// Reading: union of directed k-nearest-neighbour edges, self excluded, equal
// distances towards the lower id; weight exp(-d^2 / m^2) with m the median of
// the n*k directed neighbour distances.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace gs {

namespace {

struct UnionFind {
    std::vector<int32_t> p;
    explicit UnionFind(int64_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
    int32_t find(int32_t x) {
        while (p[x] != x) {
            p[x] = p[p[x]];
            x = p[x];
        }
        return x;
    }
    void unite(int32_t a, int32_t b) {
        a = find(a);
        b = find(b);
        if (a != b) p[std::max(a, b)] = std::min(a, b);
    }
};

double sqdist(const float* X, int d, int64_t i, int64_t j) {
    const float* a = X + i * d;
    const float* b = X + j * d;
    double s = 0.0;
    for (int c = 0; c < d; ++c) {
        const double t = (double)a[c] - (double)b[c];
        s += t * t;
    }
    return s;
}

// Degrees, bounds, component count (host only).
void graph_stats(gs_graph_s& g) {
    const int64_t n = g.n;
    g.h_deg.assign(n, 0.f);
    double dmax = 0.0;
    std::vector<double> degd(n, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t e = g.h_rowptr[i]; e < g.h_rowptr[i + 1]; ++e) s += (double)g.h_val[e];
        degd[i] = s;
        g.h_deg[i] = (float)s;
        dmax = std::max(dmax, s);
    }
    double eb = 0.0;
    UnionFind uf(n);
    for (int64_t i = 0; i < n; ++i)
        for (int32_t e = g.h_rowptr[i]; e < g.h_rowptr[i + 1]; ++e) {
            const int32_t j = g.h_col[e];
            eb = std::max(eb, degd[i] + degd[j]);
            uf.unite((int32_t)i, j);
        }
    int32_t comps = 0;
    for (int64_t i = 0; i < n; ++i) comps += uf.find((int32_t)i) == i ? 1 : 0;
    g.deg_max = dmax;
    g.edge_bound = eb;
    g.n_components = comps;
    g.nnz = (int64_t)g.h_col.size();
}

}  // namespace

// Copies the host CSR to the current device.
void upload_graph(gs_graph_s& g, hipStream_t st) {
    const int64_t n = g.n;
    GS_HIP(hipGetDevice(&g.device));
    g.rowptr.alloc(n + 1);
    g.col.alloc(std::max<int64_t>(g.nnz, 1));
    g.val.alloc(std::max<int64_t>(g.nnz, 1));
    GS_HIP(hipMemcpyAsync(g.rowptr.p, g.h_rowptr.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (g.nnz) {
        GS_HIP(hipMemcpyAsync(g.col.p, g.h_col.data(), g.nnz * sizeof(int32_t), hipMemcpyHostToDevice, st));
        GS_HIP(hipMemcpyAsync(g.val.p, g.h_val.data(), g.nnz * sizeof(float), hipMemcpyHostToDevice, st));
    }
    GS_HIP(hipStreamSynchronize(st));
}

void build_graph_from_points(const float* X, int64_t n, int d, int k, hipStream_t st, gs_graph_s& g) {
    // centre the points (distances are unchanged) so float32 Gram tiles lose
    // as little as possible to cancellation
    std::vector<double> mean(d, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < d; ++c) mean[c] += X[i * d + c];
    for (int c = 0; c < d; ++c) mean[c] /= (double)n;
    std::vector<float> Xc((size_t)n * d);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < d; ++c) Xc[i * d + c] = (float)((double)X[i * d + c] - mean[c]);

    int kk = 16;
    for (int c : {16, 24, 32, 40}) {
        kk = c;
        if (c >= k + 8) break;
    }
    std::vector<int32_t> cand((size_t)n * kk);
    {
        DevBuf<float> dX((size_t)n * d), dN(n);
        DevBuf<int32_t> dC((size_t)n * kk);
        GS_HIP(hipMemcpyAsync(dX.p, Xc.data(), (size_t)n * d * sizeof(float), hipMemcpyHostToDevice, st));
        launch_row_norms(dX.p, n, d, dN.p, st);
        launch_knn_candidates(dX.p, dN.p, n, d, kk, dC.p, st);
        GS_HIP(hipGetLastError());
        GS_HIP(hipMemcpyAsync(cand.data(), dC.p, (size_t)n * kk * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GS_HIP(hipStreamSynchronize(st));
    }

    // exact float64 ranking of the candidates: by (squared distance, id)
    std::vector<int32_t> nbr((size_t)n * k);
    std::vector<double> nd2((size_t)n * k);
    bool short_list = false;
#pragma omp parallel for schedule(dynamic, 256) reduction(|| : short_list)
    for (int64_t i = 0; i < n; ++i) {
        std::vector<std::pair<double, int32_t>> c;
        c.reserve(kk);
        for (int p = 0; p < kk; ++p) {
            const int32_t j = cand[(size_t)i * kk + p];
            if (j < 0 || j == i) continue;
            c.emplace_back(sqdist(X, d, i, j), j);
        }
        std::sort(c.begin(), c.end());
        c.erase(std::unique(c.begin(), c.end()), c.end());
        if ((int)c.size() < k) {
            short_list = true;
            continue;
        }
        for (int p = 0; p < k; ++p) {
            nbr[(size_t)i * k + p] = c[p].second;
            nd2[(size_t)i * k + p] = c[p].first;
        }
    }
    if (short_list) fail(GS_ERR_INVALID, "fewer than k candidate neighbours for some point");

    // median of the n*k directed distances (mean of the two middle values when even)
    std::vector<double> dist(nd2.size());
    for (size_t e = 0; e < nd2.size(); ++e) dist[e] = std::sqrt(nd2[e]);
    const size_t N = dist.size();
    std::nth_element(dist.begin(), dist.begin() + N / 2, dist.end());
    double med = dist[N / 2];
    if (N % 2 == 0) {
        const double lo = *std::max_element(dist.begin(), dist.begin() + N / 2);
        med = (lo + med) / 2.0;
    }
    // m = 0 (more than half of the directed neighbour pairs coincide) leaves
    // exp(-d^2 / m^2) undefined on the coincident pairs
    if (!(med > 0.0))
        fail(GS_ERR_INVALID, "the median neighbour distance is 0 (over half of the kNN pairs are duplicate points): "
                             "the Gaussian weights exp(-d^2/m^2) are undefined");
    const double m2 = med * med;

    // union of directed edges, rows sorted by column, duplicates merged
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int p = 0; p < k; ++p) {
            cnt[i + 1]++;
            cnt[(int64_t)nbr[(size_t)i * k + p] + 1]++;
        }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<std::pair<int32_t, double>> ent(cnt[n]);
    std::vector<int64_t> fillp(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int p = 0; p < k; ++p) {
            const int32_t j = nbr[(size_t)i * k + p];
            const double dd = nd2[(size_t)i * k + p];
            ent[fillp[i]++] = {j, dd};
            ent[fillp[j]++] = {(int32_t)i, dd};
        }
    std::vector<int32_t> rowlen(n);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        auto b = ent.begin() + cnt[i], e = ent.begin() + cnt[i + 1];
        std::sort(b, e, [](const auto& x, const auto& y) { return x.first < y.first; });
        auto last = std::unique(b, e, [](const auto& x, const auto& y) { return x.first == y.first; });
        rowlen[i] = (int32_t)(last - b);
    }
    g.n = n;
    g.h_rowptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) g.h_rowptr[i + 1] = g.h_rowptr[i] + rowlen[i];
    const int64_t nnz = g.h_rowptr[n];
    g.h_col.resize(nnz);
    g.h_val.resize(nnz);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        int32_t o = g.h_rowptr[i];
        for (int32_t p = 0; p < rowlen[i]; ++p) {
            const auto& x = ent[cnt[i] + p];
            g.h_col[o + p] = x.first;
            g.h_val[o + p] = (float)std::exp(-x.second / m2);
        }
    }
    g.median = med;
    graph_stats(g);
    upload_graph(g, st);
}

void build_graph_from_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const float* w,
                          gs_graph_s& g) {
    GS_REQUIRE(rowptr[0] == 0, "rowptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i) GS_REQUIRE(rowptr[i + 1] >= rowptr[i], "rowptr must be non-decreasing");
    GS_REQUIRE(rowptr[n] == nnz, "rowptr[n] must equal nnz");
    g.n = n;
    g.h_rowptr.assign(rowptr, rowptr + n + 1);
    g.h_col.resize(nnz);
    g.h_val.resize(nnz);
    for (int64_t i = 0; i < n; ++i) {
        std::vector<std::pair<int32_t, float>> r;
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            GS_REQUIRE(col[e] >= 0 && col[e] < n, "column id out of range");
            GS_REQUIRE(col[e] != i, "self loops are not allowed");
            GS_REQUIRE(std::isfinite(w[e]) && w[e] >= 0.f, "weights must be finite and >= 0");
            r.emplace_back(col[e], w[e]);
        }
        std::sort(r.begin(), r.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
        for (size_t p = 1; p < r.size(); ++p) GS_REQUIRE(r[p].first != r[p - 1].first, "duplicate entry in a row");
        for (size_t p = 0; p < r.size(); ++p) {
            g.h_col[rowptr[i] + p] = r[p].first;
            g.h_val[rowptr[i] + p] = r[p].second;
        }
    }
    // symmetry: every (i, j, w) has a bitwise-equal (j, i, w)
    for (int64_t i = 0; i < n; ++i)
        for (int32_t e = g.h_rowptr[i]; e < g.h_rowptr[i + 1]; ++e) {
            const int32_t j = g.h_col[e];
            const auto b = g.h_col.begin() + g.h_rowptr[j], en = g.h_col.begin() + g.h_rowptr[j + 1];
            const auto it = std::lower_bound(b, en, (int32_t)i);
            GS_REQUIRE(it != en && *it == i, "adjacency is not symmetric in pattern");
            const float wt = g.h_val[it - g.h_col.begin()];
            GS_REQUIRE(wt == g.h_val[e], "adjacency is not symmetric in value");
        }
    g.median = 0.0;
    graph_stats(g);
}

}  // namespace gs
