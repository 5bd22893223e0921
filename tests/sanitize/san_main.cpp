// Host-side sanitizer harness: exercises cluster_cut (heap path and the
// threaded forest path) and the CPU oracle on seeded random inputs, and
// checks them against each other and against a plain sequential cut.  Built
// three ways by tests/test_sanitizers.py: -fsanitize=address,undefined and
// -fsanitize=thread (with g++ / gcc only: host code, no GPU code).
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <random>
#include <vector>

#include "nnm.h"

extern "C" {
int oracle_prim_mst(const float*, int64_t, int32_t, int64_t, int32_t*, int32_t*, double*, double*, int);
int oracle_cut(const int32_t*, const int32_t*, const double*, const double*, int64_t, int64_t, int64_t,
               int64_t, int64_t, double, int32_t*, int64_t*);
int oracle_knn(const float*, int64_t, int32_t, int64_t, const int64_t*, int64_t, int32_t, int32_t*,
               double*, int32_t*, int);
}

static int failures = 0;
#define CHECK(c, ...)                                   \
    do {                                                \
        if (!(c)) {                                     \
            fprintf(stderr, "FAIL %s:%d ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);               \
            fprintf(stderr, "\n");                      \
            ++failures;                                 \
        }                                               \
    } while (0)

// A random spanning tree of n points with keys sorted as mst_build returns them.
static std::vector<nnm_edge> random_tree(std::mt19937_64& g, int64_t n, bool ties)
{
    std::vector<nnm_edge> e;
    std::uniform_real_distribution<double> U(0.0, 4.0);
    for (int64_t v = 1; v < n; ++v) {
        const int64_t u = std::uniform_int_distribution<int64_t>(0, v - 1)(g);
        double s = ties ? (double)std::uniform_int_distribution<int>(0, 6)(g) : U(g);
        e.push_back(nnm_edge{(int32_t)u, (int32_t)v, s, sqrt(s)});
    }
    std::sort(e.begin(), e.end(), [](const nnm_edge& a, const nnm_edge& b) {
        if (a.s != b.s) return a.s < b.s;
        if (a.u != b.u) return a.u < b.u;
        return a.v < b.v;
    });
    return e;
}

// Sequential reference of the KL1 / dmax cut: unite in key order while
// clusters > kl1 and w <= dmax; labels by first appearance.
static int64_t plain_cut(const std::vector<nnm_edge>& e, int64_t n, int64_t kl1, double dmax,
                         std::vector<int32_t>& lab)
{
    std::vector<int64_t> up((size_t)n);
    for (int64_t i = 0; i < n; ++i) up[(size_t)i] = i;
    auto root = [&](int64_t x) {
        while (up[(size_t)x] != x) x = up[(size_t)x] = up[(size_t)up[(size_t)x]];
        return x;
    };
    int64_t c = n;
    for (const nnm_edge& x : e) {
        if (kl1 > 0 && c <= kl1) break;
        if (x.w > dmax) continue;
        int64_t a = root(x.u), b = root(x.v);
        if (a != b) { up[(size_t)std::max(a, b)] = std::min(a, b); --c; }
    }
    lab.assign((size_t)n, -1);
    std::vector<int32_t> map((size_t)n, -1);
    int32_t next = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t r = root(i);
        if (map[(size_t)r] < 0) map[(size_t)r] = next++;
        lab[(size_t)i] = map[(size_t)r];
    }
    return next;
}

int main(int argc, char** argv)
{
    // oracle threads: the ASan build links OpenMP and runs it threaded; the
    // TSan build runs it on one thread (libgomp is not instrumented)
    const int nt = argc > 1 ? atoi(argv[1]) : 1;
    std::mt19937_64 g(20260101);
    // heap path against the oracle's cut, all settings
    for (int trial = 0; trial < 300; ++trial) {
        const int64_t n = 1 + (int64_t)(g() % 300);
        auto e = random_tree(g, n, trial % 2 == 0);
        const int64_t kl1 = (int64_t)(g() % 6), kl2 = (int64_t)(g() % 5) - 1, kl3 = (int64_t)(g() % 7) - 1;
        const int64_t kl4 = (int64_t)(g() % 5);
        const double dmax = (g() % 3 == 0) ? INFINITY : 1.0 + (double)(g() % 100) / 100.0;
        nnm_cut_params p{kl1, kl2 > 0 ? kl2 * 20 : -1, kl3 > 0 ? kl3 * 30 : -1, kl4, dmax};
        std::vector<int32_t> lab((size_t)n), olab((size_t)n);
        int64_t k = 0, ok = 0;
        CHECK(cluster_cut(e.data(), n, &p, lab.data(), &k) == NNM_OK, "cluster_cut trial %d", trial);
        std::vector<int32_t> u, v;
        std::vector<double> s, w;
        for (auto& x : e) { u.push_back(x.u); v.push_back(x.v); s.push_back(x.s); w.push_back(x.w); }
        CHECK(oracle_cut(u.data(), v.data(), s.data(), w.data(), n, p.kl1_max_clusters, p.kl2_max_size,
                         p.kl3_max_merged, p.kl4_min_size, p.dmax, olab.data(), &ok) == 0, "oracle_cut");
        CHECK(k == ok && lab == olab, "heap cut differs from the oracle's, trial %d", trial);
    }
    // threaded forest path (n >= 65536, KL1 and dmax only) against the plain cut
    for (int trial = 0; trial < 4; ++trial) {
        const int64_t n = 70000 + (int64_t)(g() % 30000);
        auto e = random_tree(g, n, trial % 2 == 1);
        const int64_t kl1 = trial == 0 ? 0 : (int64_t)(g() % 5000);
        const double dmax = trial == 2 ? 1.5 : INFINITY;
        nnm_cut_params p{kl1, -1, -1, 0, dmax};
        std::vector<int32_t> lab((size_t)n), ref;
        int64_t k = 0;
        CHECK(cluster_cut(e.data(), n, &p, lab.data(), &k) == NNM_OK, "forest cut trial %d", trial);
        const int64_t kr = plain_cut(e, n, kl1, dmax, ref);
        CHECK(k == kr && lab == ref, "forest cut differs, trial %d", trial);
    }
    // a cycle is refused on both paths
    {
        std::vector<nnm_edge> e = {{0, 1, 1.0, 1.0}, {1, 2, 2.0, sqrt(2.0)}, {0, 2, 3.0, sqrt(3.0)}};
        std::vector<int32_t> lab(4);
        int64_t k = 0;
        nnm_cut_params p{0, -1, -1, 0, INFINITY};
        CHECK(cluster_cut(e.data(), 4, &p, lab.data(), &k) == NNM_EINVAL, "cycle accepted");
    }
    // the oracle's Prim and kNN on small random inputs
    for (int trial = 0; trial < 20; ++trial) {
        const int64_t n = 2 + (int64_t)(g() % 200);
        const int32_t d = 1 + (int32_t)(g() % 6);
        std::vector<float> X((size_t)(n * d));
        for (auto& x : X) x = (float)(g() % 7);
        std::vector<int32_t> u((size_t)n), v((size_t)n), idx((size_t)(n * 4)), len((size_t)n);
        std::vector<double> s((size_t)n), w((size_t)n), ks((size_t)(n * 4));
        CHECK(oracle_prim_mst(X.data(), n, d, d, u.data(), v.data(), s.data(), w.data(), nt) == 0, "prim");
        for (int64_t e2 = 0; e2 + 1 < n; ++e2) CHECK(u[(size_t)e2] < v[(size_t)e2], "edge order");
        CHECK(oracle_knn(X.data(), n, d, d, nullptr, n, 4, idx.data(), ks.data(), len.data(), nt) == 0, "knn");
    }
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("sanitizer harness ok\n");
    return 0;
}
