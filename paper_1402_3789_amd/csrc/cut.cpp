// cut.cpp -- the constrained cut of the key-sorted merge tree (host code).
//
// Section "Problem settings" lists the constraints the method applies while
// uniting clusters: stop below a cluster count (KL1), refuse unions that
// involve a cluster already larger than KL2 or that would exceed KL3 points,
// and unite clusters smaller than KL4 first; the "Problem statement" adds a
// maximum distance at which built clusters may still join.  Clusters that
// exist during the process are always subtrees of the minimum spanning tree,
// and the single-link distance between two clusters adjacent in the tree is
// the weight of the tree edge between them, so the process runs over the
// N-1 tree edges:
//   - edges are taken in key order; with KL4 > 1 an edge whose smaller side
//     holds fewer than KL4 points goes first (class 0 before class 1), and
//     the class is re-evaluated whenever an edge comes up (sizes only grow,
//     so a class can only go from 0 to 1: the edge is then queued again);
//   - the cut stops as soon as the number of clusters is <= KL1;
//   - an edge with w > dmax, a larger side above KL2 or a sum above KL3 is
//     dropped for good (sizes only grow, so it can never become admissible);
//   - otherwise the two clusters are united.
// Labels are numbered in order of first appearance over the points.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <functional>
#include <memory>
#include <queue>
#include <thread>
#include <utility>
#include <vector>

#include "nnm.h"

namespace {

struct Dsu {
    std::vector<int32_t> up;
    std::vector<int32_t> size;
    explicit Dsu(int64_t n) : up((size_t)n), size((size_t)n, 1)
    {
        for (int64_t i = 0; i < n; ++i) up[(size_t)i] = (int32_t)i;
    }
    int32_t root(int32_t x)
    {
        while (up[(size_t)x] != x) {            // path halving
            const int32_t g = up[(size_t)up[(size_t)x]];
            up[(size_t)x] = g;
            x = g;
        }
        return x;
    }
};

// Without KL2, KL3 and KL4 every admissible tree edge unites two clusters,
// the admissible edges (w <= dmax) form a prefix of the key order, and the
// process takes the first m = min(prefix, n - KL1) of them: the result is the
// forest of those m edges, whatever the order they are united in.  Threads
// unite them concurrently (lock-free union-find, the larger root index is
// linked under the smaller, so each root is its component's smallest point);
// labels follow from the roots in increasing order, i.e. by first appearance.
// Returns false when an edge joins two points that the other edges already
// connect (the edges are not a forest).
bool forest_labels(const nnm_edge* edges, int64_t n, int64_t m, int32_t* labels, int64_t* n_clusters)
{
    unsigned nt = std::thread::hardware_concurrency();
    if (nt < 1) nt = 1;
    if (nt > 16) nt = 16;
    std::unique_ptr<std::atomic<int32_t>[]> up(new std::atomic<int32_t>[(size_t)n]);
    std::unique_ptr<int32_t[]> root(new int32_t[(size_t)n]);
    auto parallel = [&](int64_t count, auto&& body) {
        std::vector<std::thread> th;
        const int64_t per = (count + nt - 1) / nt;
        for (unsigned t = 0; t < nt; ++t) {
            const int64_t a = (int64_t)t * per, b = std::min<int64_t>(count, a + per);
            if (a >= b) break;
            th.emplace_back([=, &body] { body((int)t, a, b); });
        }
        for (auto& x : th) x.join();
    };
    auto find = [&](int32_t x) {
        int32_t p = up[(size_t)x].load(std::memory_order_relaxed);
        while (p != x) {
            const int32_t g = up[(size_t)p].load(std::memory_order_relaxed);
            if (g != p) up[(size_t)x].compare_exchange_weak(p, g, std::memory_order_relaxed);
            x = g;
            p = up[(size_t)x].load(std::memory_order_relaxed);
        }
        return x;
    };
    parallel(n, [&](int, int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) up[(size_t)i].store((int32_t)i, std::memory_order_relaxed);
    });
    // the union-find walks are memory-latency bound: the parent words of the
    // edges (and points) a few iterations ahead are prefetched
    constexpr int64_t AHEAD = 16;
    std::atomic<bool> cycle{false};
    parallel(m, [&](int, int64_t a, int64_t b) {
        for (int64_t e = a; e < b; ++e) {
            if (e + AHEAD < b) {
                __builtin_prefetch(&up[(size_t)edges[e + AHEAD].u]);
                __builtin_prefetch(&up[(size_t)edges[e + AHEAD].v]);
            }
            int32_t x = edges[e].u, y = edges[e].v;
            for (;;) {
                x = find(x);
                y = find(y);
                if (x == y) {
                    // in a forest the other edges never connect an edge's two
                    // ends, whatever has been linked so far
                    cycle.store(true, std::memory_order_relaxed);
                    break;
                }
                if (x > y) std::swap(x, y);          // link y (larger) under x
                int32_t expect = y;
                if (up[(size_t)y].compare_exchange_strong(expect, x, std::memory_order_acq_rel)) break;
            }
        }
    });
    std::vector<int64_t> count(nt + 1, 0);
    parallel(n, [&](int t, int64_t a, int64_t b) {
        int64_t c = 0;
        for (int64_t i = a; i < b; ++i) {
            if (i + AHEAD < b)
                __builtin_prefetch(&up[(size_t)up[(size_t)(i + AHEAD)].load(std::memory_order_relaxed)]);
            root[(size_t)i] = find((int32_t)i);
            c += root[(size_t)i] == (int32_t)i;
        }
        count[(size_t)t + 1] = c;
    });
    for (unsigned t = 0; t < nt; ++t) count[t + 1] += count[t];
    // names of the roots (a root is the smallest index of its component, so
    // every root precedes its members): rank among roots
    parallel(n, [&](int t, int64_t a, int64_t b) {
        int64_t c = count[(size_t)t];
        for (int64_t i = a; i < b; ++i)
            if (root[(size_t)i] == (int32_t)i) labels[i] = (int32_t)c++;
    });
    parallel(n, [&](int, int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i)
            if (root[(size_t)i] != (int32_t)i) labels[i] = labels[root[(size_t)i]];
    });
    *n_clusters = count[nt];
    return !cycle.load();
}

bool key_before(const nnm_edge& a, const nnm_edge& b)
{
    if (a.s != b.s) return a.s < b.s;
    if (a.u != b.u) return a.u < b.u;
    return a.v < b.v;
}

}  // namespace

extern "C" nnm_status cluster_cut(const nnm_edge* edges, int64_t n, const nnm_cut_params* prm,
                                  int32_t* labels, int64_t* n_clusters)
{
    if (n < 1 || !prm || !labels || !n_clusters) return NNM_EINVAL;
    if (n > 1 && !edges) return NNM_EINVAL;
    const int64_t ne = n - 1;
    {
        // every edge well formed and the keys strictly increasing
        auto check = [&](int64_t a, int64_t b) {
            for (int64_t e = a; e < b; ++e) {
                const nnm_edge& x = edges[e];
                if (x.u < 0 || x.u >= x.v || x.v >= n || !(x.s >= 0.0) || !(x.w >= 0.0)) return false;
                // w = sqrt(s) is nondecreasing in key order: the distance
                // threshold may then be tested on a prefix
                if (e > 0 && (!key_before(edges[e - 1], x) || edges[e - 1].w > x.w)) return false;
            }
            return true;
        };
        unsigned nt = ne >= 65536 ? std::thread::hardware_concurrency() : 1;
        if (nt < 1) nt = 1;
        if (nt > 16) nt = 16;
        std::vector<char> ok(nt, 1);
        std::vector<std::thread> th;
        const int64_t per = (ne + nt - 1) / nt;
        for (unsigned t = 1; t < nt; ++t) {
            const int64_t a = (int64_t)t * per, b = std::min<int64_t>(ne, a + per);
            if (a < b) th.emplace_back([&, t, a, b] { ok[t] = check(a, b); });
        }
        ok[0] = check(0, std::min<int64_t>(ne, per));
        for (auto& x : th) x.join();
        for (char c : ok)
            if (!c) return NNM_EINVAL;
    }
    const int64_t kl1 = prm->kl1_max_clusters;
    const int64_t kl2 = prm->kl2_max_size;
    const int64_t kl3 = prm->kl3_max_merged;
    const int64_t kl4 = prm->kl4_min_size;
    const double dmax = prm->dmax;
    const bool priority = kl4 > 1;

    if (kl2 < 0 && kl3 < 0 && !priority && n >= 65536) {
        int64_t lo = 0, hi = ne;                // admissible prefix (w <= dmax)
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (!(edges[mid].w > dmax)) lo = mid + 1;   // the discard test below
            else hi = mid;
        }
        int64_t m = lo;
        if (kl1 > 0) m = std::min<int64_t>(m, std::max<int64_t>(0, n - kl1));
        return forest_labels(edges, n, m, labels, n_clusters) ? NNM_OK : NNM_EINVAL;
    }

    Dsu dsu(n);
    int64_t clusters = n;
    // (class, edge index): edge index order is key order
    typedef std::pair<int, int64_t> Item;
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> queue;
    if (priority)
        for (int64_t e = 0; e < ne; ++e) queue.push(Item(0, e));  // all sizes are 1 at start
    int64_t next_in_order = 0;
    for (;;) {
        if (kl1 > 0 && clusters <= kl1) break;
        Item it;
        if (priority) {
            if (queue.empty()) break;
            it = queue.top();
            queue.pop();
        } else {
            if (next_in_order >= ne) break;
            it = Item(1, next_in_order++);
        }
        const nnm_edge& x = edges[it.second];
        const int32_t ra = dsu.root(x.u), rb = dsu.root(x.v);
        const int64_t sa = dsu.size[(size_t)ra], sb = dsu.size[(size_t)rb];
        if (ra == rb) return NNM_EINVAL;        // the edges are not a forest
        if (priority) {
            const int cls = ((sa < sb ? sa : sb) < kl4) ? 0 : 1;
            if (cls != it.first) {
                queue.push(Item(cls, it.second));
                continue;
            }
        }
        if (x.w > dmax) continue;
        if (kl2 >= 0 && (sa > sb ? sa : sb) > kl2) continue;
        if (kl3 >= 0 && sa + sb > kl3) continue;
        if (sa >= sb) {
            dsu.up[(size_t)rb] = ra;
            dsu.size[(size_t)ra] += (int32_t)sb;
        } else {
            dsu.up[(size_t)ra] = rb;
            dsu.size[(size_t)rb] += (int32_t)sa;
        }
        --clusters;
    }
    std::vector<int32_t> name((size_t)n, -1);
    int32_t next = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t r = dsu.root((int32_t)i);
        if (name[(size_t)r] < 0) name[(size_t)r] = next++;
        labels[i] = name[(size_t)r];
    }
    *n_clusters = next;
    return NNM_OK;
}
