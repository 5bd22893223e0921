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

#include <functional>
#include <queue>
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
    for (int64_t e = 0; e < ne; ++e) {
        const nnm_edge& x = edges[e];
        if (x.u < 0 || x.u >= x.v || x.v >= n || !(x.s >= 0.0)) return NNM_EINVAL;
        if (e > 0 && !key_before(edges[e - 1], x)) return NNM_EINVAL;
    }
    const int64_t kl1 = prm->kl1_max_clusters;
    const int64_t kl2 = prm->kl2_max_size;
    const int64_t kl3 = prm->kl3_max_merged;
    const int64_t kl4 = prm->kl4_min_size;
    const double dmax = prm->dmax;
    const bool priority = kl4 > 1;

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
