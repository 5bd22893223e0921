// cut_dev.hip -- the cut of a sorted tree on the device, for settings
// without size caps or priority.
//
// Section "Problem settings" stops uniting clusters at KL1 clusters and the
// "Problem statement" forbids unions above a distance threshold; with KL2,
// KL3 and KL4 off nothing else can refuse a tree edge.  The admissible edges
// (w <= dmax) then form a prefix of the key order (w is nondecreasing along
// it), every admissible edge unites two clusters, and the process takes the
// first m = min(prefix, n - KL1) of them: the clusters are the components of
// the forest of those m edges, whatever order the unions happen in.  Here the
// m unions run concurrently (lock-free union-find: a root is only ever
// linked under a smaller root, by compare-and-swap), so each component's
// root is its smallest point, and the labels number the roots in increasing
// order -- order of first appearance over the points, as the host cut
// numbers them.
#include "nnm_common.h"

namespace nnm {
namespace {

struct CutCtr {
    int32_t bad;        // bit 0: an edge malformed or out of key order; bit 1: a cycle
    int32_t prefix;     // admissible prefix length (w <= dmax)
    int32_t clusters;   // number of components
    int32_t m;          // edges united
};

constexpr int CUT_GRID_MAX = 4096;

unsigned cut_grid(int64_t n)
{
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > CUT_GRID_MAX ? CUT_GRID_MAX : g));
}

__device__ __forceinline__ int32_t ld_parent(const int32_t* p, int32_t x)
{
    return __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x.  Path halving: a point that is not a root never becomes one
// again and its parent only moves towards the root, so the plain (relaxed)
// store of a grandparent over a parent is safe against every concurrent
// union.
__device__ __forceinline__ int32_t cut_find(int32_t* parent, int32_t x)
{
    int32_t p = ld_parent(parent, x);
    while (p != x) {
        const int32_t g = ld_parent(parent, p);
        if (g != p) __hip_atomic_store(parent + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = p;
        p = g;
    }
    return x;
}

__device__ __forceinline__ bool edge_key_before(const nnm_edge& a, const nnm_edge& b)
{
    if (a.s != b.s) return a.s < b.s;
    if (a.u != b.u) return a.u < b.u;
    return a.v < b.v;
}

__global__ __launch_bounds__(64) void k_cut_reset(CutCtr* c)
{
    if (threadIdx.x == 0) *c = CutCtr{0, 0, 0, 0};
}

// Every edge well formed and after its predecessor in key order (with w
// not decreasing); the admissible prefix, as the largest admissible index
// plus one (one atomic per workgroup); parent[i] = i.
__global__ __launch_bounds__(256) void k_cut_check(const nnm_edge* __restrict__ e, int64_t ne, int64_t n,
                                                   double dmax, int32_t* __restrict__ parent,
                                                   CutCtr* __restrict__ c)
{
    __shared__ int32_t sb[4], sp[4];
    int32_t bad = 0, pre = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        parent[i] = (int32_t)i;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += stride) {
        const nnm_edge x = e[i];
        if (x.u < 0 || x.u >= x.v || x.v >= n || !(x.s >= 0.0) || !(x.w >= 0.0)) bad = 1;
        if (i > 0) {
            const nnm_edge y = e[i - 1];
            if (!edge_key_before(y, x) || y.w > x.w) bad = 1;
        }
        if (!(x.w > dmax)) pre = (int32_t)(i + 1);
    }
    for (int off = 32; off > 0; off >>= 1) {
        bad |= __shfl_xor(bad, off);
        const int32_t o = __shfl_xor(pre, off);
        pre = o > pre ? o : pre;
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sb[wave] = bad;
        sp[wave] = pre;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t b = sb[0] | sb[1] | sb[2] | sb[3];
        int32_t p = sp[0];
        for (int w = 1; w < 4; ++w) p = sp[w] > p ? sp[w] : p;
        if (b) atomicOr(&c->bad, 1);
        if (p > 0) atomicMax(&c->prefix, p);
    }
}

__global__ __launch_bounds__(64) void k_cut_count(int64_t n, int64_t kl1, CutCtr* c)
{
    if (threadIdx.x != 0) return;
    int64_t m = c->prefix;
    if (kl1 > 0) {
        const int64_t lim = n - kl1 > 0 ? n - kl1 : 0;
        m = m < lim ? m : lim;
    }
    c->m = (int32_t)m;
}

// Unite the ends of the first m edges: link the larger root under the
// smaller one; a failed compare-and-swap means that root was just linked,
// so look the roots up again.  Two ends already together: not a forest.
__global__ __launch_bounds__(256) void k_cut_unite(const nnm_edge* __restrict__ e, int32_t* parent,
                                                   CutCtr* c)
{
    if (c->bad) return;
    const int64_t m = c->m;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        int32_t x = e[i].u, y = e[i].v;
        for (;;) {
            x = cut_find(parent, x);
            y = cut_find(parent, y);
            if (x == y) {
                atomicOr(&c->bad, 2);
                break;
            }
            const int32_t lo = x < y ? x : y, hi = x < y ? y : x;
            if (atomicCAS(parent + hi, hi, lo) == hi) break;
            x = lo;
            y = hi;
        }
    }
}

// After every union: each point's root (into labels, for now) and the roots' flags.
__global__ __launch_bounds__(256) void k_cut_roots(int32_t* parent, int64_t n, int32_t* __restrict__ labels,
                                                   int32_t* __restrict__ flag)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t r = cut_find(parent, (int32_t)i);
        labels[i] = r;
        flag[i] = r == (int32_t)i ? 1 : 0;
    }
}

// Label of a point: the rank of its root among the roots.
__global__ __launch_bounds__(256) void k_cut_name(const int32_t* __restrict__ rank, int64_t n,
                                                  int32_t* __restrict__ labels)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        labels[i] = rank[labels[i]];
}

struct CutWS {
    int32_t* parent;
    int32_t* flag;
    int32_t* rank;
    void* scan_temp;
    CutCtr* ctr;
};

size_t cut_carve(int64_t n, void* base, CutWS* w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        void* p = base ? (char*)base + off : nullptr;
        off += bytes;
        return p;
    };
    w->parent = (int32_t*)take(sizeof(int32_t) * (size_t)n);
    w->flag = (int32_t*)take(sizeof(int32_t) * (size_t)n);
    w->rank = (int32_t*)take(sizeof(int32_t) * (size_t)n);
    w->scan_temp = take(scan_temp_bytes(n));
    w->ctr = (CutCtr*)take(sizeof(CutCtr));
    return off;
}

}  // namespace
}  // namespace nnm

using namespace nnm;

extern "C" nnm_status cluster_cut_device_workspace_size(int64_t n, size_t* bytes)
{
    if (n < 1 || n > INT32_MAX || !bytes) return NNM_EINVAL;
    CutWS w;
    *bytes = cut_carve(n, nullptr, &w);
    return NNM_OK;
}

extern "C" nnm_status cluster_cut_device(const nnm_edge* edges_dev, int64_t n, const nnm_cut_params* prm,
                                         void* ws_dev, size_t ws_bytes, int32_t* labels_dev,
                                         int64_t* n_clusters, void* stream)
{
    if (n < 1 || n > INT32_MAX || !prm || !labels_dev || !n_clusters || !ws_dev) return NNM_EINVAL;
    if (n > 1 && !edges_dev) return NNM_EINVAL;
    if (prm->kl2_max_size >= 0 || prm->kl3_max_merged >= 0 || prm->kl4_min_size > 1)
        return NNM_EUNSUPPORTED;
    CutWS w;
    if (cut_carve(n, ws_dev, &w) > ws_bytes) return NNM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t ne = n - 1;
    const unsigned g = cut_grid(n);
    k_cut_reset<<<1, 64, 0, s>>>(w.ctr);
    k_cut_check<<<g, 256, 0, s>>>(edges_dev, ne, n, prm->dmax, w.parent, w.ctr);
    k_cut_count<<<1, 64, 0, s>>>(n, prm->kl1_max_clusters, w.ctr);
    k_cut_unite<<<g, 256, 0, s>>>(edges_dev, w.parent, w.ctr);
    k_cut_roots<<<g, 256, 0, s>>>(w.parent, n, labels_dev, w.flag);
    if (launch_exclusive_scan(w.flag, w.rank, n, w.scan_temp, &w.ctr->clusters, s) != hipSuccess)
        return NNM_EDEVICE;
    k_cut_name<<<g, 256, 0, s>>>(w.rank, n, labels_dev);
    if (hipGetLastError() != hipSuccess) return NNM_EDEVICE;
    CutCtr hc;
    if (hipMemcpyAsync(&hc, w.ctr, sizeof(hc), hipMemcpyDeviceToHost, s) != hipSuccess) return NNM_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return NNM_EDEVICE;
    if (hc.bad) return NNM_EINVAL;
    *n_clusters = hc.clusters;
    return NNM_OK;
}
