// allpairs.hip -- the constrained clustering process over all pairs of
// points (not only the tree edges), exactly.
//
// The section "General description of the algorithm for constructing the
// set of minimum distances" unites clusters along the smallest pairs of
// points in different clusters; the settings of "Problem settings" (KL1..
// KL4) and the distance threshold of the "Problem statement" decide which
// pairs may be taken.  With the size caps KL2 / KL3 on, a pair blocked at one
// time can be bypassed by a longer pair between other clusters, which need
// not be a tree edge; cluster_cut (tree edges only) then differs from the
// process.  This entry point follows the process itself:
//
//   * a pair of clusters A, B is admissible when sqrt(s) <= dmax,
//     max(|A|, |B|) <= KL2 and |A| + |B| <= KL3; its class is 0 when
//     min(|A|, |B|) < KL4 (KL4 > 1), else 1; each step takes the admissible
//     pair with the smallest (class, key) and unites its clusters, until
//     KL1 clusters remain or no pair is admissible.
//   * Clusters only grow, so a pair that is not admissible never becomes
//     admissible again.  The smallest (class, key) over all pairs is the
//     smallest over clusters X of (class of X, best(X)), best(X) being the
//     smallest admissible pair leaving X and the class of X 0 when
//     |X| < KL4: a class-0 pair touches a small cluster, whose own best is
//     no larger.
//   * By the cut property the smallest pair leaving X is a tree edge; when
//     that edge is admissible it is best(X).  So every cluster keeps a heap
//     of the tree edges at its points, and only a cluster whose smallest
//     outgoing tree edge is blocked looks further:
//   * then best(X) is the smallest over X's points of each point's first
//     admissible neighbour.  Every point keeps an exact prefix of its
//     neighbours by key (from knn_build) and a cursor; an entry that is
//     inside the point's cluster or not admissible is skipped for good.  A
//     point whose prefix is used up gets the next prefix from the GPU: the k
//     smallest keys beyond its last one over the columns admissible for its
//     cluster now (an exact FP64 scan of every column), which stays an exact
//     prefix of the admissible columns later on, since those only shrink.
//   * Host side: cluster ids relabelled smaller-into-larger, one meldable
//     heap of points per cluster keyed by a lower bound of each point's next
//     pair, and one heap of clusters keyed by a lower bound of (class,
//     best); bounds are made exact when they reach the top.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <queue>
#include <random>
#include <vector>

#include "bound.h"
#include "nnm_common.h"

namespace nnm {
namespace {

// ---- GPU: the next k admissible neighbours of a batch of points ---------

// One point of a rescan batch: the point, the key (lb_s, lb_j) of the last
// neighbour already known ((s, j) order), and the largest admissible size
// of the other cluster (-1: none).
struct NextReq {
    int32_t row;
    int32_t lb_j;
    int32_t limit;
    int32_t pad_;
    double lb_s;
};

struct NextArgs {
    const float* xp;          // [n][DMAX] padded copy of the points
    int32_t d;
    int32_t k;
    int64_t n;
    const struct NextReq* req;// [nr] the points and what is known of them
    int32_t nr;
    int32_t splits;           // column ranges per point
    const int32_t* comp;      // [n] cluster of each point
    const int32_t* csize;     // [n] size of each cluster, by cluster id
    double dmax;
    int32_t* part_j;          // [nr][splits][k] per column range
    double* part_s;
    int32_t* part_len;        // [nr][splits]
    int32_t* out_j;           // [nr][k]
    double* out_s;            // [nr][k]
    int32_t* out_len;         // [nr]
};

__global__ __launch_bounds__(256) void k_pad_points(const float* __restrict__ X, int64_t ld, int d,
                                                    int64_t n, float* __restrict__ xp)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n * DMAX) return;
    const int64_t i = t / DMAX;
    const int f = (int)(t % DMAX);
    xp[t] = f < d ? X[i * ld + f] : 0.f;
}

// dst[idx[e]] = val[e] for e < m (every index listed once with its final value)
__global__ __launch_bounds__(256) void k_scatter_i32(const int2* __restrict__ upd, int64_t m,
                                                     int32_t* __restrict__ dst)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < m) dst[upd[e].x] = upd[e].y;
}

// One workgroup per (point, column range), grid-stride: every thread keeps
// the k smallest admissible (s, j) of its columns, then k rounds of a
// workgroup arg-min merge the 256 lists into the range's list.
__global__ __launch_bounds__(256) void k_next_admissible(NextArgs a)
{
    __shared__ double rs[4];
    __shared__ int rj[4], rt[4];
    __shared__ int win;
    __shared__ float uv[4];
    __shared__ int ut[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nq = (a.d + 3) / 4;
    const double crel = fp32_crel(a.d), a0 = fp32_a0(a.d);
    for (int item = blockIdx.x; item < a.nr * a.splits; item += gridDim.x) {
        __syncthreads();
        const int q = item / a.splits, sp = item % a.splits;
        const NextReq rq = a.req[q];
        const int i = rq.row;
        const int ci = a.comp[i];
        const int lim = rq.limit;
        const double ls0 = rq.lb_s;
        const int lj0 = rq.lb_j;
        float xi[DMAX];
        {
            const float4* src = reinterpret_cast<const float4*>(a.xp + (int64_t)i * DMAX);
#pragma unroll
            for (int f4 = 0; f4 < DMAX / 4; ++f4) {
                const float4 v = src[f4];
                xi[4 * f4] = v.x; xi[4 * f4 + 1] = v.y; xi[4 * f4 + 2] = v.z; xi[4 * f4 + 3] = v.w;
            }
        }
        double hs[KMAX];
        int hj[KMAX];
        for (int e = 0; e < KMAX; ++e) { hs[e] = __builtin_huge_val(); hj[e] = 0x7FFFFFFF; }
        const int k = a.k;
        const int64_t c0 = a.n * sp / a.splits, c1 = a.n * (sp + 1) / a.splits;
        // FP32 sum of squares of the pair (i, j): within crel s + a0 of its key s
        auto fp32_t = [&](const float4* yp) {
            float t = 0.f;
            for (int f4 = 0; f4 < nq; ++f4) {
                const float4 y = yp[f4];
                const float d0 = xi[4 * f4] - y.x, d1 = xi[4 * f4 + 1] - y.y;
                const float d2 = xi[4 * f4 + 2] - y.z, d3 = xi[4 * f4 + 3] - y.w;
                t = __builtin_fmaf(d0, d0, t);
                t = __builtin_fmaf(d1, d1, t);
                t = __builtin_fmaf(d2, d2, t);
                t = __builtin_fmaf(d3, d3, t);
            }
            return t;
        };
        // A bound U on the k-th key of this range: the k-th smallest upper
        // bound over columns that are surely admissible and beyond the known
        // prefix (each thread keeps its k smallest, then k rounds of a
        // workgroup minimum).  Only columns whose lower bound is <= U get the
        // FP64 key below.
        float U = __builtin_huge_valf();
        if (lim >= 0) {
            float hv[KMAX];
            for (int e = 0; e < KMAX; ++e) hv[e] = __builtin_huge_valf();
            for (int64_t j = c0 + tid; j < c1; j += 256) {
                const int cj = a.comp[j];
                if (cj == ci || a.csize[cj] > lim) continue;
                const float t = fp32_t(reinterpret_cast<const float4*>(a.xp + j * DMAX));
                const double lo = ((double)t - a0) / (1.0 + crel);
                const double hi = fp32_upper_from_t((double)t, crel, a0);
                if (!(lo > ls0) || __builtin_sqrt(hi) > a.dmax) continue;
                const float hf = d2f_up(hi);
                if (!(hf < hv[k - 1])) continue;
                int p = k - 1;
                while (p > 0 && hv[p - 1] > hf) { hv[p] = hv[p - 1]; --p; }
                hv[p] = hf;
            }
            int head = 0;
            for (int r = 0; r < k; ++r) {
                float bv = head < k ? hv[head] : __builtin_huge_valf();
                int bt = tid;
                for (int off = 32; off > 0; off >>= 1) {
                    const float ov = __shfl_xor(bv, off);
                    const int ot = __shfl_xor(bt, off);
                    if (ov < bv || (ov == bv && ot < bt)) { bv = ov; bt = ot; }
                }
                if (lane == 0) { uv[wave] = bv; ut[wave] = bt; }
                __syncthreads();
                float v0 = uv[0];
                int t0 = ut[0];
                for (int w = 1; w < 4; ++w)
                    if (uv[w] < v0 || (uv[w] == v0 && ut[w] < t0)) { v0 = uv[w]; t0 = ut[w]; }
                __syncthreads();
                if (!(v0 < __builtin_huge_valf())) break;   // fewer than k sure columns
                if (tid == t0) ++head;
                if (r == k - 1) U = v0;
            }
        }
        if (lim >= 0) {
            for (int64_t j = c0 + tid; j < c1; j += 256) {
                const int cj = a.comp[j];
                if (cj == ci || a.csize[cj] > lim) continue;
                const float4* yp = reinterpret_cast<const float4*>(a.xp + j * DMAX);
                // a column whose key is surely below the known prefix, above
                // U or above this thread's k-th key is dropped unscored
                {
                    const float t = fp32_t(yp);
                    const double lo = ((double)t - a0) / (1.0 + crel);
                    const double hi = fp32_upper_from_t((double)t, crel, a0);
                    if (hi < ls0 || lo > (double)U || lo > hs[k - 1]) continue;
                }
                // the key of eq. (1): FP64 differences and squares, summed in
                // feature order
                double s = 0.0;
                for (int f4 = 0; f4 < nq; ++f4) {
                    const float4 y = yp[f4];
                    const float yv[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        const int f = 4 * f4 + h;
                        if (f < a.d) {
                            const double df = __dsub_rn((double)xi[f], (double)yv[h]);
                            const double sq = __dmul_rn(df, df);
                            s = f == 0 ? sq : __dadd_rn(s, sq);
                        }
                    }
                }
                if (!sj_less(ls0, lj0, s, (int)j)) continue;          // not beyond the known prefix
                if (__builtin_sqrt(s) > a.dmax) continue;
                if (!sj_less(s, (int)j, hs[k - 1], hj[k - 1])) continue;
                int p = k - 1;
                while (p > 0 && sj_less(s, (int)j, hs[p - 1], hj[p - 1])) {
                    hs[p] = hs[p - 1];
                    hj[p] = hj[p - 1];
                    --p;
                }
                hs[p] = s;
                hj[p] = (int)j;
            }
        }
        int head = 0, kept = 0;
        for (int r = 0; r < k; ++r) {
            double bs = head < k ? hs[head] : __builtin_huge_val();
            int bj = head < k ? hj[head] : 0x7FFFFFFF;
            int bt = tid;
            for (int off = 32; off > 0; off >>= 1) {
                const double os = __shfl_xor(bs, off);
                const int oj = __shfl_xor(bj, off);
                const int ot = __shfl_xor(bt, off);
                if (sj_less(os, oj, bs, bj)) { bs = os; bj = oj; bt = ot; }
            }
            if (lane == 0) { rs[wave] = bs; rj[wave] = bj; rt[wave] = bt; }
            __syncthreads();
            if (tid == 0) {
                double s0 = rs[0];
                int j0 = rj[0], t0 = rt[0];
                for (int w = 1; w < 4; ++w)
                    if (sj_less(rs[w], rj[w], s0, j0)) { s0 = rs[w]; j0 = rj[w]; t0 = rt[w]; }
                win = s0 < __builtin_huge_val() ? t0 : -1;
                if (win >= 0) {
                    a.part_j[(int64_t)item * k + r] = j0;
                    a.part_s[(int64_t)item * k + r] = s0;
                }
            }
            __syncthreads();
            const int wt = win;
            __syncthreads();
            if (wt < 0) break;
            if (tid == wt) ++head;
            ++kept;
        }
        if (tid == 0) a.part_len[item] = kept;
    }
}

// The k smallest of a point's per-range lists (each ascending): one wave
// per point, lane r holding the head of range r's list; k rounds of a wave
// arg-min.
__global__ __launch_bounds__(256) void k_merge_ranges(NextArgs a)
{
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= a.nr) return;
    const int64_t it = (int64_t)q * a.splits + lane;
    const int len = lane < a.splits ? a.part_len[it] : 0;
    int pos = 0;
    int kept = 0;
    for (; kept < a.k; ++kept) {
        double bs = pos < len ? a.part_s[it * a.k + pos] : __builtin_huge_val();
        int bj = pos < len ? a.part_j[it * a.k + pos] : 0x7FFFFFFF;
        int bl = lane;
        for (int off = 32; off > 0; off >>= 1) {
            const double os = __shfl_xor(bs, off);
            const int oj = __shfl_xor(bj, off);
            const int ol = __shfl_xor(bl, off);
            if (sj_less(os, oj, bs, bj) || (os == bs && oj == bj && ol < bl)) { bs = os; bj = oj; bl = ol; }
        }
        if (!(bs < __builtin_huge_val())) break;
        if (lane == 0) {
            a.out_j[(int64_t)q * a.k + kept] = bj;
            a.out_s[(int64_t)q * a.k + kept] = bs;
        }
        if (lane == bl) ++pos;
    }
    if (lane == 0) a.out_len[q] = kept;
}

#define HIP_OK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) return NNM_EDEVICE; \
    } while (0)

// ---- host side ----------------------------------------------------------

struct PairKey {
    double s;
    int32_t lo, hi;
    bool operator<(const PairKey& o) const
    {
        if (s != o.s) return s < o.s;
        if (lo != o.lo) return lo < o.lo;
        return hi < o.hi;
    }
};

struct Workspace {
    size_t knn_bytes;
    void* knn_ws;
    int32_t* idx;             // [n][k]
    double* sd;               // [n][k]
    int32_t* len;             // [n]
    int32_t* comp;            // [n]
    int32_t* csize;           // [n]
    float* xp;                // [n][DMAX]
    int32_t* part_j;          // [max(n, PART_MIN)][k]
    double* part_s;
    int32_t* part_len;        // [max(n, PART_MIN)]
    // one upload per rescan: [2n] (index, value) updates of the cluster ids
    // and sizes, then [n] requests; one download: lengths, indices, keys
    char* upload;
    char* download;
};

// byte layout of a rescan's download for nr points of k neighbours
struct DownLayout {
    size_t len_off, j_off, s_off, bytes;
    DownLayout(int64_t nr, int32_t k)
    {
        len_off = 0;
        j_off = (size_t)nr * 4;
        s_off = (j_off + (size_t)nr * k * 4 + 7) & ~(size_t)7;
        bytes = s_off + (size_t)nr * k * 8;
    }
};

// per-range lists: a batch of nr points uses nr * splits <= max(nr, PART_MIN)
constexpr int64_t PART_MIN = 8192;
constexpr int64_t TARGET_GROUPS = 1024;

size_t carve_ap(int64_t n, int32_t k, size_t knn_bytes, char* base, Workspace* w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        off = (off + 255) & ~(size_t)255;
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const size_t N = (size_t)n, K = (size_t)k;
    w->knn_bytes = knn_bytes;
    w->knn_ws = take(knn_bytes);
    w->idx = (int32_t*)take(N * K * 4);
    w->sd = (double*)take(N * K * 8);
    w->len = (int32_t*)take(N * 4);
    w->comp = (int32_t*)take(N * 4);
    w->csize = (int32_t*)take(N * 4);
    w->xp = (float*)take(N * DMAX * 4);
    const size_t P = (size_t)std::max<int64_t>(n, PART_MIN);
    w->part_j = (int32_t*)take(P * K * 4);
    w->part_s = (double*)take(P * K * 8);
    w->part_len = (int32_t*)take(P * 4);
    w->upload = (char*)take(2 * N * sizeof(int2) + N * sizeof(NextReq) + 64);
    w->download = (char*)take(DownLayout((int64_t)N, k).bytes + 64);
    return off + 256;
}

constexpr int32_t DEFAULT_DEPTH = 16;

struct Process {
    int64_t n;
    int32_t K;
    int64_t kl1, kl2, kl3, kl4;
    double dmax;
    // points: neighbour prefix and cursor
    std::vector<int32_t> lj;
    std::vector<double> ls;
    std::vector<int32_t> len, cur;
    std::vector<uint8_t> state;      // 0 candidate at cur, 1 prefix used up, 2 no pair left
    std::vector<uint8_t> queued;     // in `spent`
    std::vector<int32_t> spent;      // points in state 1 awaiting the next prefix
    // clusters: the cluster id of every point, kept current (members of the
    // smaller side are relabelled at each union), sizes and versions by id
    std::vector<int32_t> size, ver;
    std::vector<int32_t> cid, mnext, mhead, mtail;
    // changes since the device copy was last brought up to date
    bool uploaded = false;
    std::vector<int32_t> dirty_pts, dirty_roots;   // each listed once (dmark bits 1, 2)
    std::vector<uint8_t> dmark;
    // per-cluster meldable heaps of points (randomised meld)
    std::vector<int32_t> hl, hr, hroot;
    std::vector<PairKey> hkey;
    // per-cluster meldable heaps of tree edges: node 2e and 2e + 1 are edge
    // e at its two ends (after a union both copies sit in one heap)
    const nnm_edge* tree = nullptr;
    const nnm_options* opt = nullptr;
    bool rows_ready = false;         // neighbour prefixes built
    std::vector<int32_t> tl, tr, troot;
    std::mt19937 coin{12345};
    // page-locked staging of the rescans' transfers (grown on demand)
    struct Pinned {
        void* p = nullptr;
        size_t cap = 0;
        ~Pinned()
        {
            if (p) (void)hipHostFree(p);
        }
        void* get(size_t bytes)
        {
            if (bytes > cap) {
                if (p) (void)hipHostFree(p);
                p = nullptr;
                cap = 0;
                if (hipHostMalloc(&p, bytes, 0) != hipSuccess) return nullptr;
                cap = bytes;
            }
            return p;
        }
    } up_pin, down_pin;
    int64_t refills = 0, refilled_rows = 0, merges = 0;
    double refill_ms = 0.0;

    int32_t meld(int32_t a, int32_t b)
    {
        if (a < 0) return b;
        if (b < 0) return a;
        if (hkey[b] < hkey[a]) std::swap(a, b);
        if (coin() & 1) hl[a] = meld(hl[a], b);
        else hr[a] = meld(hr[a], b);
        return a;
    }
    void push(int32_t c, int32_t r)
    {
        hl[r] = hr[r] = -1;
        hroot[c] = meld(hroot[c], r);
    }
    void pop(int32_t c)
    {
        const int32_t r = hroot[c];
        hroot[c] = meld(hl[r], hr[r]);
    }
    bool tless(int32_t a, int32_t b) const
    {
        const nnm_edge& x = tree[a >> 1];
        const nnm_edge& y = tree[b >> 1];
        if (x.s != y.s) return x.s < y.s;
        if (x.u != y.u) return x.u < y.u;
        return x.v < y.v;
    }
    int32_t tmeld(int32_t a, int32_t b)
    {
        if (a < 0) return b;
        if (b < 0) return a;
        if (tless(b, a)) std::swap(a, b);
        if (coin() & 1) tl[a] = tmeld(tl[a], b);
        else tr[a] = tmeld(tr[a], b);
        return a;
    }
    // largest admissible size of the other cluster for a cluster of size sx
    int32_t limit_of(int64_t sx) const
    {
        int64_t lim = INT32_MAX;
        if (kl2 >= 0) {
            if (sx > kl2) return -1;
            lim = std::min<int64_t>(lim, kl2);
        }
        if (kl3 >= 0) lim = std::min<int64_t>(lim, kl3 - sx);
        return lim < 0 ? -1 : (int32_t)lim;
    }
    bool admissible(int64_t sa, int64_t sb, double s) const
    {
        if (sqrt(s) > dmax) return false;
        if (kl2 >= 0 && std::max(sa, sb) > kl2) return false;
        if (kl3 >= 0 && sa + sb > kl3) return false;
        return true;
    }
    PairKey key_at(int32_t r) const
    {
        const int32_t j = lj[(size_t)r * K + cur[r]];
        return PairKey{ls[(size_t)r * K + cur[r]], std::min(r, j), std::max(r, j)};
    }
    // the prefix of r is used up: no pair left if it held every admissible
    // column, else wait for the next prefix (lower bound: its last key)
    void use_up(int32_t r)
    {
        if (len[r] < K) {
            state[r] = 2;
            return;
        }
        state[r] = 1;
        hkey[r] = PairKey{ls[(size_t)r * K + K - 1], -1, -1};
        if (!queued[r]) {
            queued[r] = 1;
            spent.push_back(r);
        }
    }
};

// The next prefixes of every point in p.spent, from the GPU.
nnm_status refill(Process& p, const float* X, int32_t d, int64_t ld, Workspace& w, hipStream_t s)
{
    const int32_t nr = (int32_t)p.spent.size();
    if (nr == 0) return NNM_OK;
    const auto t0 = std::chrono::steady_clock::now();
    // the clusters as they are now: everything the first time, then only
    // the points relabelled and the sizes changed since the last scan
    size_t nu = 0;
    if (!p.uploaded) {
        HIP_OK(hipMemcpyAsync(w.comp, p.cid.data(), 4 * (size_t)p.n, hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(w.csize, p.size.data(), 4 * (size_t)p.n, hipMemcpyHostToDevice, s));
        p.uploaded = true;
    } else {
        nu = p.dirty_pts.size() + p.dirty_roots.size();
    }
    const size_t np = p.uploaded ? p.dirty_pts.size() : 0, nc = nu - np;
    const size_t req_off = (nu * sizeof(int2) + 15) & ~(size_t)15;
    const size_t up_bytes = req_off + (size_t)nr * sizeof(NextReq);
    char* up = (char*)p.up_pin.get(up_bytes);
    if (!up) return NNM_EDEVICE;
    int2* upd = reinterpret_cast<int2*>(up);
    for (size_t e = 0; e < np; ++e) upd[e] = make_int2(p.dirty_pts[e], p.cid[(size_t)p.dirty_pts[e]]);
    for (size_t e = 0; e < nc; ++e)
        upd[np + e] = make_int2(p.dirty_roots[e], p.size[(size_t)p.dirty_roots[e]]);
    NextReq* rq = reinterpret_cast<NextReq*>(up + req_off);
    for (int32_t q = 0; q < nr; ++q) {
        const int32_t r = p.spent[(size_t)q];
        rq[q].row = r;
        rq[q].lb_j = p.lj[(size_t)r * p.K + p.K - 1];
        rq[q].limit = p.limit_of(p.size[(size_t)p.cid[(size_t)r]]);
        rq[q].pad_ = 0;
        rq[q].lb_s = p.ls[(size_t)r * p.K + p.K - 1];
    }
    HIP_OK(hipMemcpyAsync(w.upload, up, up_bytes, hipMemcpyHostToDevice, s));
    if (np > 0)
        k_scatter_i32<<<(unsigned)((np + 255) / 256), 256, 0, s>>>((const int2*)w.upload, (int64_t)np, w.comp);
    if (nc > 0)
        k_scatter_i32<<<(unsigned)((nc + 255) / 256), 256, 0, s>>>((const int2*)w.upload + np, (int64_t)nc,
                                                                   w.csize);
    for (int32_t x : p.dirty_pts) p.dmark[(size_t)x] &= (uint8_t)~1u;
    for (int32_t x : p.dirty_roots) p.dmark[(size_t)x] &= (uint8_t)~2u;
    p.dirty_pts.clear();
    p.dirty_roots.clear();
    const DownLayout L(nr, p.K);
    NextArgs a;
    a.xp = w.xp;
    a.d = d;
    a.k = p.K;
    a.n = p.n;
    a.req = reinterpret_cast<const NextReq*>(w.upload + req_off);
    a.nr = nr;
    a.comp = w.comp;
    a.csize = w.csize;
    a.dmax = p.dmax;
    a.out_len = reinterpret_cast<int32_t*>(w.download + L.len_off);
    a.out_j = reinterpret_cast<int32_t*>(w.download + L.j_off);
    a.out_s = reinterpret_cast<double*>(w.download + L.s_off);
    // enough workgroups for the chip: few points get more column ranges
    a.splits = nr >= TARGET_GROUPS / 2 ? 1 : (int32_t)std::min<int64_t>(64, (TARGET_GROUPS + nr - 1) / nr);
    a.part_j = w.part_j;
    a.part_s = w.part_s;
    a.part_len = w.part_len;
    const int64_t items = (int64_t)nr * a.splits;
    k_next_admissible<<<(unsigned)std::min<int64_t>(items, 8192), 256, 0, s>>>(a);
    k_merge_ranges<<<(unsigned)((nr + 3) / 4), 256, 0, s>>>(a);
    HIP_OK(hipGetLastError());
    char* down = (char*)p.down_pin.get(L.bytes);
    if (!down) return NNM_EDEVICE;
    HIP_OK(hipMemcpyAsync(down, w.download, L.bytes, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const int32_t* ol = reinterpret_cast<const int32_t*>(down + L.len_off);
    const int32_t* oj = reinterpret_cast<const int32_t*>(down + L.j_off);
    const double* os = reinterpret_cast<const double*>(down + L.s_off);
    for (int32_t q = 0; q < nr; ++q) {
        const int32_t r = p.spent[(size_t)q];
        p.queued[(size_t)r] = 0;
        const int32_t ln = ol[q];
        for (int32_t e = 0; e < ln; ++e) {
            p.lj[(size_t)r * p.K + e] = oj[(size_t)q * p.K + e];
            p.ls[(size_t)r * p.K + e] = os[(size_t)q * p.K + e];
        }
        p.len[(size_t)r] = ln;
        p.cur[(size_t)r] = 0;
        p.state[(size_t)r] = ln > 0 ? 0 : 2;
    }
    p.refills += 1;
    p.refilled_rows += nr;
    p.spent.clear();
    p.refill_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return NNM_OK;
}

// Every point's exact neighbour prefix (first needed when some cluster's
// smallest outgoing tree edge is blocked); each point joins the heap of its
// cluster as it is now.
nnm_status build_prefixes(Process& p, const float* X, int32_t d, int64_t ld, Workspace& w,
                          hipStream_t s)
{
    const size_t N = (size_t)p.n, K = (size_t)p.K;
    nnm_status st = knn_build(X, p.n, d, ld, p.K, p.opt, w.knn_ws, w.knn_bytes, w.idx, w.sd, w.len,
                              s, nullptr);
    if (st != NNM_OK) return st;
    k_pad_points<<<(unsigned)((p.n * DMAX + 255) / 256), 256, 0, s>>>(X, ld, d, p.n, w.xp);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(p.lj.data(), w.idx, 4 * N * K, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(p.ls.data(), w.sd, 8 * N * K, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(p.len.data(), w.len, 4 * N, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (size_t i = 0; i < N; ++i) {
        if (p.len[i] == 0) {
            p.state[i] = 2;
            continue;
        }
        p.hkey[i] = p.key_at((int32_t)i);
        p.push(p.cid[i], (int32_t)i);
    }
    p.rows_ready = true;
    return NNM_OK;
}

// Advance every point of cluster X past the prefix entries it can no longer
// use (inside X, not admissible, beyond dmax) and rebuild X's heap with
// each point's current lower bound.
nnm_status sweep(Process& p, int32_t X)
{
    std::vector<int32_t> rows, stack;
    if (p.hroot[(size_t)X] >= 0) stack.push_back(p.hroot[(size_t)X]);
    while (!stack.empty()) {
        const int32_t r = stack.back();
        stack.pop_back();
        rows.push_back(r);
        if (p.hl[(size_t)r] >= 0) stack.push_back(p.hl[(size_t)r]);
        if (p.hr[(size_t)r] >= 0) stack.push_back(p.hr[(size_t)r]);
    }
    p.hroot[(size_t)X] = -1;
    const int64_t sx = p.size[(size_t)X];
    for (int32_t r : rows) {
        while (p.state[(size_t)r] == 0) {
            const int32_t j = p.lj[(size_t)r * p.K + p.cur[(size_t)r]];
            const double sv = p.ls[(size_t)r * p.K + p.cur[(size_t)r]];
            if (sqrt(sv) > p.dmax) {
                p.state[(size_t)r] = 2;
                break;
            }
            const int32_t cj = p.cid[(size_t)j];
            if (cj != X && p.admissible(sx, p.size[(size_t)cj], sv)) break;
            if (++p.cur[(size_t)r] >= p.len[(size_t)r]) p.use_up(r);
        }
        if (p.state[(size_t)r] == 0) p.hkey[(size_t)r] = p.key_at(r);
        if (p.state[(size_t)r] != 2) p.push(X, r);
    }
    return NNM_OK;
}

// best(X): the smallest admissible pair leaving cluster X (false: none, ever).
nnm_status best_of(Process& p, int32_t X, const float* Xd, int32_t d, int64_t ld, Workspace& w,
                   hipStream_t s, PairKey* out, int32_t* partner, bool* found)
{
    // the smallest tree edge leaving X (edges now inside X are dropped)
    while (p.troot[(size_t)X] >= 0) {
        const int32_t t = p.troot[(size_t)X];
        const nnm_edge& e = p.tree[t >> 1];
        if (p.cid[(size_t)e.u] != p.cid[(size_t)e.v]) break;
        p.troot[(size_t)X] = p.tmeld(p.tl[(size_t)t], p.tr[(size_t)t]);
    }
    if (p.troot[(size_t)X] >= 0) {
        const nnm_edge& e = p.tree[p.troot[(size_t)X] >> 1];
        const int32_t Y = p.cid[(size_t)e.u] == X ? p.cid[(size_t)e.v] : p.cid[(size_t)e.u];
        if (p.admissible(p.size[(size_t)X], p.size[(size_t)Y], e.s)) {
            *out = PairKey{e.s, e.u, e.v};
            *partner = Y;
            *found = true;
            return NNM_OK;
        }
        // every pair leaving X is at least as long as this edge: beyond
        // dmax, none is admissible; and a cluster too large for any partner
        // has none either
        if (sqrt(e.s) > p.dmax || p.limit_of(p.size[(size_t)X]) < 1) {
            *found = false;
            return NNM_OK;
        }
    } else {
        *found = false;          // X holds all its instance's points
        return NNM_OK;
    }
    if (!p.rows_ready) {
        nnm_status st = build_prefixes(p, Xd, d, ld, w, s);
        if (st != NNM_OK) return st;
    }
    for (;;) {
        const int32_t r = p.hroot[(size_t)X];
        if (r < 0) {
            *found = false;
            return NNM_OK;
        }
        if (p.state[(size_t)r] == 2) {
            p.pop(X);
            continue;
        }
        if (p.state[(size_t)r] == 1) {
            // a used-up prefix at the top: bring every point of X past the
            // entries it can no longer use, then fetch all the next prefixes
            // in one scan
            nnm_status st = sweep(p, X);
            if (st == NNM_OK) st = refill(p, Xd, d, ld, w, s);
            if (st != NNM_OK) return st;
            continue;
        }
        const int32_t j = p.lj[(size_t)r * p.K + p.cur[(size_t)r]];
        const double sv = p.ls[(size_t)r * p.K + p.cur[(size_t)r]];
        const int32_t Y = p.cid[(size_t)j];
        if (Y == X || !p.admissible(p.size[(size_t)X], p.size[(size_t)Y], sv)) {
            p.pop(X);
            if (sqrt(sv) > p.dmax) {
                p.state[(size_t)r] = 2;            // every later key is larger
                continue;
            }
            if (++p.cur[(size_t)r] >= p.len[(size_t)r]) p.use_up(r);
            else p.hkey[(size_t)r] = p.key_at(r);
            if (p.state[(size_t)r] != 2) p.push(X, r);
            continue;
        }
        const PairKey kc = p.key_at(r);
        if (p.hkey[(size_t)r] < kc) {           // a stale lower bound: re-key
            p.pop(X);
            p.hkey[(size_t)r] = kc;
            p.push(X, r);
            continue;
        }
        *out = kc;
        *partner = Y;
        *found = true;
        return NNM_OK;
    }
}

struct Entry {
    int32_t cls;
    PairKey key;
    int32_t c, ver;
    bool operator>(const Entry& o) const
    {
        if (cls != o.cls) return cls > o.cls;
        return o.key < key;
    }
};

}  // namespace
}  // namespace nnm

using namespace nnm;

extern "C" nnm_status allpairs_cut_workspace_size(int64_t n, int32_t d, int32_t k,
                                                  const nnm_options* opt, size_t* bytes)
{
    if (!bytes || n < 1 || d < 1 || d > DMAX || k < 0 || k > KMAX) return NNM_EINVAL;
    const int32_t K = k > 0 ? k : DEFAULT_DEPTH;
    size_t kb = 0;
    nnm_status st = knn_workspace_size(n, d, K, opt, &kb);
    if (st != NNM_OK) return st;
    Workspace w;
    *bytes = carve_ap(n, K, kb, nullptr, &w);
    return NNM_OK;
}

extern "C" nnm_status cluster_cut_allpairs(const float* X_dev, int64_t n, int32_t d, int64_t ld,
                                           const nnm_edge* edges_host, const nnm_cut_params* prm,
                                           int32_t k, const nnm_options* opt, void* ws_dev,
                                           size_t ws_bytes, void* stream, int32_t* labels_host,
                                           int64_t* n_clusters, int64_t* stats)
{
    if (!X_dev || !prm || !ws_dev || !labels_host || !n_clusters) return NNM_EINVAL;
    if (n < 1 || n > (int64_t)0x7FFFFFF0 || d < 1 || d > DMAX || ld < d || k < 0 || k > KMAX)
        return NNM_EINVAL;
    if (n > 1 && !edges_host) return NNM_EINVAL;
    if (std::isnan(prm->dmax) || prm->dmax < 0.0) return NNM_EINVAL;
    if (opt && opt->metric != NNM_METRIC_EUCLIDEAN) return NNM_EUNSUPPORTED;
    for (int64_t e = 0; e + 1 < n; ++e) {
        const nnm_edge& x = edges_host[e];
        if (x.u < 0 || x.u >= x.v || x.v >= n || !(x.s >= 0.0)) return NNM_EINVAL;
    }
    const int32_t K = k > 0 ? k : DEFAULT_DEPTH;
    size_t need = 0;
    nnm_status st = allpairs_cut_workspace_size(n, d, K, opt, &need);
    if (st != NNM_OK) return st;
    if (ws_bytes < need) return NNM_EINVAL;
    Workspace w;
    size_t kb = 0;
    st = knn_workspace_size(n, d, K, opt, &kb);
    if (st != NNM_OK) return st;
    carve_ap(n, K, kb, (char*)ws_dev, &w);
    hipStream_t s = (hipStream_t)stream;
    Process p;
    p.n = n;
    p.K = K;
    p.kl1 = prm->kl1_max_clusters;
    p.kl2 = prm->kl2_max_size;
    p.kl3 = prm->kl3_max_merged;
    p.kl4 = prm->kl4_min_size;
    p.dmax = prm->dmax;
    const size_t N = (size_t)n;
    p.lj.assign(N * K, -1);
    p.ls.assign(N * K, 0.0);
    p.len.assign(N, 0);
    p.cur.assign(N, 0);
    p.state.assign(N, 0);
    p.queued.assign(N, 0);
    p.size.assign(N, 1);
    p.ver.assign(N, 0);
    p.hl.assign(N, -1);
    p.hr.assign(N, -1);
    p.hroot.assign(N, -1);
    p.hkey.resize(N);
    p.cid.resize(N);
    p.dmark.assign(N, 0);
    p.mnext.assign(N, -1);
    p.mhead.resize(N);
    p.mtail.resize(N);
    for (size_t i = 0; i < N; ++i) p.cid[i] = p.mhead[i] = p.mtail[i] = (int32_t)i;
    p.tree = edges_host;
    const size_t M = N > 0 ? 2 * (N - 1) : 0;
    p.tl.assign(M, -1);
    p.tr.assign(M, -1);
    p.troot.assign(N, -1);
    for (size_t e = 0; e + 1 < N; ++e) {
        p.troot[(size_t)edges_host[e].u] = p.tmeld(p.troot[(size_t)edges_host[e].u], (int32_t)(2 * e));
        p.troot[(size_t)edges_host[e].v] = p.tmeld(p.troot[(size_t)edges_host[e].v], (int32_t)(2 * e + 1));
    }
    p.opt = opt;
    const bool prio = p.kl4 > 1;
    std::priority_queue<Entry, std::vector<Entry>, std::greater<Entry>> G;
    // a point's smallest tree edge is its smallest pair: a lower bound of its best
    for (size_t i = 0; i < N; ++i) {
        const int32_t t = p.troot[i];
        if (t < 0) continue;
        const nnm_edge& e = edges_host[t >> 1];
        G.push(Entry{prio ? 0 : 1, PairKey{e.s, e.u, e.v}, (int32_t)i, 0});
    }
    int64_t clusters = n;
    while (!G.empty()) {
        if (p.kl1 > 0 && clusters <= p.kl1) break;
        const Entry e = G.top();
        G.pop();
        if (p.cid[(size_t)e.c] != e.c || p.ver[(size_t)e.c] != e.ver) continue;
        PairKey b;
        int32_t Y = -1;
        bool found = false;
        st = best_of(p, e.c, X_dev, d, ld, w, s, &b, &Y, &found);
        if (st != NNM_OK) return st;
        if (!found) continue;                    // no admissible pair, ever
        const int32_t cls = (prio && p.size[(size_t)e.c] < p.kl4) ? 0 : 1;
        const Entry now{cls, b, e.c, e.ver};
        if (!G.empty() && now > G.top()) {      // another cluster may come first
            G.push(now);
            continue;
        }
        // unite X and Y (the larger keeps its id)
        int32_t X = e.c;
        int32_t Z = X, o = Y;
        if (p.size[(size_t)Y] > p.size[(size_t)X]) std::swap(Z, o);
        p.size[(size_t)Z] += p.size[(size_t)o];
        p.hroot[(size_t)Z] = p.meld(p.hroot[(size_t)Z], p.hroot[(size_t)o]);
        p.hroot[(size_t)o] = -1;
        p.troot[(size_t)Z] = p.tmeld(p.troot[(size_t)Z], p.troot[(size_t)o]);
        p.troot[(size_t)o] = -1;
        for (int32_t x = p.mhead[(size_t)o]; x >= 0; x = p.mnext[(size_t)x]) {
            p.cid[(size_t)x] = Z;
            if (p.uploaded && !(p.dmark[(size_t)x] & 1)) {
                p.dmark[(size_t)x] |= 1;
                p.dirty_pts.push_back(x);
            }
        }
        if (p.uploaded && !(p.dmark[(size_t)Z] & 2)) {
            p.dmark[(size_t)Z] |= 2;
            p.dirty_roots.push_back(Z);
        }
        p.mnext[(size_t)p.mtail[(size_t)Z]] = p.mhead[(size_t)o];
        p.mtail[(size_t)Z] = p.mtail[(size_t)o];
        p.ver[(size_t)Z] += 1;
        p.ver[(size_t)o] += 1;
        --clusters;
        ++p.merges;
        // (class, key) of the pair just taken bounds the new cluster's from below
        G.push(Entry{cls, b, Z, p.ver[(size_t)Z]});
    }
    std::vector<int64_t> map(N, -1);
    int64_t next = 0;
    for (size_t i = 0; i < N; ++i) {
        const int32_t r = p.cid[i];
        if (map[(size_t)r] < 0) map[(size_t)r] = next++;
        labels_host[i] = (int32_t)map[(size_t)r];
    }
    *n_clusters = next;
    if (stats) {
        stats[0] = p.merges;
        stats[1] = p.refills;
        stats[2] = p.refilled_rows;
        stats[3] = K;
        stats[4] = (int64_t)(p.refill_ms * 1000.0);
    }
    return NNM_OK;
}
