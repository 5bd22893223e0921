// merge.hip -- one round of component merging (Boruvka) on the GPU.
//
// The section on constructing the set of minimum distances unites clusters
// along minimal pairs and repeats while clustering is not over.  Here every
// round takes, for every component, its smallest outgoing pair under the key
// (s, min index, max index) -- by the cut property that pair is a tree edge
// -- hooks each component to its partner, resolves the mutual pairs, and
// collapses the resulting trees by pointer jumping.
//
// Row minima come from each point's cached exact neighbour prefix: a cursor
// skips entries that are now inside the point's own component.  A point
// whose list is used up only has a lower bound (its last listed key); it is
// rescanned only if that bound does not exceed the best pair its component
// already has from other rows.  All reductions use integer atomics on keys,
// so every result is independent of scheduling.
#include "nnm_common.h"

namespace nnm {
namespace {

constexpr unsigned long long NONE = 0xFFFFFFFFFFFFFFFFull;

__device__ __forceinline__ unsigned long long sbits(double s)
{
    return (unsigned long long)__double_as_longlong(s);
}

__global__ __launch_bounds__(256) void k_init_points(MergeArgs a)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    a.comp[i] = (int32_t)i;
    a.parent[i] = (int32_t)i;
    a.ccur[i] = 0;
    a.rstat[i] = 0;
    a.cbest_s[i] = NONE;
    a.cbest_p[i] = NONE;
    a.clen[i] = 0;
    a.cflag[i] = 0;
    a.clb[i] = -1.0;              // no information yet: always scan
}

__global__ __launch_bounds__(256) void k_cursor(MergeArgs a)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int c = a.comp[i];
    const int len = a.clen[i];
    int cur = a.ccur[i];
    const int32_t* li = a.cidx + i * a.k;
    while (cur < len && a.comp[li[cur]] == c) ++cur;
    a.ccur[i] = cur;
    if (cur < len) {
        a.rstat[i] = 1;
        a.rbest_s[i] = a.cs[i * a.k + cur];
        a.rbest_j[i] = li[cur];
    } else if (a.cflag[i] & 1) {
        a.rstat[i] = 0;          // every point is in this component
    } else {
        a.rstat[i] = 2;          // list used up: only a lower bound is known
    }
}

// By sorted position: a component's points are contiguous there, so a wave
// mostly serves one component and issues one atomic for it.
__global__ __launch_bounds__(256) void k_compmin1(MergeArgs a)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool in = p < a.n;
    int c = -1;
    unsigned long long key = NONE;
    if (in) {
        const int i = a.perm[p];
        c = a.comp[i];
        if (a.rstat[i] == 1) key = sbits(a.rbest_s[i]);
    }
    const int c0 = __shfl(c, 0);      // lane 0 is in range whenever any lane is
    if (__ballot(in && c != c0) == 0ull) {
        unsigned long long m = key;
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(m, off);
            m = o < m ? o : m;
        }
        if ((threadIdx.x & 63) == 0 && m != NONE && m < __atomic_load_n(&a.cbest_s[c0], __ATOMIC_RELAXED))
            atomicMin(&a.cbest_s[c0], m);
    } else if (key != NONE && key < __atomic_load_n(&a.cbest_s[c], __ATOMIC_RELAXED)) {
        atomicMin(&a.cbest_s[c], key);
    }
}

// By sorted position, so the rescan list comes out in component order.
__global__ __launch_bounds__(256) void k_flag_rescan(MergeArgs a)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int i = a.perm[p];
    int f = 0;
    double u0 = -1.0;
    if (a.rstat[i] == 2) {
        const unsigned long long B = a.cbest_s[a.comp[i]];
        const double lb = a.clb[i];
        if (a.disable_prune || lb < 0.0 || B == NONE || sbits(lb) <= B) {
            f = 1;
            if (B != NONE && !a.disable_prune) u0 = __longlong_as_double((long long)B);
        }
    }
    a.rflag[p] = f;
    a.u0s[p] = u0;
}

// Flagged rows of components that have no bound yet (every row of such a
// component is flagged): up to REPS rows evenly spaced along the component's
// segment of the sorted order (which is spatially ordered) represent it.
constexpr int REPS = 8;

__global__ __launch_bounds__(256) void k_rep_flags(MergeArgs a, const int32_t* seg,
                                                   const int32_t* segstart, int64_t nseg,
                                                   int32_t* flag2, const int32_t* nseg_dev)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    if (nseg_dev) nseg = *nseg_dev;
    int f = 0;
    if (a.rflag[p] && a.u0s[p] < 0.0) {
        const int sg = seg[p];
        const int64_t st = segstart[sg];
        const int64_t en = (sg + 1 < nseg) ? segstart[sg + 1] : a.n;
        int64_t stride = (en - st) / REPS;
        if (stride < 1) stride = 1;
        f = ((p - st) % stride == 0) ? 1 : 0;
    }
    flag2[p] = f;
}

__global__ __launch_bounds__(64) void k_rep_select(const int32_t* nrep, const int32_t* rcount,
                                                   int32_t* eff)
{
    if (threadIdx.x != 0) return;
    const int32_t r = *nrep;
    *eff = (r > 0 && r < *rcount) ? r : 0;
}

__global__ __launch_bounds__(256) void k_copy_i32_dev(int32_t* __restrict__ dst,
                                                      const int32_t* __restrict__ src,
                                                      const int32_t* __restrict__ count)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < *count) dst[i] = src[i];
}

// ---- the P-minimal-pairs pass (mst_build_pminimal) ------------------------

__device__ __forceinline__ unsigned long long pack_pair(int i, int j)
{
    const unsigned long long lo = (unsigned long long)(i < j ? i : j);
    const unsigned long long hi = (unsigned long long)(i < j ? j : i);
    return (lo << 32) | hi;
}

// The pass threshold: the smallest pair key over the last entries of the
// lists that do not hold every outside point (any pair below it is in
// some row's list).  Two steps: the key bits, then (lo, hi) among rows that
// reach them.  thr[0] = s bits, thr[1] = packed (lo, hi).
__global__ __launch_bounds__(256) void k_pm_thr_s(MergeArgs a, unsigned long long* thr)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int len = a.clen[i];
    if ((a.cflag[i] & 1) || len <= 0) return;
    atomicMin(&thr[0], sbits(a.cs[i * a.k + len - 1]));
}

__global__ __launch_bounds__(256) void k_pm_thr_p(MergeArgs a, unsigned long long* thr)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int len = a.clen[i];
    if ((a.cflag[i] & 1) || len <= 0) return;
    if (sbits(a.cs[i * a.k + len - 1]) != thr[0]) return;
    atomicMin(&thr[1], pack_pair((int)i, a.cidx[i * a.k + len - 1]));
}

// Every listed pair below the threshold, once from each of its rows
// (duplicates sit side by side after the key sort).
__global__ __launch_bounds__(256) void k_pm_emit(MergeArgs a, const unsigned long long* thr,
                                                 SortRec* out, int32_t* count, int64_t cap)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int len = a.clen[i];
    const unsigned long long ts = thr[0], tp = thr[1];
    for (int e = 0; e < len; ++e) {
        const unsigned long long sb = sbits(a.cs[i * a.k + e]);
        const int j = a.cidx[i * a.k + e];
        const unsigned long long pp = pack_pair((int)i, j);
        if (sb > ts || (sb == ts && pp >= tp)) break;        // lists are ascending
        const int pos = atomicAdd(count, 1);
        if (pos < cap) {
            SortRec r;
            r.k0 = sb;
            r.k1 = (uint32_t)(pp >> 32);
            r.k2 = (uint32_t)(pp & 0xFFFFFFFFu);
            out[pos] = r;
        }
    }
}

__global__ __launch_bounds__(256) void k_seg_starts(const int32_t* seg, int64_t n, int32_t* segstart)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (p == 0 || seg[p] != seg[p - 1]) segstart[seg[p]] = (int32_t)p;
}

__global__ __launch_bounds__(256) void k_compmin2(MergeArgs a)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    if (a.rstat[i] != 1) return;
    const int c = a.comp[i];
    if (sbits(a.rbest_s[i]) != a.cbest_s[c]) return;
    const unsigned long long j = (unsigned long long)a.rbest_j[i];
    const unsigned long long lo = (unsigned long long)i < j ? (unsigned long long)i : j;
    const unsigned long long hi = (unsigned long long)i < j ? j : (unsigned long long)i;
    atomicMin(&a.cbest_p[c], (lo << 32) | hi);
}

__global__ __launch_bounds__(256) void k_hook(MergeArgs a)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    if (a.comp[c] != c) return;
    if (a.cbest_s[c] == NONE) { a.parent[c] = (int32_t)c; return; }
    const unsigned long long p = a.cbest_p[c];
    const int lo = (int)(p >> 32), hi = (int)(p & 0xFFFFFFFFu);
    const int cl = a.comp[lo], ch = a.comp[hi];
    a.parent[c] = (cl == c) ? ch : cl;
}

// A mutual pair picked the same edge (keys are distinct); its smaller root
// stays a root.
__global__ __launch_bounds__(256) void k_break(MergeArgs a)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    if (a.comp[c] != c) return;
    const int p = a.parent[c];
    if (p != c && a.parent[p] == c && c < p) a.parent[c] = (int32_t)c;
}

// Workgroups of the kernels below that count into one global counter: one
// atomic per workgroup (a per-wave atomic serialised some 30,000 waves on one
// address in the first round).
constexpr int AGG = 1024;

// One counter atomic per workgroup; its waves take consecutive runs of slots.
__global__ __launch_bounds__(AGG) void k_emit(MergeArgs a)
{
    __shared__ int wbase[AGG / 64];
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool emit = c < a.n && a.comp[c] == c && a.parent[c] != c;
    const unsigned long long m = __ballot(emit);
    if (lane == 0) wbase[wave] = (int)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < AGG / 64; ++w) {
            const int cnt = wbase[w];
            wbase[w] = tot;
            tot += cnt;
        }
        const int base = tot > 0 ? atomicAdd(&a.counters[0], tot) : 0;
        for (int w = 0; w < AGG / 64; ++w) wbase[w] += base;
    }
    __syncthreads();
    if (!emit) return;
    const int e = wbase[wave] + (int)__popcll(m & ((1ull << lane) - 1ull));
    if (e >= a.n) return;   // cannot happen: a tree has n - 1 edges
    const unsigned long long p = a.cbest_p[c];
    SortRec r;
    r.k0 = a.cbest_s[c];
    r.k1 = (uint32_t)(p >> 32);
    r.k2 = (uint32_t)(p & 0xFFFFFFFFu);
    a.edges[e] = r;
}

__global__ __launch_bounds__(256) void k_jump(MergeArgs a)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    if (a.comp[c] != c) return;
    const int p = a.parent[c];
    const int pp = a.parent[p];
    if (pp != p) a.parent[c] = pp;
}

// counters[1] = roots left, counters[2] = pointers not yet at a root
// (counted per workgroup in LDS, then one atomic each).
__global__ __launch_bounds__(AGG) void k_jump_check(MergeArgs a)
{
    __shared__ int cnt[2];
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool miss = false, root = false;
    if (c < a.n && a.comp[c] == c) {
        const int p = a.parent[c];
        miss = a.parent[p] != p;
        root = p == c;
    }
    const unsigned long long mm = __ballot(miss), mr = __ballot(root);
    if ((threadIdx.x & 63) == 0) {
        if (mm) atomicAdd(&cnt[0], (int)__popcll(mm));
        if (mr) atomicAdd(&cnt[1], (int)__popcll(mr));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (cnt[0]) atomicAdd(&a.counters[2], cnt[0]);
        if (cnt[1]) atomicAdd(&a.counters[1], cnt[1]);
    }
}

__global__ __launch_bounds__(256) void k_relabel(MergeArgs a)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    a.comp[i] = a.parent[a.comp[i]];
}

__global__ __launch_bounds__(256) void k_reset_comp(MergeArgs a)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    a.cbest_s[i] = NONE;
    a.cbest_p[i] = NONE;
}

__global__ __launch_bounds__(256) void k_export_knn(int64_t n, int k, const int32_t* __restrict__ cidx,
                                                    const double* __restrict__ cs,
                                                    const int32_t* __restrict__ clen,
                                                    int32_t* __restrict__ idx, double* __restrict__ sd,
                                                    int32_t* __restrict__ len)
{
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int64_t i = e / k;
    const int r = (int)(e % k);
    const int l = clen[i];
    if (r < l) {
        idx[e] = cidx[e];
        sd[e] = cs[e];
    } else {
        idx[e] = -1;
        sd[e] = __builtin_huge_val();
    }
    if (r == 0) len[i] = l;
}

inline unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256); }
inline unsigned gagg(int64_t n) { return (unsigned)((n + AGG - 1) / AGG); }

}  // namespace

hipError_t launch_export_knn(int64_t n, int k, const int32_t* cidx, const double* cs,
                             const int32_t* clen, int32_t* idx, double* sd, int32_t* len,
                             hipStream_t s)
{
    k_export_knn<<<g256(n * k), 256, 0, s>>>(n, k, cidx, cs, clen, idx, sd, len);
    return hipGetLastError();
}

#define NNM_LAUNCH1(name)                                   \
    hipError_t launch_##name(const MergeArgs& a, hipStream_t s) \
    {                                                       \
        k_##name<<<g256(a.n), 256, 0, s>>>(a);              \
        return hipGetLastError();                           \
    }

NNM_LAUNCH1(init_points)
NNM_LAUNCH1(cursor)
NNM_LAUNCH1(compmin1)
NNM_LAUNCH1(flag_rescan)
NNM_LAUNCH1(compmin2)
NNM_LAUNCH1(relabel)
NNM_LAUNCH1(reset_comp)
hipError_t launch_jump_check(const MergeArgs& a, hipStream_t s)
{
    k_jump_check<<<gagg(a.n), AGG, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_hook(const MergeArgs& a, hipStream_t s)
{
    k_hook<<<g256(a.n), 256, 0, s>>>(a);
    k_break<<<g256(a.n), 256, 0, s>>>(a);
    k_emit<<<gagg(a.n), AGG, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_pick_reps(const MergeArgs& a, const int32_t* seg, int32_t* segstart,
                            int64_t nseg, int32_t* flag2, hipStream_t s)
{
    k_seg_starts<<<g256(a.n), 256, 0, s>>>(seg, a.n, segstart);
    k_rep_flags<<<g256(a.n), 256, 0, s>>>(a, seg, segstart, nseg, flag2, nullptr);
    return hipGetLastError();
}

hipError_t launch_pick_reps_dev(const MergeArgs& a, const int32_t* seg, int32_t* segstart,
                                const int32_t* nseg, int32_t* flag2, hipStream_t s)
{
    k_seg_starts<<<g256(a.n), 256, 0, s>>>(seg, a.n, segstart);
    k_rep_flags<<<g256(a.n), 256, 0, s>>>(a, seg, segstart, 0, flag2, nseg);
    return hipGetLastError();
}

hipError_t launch_pm_candidates(const MergeArgs& a, unsigned long long* thr, SortRec* out,
                                int32_t* count, int64_t cap, hipStream_t s)
{
    k_pm_thr_s<<<g256(a.n), 256, 0, s>>>(a, thr);
    k_pm_thr_p<<<g256(a.n), 256, 0, s>>>(a, thr);
    k_pm_emit<<<g256(a.n), 256, 0, s>>>(a, thr, out, count, cap);
    return hipGetLastError();
}

hipError_t launch_rep_select(const int32_t* nrep, const int32_t* rcount, int32_t* eff, hipStream_t s)
{
    k_rep_select<<<1, 64, 0, s>>>(nrep, rcount, eff);
    return hipGetLastError();
}

hipError_t launch_copy_i32_dev(int32_t* dst, const int32_t* src, const int32_t* count, int64_t cap,
                               hipStream_t s)
{
    k_copy_i32_dev<<<g256(cap), 256, 0, s>>>(dst, src, count);
    return hipGetLastError();
}

hipError_t launch_jump(const MergeArgs& a, int iters, hipStream_t s)
{
    for (int it = 0; it < iters; ++it) k_jump<<<g256(a.n), 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace nnm
