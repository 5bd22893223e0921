// sort_scan.hip -- prefix sums, stream compaction and a stable LSD radix sort.
//
// Used to order points by component before every round (so that a tile of
// rows and a chunk of columns either share no component or are masked) and
// to sort the tree edges by key (s, u, v) at the end -- the paper's kernels
// sort the minimal pairs they select by distance before handing them on.
#include "nnm_common.h"

namespace nnm {
namespace {

constexpr int SCAN_TILE = 2048;   // 256 threads x 8
constexpr int RADIX_TILE = 2048;

__global__ __launch_bounds__(256) void k_scan_partial(const int32_t* __restrict__ in, int64_t n,
                                                      int32_t* __restrict__ bsum)
{
    __shared__ int32_t ws[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t acc = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t idx = base + e * 256 + threadIdx.x;
        if (idx < n) acc += in[idx];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Exclusive scan of the block sums in one workgroup (chunks of 1024).
__global__ __launch_bounds__(1024) void k_scan_top(int32_t* bsum, int64_t nb, int32_t* total)
{
    __shared__ int32_t buf[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        const int64_t idx = c0 + threadIdx.x;
        const int32_t v = idx < nb ? bsum[idx] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (idx < nb) bsum[idx] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                    const int32_t* __restrict__ bsum,
                                                    int32_t* __restrict__ out)
{
    __shared__ int32_t tsum[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 8;
    int32_t v[8];
    int32_t acc = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t idx = base + e;
        v[e] = idx < n ? in[idx] : 0;
        acc += v[e];
    }
    tsum[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t t = threadIdx.x >= off ? tsum[threadIdx.x - off] : 0;
        __syncthreads();
        tsum[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t run = bsum[blockIdx.x] + tsum[threadIdx.x] - acc;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t idx = base + e;
        if (idx < n) out[idx] = run;
        run += v[e];
    }
}

// clear (may alias flags): the flags, zeroed once read
__global__ __launch_bounds__(256) void k_compact_scatter(const int32_t* flags,
                                                         const int32_t* __restrict__ pos, int64_t n,
                                                         int32_t* __restrict__ out, int32_t* clear)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n && flags[i]) {
        out[pos[i]] = (int32_t)i;
        if (clear) clear[i] = 0;
    }
}

__device__ __forceinline__ uint32_t digit_of(const SortRec& r, int field, int shift)
{
    if (field == 0) return (uint32_t)((r.k0 >> shift) & 0xFFu);
    if (field == 1) return (r.k1 >> shift) & 0xFFu;
    return (r.k2 >> shift) & 0xFFu;
}

__global__ __launch_bounds__(256) void k_radix_hist(const SortRec* __restrict__ a, int64_t n,
                                                    int field, int shift, int32_t* __restrict__ hist,
                                                    int64_t nblocks)
{
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
#pragma unroll
    for (int e = 0; e < RADIX_TILE / 256; ++e) {
        const int64_t idx = base + e * 256 + threadIdx.x;
        if (idx < n) atomicAdd(&h[digit_of(a[idx], field, shift)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: items are ranked in index order (round by round, wave by
// wave, lane by lane) using ballots to find lanes holding the same digit.
__global__ __launch_bounds__(256) void k_radix_scatter(const SortRec* __restrict__ a,
                                                       SortRec* __restrict__ b, int64_t n,
                                                       int field, int shift,
                                                       const int32_t* __restrict__ offs,
                                                       int64_t nblocks)
{
    __shared__ int32_t base[256];
    __shared__ int32_t cnt[4][256];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    base[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t tile = (int64_t)blockIdx.x * RADIX_TILE;
    for (int r = 0; r < RADIX_TILE / 256; ++r) {
        cnt[0][tid] = 0; cnt[1][tid] = 0; cnt[2][tid] = 0; cnt[3][tid] = 0;
        __syncthreads();
        const int64_t idx = tile + r * 256 + tid;
        const bool valid = idx < n;
        SortRec rec;
        uint32_t dg = 0;
        if (valid) {
            rec = a[idx];
            dg = digit_of(rec, field, shift);
        }
        unsigned long long m = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (dg >> bit) & 1u;
            const unsigned long long bb = __ballot(on);
            m &= on ? bb : ~bb;
        }
        const int rank = __popcll(m & lt);
        if (valid && rank == 0) cnt[wave][dg] = __popcll(m);
        __syncthreads();
        if (valid) {
            int pre = 0;
            for (int w = 0; w < wave; ++w) pre += cnt[w][dg];
            const int64_t dst = (int64_t)base[dg] + pre + rank;
            if (dst >= 0 && dst < n) b[dst] = rec;
        }
        __syncthreads();
        base[tid] += cnt[0][tid] + cnt[1][tid] + cnt[2][tid] + cnt[3][tid];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_comp_records(const int32_t* __restrict__ comp, int64_t n,
                                                      SortRec* __restrict__ rec)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    SortRec r;
    r.k0 = 0;
    r.k1 = (uint32_t)comp[i];
    r.k2 = (uint32_t)i;
    rec[i] = r;
}

__global__ __launch_bounds__(256) void k_perm_from_records(const SortRec* __restrict__ rec, int64_t n,
                                                           int32_t* __restrict__ perm)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) perm[i] = (int32_t)rec[i].k2;
}

__global__ __launch_bounds__(256) void k_write_edges(const SortRec* __restrict__ rec, int64_t ne,
                                                     nnm_edge* __restrict__ out, int metric)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const SortRec r = rec[e];
    nnm_edge o;
    o.u = (int32_t)r.k1;
    o.v = (int32_t)r.k2;
    o.s = __longlong_as_double((long long)r.k0);
    o.w = metric_key_is_distance(metric) ? o.s : __dsqrt_rn(o.s);
    out[e] = o;
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* p, int32_t v, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// p[0 .. d->n_rows) = v over a fixed grid
__global__ __launch_bounds__(256) void k_fill_i32_desc(int32_t* p, int32_t v, const LaunchDesc* d)
{
    const int64_t n = d->n_rows;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Column splits per row tile for a launch of `tiles` tiles: enough
// workgroups for `target` in all, at most one split per 65536 columns and
// at most 64 (the host's rule for host-sized launches).
__device__ __forceinline__ int32_t splits_for(int64_t tiles, int64_t np, int32_t target, int32_t fixed)
{
    if (fixed > 0) return fixed;
    if (tiles < 1) tiles = 1;
    int64_t want = (target + tiles - 1) / tiles;
    const int64_t cap = np / 65536;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    if (want > 64) want = 64;
    return (int32_t)want;
}

__global__ __launch_bounds__(64) void k_desc_rows(LaunchDesc* d, const int32_t* count, int32_t off,
                                                  int32_t cap, int64_t np, int32_t target,
                                                  int32_t fixed)
{
    if (threadIdx.x != 0) return;
    int32_t n = *count - off;
    n = n < 0 ? 0 : (n > cap ? cap : n);
    d->n_rows = n;
    d->n_tiles = (n + 255) / 256;
    d->splits = splits_for(d->n_tiles, np, target, fixed);
    d->queue = 0;
    d->over = 0;
}

// k_desc_rows and the clearing of a launch's per-row buffers in one kernel:
// every thread derives n_rows from *count itself
__global__ __launch_bounds__(256) void k_prep_launch(LaunchDesc* d, const int32_t* count, int32_t off,
                                                     int32_t cap, int64_t np, int32_t target,
                                                     int32_t fixed, int32_t* surv_cnt, uint32_t* tfin,
                                                     uint32_t* gT, uint32_t* gU)
{
    int32_t n = *count - off;
    n = n < 0 ? 0 : (n > cap ? cap : n);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d->n_rows = n;
        d->n_tiles = (n + 255) / 256;
        d->splits = splits_for(d->n_tiles, np, target, fixed);
        d->queue = 0;
        d->over = 0;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        surv_cnt[i] = 0;
        if (tfin) tfin[i] = 0x7F800000u;
        gT[i] = 0x7F800000u;
        gU[i] = 0x7F800000u;
    }
}

__global__ __launch_bounds__(64) void k_desc_splits(LaunchDesc* d, int64_t np, int32_t target,
                                                    int32_t fixed)
{
    if (threadIdx.x != 0) return;
    d->splits = splits_for(d->n_tiles, np, target, fixed);
}

__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t scan_temp_bytes(int64_t n)
{
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    return (size_t)(nb + 64) * sizeof(int32_t) + (size_t)n * sizeof(int32_t) + 256;
}

hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, void* temp,
                                 int32_t* total, hipStream_t s)
{
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    int32_t* bsum = (int32_t*)temp;
    if (n <= 0) return hipSuccess;
    k_scan_partial<<<(unsigned)nb, 256, 0, s>>>(in, n, bsum);
    k_scan_top<<<1, 1024, 0, s>>>(bsum, nb, total);
    k_scan_apply<<<(unsigned)nb, 256, 0, s>>>(in, n, bsum, out);
    return hipGetLastError();
}

hipError_t launch_compact(const int32_t* flags, int64_t n, int32_t* out_list, int32_t* out_count,
                          void* temp, hipStream_t s)
{
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    int32_t* pos = (int32_t*)temp + (nb + 64);
    hipError_t e = launch_exclusive_scan(flags, pos, n, temp, out_count, s);
    if (e != hipSuccess) return e;
    k_compact_scatter<<<g256(n), 256, 0, s>>>(flags, pos, n, out_list, nullptr);
    return hipGetLastError();
}

hipError_t launch_compact_clear(int32_t* flags, int64_t n, int32_t* out_list, int32_t* out_count,
                                void* temp, hipStream_t s)
{
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    int32_t* pos = (int32_t*)temp + (nb + 64);
    hipError_t e = launch_exclusive_scan(flags, pos, n, temp, out_count, s);
    if (e != hipSuccess) return e;
    k_compact_scatter<<<g256(n), 256, 0, s>>>(flags, pos, n, out_list, flags);
    return hipGetLastError();
}

size_t radix_temp_bytes(int64_t n)
{
    const int64_t nb = (n + RADIX_TILE - 1) / RADIX_TILE;
    const int64_t h = 256 * nb;
    return (size_t)h * sizeof(int32_t) * 2 + scan_temp_bytes(h) + 256;
}

hipError_t launch_radix_sort(SortRec* a, SortRec* b, int64_t n, const int* fields, const int* bits,
                             int nfields, void* temp, SortRec** result, hipStream_t s)
{
    *result = a;
    if (n <= 1) return hipSuccess;
    const int64_t nb = (n + RADIX_TILE - 1) / RADIX_TILE;
    const int64_t h = 256 * nb;
    int32_t* hist = (int32_t*)temp;
    int32_t* offs = hist + h;
    void* stemp = offs + h;
    SortRec* src = a;
    SortRec* dst = b;
    for (int f = 0; f < nfields; ++f) {
        for (int shift = 0; shift < bits[f]; shift += 8) {
            k_radix_hist<<<(unsigned)nb, 256, 0, s>>>(src, n, fields[f], shift, hist, nb);
            hipError_t e = launch_exclusive_scan(hist, offs, h, stemp, nullptr, s);
            if (e != hipSuccess) return e;
            k_radix_scatter<<<(unsigned)nb, 256, 0, s>>>(src, dst, n, fields[f], shift, offs, nb);
            SortRec* t = src;
            src = dst;
            dst = t;
        }
    }
    *result = src;
    return hipGetLastError();
}

hipError_t launch_comp_records(const int32_t* comp, int64_t n, SortRec* rec, hipStream_t s)
{
    k_comp_records<<<g256(n), 256, 0, s>>>(comp, n, rec);
    return hipGetLastError();
}

hipError_t launch_perm_from_records(const SortRec* rec, int64_t n, int32_t* perm, hipStream_t s)
{
    k_perm_from_records<<<g256(n), 256, 0, s>>>(rec, n, perm);
    return hipGetLastError();
}

hipError_t launch_write_edges(const SortRec* rec, int64_t ne, nnm_edge* out, int metric,
                              hipStream_t s)
{
    if (ne <= 0) return hipSuccess;
    k_write_edges<<<g256(ne), 256, 0, s>>>(rec, ne, out, metric);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<g256(n), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_i32_desc(int32_t* p, int32_t v, const LaunchDesc* d, hipStream_t s)
{
    k_fill_i32_desc<<<1024, 256, 0, s>>>(p, v, d);
    return hipGetLastError();
}

hipError_t launch_desc_rows(LaunchDesc* d, const int32_t* count, int32_t off, int32_t cap,
                            int64_t np, int32_t target, int32_t fixed_splits, hipStream_t s)
{
    k_desc_rows<<<1, 64, 0, s>>>(d, count, off, cap, np, target, fixed_splits);
    return hipGetLastError();
}

hipError_t launch_prep_launch(LaunchDesc* d, const int32_t* count, int32_t off, int32_t cap,
                              int64_t np, int32_t target, int32_t fixed_splits, int32_t* surv_cnt,
                              uint32_t* tfin, uint32_t* gT, uint32_t* gU, hipStream_t s)
{
    k_prep_launch<<<1024, 256, 0, s>>>(d, count, off, cap, np, target, fixed_splits, surv_cnt, tfin,
                                       gT, gU);
    return hipGetLastError();
}

hipError_t launch_desc_splits(LaunchDesc* d, int64_t np, int32_t target, int32_t fixed_splits,
                              hipStream_t s)
{
    k_desc_splits<<<1, 64, 0, s>>>(d, np, target, fixed_splits);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_u64<<<g256(n), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

}  // namespace nnm
