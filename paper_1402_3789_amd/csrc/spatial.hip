// spatial.hip -- a spatial order of the points and bounding balls of chunks.
//
// The candidate pass visits, for every tile of rows, the chunks of columns
// nearest to it first and skips chunks that provably hold no pair the rows
// still need.  Both rely on consecutive points being close in space:
//   - a two-level landmark partition: every point goes to its nearest of
//     L2 coarse landmarks, then to its nearest fine landmark among those
//     that fell into the same coarse cell; points are ordered by fine cell
//     (cells of one coarse cell adjacent).  The order only steers the
//     search; results never depend on it.
//   - after each merge round components are ordered by the earliest spatial
//     position of their members, points inside a component by spatial
//     position, and every sorted position gets a monotone segment id.
//   - per chunk of BN sorted positions: a centre (FP32) and a radius rounded
//     up in FP64, so that ||x_i - x_j|| >= ||c_R - c_C|| - r_R - r_C holds
//     for every pair across two balls.
#include <vector>

#include "nnm_common.h"

namespace nnm {
namespace {

inline unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256); }

// nearest of L2 coarse landmarks (landmark l is point lm[l]); FP32, ties to
// the smaller landmark number
__global__ __launch_bounds__(256) void k_assign_coarse(const float* __restrict__ X, int64_t n, int d,
                                                       int64_t ld, const int32_t* __restrict__ lm,
                                                       int L2, int32_t* __restrict__ coarse)
{
    extern __shared__ float lc[];   // [L2][d]
    for (int e = threadIdx.x; e < L2 * d; e += blockDim.x) {
        const int l = e / d, f = e % d;
        lc[e] = X[(int64_t)lm[l] * ld + f];
    }
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[DMAX];
    for (int f = 0; f < d; ++f) x[f] = X[i * ld + f];
    float best = __builtin_huge_valf();
    int bl = 0;
    for (int l = 0; l < L2; ++l) {
        float t = 0.f;
        for (int f = 0; f < d; ++f) {
            const float df = x[f] - lc[l * d + f];
            t = __builtin_fmaf(df, df, t);
        }
        if (t < best) { best = t; bl = l; }
    }
    coarse[i] = bl;
}

// Fine landmarks sorted by coarse cell: flm[q] (point id), q in
// [goff[c], goff[c+1]) for coarse cell c.  key[i] = fine position.
__global__ __launch_bounds__(256) void k_assign_fine(const float* __restrict__ X, int64_t n, int d,
                                                     int64_t ld, const int32_t* __restrict__ coarse,
                                                     const int32_t* __restrict__ flm,
                                                     const int32_t* __restrict__ goff,
                                                     uint32_t* __restrict__ key)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = coarse[i];
    const int q0 = goff[c], q1 = goff[c + 1];
    float x[DMAX];
    for (int f = 0; f < d; ++f) x[f] = X[i * ld + f];
    float best = __builtin_huge_valf();
    int bq = q0;
    for (int q = q0; q < q1; ++q) {
        const float* y = X + (int64_t)flm[q] * ld;
        float t = 0.f;
        for (int f = 0; f < d; ++f) {
            const float df = x[f] - y[f];
            t = __builtin_fmaf(df, df, t);
        }
        if (t < best) { best = t; bq = q; }
    }
    key[i] = (uint32_t)bq;
}

__global__ __launch_bounds__(256) void k_records_u32(const uint32_t* __restrict__ key, int64_t n,
                                                     SortRec* __restrict__ rec)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    SortRec r;
    r.k0 = 0;
    r.k1 = key[i];
    r.k2 = (uint32_t)i;
    rec[i] = r;
}

// fine landmark records: k1 = coarse cell of the landmark, k2 = point id
__global__ __launch_bounds__(256) void k_fine_records(const int32_t* __restrict__ coarse,
                                                      const int32_t* __restrict__ lm, int L1,
                                                      SortRec* __restrict__ rec)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= L1) return;
    SortRec r;
    r.k0 = 0;
    r.k1 = (uint32_t)coarse[lm[q]];
    r.k2 = (uint32_t)lm[q];
    rec[q] = r;
}

// One block: flm from the sorted records, goff[c] = first q of cell c.
__global__ __launch_bounds__(1024) void k_fine_groups(const SortRec* __restrict__ rec, int L1, int L2,
                                                      int32_t* __restrict__ flm,
                                                      int32_t* __restrict__ goff)
{
    for (int q = threadIdx.x; q < L1; q += blockDim.x) flm[q] = (int32_t)rec[q].k2;
    for (int c = threadIdx.x; c <= L2; c += blockDim.x) {
        // lower bound of c among the sorted coarse ids
        int lo = 0, hi = L1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((int)rec[mid].k1 < c) lo = mid + 1;
            else hi = mid;
        }
        goff[c] = lo;
    }
}

__global__ __launch_bounds__(256) void k_rank_of(const int32_t* __restrict__ perm, int64_t n,
                                                 int32_t* __restrict__ rank)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n) rank[perm[p]] = (int32_t)p;
}

__global__ __launch_bounds__(256) void k_ckey_reset(int32_t* __restrict__ ckey, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) ckey[i] = 0x7FFFFFFF;
}

__global__ __launch_bounds__(256) void k_ckey_min(const int32_t* __restrict__ comp,
                                                  const int32_t* __restrict__ rank0, int64_t n,
                                                  int32_t* __restrict__ ckey)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) atomicMin(&ckey[comp[i]], rank0[i]);
}

// records in spatial order: k1 = key of the point's component, k2 = point
__global__ __launch_bounds__(256) void k_comp_records_spatial(const int32_t* __restrict__ perm0,
                                                              const int32_t* __restrict__ comp,
                                                              const int32_t* __restrict__ ckey,
                                                              int64_t n, SortRec* __restrict__ rec)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int i = perm0[q];
    SortRec r;
    r.k0 = 0;
    r.k1 = (uint32_t)ckey[comp[i]];
    r.k2 = (uint32_t)i;
    rec[q] = r;
}

__global__ __launch_bounds__(256) void k_segment_flags(const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ comp, int64_t n,
                                                       int32_t* __restrict__ flag)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    flag[p] = (p == 0 || comp[perm[p]] != comp[perm[p - 1]]) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_segment_ids(const int32_t* __restrict__ flag,
                                                     const int32_t* __restrict__ excl, int64_t n,
                                                     int32_t* __restrict__ seg)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n) seg[p] = excl[p] + flag[p] - 1;
}

// One block per chunk of `bn` sorted positions: centre = FP64 mean rounded
// to FP32, radius = FP64 max distance to that centre, rounded up.
__global__ __launch_bounds__(256) void k_chunk_balls(const float* __restrict__ X, int64_t n, int d,
                                                     int64_t ld, const int32_t* __restrict__ perm,
                                                     int bn, float* __restrict__ balls)
{
    __shared__ double acc[4][DMAX];
    __shared__ float cen[DMAX];
    __shared__ double rmax[4];
    const int64_t c0 = (int64_t)blockIdx.x * bn;
    int64_t c1 = c0 + bn;
    if (c1 > n) c1 = n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double sum[DMAX];
    for (int f = 0; f < DMAX; ++f) sum[f] = 0.0;
    for (int64_t p = c0 + threadIdx.x; p < c1; p += blockDim.x) {
        const float* x = X + (int64_t)perm[p] * ld;
        for (int f = 0; f < d; ++f) sum[f] += (double)x[f];
    }
    for (int f = 0; f < d; ++f) {
        double v = sum[f];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) acc[wave][f] = v;
    }
    __syncthreads();
    if (threadIdx.x < d) {
        const double m = (acc[0][threadIdx.x] + acc[1][threadIdx.x] + acc[2][threadIdx.x] +
                          acc[3][threadIdx.x]) / (double)(c1 - c0);
        cen[threadIdx.x] = (float)m;
    }
    __syncthreads();
    double r2 = 0.0;
    for (int64_t p = c0 + threadIdx.x; p < c1; p += blockDim.x) {
        const float* x = X + (int64_t)perm[p] * ld;
        double s = 0.0;
        for (int f = 0; f < d; ++f) {
            const double df = (double)x[f] - (double)cen[f];
            s += df * df;
        }
        r2 = s > r2 ? s : r2;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(r2, off);
        r2 = o > r2 ? o : r2;
    }
    if (lane == 0) rmax[wave] = r2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = rmax[0];
        for (int w = 1; w < 4; ++w) m = rmax[w] > m ? rmax[w] : m;
        balls[(int64_t)blockIdx.x * (DMAX + 1) + DMAX] = d2f_up(__builtin_sqrt(m) * (1.0 + 0x1p-40));
    }
    if (threadIdx.x < DMAX)
        balls[(int64_t)blockIdx.x * (DMAX + 1) + threadIdx.x] = threadIdx.x < d ? cen[threadIdx.x] : 0.f;
}

}  // namespace

size_t spatial_temp_bytes(int64_t n, int L1, int L2)
{
    return (size_t)n * 4 * 3 + (size_t)L1 * 4 * 2 + (size_t)(L2 + 1) * 4 + (size_t)L1 * sizeof(SortRec) * 2 +
           radix_temp_bytes(L1 > n ? L1 : n) + 4096;
}

// perm0 (spatial order) and rank0 (its inverse) for n points.
hipError_t launch_spatial_order(const float* X, int64_t n, int d, int64_t ld, int L1, int L2,
                                int32_t* perm0, int32_t* rank0, SortRec* recA, SortRec* recB,
                                void* temp, hipStream_t s)
{
    char* t = (char*)temp;
    auto take = [&](size_t bytes) { char* p = t; t += (bytes + 255) & ~(size_t)255; return p; };
    int32_t* coarse = (int32_t*)take((size_t)n * 4);
    uint32_t* key = (uint32_t*)take((size_t)n * 4);
    int32_t* lm2 = (int32_t*)take((size_t)L2 * 4);
    int32_t* lm1 = (int32_t*)take((size_t)L1 * 4);
    int32_t* flm = (int32_t*)take((size_t)L1 * 4);
    int32_t* goff = (int32_t*)take((size_t)(L2 + 1) * 4);
    SortRec* fa = (SortRec*)take((size_t)L1 * sizeof(SortRec));
    SortRec* fb = (SortRec*)take((size_t)L1 * sizeof(SortRec));
    void* rtemp = take(radix_temp_bytes(L1 > n ? L1 : n));
    // landmarks: evenly strided point ids
    std::vector<int32_t> h2(L2), h1(L1);
    for (int l = 0; l < L2; ++l) h2[l] = (int32_t)((int64_t)l * n / L2);
    for (int l = 0; l < L1; ++l) h1[l] = (int32_t)((int64_t)l * n / L1);
    hipError_t e = hipMemcpyAsync(lm2, h2.data(), (size_t)L2 * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(lm1, h1.data(), (size_t)L1 * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    k_assign_coarse<<<g256(n), 256, (size_t)L2 * d * sizeof(float), s>>>(X, n, d, ld, lm2, L2, coarse);
    k_fine_records<<<g256(L1), 256, 0, s>>>(coarse, lm1, L1, fa);
    const int lgL2 = L2 > 1 ? 32 - __builtin_clz((unsigned)(L2 - 1)) : 1;
    const int f1[1] = {1};
    const int b1[1] = {lgL2};
    SortRec* fs = nullptr;
    e = launch_radix_sort(fa, fb, L1, f1, b1, 1, rtemp, &fs, s);
    if (e != hipSuccess) return e;
    k_fine_groups<<<1, 1024, 0, s>>>(fs, L1, L2, flm, goff);
    k_assign_fine<<<g256(n), 256, 0, s>>>(X, n, d, ld, coarse, flm, goff, key);
    k_records_u32<<<g256(n), 256, 0, s>>>(key, n, recA);
    const int lgL1 = L1 > 1 ? 32 - __builtin_clz((unsigned)(L1 - 1)) : 1;
    const int b2[1] = {lgL1};
    SortRec* ps = nullptr;
    e = launch_radix_sort(recA, recB, n, f1, b2, 1, rtemp, &ps, s);
    if (e != hipSuccess) return e;
    e = launch_perm_from_records(ps, n, perm0, s);
    if (e != hipSuccess) return e;
    k_rank_of<<<g256(n), 256, 0, s>>>(perm0, n, rank0);
    return hipGetLastError();
}

// perm: components ordered by their earliest spatial rank, members by rank;
// seg: monotone segment id of every sorted position.
hipError_t launch_component_order(const int32_t* comp, const int32_t* perm0, const int32_t* rank0,
                                  int64_t n, int32_t* ckey, SortRec* recA, SortRec* recB,
                                  int32_t* perm, int32_t* seg, int32_t* flag, int32_t* excl,
                                  void* radix_temp, void* scan_temp, hipStream_t s)
{
    k_ckey_reset<<<g256(n), 256, 0, s>>>(ckey, n);
    k_ckey_min<<<g256(n), 256, 0, s>>>(comp, rank0, n, ckey);
    k_comp_records_spatial<<<g256(n), 256, 0, s>>>(perm0, comp, ckey, n, recA);
    int lg = 1;
    while (((int64_t)1 << lg) < n) ++lg;
    const int f1[1] = {1};
    const int b1[1] = {lg};
    SortRec* res = nullptr;
    hipError_t e = launch_radix_sort(recA, recB, n, f1, b1, 1, radix_temp, &res, s);
    if (e != hipSuccess) return e;
    e = launch_perm_from_records(res, n, perm, s);
    if (e != hipSuccess) return e;
    k_segment_flags<<<g256(n), 256, 0, s>>>(perm, comp, n, flag);
    e = launch_exclusive_scan(flag, excl, n, scan_temp, nullptr, s);
    if (e != hipSuccess) return e;
    k_segment_ids<<<g256(n), 256, 0, s>>>(flag, excl, n, seg);
    return hipGetLastError();
}

hipError_t launch_chunk_balls(const float* X, int64_t n, int d, int64_t ld, const int32_t* perm,
                              int bn, float* balls, hipStream_t s)
{
    const int64_t nc = (n + bn - 1) / bn;
    k_chunk_balls<<<(unsigned)nc, 256, 0, s>>>(X, n, d, ld, perm, bn, balls);
    return hipGetLastError();
}

}  // namespace nnm

// ---- many instances in one point set --------------------------------------
namespace nnm {
namespace {

__device__ __forceinline__ int instance_of(const int32_t* off, int ninst, int64_t p)
{
    int lo = 0, hi = ninst;          // off[lo] <= p < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)off[mid] <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

// first r in [0, nb) whose position is >= pos (rows ascending; NULL = row0 + r)
__device__ __forceinline__ int64_t first_row_at(const int32_t* rows, int32_t row0, int64_t nb,
                                                int64_t pos)
{
    if (!rows) {
        int64_t r = pos - row0;
        return r < 0 ? 0 : (r > nb ? nb : r);
    }
    int64_t lo = 0, hi = nb;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rows[mid] < pos) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_concat(const InstDev* __restrict__ inst,
                                                const int32_t* __restrict__ off, int ninst,
                                                int64_t n, int dmax, float* __restrict__ Xc)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = instance_of(off, ninst, i);
    const InstDev in = inst[b];
    const float* src = in.X + (i - off[b]) * in.ld;
    for (int f = 0; f < dmax; ++f) Xc[i * dmax + f] = f < in.d ? src[f] : 0.f;
}

__global__ __launch_bounds__(256) void k_inst_records(const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ off, int ninst,
                                                      int64_t n, SortRec* __restrict__ rec)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    SortRec r;
    r.k0 = 0;
    r.k1 = (uint32_t)instance_of(off, ninst, perm[q]);
    r.k2 = (uint32_t)perm[q];
    rec[q] = r;
}

__global__ __launch_bounds__(256) void k_tile_flags(const int32_t* __restrict__ rows, int32_t row0,
                                                    int64_t nb, const int32_t* __restrict__ off,
                                                    int ninst, int bm, int32_t* __restrict__ flag)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= nb) return;
    const int64_t p = rows ? rows[r] : row0 + r;
    const int b = instance_of(off, ninst, p);
    const int64_t st = first_row_at(rows, row0, nb, off[b]);
    flag[r] = ((r - st) % bm == 0) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_tile_desc(const int32_t* __restrict__ tstart, int ntiles,
                                                   const int32_t* __restrict__ rows, int32_t row0,
                                                   int64_t nb, const int32_t* __restrict__ off,
                                                   int ninst, int bm, int4* __restrict__ tiles)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const int64_t rbeg = tstart[t];
    const int64_t p = rows ? rows[rbeg] : row0 + rbeg;
    const int b = instance_of(off, ninst, p);
    const int64_t run_end = first_row_at(rows, row0, nb, off[b + 1]);
    const int64_t rend = rbeg + bm < run_end ? rbeg + bm : run_end;
    tiles[t] = make_int4((int)rbeg, (int)rend, off[b], off[b + 1]);
}

// sorted edges -> records (k0 = edge index, k1 = instance of u)
__global__ __launch_bounds__(256) void k_edge_inst_records(const SortRec* __restrict__ e, int64_t ne,
                                                           const int32_t* __restrict__ off, int ninst,
                                                           SortRec* __restrict__ rec)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= ne) return;
    SortRec r;
    r.k0 = (uint64_t)q;
    r.k1 = (uint32_t)instance_of(off, ninst, e[q].k1);
    r.k2 = 0;
    rec[q] = r;
}

__global__ __launch_bounds__(256) void k_write_edges_inst(const SortRec* __restrict__ sorted,
                                                          const SortRec* __restrict__ order, int64_t ne,
                                                          const int32_t* __restrict__ off,
                                                          nnm_edge* const* __restrict__ out)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= ne) return;
    const int b = (int)order[q].k1;
    const SortRec r = sorted[order[q].k0];
    const int64_t local = q - ((int64_t)off[b] - b);   // instance b owns edges [off_b - b, ...)
    nnm_edge o;
    o.u = (int32_t)(r.k1 - (uint32_t)off[b]);
    o.v = (int32_t)(r.k2 - (uint32_t)off[b]);
    o.s = __longlong_as_double((long long)r.k0);
    o.w = __dsqrt_rn(o.s);
    out[b][local] = o;
}

}  // namespace

hipError_t launch_concat(const InstDev* inst, const int32_t* off, int ninst, int64_t n, int dmax,
                         float* Xc, hipStream_t s)
{
    k_concat<<<g256(n), 256, 0, s>>>(inst, off, ninst, n, dmax, Xc);
    return hipGetLastError();
}

// perm0 made instance-major (stable: spatial order kept inside instances)
hipError_t launch_instance_major(int32_t* perm0, int32_t* rank0, const int32_t* off, int ninst,
                                 int64_t n, SortRec* recA, SortRec* recB, void* radix_temp,
                                 hipStream_t s)
{
    k_inst_records<<<g256(n), 256, 0, s>>>(perm0, off, ninst, n, recA);
    int lg = 1;
    while ((1 << lg) < ninst) ++lg;
    const int f1[1] = {1};
    const int b1[1] = {lg};
    SortRec* res = nullptr;
    hipError_t e = launch_radix_sort(recA, recB, n, f1, b1, 1, radix_temp, &res, s);
    if (e != hipSuccess) return e;
    e = launch_perm_from_records(res, n, perm0, s);
    if (e != hipSuccess) return e;
    k_rank_of<<<g256(n), 256, 0, s>>>(perm0, n, rank0);
    return hipGetLastError();
}

hipError_t launch_tiles(const int32_t* rows, int32_t row0, int64_t nb, const int32_t* off, int ninst,
                        int bm, int32_t* flag, int32_t* tstart, int32_t* ntiles_dev, void* scan_temp,
                        hipStream_t s)
{
    k_tile_flags<<<g256(nb), 256, 0, s>>>(rows, row0, nb, off, ninst, bm, flag);
    return launch_compact(flag, nb, tstart, ntiles_dev, scan_temp, s);
}

hipError_t launch_tile_desc(const int32_t* tstart, int ntiles, const int32_t* rows, int32_t row0,
                            int64_t nb, const int32_t* off, int ninst, int bm, int4* tiles,
                            hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    k_tile_desc<<<g256(ntiles), 256, 0, s>>>(tstart, ntiles, rows, row0, nb, off, ninst, bm, tiles);
    return hipGetLastError();
}

hipError_t launch_write_edges_batched(const SortRec* sorted, int64_t ne, const int32_t* off, int ninst,
                                      SortRec* recA, SortRec* recB, void* radix_temp,
                                      nnm_edge* const* out, hipStream_t s)
{
    if (ne <= 0) return hipSuccess;
    k_edge_inst_records<<<g256(ne), 256, 0, s>>>(sorted, ne, off, ninst, recA);
    int lg = 1;
    while ((1 << lg) < ninst) ++lg;
    const int f1[1] = {1};
    const int b1[1] = {lg};
    SortRec* res = nullptr;
    hipError_t e = launch_radix_sort(recA, recB, ne, f1, b1, 1, radix_temp, &res, s);
    if (e != hipSuccess) return e;
    k_write_edges_inst<<<g256(ne), 256, 0, s>>>(sorted, res, ne, off, out);
    return hipGetLastError();
}

}  // namespace nnm
