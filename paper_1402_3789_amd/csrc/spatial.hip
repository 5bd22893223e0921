// spatial.hip -- a spatial order of the points and bounding balls of chunks.
//
// The candidate pass visits, for every tile of rows, the chunks of columns
// nearest to it first and skips chunks that provably hold no pair the rows
// still need.  Both rely on consecutive points being close in space:
//   - a hierarchical landmark partition: level by level, every cell picks up
//     to 32 of its points as landmarks, orders them along a greedy
//     nearest-neighbour chain (so neighbouring landmarks get neighbouring
//     numbers) and every point moves to the child cell of its nearest
//     landmark; at the finest level points are ordered by their distance to
//     that landmark.  A compact cluster stays in one cell at every level
//     above its own scale and therefore forms one contiguous run.  The order
//     only steers the search; results never depend on it.
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

// Visits the points in spatial order (rank q of point perm0[q] is q), so the
// smallest rank of each run of equal components inside a wave is its first
// lane's: one atomic per run instead of one per point.  Keys only decrease,
// so a run whose rank is not below the key already read needs no atomic
// (with few components left, most waves' runs fall on the same addresses).
__global__ __launch_bounds__(256) void k_ckey_min(const int32_t* __restrict__ comp,
                                                  const int32_t* __restrict__ perm0, int64_t n,
                                                  int32_t* ckey)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int c = q < n ? comp[perm0[q]] : -1;
    const int prev = __shfl_up(c, 1);
    if (q < n && (lane == 0 || prev != c) && (int32_t)q < __atomic_load_n(&ckey[c], __ATOMIC_RELAXED))
        atomicMin(&ckey[c], (int32_t)q);
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

// One block per chunk of `bn` consecutive rows of the sorted FP32 copy
// (DMAX floats a row, zero beyond the data's features): centre = FP64 mean
// rounded to FP32, radius = FP64 max distance to that centre, rounded up.
// Eight lanes per row, one float4 each, so every read is a whole row.
// Ball of the sorted positions [c0, c1) of block b: fixed blocks of bn
// positions, or (starts != NULL) [starts[b], starts[b + 1]) for the first
// *count blocks (blocks past the count return at once).
__global__ __launch_bounds__(256) void k_chunk_balls(const float* __restrict__ xs, int64_t n, int bn,
                                                     const int32_t* __restrict__ starts,
                                                     const int32_t* __restrict__ count,
                                                     float* __restrict__ balls)
{
    __shared__ double acc[4][DMAX];
    __shared__ alignas(16) float cen[DMAX];
    __shared__ double rmax[4];
    if (starts && (int)blockIdx.x >= *count) return;
    const int64_t c0 = starts ? (int64_t)starts[blockIdx.x] : (int64_t)blockIdx.x * bn;
    const int64_t c1 = starts ? (int64_t)starts[blockIdx.x + 1] : (c0 + bn < n ? c0 + bn : n);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = threadIdx.x & 7;               // float4 of the row
    const int r = threadIdx.x >> 3;              // row of a pass of 32
    const float4* x4 = reinterpret_cast<const float4*>(xs);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int64_t p = c0 + r; p < c1; p += 32) {
        const float4 v = x4[p * (DMAX / 4) + q];
        s0 += (double)v.x;
        s1 += (double)v.y;
        s2 += (double)v.z;
        s3 += (double)v.w;
    }
    // over the eight rows of the wave that share q
    for (int off = 8; off < 64; off <<= 1) {
        s0 += __shfl_xor(s0, off);
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
        s3 += __shfl_xor(s3, off);
    }
    if (lane < 8) {
        acc[wave][4 * q + 0] = s0;
        acc[wave][4 * q + 1] = s1;
        acc[wave][4 * q + 2] = s2;
        acc[wave][4 * q + 3] = s3;
    }
    __syncthreads();
    if (threadIdx.x < DMAX) {
        const int f = threadIdx.x;
        cen[f] = (float)((acc[0][f] + acc[1][f] + acc[2][f] + acc[3][f]) / (double)(c1 - c0));
    }
    __syncthreads();
    const float4 c = reinterpret_cast<const float4*>(cen)[q];
    double r2 = 0.0;
    for (int64_t p = c0 + r; p < c1; p += 32) {
        const float4 v = x4[p * (DMAX / 4) + q];
        const double d0 = (double)v.x - (double)c.x, d1 = (double)v.y - (double)c.y;
        const double d2 = (double)v.z - (double)c.z, d3 = (double)v.w - (double)c.w;
        double part = d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
        // the row's eight lanes run the same trips: its full squared distance
        part += __shfl_xor(part, 1);
        part += __shfl_xor(part, 2);
        part += __shfl_xor(part, 4);
        r2 = part > r2 ? part : r2;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(r2, off);
        r2 = o > r2 ? o : r2;
    }
    if (lane == 0) rmax[wave] = r2;
    __syncthreads();
    float* out = balls + (int64_t)blockIdx.x * BALL_STRIDE;
    if (threadIdx.x == 0) {
        double m = rmax[0];
        for (int w = 1; w < 4; ++w) m = rmax[w] > m ? rmax[w] : m;
        out[DMAX] = d2f_up(__builtin_sqrt(m) * (1.0 + 0x1p-40));
    }
    if (threadIdx.x < DMAX) out[threadIdx.x] = cen[threadIdx.x];
    else if (threadIdx.x > DMAX && threadIdx.x < BALL_STRIDE) out[threadIdx.x] = 0.f;
}

constexpr int FANOUT = 32;

__global__ __launch_bounds__(256) void k_cell_records(const int32_t* __restrict__ order,
                                                      const int32_t* __restrict__ cell, int64_t n,
                                                      SortRec* __restrict__ rec)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int i = order ? order[q] : (int)q;
    SortRec r;
    r.k0 = 0;
    r.k1 = (uint32_t)cell[i];
    r.k2 = (uint32_t)i;
    rec[q] = r;
}

// cstart / cend of every non-empty cell in the cell-sorted order
__global__ __launch_bounds__(256) void k_cell_bounds(const SortRec* __restrict__ rec, int64_t n,
                                                     int32_t* __restrict__ cstart,
                                                     int32_t* __restrict__ cend)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    const uint32_t c = rec[q].k1;
    if (q == 0 || rec[q - 1].k1 != c) cstart[c] = (int32_t)q;
    if (q == n - 1 || rec[q + 1].k1 != c) cend[c] = (int32_t)(q + 1);
}

// One wave per cell: up to FANOUT landmarks strided over the cell's members,
// numbered along a greedy nearest-neighbour chain starting at the first.
__global__ __launch_bounds__(64) void k_cell_landmarks(const float* __restrict__ X, int d, int64_t ld,
                                                       const SortRec* __restrict__ rec,
                                                       const int32_t* __restrict__ cstart,
                                                       const int32_t* __restrict__ cend, int ncells,
                                                       int32_t* __restrict__ lm, int32_t* __restrict__ lrank,
                                                       int32_t* __restrict__ lcount)
{
    __shared__ float dist[FANOUT][FANOUT];
    __shared__ int ids[FANOUT];
    const int c = blockIdx.x;
    if (c >= ncells) return;
    const int st = cstart[c], en = cend[c];
    const int lane = threadIdx.x;
    if (en <= st) {
        if (lane == 0) lcount[c] = 0;
        return;
    }
    const int sz = en - st;
    const int m = sz < FANOUT ? sz : FANOUT;
    if (lane < m) ids[lane] = (int)rec[st + (int64_t)lane * sz / m].k2;
    __syncthreads();
    if (lane < m) {
        const float* xa = X + (int64_t)ids[lane] * ld;
        for (int b = 0; b < m; ++b) {
            const float* xb = X + (int64_t)ids[b] * ld;
            float t = 0.f;
            for (int f = 0; f < d; ++f) {
                const float df = xa[f] - xb[f];
                t = __builtin_fmaf(df, df, t);
            }
            dist[lane][b] = t;
        }
    }
    __syncthreads();
    if (lane == 0) {
        unsigned int seen = 1u;
        int cur = 0;
        lrank[c * FANOUT + 0] = 0;
        for (int r = 1; r < m; ++r) {
            int nx = -1;
            float best = __builtin_huge_valf();
            for (int b = 0; b < m; ++b)
                if (!((seen >> b) & 1u) && dist[cur][b] < best) { best = dist[cur][b]; nx = b; }
            if (nx < 0) {   // equal or infinite distances: take the first unvisited
                for (int b = 0; b < m; ++b) if (!((seen >> b) & 1u)) { nx = b; break; }
            }
            seen |= 1u << nx;
            lrank[c * FANOUT + nx] = r;
            cur = nx;
        }
        lcount[c] = m;
    }
    if (lane < m) lm[c * FANOUT + lane] = ids[lane];
}

// Each point takes the nearest of its cell's landmarks (FP32; any choice is
// a valid order).  Workgroups run over the cell-sorted order, so the few
// cells one workgroup touches have their landmarks staged in LDS in turn.
__global__ __launch_bounds__(256) void k_cell_assign(const float* __restrict__ X, int64_t n, int d,
                                                     int64_t ld, const SortRec* __restrict__ rec,
                                                     int32_t* __restrict__ cell,
                                                     const int32_t* __restrict__ lm,
                                                     const int32_t* __restrict__ lrank,
                                                     const int32_t* __restrict__ lcount,
                                                     float* __restrict__ dist)
{
    __shared__ float L[FANOUT][DMAX + 1];
    __shared__ uint32_t next_c;
    const int64_t q0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t q = q0 + threadIdx.x;
    const bool valid = q < n;
    const int64_t qe = (q0 + blockDim.x < n ? q0 + blockDim.x : n) - 1;
    const uint32_t clast = rec[qe].k1;
    const int i = valid ? (int)rec[q].k2 : 0;
    const uint32_t myc = valid ? rec[q].k1 : 0xFFFFFFFFu;
    float xi[DMAX];
    for (int f = 0; f < DMAX; ++f) xi[f] = (valid && f < d) ? X[(int64_t)i * ld + f] : 0.f;
    float best = __builtin_huge_valf();
    int bj = 0;
    uint32_t c = rec[q0].k1;
    for (;;) {
        const int m = lcount[c];
        for (int idx = threadIdx.x; idx < m * d; idx += blockDim.x) {
            const int j = idx / d, f = idx - j * d;
            L[j][f] = X[(int64_t)lm[c * FANOUT + j] * ld + f];
        }
        if (threadIdx.x == 0) next_c = 0xFFFFFFFFu;
        __syncthreads();
        if (myc == c) {
            for (int j = 0; j < m; ++j) {
                float t = 0.f;
                for (int f = 0; f < d; ++f) {
                    const float df = xi[f] - L[j][f];
                    t = __builtin_fmaf(df, df, t);
                }
                if (t < best) { best = t; bj = j; }
            }
        } else if (valid && myc > c) {
            atomicMin(&next_c, myc);
        }
        __syncthreads();
        if (c == clast) break;
        c = next_c;
        __syncthreads();
    }
    if (!valid) return;
    const int m = lcount[myc];
    cell[i] = (int)myc * FANOUT + (m > 0 ? lrank[myc * FANOUT + bj] : 0);
    dist[i] = m > 0 ? best : 0.f;
}

__global__ __launch_bounds__(256) void k_dist_records(const float* __restrict__ dist,
                                                      const int32_t* __restrict__ cell, int64_t n,
                                                      SortRec* __restrict__ rec)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    SortRec r;
    r.k0 = (uint64_t)__float_as_uint(dist[i]);   // non-negative: bits order as values
    r.k1 = (uint32_t)cell[i];
    r.k2 = (uint32_t)i;
    rec[i] = r;
}

int order_levels(int64_t n)
{
    int lev = 0;
    double cells = 1.0;
    while ((double)n / cells > 64.0 && lev < 3) { cells *= FANOUT; ++lev; }
    return lev < 1 ? 1 : lev;
}

}  // namespace

size_t spatial_temp_bytes(int64_t n, int, int)
{
    const int64_t maxcells = (int64_t)FANOUT * FANOUT * FANOUT;
    return (size_t)n * 4 * 3 + (size_t)maxcells * 4 * (3 + 2 * FANOUT) + radix_temp_bytes(n) + 8192;
}

// perm0 (spatial order) and rank0 (its inverse) for n points.
hipError_t launch_spatial_order(const float* X, int64_t n, int d, int64_t ld, int, int,
                                int32_t* perm0, int32_t* rank0, SortRec* recA, SortRec* recB,
                                void* temp, hipStream_t s)
{
    char* t = (char*)temp;
    auto take = [&](size_t bytes) { char* p = t; t += (bytes + 255) & ~(size_t)255; return p; };
    const int levels = order_levels(n);
    int64_t maxcells = 1;
    for (int l = 0; l < levels; ++l) maxcells *= FANOUT;
    int32_t* cell = (int32_t*)take((size_t)n * 4);
    float* dist = (float*)take((size_t)n * 4);
    int32_t* order = (int32_t*)take((size_t)n * 4);
    int32_t* cstart = (int32_t*)take((size_t)maxcells * 4);
    int32_t* cend = (int32_t*)take((size_t)maxcells * 4);
    int32_t* lcount = (int32_t*)take((size_t)maxcells * 4);
    int32_t* lm = (int32_t*)take((size_t)maxcells * FANOUT * 4);
    int32_t* lrank = (int32_t*)take((size_t)maxcells * FANOUT * 4);
    void* rtemp = take(radix_temp_bytes(n));
    hipError_t e = hipMemsetAsync(cell, 0, (size_t)n * 4, s);
    if (e != hipSuccess) return e;
    int64_t ncells = 1;
    const int32_t* prev = nullptr;     // order of the previous level (NULL = identity)
    for (int lev = 0; lev < levels; ++lev) {
        k_cell_records<<<g256(n), 256, 0, s>>>(prev, cell, n, recA);
        int bits = 5 * lev;
        SortRec* res = recA;
        if (bits > 0) {
            const int f1[1] = {1};
            const int b1[1] = {bits};
            e = launch_radix_sort(recA, recB, n, f1, b1, 1, rtemp, &res, s);
            if (e != hipSuccess) return e;
        }
        e = hipMemsetAsync(cstart, 0, (size_t)ncells * 4, s);
        if (e != hipSuccess) return e;
        e = hipMemsetAsync(cend, 0, (size_t)ncells * 4, s);
        if (e != hipSuccess) return e;
        k_cell_bounds<<<g256(n), 256, 0, s>>>(res, n, cstart, cend);
        k_cell_landmarks<<<(unsigned)ncells, 64, 0, s>>>(X, d, ld, res, cstart, cend, (int)ncells, lm,
                                                        lrank, lcount);
        k_cell_assign<<<g256(n), 256, 0, s>>>(X, n, d, ld, res, cell, lm, lrank, lcount, dist);
        e = launch_perm_from_records(res, n, order, s);
        if (e != hipSuccess) return e;
        prev = order;
        ncells *= FANOUT;
    }
    // finest cells, each ordered by distance to its landmark
    k_dist_records<<<g256(n), 256, 0, s>>>(dist, cell, n, recA);
    const int f2[2] = {0, 1};
    const int b2[2] = {32, 5 * levels};
    SortRec* res = nullptr;
    e = launch_radix_sort(recA, recB, n, f2, b2, 2, rtemp, &res, s);
    if (e != hipSuccess) return e;
    e = launch_perm_from_records(res, n, perm0, s);
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
    k_ckey_min<<<g256(n), 256, 0, s>>>(comp, perm0, n, ckey);
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

hipError_t launch_chunk_balls(const float* xs, int64_t n, int bn, float* balls, hipStream_t s)
{
    static_assert(DMAX == 32, "eight float4 per padded row");
    const int64_t nc = (n + bn - 1) / bn;
    if (nc <= 0) return hipSuccess;
    k_chunk_balls<<<(unsigned)nc, 256, 0, s>>>(xs, n, bn, nullptr, nullptr, balls);
    return hipGetLastError();
}

// ---- component-aligned column chunks --------------------------------------
// In the merge rounds the sorted order holds each component as one segment.
// A fixed chunk that straddles two segments has a bounding ball spanning two
// components, far apart, which nearly every row's ball test passes; so once
// components are large each segment [a, b) is cut on its own into chunks
// starting at a, a + CHUNK, ... and its chunks into super-chunks of SUPER.

namespace {

__global__ __launch_bounds__(256) void k_tab_segstart(const int32_t* __restrict__ seg, int64_t n,
                                                      int32_t* __restrict__ segstart)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (p == 0 || seg[p] != seg[p - 1]) segstart[seg[p]] = (int32_t)p;
    if (p == n - 1) segstart[seg[p] + 1] = (int32_t)n;
}

__global__ __launch_bounds__(256) void k_tab_counts(const int32_t* __restrict__ segstart, int64_t nseg,
                                                    int32_t* __restrict__ ccnt, int32_t* __restrict__ scnt)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= nseg) return;
    const int len = segstart[g + 1] - segstart[g];
    const int c = (len + CHUNK - 1) / CHUNK;
    ccnt[g] = c;
    scnt[g] = (c + SUPER - 1) / SUPER;
}

// One block per segment.
__global__ __launch_bounds__(256) void k_tab_fill(const int32_t* __restrict__ segstart, int64_t nseg,
                                                  int64_t n, const int32_t* __restrict__ ccnt,
                                                  const int32_t* __restrict__ scnt,
                                                  const int32_t* __restrict__ cbase,
                                                  const int32_t* __restrict__ sbase,
                                                  int32_t* __restrict__ cstart, int32_t* __restrict__ csup,
                                                  int32_t* __restrict__ sfirst, int32_t* __restrict__ spos,
                                                  int32_t* __restrict__ ccomp, int32_t* __restrict__ scomp,
                                                  int32_t* __restrict__ tabn)
{
    const int64_t g = blockIdx.x;
    const int a = segstart[g];
    const int cb = cbase[g], sb = sbase[g];
    for (int c = threadIdx.x; c < ccnt[g]; c += 256) {
        cstart[cb + c] = a + c * CHUNK;
        csup[cb + c] = sb + c / SUPER;
        ccomp[cb + c] = (int32_t)g;
    }
    for (int q = threadIdx.x; q < scnt[g]; q += 256) {
        sfirst[sb + q] = cb + q * SUPER;
        spos[sb + q] = a + q * SUPER * CHUNK;
        scomp[sb + q] = (int32_t)g;
    }
    if (g == nseg - 1 && threadIdx.x == 0) {
        const int nch = cb + ccnt[g], nsc = sb + scnt[g];
        cstart[nch] = (int32_t)n;
        sfirst[nsc] = nch;
        spos[nsc] = (int32_t)n;
        tabn[0] = nch;
        tabn[1] = nsc;
    }
}

__global__ __launch_bounds__(256) void k_tab_pos2chunk(const int32_t* __restrict__ seg, int64_t n,
                                                       const int32_t* __restrict__ segstart,
                                                       const int32_t* __restrict__ cbase,
                                                       int32_t* __restrict__ pos2chunk)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int g = seg[p];
    pos2chunk[p] = cbase[g] + (int)((p - segstart[g]) / CHUNK);
}

}  // namespace

hipError_t launch_chunk_tables(const int32_t* seg, int64_t n, int64_t nseg, const ChunkTabs& t,
                               const float* xs, float* balls, float* sballs, void* scan_temp,
                               hipStream_t s)
{
    static_assert(DMAX == 32, "eight float4 per padded row");
    if (n <= 0 || nseg <= 0) return hipSuccess;
    k_tab_segstart<<<g256(n), 256, 0, s>>>(seg, n, t.segstart);
    k_tab_counts<<<g256(nseg), 256, 0, s>>>(t.segstart, nseg, t.ccnt, t.scnt);
    hipError_t e = launch_exclusive_scan(t.ccnt, t.cbase, nseg, scan_temp, nullptr, s);
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan(t.scnt, t.sbase, nseg, scan_temp, nullptr, s);
    if (e != hipSuccess) return e;
    k_tab_fill<<<(unsigned)nseg, 256, 0, s>>>(t.segstart, nseg, n, t.ccnt, t.scnt, t.cbase, t.sbase,
                                              t.cstart, t.csup, t.sfirst, t.spos, t.ccomp, t.scomp,
                                              t.tabn);
    k_tab_pos2chunk<<<g256(n), 256, 0, s>>>(seg, n, t.segstart, t.cbase, t.pos2chunk);
    // at most n / CHUNK + nseg chunks and n / (CHUNK SUPER) + nseg super-chunks
    const int64_t mc = (n + CHUNK - 1) / CHUNK + nseg;
    const int64_t ms = (n + CHUNK * SUPER - 1) / (CHUNK * SUPER) + nseg;
    k_chunk_balls<<<(unsigned)mc, 256, 0, s>>>(xs, n, CHUNK, t.cstart, t.tabn, balls);
    k_chunk_balls<<<(unsigned)ms, 256, 0, s>>>(xs, n, CHUNK, t.spos, t.tabn + 1, sballs);
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

// nb rows, or (desc) the first desc->n_rows of the nb row slots; the rest
// of the slots are flagged 0
__global__ __launch_bounds__(256) void k_tile_flags(const int32_t* __restrict__ rows, int32_t row0,
                                                    int64_t nb, const int32_t* __restrict__ off,
                                                    int ninst, int bm, int32_t* __restrict__ flag,
                                                    const LaunchDesc* __restrict__ desc)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= nb) return;
    if (desc) {
        const int64_t nr = desc->n_rows;
        if (r >= nr) {
            flag[r] = 0;
            return;
        }
        nb = nr;
    }
    const int64_t p = rows ? rows[r] : row0 + r;
    const int b = instance_of(off, ninst, p);
    const int64_t st = first_row_at(rows, row0, nb, off[b]);
    flag[r] = ((r - st) % bm == 0) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_tile_desc(const int32_t* __restrict__ tstart, int ntiles,
                                                   const int32_t* __restrict__ rows, int32_t row0,
                                                   int64_t nb, const int32_t* __restrict__ off,
                                                   int ninst, int bm, int4* __restrict__ tiles,
                                                   const LaunchDesc* __restrict__ desc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (desc) {
        ntiles = desc->n_tiles;
        nb = desc->n_rows;
    }
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
                                                          nnm_edge* const* __restrict__ out,
                                                          int metric)
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
    o.w = metric_key_is_distance(metric) ? o.s : __dsqrt_rn(o.s);
    out[b][local] = o;
}

// The cosine metric's rows: scaled to unit Euclidean length (FP64 norm from
// the sum of squares in feature order, one division and one rounding per
// feature; a zero row stays zero).  One thread per row.
__global__ __launch_bounds__(256) void k_normalize_rows(const float* __restrict__ X, int64_t n, int d,
                                                        int64_t ld, float* __restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* x = X + i * ld;
    double q = 0.0;
    for (int f = 0; f < d; ++f) {
        const double v = (double)x[f];
        const double sq = __dmul_rn(v, v);
        q = (f == 0) ? sq : __dadd_rn(q, sq);
    }
    const double nrm = __dsqrt_rn(q);
    for (int f = 0; f < d; ++f)
        out[i * d + f] = nrm > 0.0 ? (float)__ddiv_rn((double)x[f], nrm) : 0.0f;
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
    k_tile_flags<<<g256(nb), 256, 0, s>>>(rows, row0, nb, off, ninst, bm, flag, nullptr);
    return launch_compact(flag, nb, tstart, ntiles_dev, scan_temp, s);
}

hipError_t launch_tiles_dev(const int32_t* rows, int64_t cap, const int32_t* off, int ninst, int bm,
                            int32_t* flag, int32_t* tstart, LaunchDesc* d, void* scan_temp,
                            hipStream_t s)
{
    k_tile_flags<<<g256(cap), 256, 0, s>>>(rows, 0, cap, off, ninst, bm, flag, d);
    return launch_compact(flag, cap, tstart, &d->n_tiles, scan_temp, s);
}

hipError_t launch_tile_desc_dev(const int32_t* tstart, int max_tiles, const int32_t* rows,
                                const int32_t* off, int ninst, int bm, int4* tiles,
                                const LaunchDesc* d, hipStream_t s)
{
    k_tile_desc<<<g256(max_tiles), 256, 0, s>>>(tstart, max_tiles, rows, 0, 0, off, ninst, bm, tiles, d);
    return hipGetLastError();
}

hipError_t launch_tile_desc(const int32_t* tstart, int ntiles, const int32_t* rows, int32_t row0,
                            int64_t nb, const int32_t* off, int ninst, int bm, int4* tiles,
                            hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    k_tile_desc<<<g256(ntiles), 256, 0, s>>>(tstart, ntiles, rows, row0, nb, off, ninst, bm, tiles,
                                             nullptr);
    return hipGetLastError();
}

hipError_t launch_write_edges_batched(const SortRec* sorted, int64_t ne, const int32_t* off, int ninst,
                                      SortRec* recA, SortRec* recB, void* radix_temp,
                                      nnm_edge* const* out, int metric, hipStream_t s)
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
    k_write_edges_inst<<<g256(ne), 256, 0, s>>>(sorted, res, ne, off, out, metric);
    return hipGetLastError();
}

hipError_t launch_normalize_rows(const float* X, int64_t n, int d, int64_t ld, float* out,
                                 hipStream_t s)
{
    k_normalize_rows<<<g256(n), 256, 0, s>>>(X, n, d, ld, out);
    return hipGetLastError();
}

}  // namespace nnm
