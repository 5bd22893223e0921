// cand_common.h -- pieces shared by the matrix-core and the FP32 candidate
// passes: the bounding ball of a tile of rows, the near-first order of column
// chunks and the chunk pruning test.
#pragma once

#include "bound.h"
#include "nnm_common.h"

namespace nnm {


// Shared-memory scratch for the per-workgroup tile ball and the per-chunk
// pruning decision (one instance per workgroup).
struct TileShared {
    double acc[4][DMAX];
    alignas(16) float cen[DMAX];   // zero beyond the data's features
    double red[4];
    float wmax[4];
    float rball;
    float umax;
    int decision;
    int lo, hi, rows, first_pos;
    int col_lo, col_hi;      // columns this tile may pair with (sorted positions)
    int wneed[4];            // per wave: does any of its rows need the current chunk
};

// Workgroups are dealt to the 8 XCDs round-robin; neighbouring tiles sweep
// mostly the same column chunks, so give each XCD (and its L2) a contiguous
// run of tiles: workgroup b -> tile (b mod 8) * q + min(b mod 8, r) + b / 8
// for G = 8 q + r workgroups, a bijection onto [0, G).
__device__ __forceinline__ int xcd_tile(int b, int G)
{
    if (gridDim.y != 1) return b;
    const int x = b & 7, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// One work item of a candidate launch: row tile t, column split sp of nsp,
// in a launch of n_rows rows.  A host-sized launch has one item per
// workgroup (the grid is tiles x splits); a device-sized one pops items
// from its descriptor's queue.
struct Item {
    int t, sp, nsp, n_rows;
};

// Workgroups of a device-sized candidate launch (two per compute unit, twice over).
constexpr unsigned QGRID = 1024;

__device__ __forceinline__ Item grid_item(const CandArgs& a)
{
    return Item{xcd_tile((int)blockIdx.x, (int)gridDim.x), (int)blockIdx.y, a.col_splits, a.n_rows};
}

// Row slots [rbeg, rend) and column range [cl, ch) of a work item's tile.
__device__ __forceinline__ int4 tile_of(const CandArgs& a, int bm, const Item& it)
{
    if (a.tiles) return a.tiles[it.t];
    const int rbeg = it.t * bm;
    const int rend = rbeg + bm < it.n_rows ? rbeg + bm : it.n_rows;
    return make_int4(rbeg, rend, 0, a.np);
}

// The next item of a device-sized launch (all 256 threads call it; `slot`
// is a shared int); false once the launch's items are used up.
__device__ __forceinline__ bool pop_item(const CandArgs& a, int& slot, Item& it)
{
    __syncthreads();                  // the previous item is finished
    if (threadIdx.x == 0) slot = atomicAdd(&a.desc->queue, 1);
    __syncthreads();
    const int w = slot;
    const int nt = a.desc->n_tiles, nsp = a.desc->splits;
    if (w >= nt * nsp) return false;
    it = Item{w % nt, w / nt, nsp, a.desc->n_rows};
    return true;
}

// Centre (FP32, from an FP64 mean) and radius (FP64 max, rounded up) of the
// rows of this tile; thread t owns row t (valid = row exists), x holds its
// first d features.  All 256 threads of the workgroup must call it.
template <int DM>
__device__ inline void tile_ball(TileShared& sh, const float (&x)[DM], bool valid, int d)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double cnt = valid ? 1.0 : 0.0;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
#pragma unroll
    for (int f = 0; f < DM; ++f) {
        if (f < d) {
            double v = valid ? (double)x[f] : 0.0;
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) sh.acc[wave][f] = v;
        }
    }
    if (lane == 0) sh.red[wave] = cnt;
    __syncthreads();
    if (threadIdx.x < d) {
        const double tot = sh.red[0] + sh.red[1] + sh.red[2] + sh.red[3];
        const double m = (sh.acc[0][threadIdx.x] + sh.acc[1][threadIdx.x] + sh.acc[2][threadIdx.x] +
                          sh.acc[3][threadIdx.x]) / (tot > 0.0 ? tot : 1.0);
        sh.cen[threadIdx.x] = (float)m;
    } else if (threadIdx.x < DMAX) {
        sh.cen[threadIdx.x] = 0.f;
    }
    __syncthreads();
    double r2 = 0.0;
    if (valid) {
#pragma unroll
        for (int f = 0; f < DM; ++f) {
            if (f < d) {
                const double df = (double)x[f] - (double)sh.cen[f];
                r2 += df * df;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(r2, off);
        r2 = o > r2 ? o : r2;
    }
    __syncthreads();
    if (lane == 0) sh.red[wave] = r2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh.red[0];
        for (int w = 1; w < 4; ++w) m = sh.red[w] > m ? sh.red[w] : m;
        sh.rball = d2f_up(__builtin_sqrt(m) * (1.0 + 0x1p-40));
    }
    __syncthreads();
}

// Bounding ball of the calling wave's rows (lane l owns row l; valid = the
// row exists; x its first d features): centre (FP32, from an FP64 mean) into
// wc[DMAX], zero beyond the data's features, and radius (FP64 max, rounded
// up) into *wr.  Wave-local: no workgroup barrier.
template <int DM>
__device__ inline void wave_ball(float* wc, float* wr, const float (&x)[DM], bool valid, int d)
{
    const int lane = threadIdx.x & 63;
    const double cnt = (double)__popcll(__ballot(valid));
#pragma unroll
    for (int f = 0; f < DMAX; ++f) {
        double v = (f < DM && f < d && valid) ? (double)x[f < DM ? f : 0] : 0.0;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) wc[f] = (f < d) ? (float)(v / (cnt > 0.0 ? cnt : 1.0)) : 0.f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double r2 = 0.0;
    if (valid) {
#pragma unroll
        for (int f = 0; f < DM; ++f) {
            if (f < d) {
                const double df = (double)x[f] - (double)wc[f];
                r2 += df * df;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(r2, off);
        r2 = o > r2 ? o : r2;
    }
    if (lane == 0) *wr = d2f_up(__builtin_sqrt(r2) * (1.0 + 0x1p-40));
}

// Lower bound, rounded down, on the squared distance of any pair across the
// ball (centre cen[DMAX], radius rad) and the ball `ball` (BALL_STRIDE
// floats, 16-byte aligned); the margins are those of ball_lb2 below.
__device__ inline float balls_lb2(const float* cen, float rad, const float* ball)
{
    const float4* b4 = reinterpret_cast<const float4*>(ball);
    const float4* c4 = reinterpret_cast<const float4*>(cen);
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < DMAX / 4; ++q) {
        const float4 c = c4[q], bv = b4[q];
        const float d0 = c.x - bv.x, d1 = c.y - bv.y;
        const float d2 = c.z - bv.z, d3 = c.w - bv.w;
        s = __builtin_fmaf(d0, d0, s);
        s = __builtin_fmaf(d1, d1, s);
        s = __builtin_fmaf(d2, d2, s);
        s = __builtin_fmaf(d3, d3, s);
    }
    const float lb = __builtin_sqrtf(s) * (1.0f - 0x1p-18f) - rad - ball[DMAX];
    if (!(lb > 0.f)) return 0.f;
    return lb * lb * (1.0f - 0x1p-20f);
}

// Lower bound on the squared distance of any pair across the tile ball and
// the ball `ball` (BALL_STRIDE floats, 16-byte aligned), rounded down.  Both
// centres are zero beyond the data's features, so all DMAX features are
// summed: the loads carry no dependence on d and issue together.  FP32: the
// computed sum of squares is within (DMAX + 2) 2^-24 of the exact one and the
// root within half that plus one rounding, which the factor 1 - 2^-18 on the
// root covers; the two subtractions of the radii (rounded up) round by at
// most 2^-24 of the root each, and the square by 2^-24, covered by 1 - 2^-20.
__device__ inline float ball_lb2(const TileShared& sh, const float* ball)
{
    const float4* b4 = reinterpret_cast<const float4*>(ball);
    const float4* c4 = reinterpret_cast<const float4*>(sh.cen);
    float4 bv[DMAX / 4];
#pragma unroll
    for (int q = 0; q < DMAX / 4; ++q) bv[q] = b4[q];
    const float rad = ball[DMAX];
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < DMAX / 4; ++q) {
        const float4 c = c4[q];
        const float d0 = c.x - bv[q].x, d1 = c.y - bv[q].y;
        const float d2 = c.z - bv[q].z, d3 = c.w - bv[q].w;
        s = __builtin_fmaf(d0, d0, s);
        s = __builtin_fmaf(d1, d1, s);
        s = __builtin_fmaf(d2, d2, s);
        s = __builtin_fmaf(d3, d3, s);
    }
    const float lb = __builtin_sqrtf(s) * (1.0f - 0x1p-18f) - sh.rball - rad;
    if (!(lb > 0.f)) return 0.f;
    return lb * lb * (1.0f - 0x1p-20f);
}

// Lower bound, rounded down, on the squared distance between the point x
// (FP32, NQ float4s, zero beyond the data's features) and every point of the
// ball `ball` (BALL_STRIDE floats, 16-byte aligned, radius rounded up).
// Plain FP32 over all 4 NQ features (the padding adds exact zeros): the
// computed sum of squares is within (4 NQ + 2) 2^-24 of the exact one, which
// the margins on the root and on the square cover for NQ <= 8.
template <int NQ>
__device__ __forceinline__ float point_ball_lb2(const float4 (&x)[NQ], const float* ball)
{
    const float4* b4 = reinterpret_cast<const float4*>(ball);
    float4 bv[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) bv[q] = b4[q];
    const float rad = ball[DMAX];
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const float d0 = x[q].x - bv[q].x, d1 = x[q].y - bv[q].y;
        const float d2 = x[q].z - bv[q].z, d3 = x[q].w - bv[q].w;
        s = __builtin_fmaf(d0, d0, s);
        s = __builtin_fmaf(d1, d1, s);
        s = __builtin_fmaf(d2, d2, s);
        s = __builtin_fmaf(d3, d3, s);
    }
    const float lb = __builtin_sqrtf(s) * (1.0f - 0x1p-18f) - rad;
    if (!(lb > 0.f)) return 0.f;
    return lb * lb * (1.0f - 0x1p-20f);
}

// Upper bound on sqrt(U) for the per-row ball test below (U >= 0 or +inf):
// the correctly rounded root times 1 + 2^-20, rounded, stays above it.
__device__ __forceinline__ float reach_of(float U)
{
    return __builtin_sqrtf(U) * (1.0f + 0x1p-20f);
}

// Whether the point x (as for point_ball_lb2) may hold a pair with the ball
// `ball` whose key is at most U, given reach >= sqrt(U): such a pair needs
// |x - centre| <= radius + sqrt(U).  No root per test: the computed sum of
// squares s is within (4 NQ + 2) 2^-24 of the exact one (NQ <= 8), and the
// sum radius + reach and its square round by 2^-24 each, so comparing s with
// the square times 1 + 2^-16 never drops a ball that holds such a pair.
template <int NQ>
__device__ __forceinline__ bool point_ball_reach(const float4 (&x)[NQ], const float* ball, float reach)
{
    const float4* b4 = reinterpret_cast<const float4*>(ball);
    float4 bv[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) bv[q] = b4[q];
    const float rad = ball[DMAX];
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const float d0 = x[q].x - bv[q].x, d1 = x[q].y - bv[q].y;
        const float d2 = x[q].z - bv[q].z, d3 = x[q].w - bv[q].w;
        s = __builtin_fmaf(d0, d0, s);
        s = __builtin_fmaf(d1, d1, s);
        s = __builtin_fmaf(d2, d2, s);
        s = __builtin_fmaf(d3, d3, s);
    }
    const float r = rad + reach;
    return s <= r * r * (1.0f + 0x1p-16f);
}

// Workgroup-wide max of one float per thread (all 256 threads call it).
__device__ inline float block_max(TileShared& sh, float v)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    if (lane == 0) sh.red[wave] = (double)v;
    __syncthreads();
    float m = (float)sh.red[0];
    for (int w = 1; w < 4; ++w) m = fmaxf(m, (float)sh.red[w]);
    __syncthreads();
    return m;
}

// Column chunks of the sweep: CHUNK consecutive sorted positions each
// (super-chunks of SUPER consecutive chunks), or (TAB) the component-aligned
// tables of CandArgs, in which no chunk or super-chunk crosses a component.
// TAB is a template parameter of the kernels, so each kernel carries the
// arithmetic of one kind only.
template <bool TAB>
__device__ __forceinline__ int n_chunks(const CandArgs& a)
{
    if constexpr (TAB) return a.tabn[0];
    else return (a.np + CHUNK - 1) / CHUNK;
}

template <bool TAB>
__device__ __forceinline__ int64_t chunk_begin(const CandArgs& a, int ci)
{
    if constexpr (TAB) return (int64_t)a.cstart[ci];
    else return (int64_t)ci * CHUNK;
}

template <bool TAB>
__device__ __forceinline__ int64_t chunk_end(const CandArgs& a, int ci)
{
    if constexpr (TAB) {
        return (int64_t)a.cstart[ci + 1];
    } else {
        const int64_t e = (int64_t)(ci + 1) * CHUNK;
        return e < a.np ? e : (int64_t)a.np;
    }
}

// The chunk holding sorted position p (0 <= p < np).
template <bool TAB>
__device__ __forceinline__ int chunk_at(const CandArgs& a, int64_t p)
{
    if constexpr (TAB) return a.pos2chunk[p];
    else return (int)(p / CHUNK);
}

// First chunk, and end chunk, of the columns [lo, hi) of a tile (in the
// aligned tables an instance's range starts and ends on chunk boundaries).
template <bool TAB>
__device__ __forceinline__ int chunk_first_of(const CandArgs& a, int64_t lo)
{
    if constexpr (TAB) return lo < a.np ? a.pos2chunk[lo] : a.tabn[0];
    else return (int)(lo / CHUNK);
}

template <bool TAB>
__device__ __forceinline__ int chunk_end_of(const CandArgs& a, int64_t hi)
{
    if constexpr (TAB) return hi < a.np ? a.pos2chunk[hi] : a.tabn[0];
    else return (int)((hi + CHUNK - 1) / CHUNK);
}

template <bool TAB>
__device__ __forceinline__ int super_of(const CandArgs& a, int ci)
{
    if constexpr (TAB) return a.csup[ci];
    else return ci / SUPER;
}

template <bool TAB>
__device__ __forceinline__ int super_first(const CandArgs& a, int sc)
{
    if constexpr (TAB) return a.sfirst[sc];
    else return sc * SUPER;
}

template <bool TAB>
__device__ __forceinline__ int super_end(const CandArgs& a, int sc)
{
    if constexpr (TAB) {
        return a.sfirst[sc + 1];
    } else {
        const int e = (sc + 1) * SUPER, nc = n_chunks<TAB>(a);
        return e < nc ? e : nc;
    }
}

// Near-first visiting order of the chunks [lo, hi) around `start`:
// start, start+1, start-1, start+2, ...  step -> chunk index or -1.
__device__ __forceinline__ int zigzag(int step, int start, int lo, int hi)
{
    // positions alternate right/left; skip sides that ran out of range
    const int right = hi - 1 - start;   // chunks available to the right
    const int left = start - lo;        // and to the left
    if (step == 0) return start;
    const int both = 2 * (right < left ? right : left);
    if (step <= both) {
        const int k = (step + 1) >> 1;
        return (step & 1) ? start + k : start - k;
    }
    const int rest = step - both;
    if (right > left) return start + left + rest;
    return start - right - rest;
}

// Visit the chunks of this workgroup's column range nearest-first and call
// process(ci) for every chunk that (1) does not lie entirely inside the
// tile's only component and (2) survives the ball tests against the tile's
// bound umax = max over its rows of U_i (first per super-chunk, then per
// chunk).  process() must end by storing its waves' maxima of U_i in
// sh.wmax; umax is refreshed from them, behind one barrier, only after a
// chunk was processed.  All 256 threads call this with identical arguments.
template <bool TAB, typename Fn>
__device__ inline void sweep_chunks(TileShared& sh, const CandArgs& a, const Item& it, int lo_r,
                                    int hi_r, float umax, Fn&& process)
{
    const int first_ch = chunk_first_of<TAB>(a, sh.col_lo);
    const int nch = chunk_end_of<TAB>(a, sh.col_hi) - first_ch;
    const int cps = (nch + it.nsp - 1) / it.nsp;
    const int ch_lo = first_ch + it.sp * cps;
    const int ch_hi = ch_lo + cps < first_ch + nch ? ch_lo + cps : first_ch + nch;
    if (ch_lo >= ch_hi) return;
    int start = chunk_at<TAB>(a, sh.first_pos);
    start = start < ch_lo ? ch_lo : (start >= ch_hi ? ch_hi - 1 : start);
    const int sc_lo = super_of<TAB>(a, ch_lo), sc_hi = super_of<TAB>(a, ch_hi - 1) + 1;
    const int sc_start = super_of<TAB>(a, start);
    bool stale = false;
    for (int ss = 0; ss < sc_hi - sc_lo; ++ss) {
        const int sc = zigzag(ss, sc_start, sc_lo, sc_hi);
        if (a.prune) {
            if (stale) {
                __syncthreads();
                umax = fmaxf(fmaxf(sh.wmax[0], sh.wmax[1]), fmaxf(sh.wmax[2], sh.wmax[3]));
                stale = false;
            }
            if (ball_lb2(sh, a.sballs + (int64_t)sc * BALL_STRIDE) > umax) continue;
        }
        const int sf = super_first<TAB>(a, sc), se = super_end<TAB>(a, sc);
        const int c_lo = sf > ch_lo ? sf : ch_lo;
        const int c_hi = se < ch_hi ? se : ch_hi;
        const int cstart = (sc == sc_start) ? start : (sc > sc_start ? c_lo : c_hi - 1);
        for (int cs = 0; cs < c_hi - c_lo; ++cs) {
            const int ci = zigzag(cs, cstart, c_lo, c_hi);
            const int64_t c0 = chunk_begin<TAB>(a, ci);
            const int64_t c1 = chunk_end<TAB>(a, ci) - 1;
            const int lo_c = a.compS[c0], hi_c = a.compS[c1];
            if (lo_r == hi_r && lo_c == hi_c && lo_r == lo_c) continue;   // all one component
            if (a.prune) {
                if (stale) {
                    __syncthreads();
                    umax = fmaxf(fmaxf(sh.wmax[0], sh.wmax[1]), fmaxf(sh.wmax[2], sh.wmax[3]));
                    stale = false;
                }
                if (ball_lb2(sh, a.balls + (int64_t)ci * BALL_STRIDE) > umax) continue;
            }
            process(ci, lo_c, hi_c);
            stale = true;
        }
    }
}

// Max over the 64 rows of the calling wave of v (one value per lane), stored
// in sh.wmax[wave].
__device__ __forceinline__ void wave_max_store(TileShared& sh, float v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) sh.wmax[threadIdx.x >> 6] = v;
}

}  // namespace nnm
