// cand_common.h -- pieces shared by the matrix-core and the FP32 candidate
// passes: the bounding ball of a tile of rows, the near-first order of column
// chunks and the chunk pruning test.
#pragma once

#include "nnm_common.h"

namespace nnm {

// Chunk size of the candidate sweep; chunk balls are built for it, and for
// super-chunks of SUPER consecutive chunks.
constexpr int CHUNK = 256;
constexpr int SUPER = 16;
constexpr int BALL_STRIDE = DMAX + 1;   // centre[DMAX], radius

// Shared-memory scratch for the per-workgroup tile ball and the per-chunk
// pruning decision (one instance per workgroup).
struct TileShared {
    double acc[4][DMAX];
    float cen[DMAX];
    double red[4];
    float wmax[4];
    float rball;
    float umax;
    int decision;
    int lo, hi, rows, first_pos;
    int col_lo, col_hi;      // columns this tile may pair with (sorted positions)
};

// Row slots [rbeg, rend) and column range [cl, ch) of this workgroup's tile.
__device__ __forceinline__ int4 tile_of(const CandArgs& a, int bm)
{
    if (a.tiles) return a.tiles[blockIdx.x];
    const int rbeg = (int)blockIdx.x * bm;
    const int rend = rbeg + bm < a.n_rows ? rbeg + bm : a.n_rows;
    return make_int4(rbeg, rend, 0, a.np);
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

// Lower bound on the squared distance of any pair across the tile ball and
// chunk ball `ball` (centre[DMAX], radius), rounded down.
__device__ inline double ball_lb2(const TileShared& sh, const float* ball, int d)
{
    double s = 0.0;
    for (int f = 0; f < d; ++f) {
        const double df = (double)sh.cen[f] - (double)ball[f];
        s += df * df;
    }
    const double dist = __builtin_sqrt(s) * (1.0 - 0x1p-40);
    const double lb = dist - (double)sh.rball - (double)ball[DMAX];
    if (!(lb > 0.0)) return 0.0;
    return lb * lb * (1.0 - 0x1p-40);
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
template <typename Fn>
__device__ inline void sweep_chunks(TileShared& sh, const CandArgs& a, int lo_r, int hi_r,
                                    float umax, Fn&& process)
{
    const int first_ch = sh.col_lo / CHUNK;
    const int nch = (sh.col_hi + CHUNK - 1) / CHUNK - first_ch;
    const int cps = (nch + a.col_splits - 1) / a.col_splits;
    const int ch_lo = first_ch + (int)blockIdx.y * cps;
    const int ch_hi = ch_lo + cps < first_ch + nch ? ch_lo + cps : first_ch + nch;
    if (ch_lo >= ch_hi) return;
    int start = sh.first_pos / CHUNK;
    start = start < ch_lo ? ch_lo : (start >= ch_hi ? ch_hi - 1 : start);
    const int sc_lo = ch_lo / SUPER, sc_hi = (ch_hi - 1) / SUPER + 1;
    const int sc_start = start / SUPER;
    bool stale = false;
    for (int ss = 0; ss < sc_hi - sc_lo; ++ss) {
        const int sc = zigzag(ss, sc_start, sc_lo, sc_hi);
        if (a.prune) {
            if (stale) {
                __syncthreads();
                umax = fmaxf(fmaxf(sh.wmax[0], sh.wmax[1]), fmaxf(sh.wmax[2], sh.wmax[3]));
                stale = false;
            }
            if (ball_lb2(sh, a.sballs + (int64_t)sc * BALL_STRIDE, a.d) > (double)umax) continue;
        }
        const int c_lo = sc * SUPER > ch_lo ? sc * SUPER : ch_lo;
        const int c_hi = sc * SUPER + SUPER < ch_hi ? sc * SUPER + SUPER : ch_hi;
        const int cstart = (sc == sc_start) ? start : (sc > sc_start ? c_lo : c_hi - 1);
        for (int cs = 0; cs < c_hi - c_lo; ++cs) {
            const int ci = zigzag(cs, cstart, c_lo, c_hi);
            const int64_t c0 = (int64_t)ci * CHUNK;
            const int64_t c1 = (a.np - c0) < CHUNK ? a.np - 1 : c0 + CHUNK - 1;
            const int lo_c = a.compS[c0], hi_c = a.compS[c1];
            if (lo_r == hi_r && lo_c == hi_c && lo_r == lo_c) continue;   // all one component
            if (a.prune) {
                if (stale) {
                    __syncthreads();
                    umax = fmaxf(fmaxf(sh.wmax[0], sh.wmax[1]), fmaxf(sh.wmax[2], sh.wmax[3]));
                    stale = false;
                }
                if (ball_lb2(sh, a.balls + (int64_t)ci * BALL_STRIDE, a.d) > (double)umax) continue;
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
