// cand_common.h -- pieces shared by the matrix-core and the FP32 candidate
// passes: the bounding ball of a tile of rows, the near-first order of column
// chunks and the chunk pruning test.
#pragma once

#include "nnm_common.h"

namespace nnm {

// Chunk size of the candidate sweep; chunk balls are built for it.
constexpr int CHUNK = 256;
constexpr int BALL_STRIDE = DMAX + 1;   // centre[DMAX], radius

// Shared-memory scratch for the per-workgroup tile ball and the per-chunk
// pruning decision (one instance per workgroup).
struct TileShared {
    double acc[4][DMAX];
    float cen[DMAX];
    double red[4];
    float rball;
    float umax;
    int decision;
    int lo, hi, rows, first_pos;
};

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

}  // namespace nnm
