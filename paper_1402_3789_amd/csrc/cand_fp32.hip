// cand_fp32.hip -- the plain FP32 candidate pass on the vector ALUs.
//
// Same contract as the matrix-core pass (pair distances fused with the
// selection of the k smallest per row, component mask, survivor lists), but
// the candidate is the FP32 direct-difference sum
//     t_ij = sum_f fma((x_if - x_jf), (x_if - x_jf), .)
// which is within a relative (D + 3) 2^-24 of the exact FP64 key.  One row
// per thread (features in registers); column chunks are broadcast from LDS.
#include "nnm_common.h"

namespace nnm {
namespace {

constexpr int BM = 256;
constexpr int BN = 128;

__device__ __forceinline__ float fp32_thresh_from_U(double U, double crel, double a0)
{
    return d2f_up((U * (1.0 + crel) + a0) * (1.0 + 0x1p-40));
}

__device__ __forceinline__ double fp32_upper_from_t(double t, double crel, double a0)
{
    return (t + a0) / (1.0 - crel);
}

template <int DP>
__global__ __launch_bounds__(256, 2) void k_cand_fp32(CandArgs a)
{
    constexpr int F4 = DP / 4;
    __shared__ float4 cbuf[BN * F4];
    __shared__ int32_t ccomp[BN];
    __shared__ int32_t tileLo, tileHi, tileRows;
    extern __shared__ float topk[];   // [BM][k]

    const int tid = threadIdx.x;
    const int k = a.k;
    const int64_t slot = (int64_t)blockIdx.x * BM + tid;
    const bool valid = slot < a.n_rows;
    const int rp = valid ? (a.rows ? a.rows[slot] : a.row0 + (int)slot) : 0;
    const double crel = (double)(a.d + 3) * 0x1p-24 + 0x1p-40;
    const double a0 = (double)a.d * 0x1p-148;

    float xr[DP];
    {
        const float4* src = reinterpret_cast<const float4*>(a.xs + (int64_t)rp * DMAX);
#pragma unroll
        for (int q = 0; q < F4; ++q) {
            float4 v = src[q];
            xr[4 * q + 0] = v.x; xr[4 * q + 1] = v.y; xr[4 * q + 2] = v.z; xr[4 * q + 3] = v.w;
        }
    }
    const int rc = valid ? a.compS[rp] : -2;
    float T = -__builtin_huge_valf();
    if (valid) {
        T = 3.402823466e38f;
        if (a.u0) {
            const double u0 = a.u0[rp];
            if (u0 >= 0.0) T = fminf(T, fp32_thresh_from_U(u0, crel, a0));
        }
    }
    float* tk = topk + tid * k;
    for (int e = 0; e < k; ++e) tk[e] = __builtin_huge_valf();
    if (tid == 0) {
        int64_t last = (int64_t)blockIdx.x * BM + BM - 1;
        if (last >= a.n_rows) last = a.n_rows - 1;
        const int64_t first = (int64_t)blockIdx.x * BM;
        tileLo = a.compS[a.rows ? a.rows[first] : a.row0 + (int)first];
        tileHi = a.compS[a.rows ? a.rows[last] : a.row0 + (int)last];
        tileRows = (int)(last - first + 1);
    }
    __syncthreads();
    const int lo_r = tileLo, hi_r = tileHi;

    int64_t cps = ((int64_t)a.np + a.col_splits - 1) / a.col_splits;
    cps = (cps + BN - 1) / BN * BN;
    const int64_t c_begin = (int64_t)blockIdx.y * cps;
    int64_t c_end = c_begin + cps;
    if (c_end > a.np) c_end = a.np;
    unsigned long long pairs = 0;

    for (int64_t c0 = c_begin; c0 < c_end; c0 += BN) {
        const int ncols = (int)((c_end - c0) < BN ? (c_end - c0) : BN);
        const int lo_c = a.compS[c0];
        const int hi_c = a.compS[c0 + ncols - 1];
        if (lo_r == hi_r && lo_c == hi_c && lo_r == lo_c) continue;
        const bool masked = !(hi_c < lo_r || lo_c > hi_r);
        __syncthreads();
        for (int idx = tid; idx < BN * F4; idx += 256) {
            const int c = idx / F4, q = idx % F4;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < ncols) v = reinterpret_cast<const float4*>(a.xs + (c0 + c) * DMAX)[q];
            cbuf[idx] = v;
        }
        if (tid < BN) ccomp[tid] = (tid < ncols) ? a.compS[c0 + tid] : -1;
        __syncthreads();
        pairs += (unsigned long long)ncols;
        for (int c = 0; c < ncols; ++c) {
            float t = 0.f;
#pragma unroll
            for (int q = 0; q < F4; ++q) {
                const float4 y = cbuf[c * F4 + q];
                const float d0 = xr[4 * q + 0] - y.x;
                const float d1 = xr[4 * q + 1] - y.y;
                const float d2 = xr[4 * q + 2] - y.z;
                const float d3 = xr[4 * q + 3] - y.w;
                t = __builtin_fmaf(d0, d0, t);
                t = __builtin_fmaf(d1, d1, t);
                t = __builtin_fmaf(d2, d2, t);
                t = __builtin_fmaf(d3, d3, t);
            }
            if (masked && ccomp[c] == rc) t = __builtin_huge_valf();
            if (t <= T) {
                const int pos = atomicAdd(&a.surv_cnt[slot], 1);
                if (pos < a.S) {
                    a.surv_j[slot * a.S + pos] = (int)(c0 + c);
                    a.surv_t[slot * a.S + pos] = t;
                }
                if (t < tk[k - 1]) {
                    int p = k - 1;
                    while (p > 0 && tk[p - 1] > t) { tk[p] = tk[p - 1]; --p; }
                    tk[p] = t;
                    const float kth = tk[k - 1];
                    if (kth < __builtin_huge_valf()) {
                        const float Tn = fp32_thresh_from_U(fp32_upper_from_t((double)kth, crel, a0), crel, a0);
                        T = fminf(T, Tn);
                    }
                }
            }
        }
    }
    if (tid == 0 && a.pairs) atomicAdd(a.pairs, pairs * (unsigned long long)tileRows);
}

}  // namespace

hipError_t launch_cand_fp32(const CandArgs& a, hipStream_t s)
{
    if (a.n_rows <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.n_rows + BM - 1) / BM), (unsigned)a.col_splits);
    size_t shm = (size_t)BM * a.k * sizeof(float);
    const int dp = (a.d + 3) / 4 * 4;
    switch (dp) {
    case 4: k_cand_fp32<4><<<grid, 256, shm, s>>>(a); break;
    case 8: k_cand_fp32<8><<<grid, 256, shm, s>>>(a); break;
    case 12: k_cand_fp32<12><<<grid, 256, shm, s>>>(a); break;
    case 16: k_cand_fp32<16><<<grid, 256, shm, s>>>(a); break;
    case 20: k_cand_fp32<20><<<grid, 256, shm, s>>>(a); break;
    case 24: k_cand_fp32<24><<<grid, 256, shm, s>>>(a); break;
    case 28: k_cand_fp32<28><<<grid, 256, shm, s>>>(a); break;
    case 32: k_cand_fp32<32><<<grid, 256, shm, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nnm
