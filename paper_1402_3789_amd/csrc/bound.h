// bound.h -- the proven error bound of the candidate distances and the
// selection thresholds derived from it, shared by the candidate passes (which
// apply them) and FP64 rescoring (which reports, for every rescored
// survivor, the bound that was applied to it next to the observed error).
#pragma once

#include "nnm_common.h"

namespace nnm {

// Matrix-core candidates.  For row i and column j the FP32 accumulator is
// t = ||q_i||^2 + ||q_j||^2 - 2 q_i.q_j over the low-precision operands q in
// a frame scaled by sigma; with eps (accumulation and norm-slot slack) and
// eta (quantisation slack) of the pair,
//     |t - sigma^2 s| <= E(t) = KFAC (eps + eta (2 sqrt(t+ + eps) + eta)),
// where s is the FP64 key of eq. (1); KFAC covers the FP64 key's own
// rounding ((D + 2) 2^-53 relative).
constexpr float KFAC = 1.0f + 0x1p-20f;

// Upper bound on the exact (scaled) key of a column whose candidate is t:
// t + E(t), evaluated in FP32 with a relative margin of 2^-18 that covers
// the roundings of the expression (square root within 1 ulp, a dozen
// operations).  exact: t == sigma^2 s.
__device__ __forceinline__ float upper_from_t(float t, float eps, float eta, int exact)
{
    if (exact) return t;
    const float e = KFAC * (eps + eta * (2.f * __builtin_sqrtf(fmaxf(t, 0.f) + eps) + eta));
    return (t + e) + (__builtin_fabsf(t) + e) * 0x1p-18f;
}

// Largest candidate value that can still belong to a column whose exact key
// is <= U (scaled units): t - E(t) <= U  iff  sqrt(t + eps) <= W with
// W = KFAC eta + sqrt(KFAC^2 eta^2 + U + eps (1 + KFAC) + KFAC eta^2).
// Never above FLT_MAX, so +inf candidates (masked columns) never pass.
__device__ __forceinline__ float thresh_from_U(float U, float eps, float eta, int exact)
{
    float T;
    if (exact) {
        T = U;
    } else {
        const float ke = KFAC * eta;
        const float W = ke + __builtin_sqrtf(ke * ke + U + eps * (1.f + KFAC) + ke * eta);
        T = (W * W - eps) + (W * W + eps) * 0x1p-18f;
    }
    return fminf(T, 3.402823466e38f);
}

// Global frame (one centre and scale for every pair): the slack of row
// point r against any column, from the maxima of the columns' bound inputs.
__device__ __forceinline__ float global_eps(const PointConst& r, const BoundConst& b)
{
    return (b.gamma * (2.f * r.Q * b.colQ + r.P + b.colP) + r.rho + b.colRho) * (1.f + 0x1p-20f);
}

__device__ __forceinline__ float global_eta(const PointConst& r, const BoundConst& b)
{
    return (r.eta + b.colEta) * (1.f + 0x1p-22f);
}

// FP32 direct differences: the computed sum of squares t over d features
// satisfies |t - s| <= crel s + a0 (relative (d + 3) 2^-24 and an underflow
// floor), so s <= (t + a0) / (1 - crel).
__host__ __device__ __forceinline__ double fp32_crel(int d) { return (double)(d + 3) * 0x1p-24 + 0x1p-40; }
__host__ __device__ __forceinline__ double fp32_a0(int d) { return (double)d * 0x1p-148; }

__device__ __forceinline__ float fp32_thresh_from_U(double U, double crel, double a0)
{
    return d2f_up((U * (1.0 + crel) + a0) * (1.0 + 0x1p-40));
}

__device__ __forceinline__ double fp32_upper_from_t(double t, double crel, double a0)
{
    return (t + a0) / (1.0 - crel) * (1.0 + 0x1p-40);
}

// How rescoring recovers the bound applied to a survivor.
enum BoundMode : int {
    BOUND_FP32 = 0,     // FP32 direct differences: fp32_upper_from_t(t) - t
    BOUND_GLOBAL = 1,   // matrix cores, global frame: from the row's PointConst
    BOUND_LOCAL = 2,    // matrix cores, super-chunk frames: t + E(t) stored per survivor
    BOUND_EXACT = 3     // exact integer data: E = 0
};

}  // namespace nnm
