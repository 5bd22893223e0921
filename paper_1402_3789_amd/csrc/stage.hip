// stage.hip -- input validation and operand staging.
//
// The paper leaves scaling and shifting of the data to the caller (section
// "Overall idea of the algorithm") and asks the main module to check the
// data array (section "Objectives of the main module").  Staging therefore
// (1) scans X once for non-finite values, per-feature ranges and whether
// every feature is an integer in [-16, 16], and (2) writes the low-precision
// operands of the candidate pass together with the inputs of their error
// bound.  The candidate value of a pair is
//     t = ||q_i||^2 + ||q_j||^2 - 2 q_i . q_j,   q = lowp(sigma (x - c)),
// with both squared norms folded into spare K slots so the matrix-core
// output is t itself.
#include "nnm_common.h"

namespace nnm {
namespace {

__device__ __forceinline__ uint32_t ord_enc(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// One pass over X: eight lanes per point, lane q covering features
// 4q..4q+3, so the reads of a row are contiguous across its lanes.
__global__ __launch_bounds__(256) void k_stage_stats(const float* __restrict__ X,
                                                     int64_t n, int d, int64_t ld,
                                                     StageStats* st)
{
    static_assert(DMAX == 32, "eight lanes of four features");
    __shared__ uint32_t smin[DMAX], smax[DMAX];
    __shared__ int sbad, snonint;
    if (threadIdx.x < DMAX) {
        smin[threadIdx.x] = 0xFFFFFFFFu;
        smax[threadIdx.x] = 0u;
    }
    if (threadIdx.x == 0) { sbad = 0; snonint = 0; }
    __syncthreads();
    const int q = threadIdx.x & 7;
    int bad = 0, nonint = 0;
    uint32_t lo[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    uint32_t hi[4] = {0u, 0u, 0u, 0u};
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 3);
    for (int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 3) + (threadIdx.x >> 3); i < n; i += stride) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int f = 4 * q + h;
            if (f >= d) continue;
            const float v = X[i * ld + f];
            if (!__builtin_isfinite(v)) { bad = 1; continue; }
            if (v != __builtin_rintf(v) || __builtin_fabsf(v) > 16.0f) nonint = 1;
            const uint32_t e = ord_enc(v);
            lo[h] = lo[h] < e ? lo[h] : e;
            hi[h] = hi[h] > e ? hi[h] : e;
        }
    }
    // over the eight points of the wave that share q, then one LDS atomic
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        for (int off = 8; off < 64; off <<= 1) {
            const uint32_t olo = __shfl_xor(lo[h], off);
            const uint32_t ohi = __shfl_xor(hi[h], off);
            lo[h] = lo[h] < olo ? lo[h] : olo;
            hi[h] = hi[h] > ohi ? hi[h] : ohi;
        }
        if ((threadIdx.x & 63) < 8 && 4 * q + h < d) {
            atomicMin(&smin[4 * q + h], lo[h]);
            atomicMax(&smax[4 * q + h], hi[h]);
        }
    }
    if (bad) atomicOr(&sbad, 1);
    if (nonint) atomicOr(&snonint, 1);
    __syncthreads();
    if (threadIdx.x < d) {
        atomicMin(&st->fmin[threadIdx.x], smin[threadIdx.x]);
        atomicMax(&st->fmax[threadIdx.x], smax[threadIdx.x]);
    }
    if (threadIdx.x == 0) {
        if (sbad) atomicOr(&st->nonfinite, 1);
        if (snonint) atomicOr(&st->nonint, 1);
    }
}

// Low-precision rounding of one value (round to nearest even).
template <int OP>
__device__ __forceinline__ uint16_t to_lp(float f);
template <>
__device__ __forceinline__ uint16_t to_lp<OP_BF16>(float f) { return f32_to_bf16_rn(f); }
template <>
__device__ __forceinline__ uint16_t to_lp<OP_FP16>(float f) { return f32_to_f16_rn(f); }

template <int OP>
__device__ __forceinline__ float from_lp(uint16_t h);
template <>
__device__ __forceinline__ float from_lp<OP_BF16>(uint16_t h) { return bf16_to_f32(h); }
template <>
__device__ __forceinline__ float from_lp<OP_FP16>(uint16_t h) { return f16_to_f32(h); }

// Unit roundoff of the operand format plus the FP32 / FP64 roundings on the
// way (x - c in FP64, then to FP32, then to the operand format), and the
// absolute error floor of its subnormal range.
template <int OP> struct LpBound;
template <> struct LpBound<OP_BF16> {
    static constexpr double alpha = 0x1p-8 + 0x1p-23 + 0x1p-50;
    static constexpr double beta = 0x1p-125;
};
template <> struct LpBound<OP_FP16> {
    static constexpr double alpha = 0x1p-11 + 0x1p-23 + 0x1p-50;
    static constexpr double beta = 0x1p-25 + 0x1p-149;
};

template <int OP>
__global__ __launch_bounds__(256) void k_stage_operands_16(
    const float* __restrict__ X, int64_t n, int d, int64_t ld, int exact,
    const float* __restrict__ centre, float sigma, uint16_t* __restrict__ opR,
    uint16_t* __restrict__ opC, PointConst* __restrict__ pc, StageStats* st)
{
    // lanes past the end repeat the last point (for the wave maxima) and
    // store nothing
    const int64_t b0 = blockIdx.x * (int64_t)blockDim.x;
    const int64_t gi = b0 + threadIdx.x;
    if (b0 >= n) return;
    const bool valid = gi < n;
    const int64_t i = valid ? gi : n - 1;
    // the block's rows, read whole and together (row-major X: consecutive
    // threads read consecutive features), then each thread's own row from LDS
    __shared__ float tile[256 * DMAX_MFMA];
    __shared__ float bmax[4][4];
    {
        // 32 lanes a row (d <= 26 of them load), 8 rows a pass
        const int rows = (int)((n - b0) < 256 ? (n - b0) : 256);
        const int f = threadIdx.x & 31;
        for (int r = threadIdx.x >> 5; r < rows; r += 8)
            if (f < d) tile[r * d + f] = X[(b0 + r) * ld + f];
    }
    __syncthreads();
    const float* xrow = tile + (int)(i - b0) * d;
    uint16_t q[KSLOT];
    double nrm = 0.0, vn = 0.0;
#pragma unroll
    for (int f = 0; f < KSLOT; ++f) q[f] = 0;
    for (int f = 0; f < d; ++f) {
        double v = ((double)xrow[f] - (double)centre[f]) * (double)sigma;
        uint16_t h = to_lp<OP>((float)v);
        q[f] = h;
        double qd = (double)from_lp<OP>(h);
        nrm += qd * qd;
        vn += v * v;
    }
    // three-part split of ||q||^2 into operand-format values
    double r = nrm;
    uint16_t part[NORM_PARTS];
    double psum = 0.0;
    for (int k = 0; k < NORM_PARTS; ++k) {
        part[k] = to_lp<OP>((float)r);
        double pv = (double)from_lp<OP>(part[k]);
        psum += __builtin_fabs(pv);
        r -= pv;
    }
    const uint16_t one = to_lp<OP>(1.0f);
    // row form: [q, parts, 1,1,1]; column form: [-2q, 1,1,1, parts]
    uint16_t row[KSLOT], col[KSLOT];
#pragma unroll
    for (int f = 0; f < KSLOT; ++f) {
        row[f] = q[f];
        uint16_t c = q[f];
        if (f < d) c = to_lp<OP>(-2.0f * from_lp<OP>(q[f]));  // exact scaling
        col[f] = c;
    }
#pragma unroll
    for (int k = 0; k < NORM_PARTS; ++k) {
        row[DMAX_MFMA + k] = part[k];
        row[DMAX_MFMA + NORM_PARTS + k] = one;
        col[DMAX_MFMA + k] = one;
        col[DMAX_MFMA + NORM_PARTS + k] = part[k];
    }
    if (valid) {
        uint4* dR = reinterpret_cast<uint4*>(opR + i * KSLOT);
        uint4* dC = reinterpret_cast<uint4*>(opC + i * KSLOT);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            uint4 a, b;
            a.x = row[8 * w + 0] | ((uint32_t)row[8 * w + 1] << 16);
            a.y = row[8 * w + 2] | ((uint32_t)row[8 * w + 3] << 16);
            a.z = row[8 * w + 4] | ((uint32_t)row[8 * w + 5] << 16);
            a.w = row[8 * w + 6] | ((uint32_t)row[8 * w + 7] << 16);
            b.x = col[8 * w + 0] | ((uint32_t)col[8 * w + 1] << 16);
            b.y = col[8 * w + 2] | ((uint32_t)col[8 * w + 3] << 16);
            b.z = col[8 * w + 4] | ((uint32_t)col[8 * w + 5] << 16);
            b.w = col[8 * w + 6] | ((uint32_t)col[8 * w + 7] << 16);
            dR[w] = a;
            dC[w] = b;
        }
    }
    PointConst p;
    if (exact) {
        p.Q = 0.f; p.P = 0.f; p.rho = 0.f; p.eta = 0.f;
    } else {
        p.Q = d2f_up(__builtin_sqrt(nrm) * (1.0 + 0x1p-40));
        p.P = d2f_up(psum * (1.0 + 0x1p-40));
        p.rho = d2f_up(__builtin_fabs(r) + nrm * 0x1p-47);
        p.eta = d2f_up((LpBound<OP>::alpha * __builtin_sqrt(vn) * (1.0 + 0x1p-40) +
                        LpBound<OP>::beta * __builtin_sqrt((double)d)) * (1.0 + 0x1p-40));
    }
    if (valid) pc[i] = p;
    // column maxima: one atomic per workgroup and quantity, skipped when the
    // maximum already read is not smaller (non-negative floats order as
    // their bits; maxima only grow)
    float m4[4] = {p.Q, p.P, p.rho, p.eta};
#pragma unroll
    for (int q = 0; q < 4; ++q)
        for (int off = 32; off > 0; off >>= 1) m4[q] = fmaxf(m4[q], __shfl_xor(m4[q], off));
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 4; ++q) bmax[threadIdx.x >> 6][q] = m4[q];
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        const float m = fmaxf(fmaxf(bmax[0][q], bmax[1][q]), fmaxf(bmax[2][q], bmax[3][q]));
        const uint32_t bits = __float_as_uint(m);
        if (bits > __atomic_load_n(&st->colmax[q], __ATOMIC_RELAXED)) atomicMax(&st->colmax[q], bits);
    }
}

__device__ __forceinline__ uint8_t to_fp8(float f)
{
    // hardware conversion to the target's native e4m3 encoding
    int packed = __builtin_amdgcn_cvt_pk_fp8_f32(f, 0.0f, 0, false);
    return (uint8_t)(packed & 0xFF);
}

// FP8 operands, integer mode only: q = x exactly (|x| <= 16).  ||q||^2 is
// carried in balanced base-32 digits, n = (32a) * 32 + b * 32 + c * 1.
__global__ __launch_bounds__(256) void k_stage_operands_fp8(
    const float* __restrict__ X, int64_t n, int d, int64_t ld,
    uint8_t* __restrict__ opR, uint8_t* __restrict__ opC,
    PointConst* __restrict__ pc)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint8_t row[KSLOT], col[KSLOT];
    int nrm = 0;
#pragma unroll
    for (int f = 0; f < KSLOT; ++f) { row[f] = to_fp8(0.f); col[f] = row[f]; }
    for (int f = 0; f < d; ++f) {
        float v = X[i * ld + f];
        int iv = (int)v;
        nrm += iv * iv;
        row[f] = to_fp8(v);
        col[f] = to_fp8(-2.0f * v);
    }
    int c = ((nrm + 16) & 31) - 16;
    int t = (nrm - c) / 32;
    int b = ((t + 16) & 31) - 16;
    int a = (t - b) / 32;
    float val[NORM_PARTS] = {32.0f * a, (float)b, (float)c};
    float cst[NORM_PARTS] = {32.0f, 32.0f, 1.0f};
#pragma unroll
    for (int k = 0; k < NORM_PARTS; ++k) {
        row[DMAX_MFMA + k] = to_fp8(val[k]);
        row[DMAX_MFMA + NORM_PARTS + k] = to_fp8(cst[k]);
        col[DMAX_MFMA + k] = to_fp8(cst[k]);
        col[DMAX_MFMA + NORM_PARTS + k] = to_fp8(val[k]);
    }
    uint4* dR = reinterpret_cast<uint4*>(opR + i * KSLOT);
    uint4* dC = reinterpret_cast<uint4*>(opC + i * KSLOT);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        uint4 x, y;
        uint32_t* px = reinterpret_cast<uint32_t*>(&x);
        uint32_t* py = reinterpret_cast<uint32_t*>(&y);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int o = 16 * w + 4 * e;
            px[e] = row[o] | (row[o + 1] << 8) | (row[o + 2] << 16) | ((uint32_t)row[o + 3] << 24);
            py[e] = col[o] | (col[o + 1] << 8) | (col[o + 2] << 16) | ((uint32_t)col[o + 3] << 24);
        }
        dR[w] = x;
        dC[w] = y;
    }
    pc[i] = PointConst{0.f, 0.f, 0.f, 0.f};
}

// Gather everything the candidate pass reads into component-sorted order.
template <int BYTES>
__global__ __launch_bounds__(256) void k_gather(int64_t n, const int32_t* __restrict__ perm,
                                                const uint4* __restrict__ opR,
                                                const uint4* __restrict__ opC,
                                                const PointConst* __restrict__ pc,
                                                const int32_t* __restrict__ comp,
                                                uint4* __restrict__ opRs,
                                                uint4* __restrict__ opCs,
                                                PointConst* __restrict__ pcs,
                                                int32_t* __restrict__ compS)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    int64_t i = perm[p];
    constexpr int W = BYTES / 16;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        opRs[p * W + w] = opR[i * W + w];
        opCs[p * W + w] = opC[i * W + w];
    }
    pcs[p] = pc[i];
}

__global__ __launch_bounds__(256) void k_gather_fp32(int64_t n, const int32_t* __restrict__ perm,
                                                     const float* __restrict__ X, int d,
                                                     int64_t ld, float* __restrict__ xs)
{
    // eight lanes per point, one float4 of the padded row each: the reads of
    // a row and the 128-byte write are contiguous across its lanes
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t p = t >> 3;
    const int q = (int)(t & 7);
    if (p >= n) return;
    const float* src = X + (int64_t)perm[p] * ld + 4 * q;
    float4 v;
    v.x = (4 * q + 0 < d) ? src[0] : 0.f;
    v.y = (4 * q + 1 < d) ? src[1] : 0.f;
    v.z = (4 * q + 2 < d) ? src[2] : 0.f;
    v.w = (4 * q + 3 < d) ? src[3] : 0.f;
    reinterpret_cast<float4*>(xs + p * DMAX)[q] = v;
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_stage_stats(const float* X, int64_t n, int d, int64_t ld,
                              StageStats* st, hipStream_t s)
{
    int64_t blocks = (n + 31) / 32;          // 32 points per pass of a block
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    k_stage_stats<<<(unsigned)blocks, 256, 0, s>>>(X, n, d, ld, st);
    return hipGetLastError();
}

hipError_t launch_stage_operands(const float* X, int64_t n, int d, int64_t ld,
                                 int opkind, int exact, const float* centre,
                                 float sigma, void* opR, void* opC,
                                 PointConst* pc, StageStats* st, hipStream_t s)
{
    if (d < 1 || d > DMAX_MFMA) return hipErrorInvalidValue;   // the row tile holds DMAX_MFMA
    unsigned g = grid_for(n, 256);
    switch (opkind) {
    case OP_BF16:
        k_stage_operands_16<OP_BF16><<<g, 256, 0, s>>>(X, n, d, ld, exact, centre, sigma,
                                                       (uint16_t*)opR, (uint16_t*)opC, pc, st);
        break;
    case OP_FP16:
        k_stage_operands_16<OP_FP16><<<g, 256, 0, s>>>(X, n, d, ld, exact, centre, sigma,
                                                       (uint16_t*)opR, (uint16_t*)opC, pc, st);
        break;
    case OP_FP8:
        k_stage_operands_fp8<<<g, 256, 0, s>>>(X, n, d, ld, (uint8_t*)opR, (uint8_t*)opC, pc);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gather_points(int64_t n, int opkind, const int32_t* perm,
                                const void* opR, const void* opC,
                                const PointConst* pc, const float* X, int d,
                                int64_t ld, const int32_t* comp, void* opRs,
                                void* opCs, PointConst* pcs, float* xs,
                                int32_t* compS, hipStream_t s)
{
    unsigned g = grid_for(n, 256);
    if (opkind == OP_FP32) {
        static_assert(DMAX == 32, "eight float4 per padded row");
        k_gather_fp32<<<grid_for(n * 8, 256), 256, 0, s>>>(n, perm, X, d, ld, xs);
    } else if (opkind == OP_FP8) {
        k_gather<32><<<g, 256, 0, s>>>(n, perm, (const uint4*)opR, (const uint4*)opC, pc, comp,
                                       (uint4*)opRs, (uint4*)opCs, pcs, compS);
    } else {
        k_gather<64><<<g, 256, 0, s>>>(n, perm, (const uint4*)opR, (const uint4*)opC, pc, comp,
                                       (uint4*)opRs, (uint4*)opCs, pcs, compS);
    }
    return hipGetLastError();
}

}  // namespace nnm
