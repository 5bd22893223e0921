// cand_fp32.hip -- the plain FP32 candidate pass on the vector ALUs.
//
// Same contract as the matrix-core pass (pair distances fused with the
// selection of the k smallest per row, component mask, survivor lists,
// nearest-first chunk order, ball pruning), but the candidate is the FP32
// direct-difference sum
//     t_ij = sum_f fma((x_if - x_jf), (x_if - x_jf), .)
// which is within a relative (D + 3) 2^-24 (plus an underflow floor) of the
// exact FP64 key.  One row per thread (features in registers); column
// chunks are broadcast from LDS.
//
// The L1 and L-infinity metrics (nnm_metric) run here too, with the FP32
// sum or maximum of |x_if - x_jf|: one rounding per difference and per
// addition, within the same relative bound of their FP64 keys.  The chunk
// balls are Euclidean; since the L1 distance is at least the Euclidean one
// and the L-infinity distance at least 1/sqrt(D) of it, a ball whose squared
// Euclidean gap exceeds U^2 (L1) or D U^2 (L-infinity) holds no candidate.
#include "cand_common.h"

namespace nnm {
namespace {

template <int M>
__device__ __forceinline__ float prune_bound(float U, int d)
{
    if constexpr (M == NNM_METRIC_L1) return U * U * (1.0f + 0x1p-20f);
    else if constexpr (M == NNM_METRIC_LINF) return (float)d * U * U * (1.0f + 0x1p-20f);
    else return U;
}

// one feature's contribution to the candidate t
template <int M>
__device__ __forceinline__ float acc_term(float t, float diff)
{
    if constexpr (M == NNM_METRIC_L1) return t + __builtin_fabsf(diff);
    else if constexpr (M == NNM_METRIC_LINF) return fmaxf(t, __builtin_fabsf(diff));
    else return __builtin_fmaf(diff, diff, t);
}

constexpr int BM = 256;
constexpr int BN = CHUNK;

// One work item (row tile, column split); share: the row thresholds are
// shared with the item's other column splits through gT / gU.
template <int DP, bool TAB, int M>
__device__ __forceinline__ void cand_fp32_item(const CandArgs& a, const Item& it, const bool share)
{
    constexpr int F4 = DP / 4;
    __shared__ float4 cbuf[BN * F4];
    __shared__ int32_t ccomp[BN];
    __shared__ TileShared sh;
    extern __shared__ float topk[];   // [BM][k]

    const int tid = threadIdx.x;
    const int k = a.k;
    const int4 tile = tile_of(a, BM, it);
    const int64_t slot = (int64_t)tile.x + tid;
    const bool valid = slot < tile.y;
    const int rp = valid ? (a.rows ? a.rows[slot] : a.row0 + (int)slot) : 0;
    const double crel = fp32_crel(a.d);
    const double a0 = fp32_a0(a.d);

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
    float U = 0.f;
    if (valid) {
        T = 3.402823466e38f;
        U = __builtin_huge_valf();
        if (a.u0) {
            const double u0 = a.u0[rp];
            if (u0 >= 0.0) {
                T = fminf(T, fp32_thresh_from_U(u0, crel, a0));
                U = d2f_up(u0);
            }
        }
    }
    float* tk = topk + tid * k;
    for (int e = 0; e < k; ++e) tk[e] = __builtin_huge_valf();
    if (valid && !(U < __builtin_huge_valf())) {
        // no bound yet: seed one from the row's neighbours in the sorted
        // order (distinct admissible columns, keys bounded from FP32)
        for (int o = -k; o <= k; ++o) {
            const int64_t q = (int64_t)rp + o;
            if (o == 0 || q < tile.z || q >= tile.w || q >= a.np || a.compS[q] == rc) continue;
            const float4* src = reinterpret_cast<const float4*>(a.xs + q * DMAX);
            float sq = 0.f;
#pragma unroll
            for (int f4 = 0; f4 < F4; ++f4) {
                const float4 y = src[f4];
                const float d0 = xr[4 * f4 + 0] - y.x, d1 = xr[4 * f4 + 1] - y.y;
                const float d2 = xr[4 * f4 + 2] - y.z, d3 = xr[4 * f4 + 3] - y.w;
                sq = acc_term<M>(sq, d0);
                sq = acc_term<M>(sq, d1);
                sq = acc_term<M>(sq, d2);
                sq = acc_term<M>(sq, d3);
            }
            const float ub = __builtin_fmaf(sq, (float)(a.d + 6) * 0x1p-24f, sq) + 0x1p-126f;
            if (ub < tk[k - 1]) {
                int p = k - 1;
                while (p > 0 && tk[p - 1] > ub) { tk[p] = tk[p - 1]; --p; }
                tk[p] = ub;
            }
        }
        if (tk[k - 1] < __builtin_huge_valf()) {
            U = tk[k - 1];
            T = fminf(T, fp32_thresh_from_U((double)U, crel, a0));
        }
        for (int e = 0; e < k; ++e) tk[e] = __builtin_huge_valf();
    }
    int cnt = 0;                         // survivors (rows not shared by splits)
    if (a.prune) tile_ball<DP>(sh, xr, valid, a.d);
    if (tid == 0) {
        const int64_t last = (int64_t)tile.y - 1;
        const int64_t first = tile.x;
        sh.col_lo = tile.z;
        sh.col_hi = tile.w;
        const int r0 = a.rows ? a.rows[first] : a.row0 + (int)first;
        sh.lo = a.compS[r0];
        sh.hi = a.compS[a.rows ? a.rows[last] : a.row0 + (int)last];
        sh.rows = (int)(last - first + 1);
        sh.first_pos = r0;
    }
    __syncthreads();
    const int lo_r = sh.lo, hi_r = sh.hi;

    unsigned long long pairs = 0;
    wave_max_store(sh, valid ? prune_bound<M>(U, a.d) : 0.f);
    __syncthreads();
    const float umax0 = fmaxf(fmaxf(sh.wmax[0], sh.wmax[1]), fmaxf(sh.wmax[2], sh.wmax[3]));

    sweep_chunks<TAB>(sh, a, it, lo_r, hi_r, umax0, [&](int ci, int lo_c, int hi_c) {
        // a chunk made only of the row's own component holds no candidate
        const bool own = lo_c == hi_c && lo_c == rc;
        const int64_t c0 = chunk_begin<TAB>(a, ci);
        const int ncols = (int)(chunk_end<TAB>(a, ci) - c0);
        const int cl = sh.col_lo, ch = sh.col_hi;
        if (share && valid) {
            T = fminf(T, __uint_as_float(a.gT[slot]));
            U = fminf(U, __uint_as_float(a.gU[slot]));
        }

        // per-row ball test: a wave whose rows are all farther from the
        // chunk's ball than their bounds skips the chunk; if every wave
        // does, so does the workgroup
        {
            bool need = valid && !own;
            if (a.prune && need) {
                float4 x4[F4];
#pragma unroll
                for (int q = 0; q < F4; ++q) x4[q] = make_float4(xr[4 * q], xr[4 * q + 1], xr[4 * q + 2], xr[4 * q + 3]);
                need = point_ball_lb2(x4, a.balls + (int64_t)ci * BALL_STRIDE) <= prune_bound<M>(U, a.d);
            }
            const unsigned long long b = __ballot(need);
            if ((tid & 63) == 0) sh.wneed[tid >> 6] = b != 0ull;
        }
        __syncthreads();
        if (!(sh.wneed[0] | sh.wneed[1] | sh.wneed[2] | sh.wneed[3])) return;
        const bool wrun = sh.wneed[tid >> 6] != 0;
        for (int idx = tid; idx < BN * F4; idx += 256) {
            const int c = idx / F4, q = idx % F4;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < ncols) v = reinterpret_cast<const float4*>(a.xs + (c0 + c) * DMAX)[q];
            cbuf[idx] = v;
        }
        ccomp[tid] = (tid < ncols && c0 + tid >= cl && c0 + tid < ch) ? a.compS[c0 + tid] : -1;
        __syncthreads();
        if (!wrun) {
            wave_max_store(sh, valid ? prune_bound<M>(U, a.d) : 0.f);
            return;
        }
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
                t = acc_term<M>(t, d0);
                t = acc_term<M>(t, d1);
                t = acc_term<M>(t, d2);
                t = acc_term<M>(t, d3);
            }
            if (t <= T && !own) {
                // same component, or a column this tile must not pair with
                const int cc = ccomp[c];
                if (cc < 0 || cc == rc) continue;
                const int pos = share ? atomicAdd(&a.surv_cnt[slot], 1) : cnt++;
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
                        const double Ud = fp32_upper_from_t((double)kth, crel, a0);
                        const float Tn = fp32_thresh_from_U(Ud, crel, a0);
                        const float Un = d2f_up(Ud);
                        if (Tn < T) {
                            T = Tn;
                            if (share) atomicMin(&a.gT[slot], __float_as_uint(T));
                        }
                        if (Un < U) {
                            U = Un;
                            if (share) atomicMin(&a.gU[slot], __float_as_uint(U));
                        }
                    }
                }
            }
        }
        wave_max_store(sh, valid ? prune_bound<M>(U, a.d) : 0.f);
    });
    if (!share && valid) a.surv_cnt[slot] = cnt;
    const int wrows = sh.rows - (tid >> 6) * 64;
    if ((tid & 63) == 0 && a.pairs && wrows > 0)
        atomicAdd(&a.pairs[((blockIdx.x * 4 + (tid >> 6)) & (NSPREAD - 1)) * SPREAD_STRIDE],
                  pairs * (unsigned long long)(wrows < 64 ? wrows : 64));
}

template <int DP, bool TAB, int M>
__global__ __launch_bounds__(256, 2) void k_cand_fp32(CandArgs a)
{
    cand_fp32_item<DP, TAB, M>(a, grid_item(a), a.share != 0);
}

// device-sized launch: a fixed grid pops (tile, split) items
template <int DP, int M>
__global__ __launch_bounds__(256, 2) void k_cand_fp32_q(CandArgs a)
{
    __shared__ int slot;
    Item it;
    while (pop_item(a, slot, it)) cand_fp32_item<DP, false, M>(a, it, it.nsp > 1);
}

template <int DP>
void launch_q(const CandArgs& a, size_t shm, hipStream_t s)
{
    switch (a.metric) {
    case NNM_METRIC_L1: k_cand_fp32_q<DP, NNM_METRIC_L1><<<QGRID, 256, shm, s>>>(a); break;
    case NNM_METRIC_LINF: k_cand_fp32_q<DP, NNM_METRIC_LINF><<<QGRID, 256, shm, s>>>(a); break;
    default: k_cand_fp32_q<DP, NNM_METRIC_EUCLIDEAN><<<QGRID, 256, shm, s>>>(a); break;
    }
}

template <int DP, bool TAB>
void launch_m(const CandArgs& a, dim3 grid, size_t shm, hipStream_t s)
{
    switch (a.metric) {
    case NNM_METRIC_L1: k_cand_fp32<DP, TAB, NNM_METRIC_L1><<<grid, 256, shm, s>>>(a); break;
    case NNM_METRIC_LINF: k_cand_fp32<DP, TAB, NNM_METRIC_LINF><<<grid, 256, shm, s>>>(a); break;
    default: k_cand_fp32<DP, TAB, NNM_METRIC_EUCLIDEAN><<<grid, 256, shm, s>>>(a); break;
    }
}

hipError_t launch_dp_q(const CandArgs& a, int dp, size_t shm, hipStream_t s)
{
    switch (dp) {
    case 4: launch_q<4>(a, shm, s); break;
    case 8: launch_q<8>(a, shm, s); break;
    case 12: launch_q<12>(a, shm, s); break;
    case 16: launch_q<16>(a, shm, s); break;
    case 20: launch_q<20>(a, shm, s); break;
    case 24: launch_q<24>(a, shm, s); break;
    case 28: launch_q<28>(a, shm, s); break;
    case 32: launch_q<32>(a, shm, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool TAB>
hipError_t launch_dp(const CandArgs& a, int dp, dim3 grid, size_t shm, hipStream_t s)
{
    switch (dp) {
    case 4: launch_m<4, TAB>(a, grid, shm, s); break;
    case 8: launch_m<8, TAB>(a, grid, shm, s); break;
    case 12: launch_m<12, TAB>(a, grid, shm, s); break;
    case 16: launch_m<16, TAB>(a, grid, shm, s); break;
    case 20: launch_m<20, TAB>(a, grid, shm, s); break;
    case 24: launch_m<24, TAB>(a, grid, shm, s); break;
    case 28: launch_m<28, TAB>(a, grid, shm, s); break;
    case 32: launch_m<32, TAB>(a, grid, shm, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cand_fp32(const CandArgs& a, hipStream_t s)
{
    if (a.desc) {
        if (a.cstart) return hipErrorInvalidValue;   // device-sized launches use fixed chunks
        return launch_dp_q(a, (a.d + 3) / 4 * 4, (size_t)BM * a.k * sizeof(float), s);
    }
    if (a.n_rows <= 0) return hipSuccess;
    const unsigned nt = a.tiles ? (unsigned)a.n_tiles : (unsigned)((a.n_rows + BM - 1) / BM);
    if (nt == 0) return hipSuccess;
    dim3 grid(nt, (unsigned)a.col_splits);
    size_t shm = (size_t)BM * a.k * sizeof(float);
    const int dp = (a.d + 3) / 4 * 4;
    if (a.cstart) return launch_dp<true>(a, dp, grid, shm, s);
    return launch_dp<false>(a, dp, grid, shm, s);
}

}  // namespace nnm
