// cand_mfma.hip -- the candidate pass on the matrix cores (gfx950).
//
// This is the hot loop of the method: distances between all pairs of points
// (section "Overall idea of the algorithm", item two) fused with the
// selection of the minimal ones (item three, and the per-portion selection of
// the section on constructing the set of minimum distances).  The pair space
// is the product of two blocks of the data -- a row tile held in registers
// and column chunks streamed through LDS -- including the diagonal tiles;
// self pairs and pairs inside one component are masked out.
//
// For row i and column j the kernel evaluates the low-precision candidate
//     t_ij = ||q_i||^2 + ||q_j||^2 - 2 q_i . q_j        (scaled by sigma^2)
// as one v_mfma_f32_16x16x32_{bf16,f16,fp8} per 16x16 block: features occupy
// K slots 0..D-1, the two squared norms ride in slots 26..31 as
// (value, constant) pairs, so the FP32 accumulator is t itself.
//
// Selection.  Each row keeps, in LDS, the k smallest t it has seen; from the
// k-th of them the proven error bound gives (1) U_i, an upper bound on the
// exact key of the row's k-th nearest column, and (2) a threshold T_i such
// that every column whose exact key is <= U_i has t <= T_i.  Every column
// with t <= T_i is appended to the row's survivor list (global memory) for
// exact FP64 rescoring.  The per-element work is one min3 chain and one
// compare per eight pairs; hits take a wave-uniform slow path, which also
// applies the component mask.
//
// Search order and pruning.  Points are stored in a spatial order, so the
// chunks are visited nearest-first starting at the tile's own position, and
// a chunk is skipped when the distance between the tile's bounding ball and
// the chunk's bounding ball already exceeds every row's U_i.
//
// MFMA layouts used (16x16x32): lane l supplies A[m = l%16][k-slice l/16]
// and B[k-slice l/16][n = l%16]; result register r of lane l is
// D[m = 4(l/16) + r][n = l%16].  Columns j are the A (M) side, rows i the
// B (N) side, so each lane ends up with four columns of one row.
#include "cand_common.h"

namespace nnm {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int WAVES = 4;
constexpr int RB = 4;                 // 16-row blocks per wave
constexpr int BM = WAVES * RB * 16;   // rows per workgroup (= threads)
constexpr int BN = CHUNK;             // columns per LDS chunk
constexpr float KFAC = 1.0f + 0x1p-20f;

template <int OP> struct OpTraits;
template <> struct OpTraits<OP_BF16> {
    typedef uint4 frag_t;             // 8 x bf16 per lane
    static constexpr int BYTES = 64;
    __device__ static f32x4_t mma(uint4 a, uint4 b) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                      __builtin_bit_cast(bf16x8_t, b),
                                                      f32x4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
};
template <> struct OpTraits<OP_FP16> {
    typedef uint4 frag_t;             // 8 x f16 per lane
    static constexpr int BYTES = 64;
    __device__ static f32x4_t mma(uint4 a, uint4 b) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a),
                                                     __builtin_bit_cast(f16x8_t, b),
                                                     f32x4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
};
template <> struct OpTraits<OP_FP8> {
    typedef uint2 frag_t;             // 8 x e4m3 per lane
    static constexpr int BYTES = 32;
    __device__ static f32x4_t mma(uint2 a, uint2 b) {
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a),
                                                         __builtin_bit_cast(long, b),
                                                         f32x4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
};

// Largest candidate value that can still belong to a column whose exact key
// is <= U (scaled units), for a row with accumulation slack eps and
// quantisation slack eta (both already combined with the column maxima).
// With E(t) = KFAC * (eps + eta * (2 sqrt(t + eps) + eta)) bounding |t - s|,
// t - E(t) <= U  iff  sqrt(t + eps) <= W, W = KFAC eta + sqrt(...).
__device__ __forceinline__ float thresh_from_U(double U, double eps, double eta, int exact)
{
    if (exact) return d2f_up(U);
    const double kf = (double)KFAC;
    double W = kf * eta + __builtin_sqrt(kf * kf * eta * eta + U + eps * (1.0 + kf) + kf * eta * eta);
    double T = (W * W - eps) * (1.0 + 0x1p-40) + 0x1p-1000;
    return d2f_up(T);
}

// Upper bound on the exact (scaled) key of a column whose candidate is t.
__device__ __forceinline__ double upper_from_t(double t, double eps, double eta, int exact)
{
    if (exact) return t;
    const double kf = (double)KFAC;
    double tp = t > 0.0 ? t : 0.0;
    return (t + kf * (eps + eta * (2.0 * __builtin_sqrt(tp + eps) + eta))) * (1.0 + 0x1p-40);
}

template <int OP>
__global__ __launch_bounds__(256, 3) void k_cand_mfma(CandArgs a)
{
    typedef OpTraits<OP> Tr;
    typedef typename Tr::frag_t frag_t;
    constexpr int LOADS = BN * Tr::BYTES / 16 / 256;       // uint4 loads per thread

    __shared__ frag_t colbuf[BN / 16 * 4 * 16];
    __shared__ __align__(16) int32_t colcomp[BN];
    __shared__ float rowT[BM], rowU[BM];
    __shared__ double rowEps[BM], rowEta[BM];
    __shared__ TileShared sh;
    extern __shared__ float topk[];                        // [BM][k]

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int grp = lane >> 4;
    const int k = a.k;
    const int4 tile = tile_of(a, BM);
    const int64_t row_base = tile.x;
    const int64_t row_end = tile.y;
    const int exact = a.bc.exact;
    const double inv_s2 = 1.0 / (double)a.bc.sigma2;

    // ---- per-row state (thread t owns row t of the tile) -----------------
    const int64_t my_slot = row_base + tid;
    const bool my_valid = my_slot < row_end;
    const int my_rp = my_valid ? (a.rows ? a.rows[my_slot] : a.row0 + (int)my_slot) : 0;
    {
        float T = -__builtin_huge_valf(), U = 0.f;
        double eps = 0.0, eta = 0.0;
        if (my_valid) {
            const PointConst p = a.pc[my_rp];
            eps = ((double)a.bc.gamma * (2.0 * (double)p.Q * (double)a.bc.colQ + (double)p.P +
                                         (double)a.bc.colP) +
                   (double)p.rho + (double)a.bc.colRho) * (1.0 + 0x1p-40);
            eta = ((double)p.eta + (double)a.bc.colEta) * (1.0 + 0x1p-40);
            T = 3.402823466e38f;                           // FLT_MAX: keep all
            U = __builtin_huge_valf();
            if (a.u0) {
                const double u0 = a.u0[my_rp];
                if (u0 >= 0.0) {
                    T = fminf(T, thresh_from_U(u0 * (double)a.bc.sigma2 * (1.0 + 0x1p-50), eps, eta, exact));
                    U = d2f_up(u0);
                }
            }
        }
        rowT[tid] = T;
        rowU[tid] = U;
        rowEps[tid] = eps;
        rowEta[tid] = eta;
        for (int e = 0; e < k; ++e) topk[tid * k + e] = __builtin_huge_valf();
    }
    if (a.prune) {
        float x[DMAX];
        const float* src = a.X + (int64_t)(my_valid ? a.perm[my_rp] : 0) * a.ld;
#pragma unroll
        for (int f = 0; f < DMAX; ++f) x[f] = (f < a.d && my_valid) ? src[f] : 0.f;
        tile_ball<DMAX>(sh, x, my_valid, a.d);
    }
    if (tid == 0) {
        const int64_t last = row_end - 1;
        const int r0 = a.rows ? a.rows[row_base] : a.row0 + (int)row_base;
        const int r1 = a.rows ? a.rows[last] : a.row0 + (int)last;
        sh.lo = a.compS[r0];
        sh.hi = a.compS[r1];
        sh.rows = (int)(last - row_base + 1);
        sh.first_pos = r0;
        sh.col_lo = tile.z;
        sh.col_hi = tile.w;
    }
    // row fragments stay in registers for the whole sweep
    frag_t bfrag[RB];
    int32_t rcomp[RB];
    bool rvalid[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int rl = wave * RB * 16 + rb * 16 + (lane & 15);
        const int64_t slot = row_base + rl;
        rvalid[rb] = slot < row_end;
        const int rp = rvalid[rb] ? (a.rows ? a.rows[slot] : a.row0 + (int)slot) : 0;
        const frag_t* src = reinterpret_cast<const frag_t*>(a.opR) + (int64_t)rp * 4 + grp;
        bfrag[rb] = *src;
        rcomp[rb] = rvalid[rb] ? a.compS[rp] : -2;
    }
    __syncthreads();
    float Treg[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) Treg[rb] = rowT[wave * RB * 16 + rb * 16 + (lane & 15)];
    const int lo_r = sh.lo, hi_r = sh.hi;

    // ---- column sweep, nearest chunks first ------------------------------
    unsigned long long pairs = 0;
    wave_max_store(sh, my_valid ? rowU[tid] : 0.f);
    __syncthreads();
    const float umax0 = fmaxf(fmaxf(sh.wmax[0], sh.wmax[1]), fmaxf(sh.wmax[2], sh.wmax[3]));

    sweep_chunks(sh, a, lo_r, hi_r, umax0, [&](int ci, int lo_c, int hi_c) {
        const int64_t c0 = (int64_t)ci * BN;
        const int ncols = (int)((a.np - c0) < BN ? (a.np - c0) : BN);
        const int cl = sh.col_lo, ch = sh.col_hi;
        if (a.share && my_valid) {
            rowT[tid] = fminf(rowT[tid], __uint_as_float(a.gT[my_slot]));
            rowU[tid] = fminf(rowU[tid], __uint_as_float(a.gU[my_slot]));
        }
        __syncthreads();
        // stage the column chunk into LDS in fragment order
        const uint4* gsrc = reinterpret_cast<const uint4*>(a.opC) + c0 * (Tr::BYTES / 16);
#pragma unroll
        for (int it = 0; it < LOADS; ++it) {
            const int idx = it * 256 + tid;
            if constexpr (Tr::BYTES == 64) {
                const int c = idx >> 2, q = idx & 3;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (c < ncols) v = gsrc[idx];
                reinterpret_cast<uint4*>(colbuf)[((c >> 4) * 4 + q) * 16 + (c & 15)] = v;
            } else {
                const int c = idx >> 1, h = idx & 1;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (c < ncols) v = gsrc[idx];
                uint2* cb2 = reinterpret_cast<uint2*>(colbuf);
                cb2[((c >> 4) * 4 + 2 * h) * 16 + (c & 15)] = make_uint2(v.x, v.y);
                cb2[((c >> 4) * 4 + 2 * h + 1) * 16 + (c & 15)] = make_uint2(v.z, v.w);
            }
        }
        colcomp[tid] = (tid < ncols && c0 + tid >= cl && c0 + tid < ch) ? a.compS[c0 + tid] : -1;
        __syncthreads();
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) Treg[rb] = rowT[wave * RB * 16 + rb * 16 + (lane & 15)];
        pairs += (unsigned long long)ncols;

        const int nblk = (ncols + 15) >> 4;
        // slow path for one 16-column block: one lane group at a time so the
        // 4 lanes of a row never touch its LDS state together
        auto slow = [&](int cb, const f32x4_t (&acc)[RB]) {
            for (int g = 0; g < 4; ++g) {
                if (grp == g) {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        if (!rvalid[rb]) continue;
                        const int rl = wave * RB * 16 + rb * 16 + (lane & 15);
                        const int64_t slot = row_base + rl;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float v = acc[rb][r];
                            if (!(v <= rowT[rl])) continue;
                            // same component, or a column this tile must not pair with
                            const int cc = colcomp[cb * 16 + 4 * g + r];
                            if (cc < 0 || cc == rcomp[rb]) continue;
                            const int col = (int)(c0 + cb * 16 + 4 * g + r);
                            const int pos = atomicAdd(&a.surv_cnt[slot], 1);
                            if (pos < a.S) {
                                a.surv_j[slot * a.S + pos] = col;
                                a.surv_t[slot * a.S + pos] = v;
                            }
                            float* tk = topk + rl * k;
                            if (v < tk[k - 1]) {
                                int p = k - 1;
                                while (p > 0 && tk[p - 1] > v) { tk[p] = tk[p - 1]; --p; }
                                tk[p] = v;
                                const float kth = tk[k - 1];
                                if (kth < __builtin_huge_valf()) {
                                    const double U = upper_from_t((double)kth, rowEps[rl], rowEta[rl], exact);
                                    const float T = thresh_from_U(U, rowEps[rl], rowEta[rl], exact);
                                    const float Us = d2f_up(exact ? U : U * inv_s2 * (1.0 + 0x1p-40));
                                    if (T < rowT[rl]) {
                                        rowT[rl] = T;
                                        if (a.share) atomicMin(&a.gT[slot], __float_as_uint(T));
                                    }
                                    if (Us < rowU[rl]) {
                                        rowU[rl] = Us;
                                        if (a.share) atomicMin(&a.gU[slot], __float_as_uint(Us));
                                    }
                                }
                            }
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
        };
        auto reload_T = [&]() {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) Treg[rb] = rowT[wave * RB * 16 + rb * 16 + (lane & 15)];
        };
        // two 16-column blocks per step: 8 MFMAs, then one min3 chain and
        // one compare per row block for 8 candidates.  The component mask is
        // applied in the slow path only: masked columns (same component,
        // outside the tile's column range) are rare and merely cause a
        // detour there.
        int cb = 0;
        for (; cb + 1 < nblk; cb += 2) {
            const frag_t af0 = colbuf[(cb * 4 + grp) * 16 + (lane & 15)];
            const frag_t af1 = colbuf[((cb + 1) * 4 + grp) * 16 + (lane & 15)];
            f32x4_t acc0[RB], acc1[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc0[rb] = Tr::mma(af0, bfrag[rb]);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc1[rb] = Tr::mma(af1, bfrag[rb]);
            bool hit = false;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                float m = fminf(fminf(acc0[rb][0], acc0[rb][1]), acc0[rb][2]);
                m = fminf(fminf(m, acc0[rb][3]), acc1[rb][0]);
                m = fminf(fminf(m, acc1[rb][1]), acc1[rb][2]);
                m = fminf(m, acc1[rb][3]);
                hit |= (m <= Treg[rb]);
            }
            if (__ballot(hit)) {
                slow(cb, acc0);
                slow(cb + 1, acc1);
                reload_T();
            }
        }
        if (cb < nblk) {
            const frag_t af = colbuf[(cb * 4 + grp) * 16 + (lane & 15)];
            f32x4_t acc[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[rb] = Tr::mma(af, bfrag[rb]);
            bool hit = false;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const float m = fminf(fminf(acc[rb][0], acc[rb][1]), fminf(acc[rb][2], acc[rb][3]));
                hit |= (m <= Treg[rb]);
            }
            if (__ballot(hit)) {
                slow(cb, acc);
                reload_T();
            }
        }
        wave_max_store(sh, my_valid ? rowU[tid] : 0.f);
    });
    if (tid == 0 && a.pairs) atomicAdd(a.pairs, pairs * (unsigned long long)sh.rows);
}

}  // namespace

hipError_t launch_cand_mfma(int opkind, const CandArgs& a, hipStream_t s)
{
    if (a.n_rows <= 0) return hipSuccess;
    const unsigned nt = a.tiles ? (unsigned)a.n_tiles : (unsigned)((a.n_rows + BM - 1) / BM);
    if (nt == 0) return hipSuccess;
    dim3 grid(nt, (unsigned)a.col_splits);
    size_t shm = (size_t)BM * a.k * sizeof(float);
    switch (opkind) {
    case OP_BF16: k_cand_mfma<OP_BF16><<<grid, 256, shm, s>>>(a); break;
    case OP_FP16: k_cand_mfma<OP_FP16><<<grid, 256, shm, s>>>(a); break;
    case OP_FP8: k_cand_mfma<OP_FP8><<<grid, 256, shm, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nnm
