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
// Frame.  FP16 on general data, and exact integer data (FP8, or BF16/FP16 on
// integer grids), use precomputed operands in one global frame.  BF16 on
// general data (8 significant bits) uses two frames per pair: the column
// operands are built once per round in the frame of their own super-chunk
// (k_split_columns, centre c_S = the super-chunk's ball centre), and the
// rows once per tile in the frame of the tile's centre c_T, as a sum of two
// BF16 values (a = ah + al, both multiplied in by two chained MFMAs).  The
// frames meet through delta = sigma (c_T - c_S): the rows' norm slots carry
// ||a + delta||^2 (rewritten when a wave moves to another super-chunk) and
// the columns' ||p||^2 - 2 delta.p (rewritten when staged).  The column
// error then scales with the super-chunk's radius and the row error is
// ~2^-16 of the row's offset from its tile's centre.
//
// Selection.  For every column that reaches the slow path the proven error
// bound gives an upper bound on its exact key; each row keeps, in LDS, the k
// smallest such bounds, whose k-th is U_i >= the row's k-th smallest key.  Per
// chunk the bound also gives a threshold T_i such that every column of the
// chunk whose exact key is <= U_i has t <= T_i.  Every column with t <= T_i
// is appended to the row's survivor list (global memory) for exact FP64
// rescoring.  The per-element work is one min3 chain and one
// compare per eight pairs; hits take a wave-uniform slow path, which also
// applies the component mask.
//
// Search order and pruning.  Points are stored in a spatial order, so the
// chunks are visited nearest-first starting at the tile's own position, a
// group of candidate chunks at a time: a chunk is a candidate unless the
// distance between the tile's bounding ball and the chunk's already exceeds
// every row's U_i; each row then tests its own distance to every
// candidate's ball against its U_i, and only the chunks some wave's rows
// need are staged and evaluated -- by the waves that need them.
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
constexpr int SEEDW = 32;             // seeding window: sweep-order neighbours on each side
constexpr int NQR = (DMAX_MFMA + 3) / 4;   // float4s of a row's coordinates

template <int OP> struct OpTraits;
template <> struct OpTraits<OP_BF16> {
    typedef uint4 frag_t;             // 8 x bf16 per lane
    static constexpr int BYTES = 64;
    __device__ static f32x4_t mma(uint4 a, uint4 b) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                      __builtin_bit_cast(bf16x8_t, b),
                                                      f32x4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
    __device__ static f32x4_t mma_acc(uint4 a, uint4 b, f32x4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                      __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
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
    __device__ static f32x4_t mma_acc(uint4, uint4, f32x4_t c) { return c; }   // not used
};
template <> struct OpTraits<OP_FP8> {
    typedef uint2 frag_t;             // 8 x e4m3 per lane
    static constexpr int BYTES = 32;
    __device__ static f32x4_t mma(uint2 a, uint2 b) {
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a),
                                                         __builtin_bit_cast(long, b),
                                                         f32x4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
    __device__ static f32x4_t mma_acc(uint2, uint2, f32x4_t c) { return c; }   // not used
};

// Upper bound, in FP32, on the exact key of a pair whose FP32 direct-difference
// sum of squares over d features is s (relative error below (d + 2) 2^-24,
// plus subnormal flushes far below 2^-126).
__device__ __forceinline__ float fp32_key_upper(float s, int d)
{
    return __builtin_fmaf(s, (float)(d + 6) * 0x1p-24f, s) + 0x1p-126f;
}

// Element e = b * 16 + rb * 4 + r of the pair of accumulator sets, by a tree
// of selects (no dynamic register indexing).
__device__ __forceinline__ float pick32(const f32x4_t (&a0)[RB], const f32x4_t (&a1)[RB], int e)
{
    f32x4_t q[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) q[rb] = (e & 16) ? a1[rb] : a0[rb];
    const f32x4_t h0 = (e & 4) ? q[1] : q[0];
    const f32x4_t h1 = (e & 4) ? q[3] : q[2];
    const f32x4_t w = (e & 8) ? h1 : h0;
    const float lo = (e & 1) ? w[1] : w[0];
    const float hi = (e & 1) ? w[3] : w[2];
    return (e & 2) ? hi : lo;
}

// Candidate chunks of the sweep, a group at a time.  The super-chunks of the
// workgroup's column range are visited nearest-first (zigzag around the
// tile's own) and tested 64 at a time against the tile ball, one lane each;
// a group takes the next GS passing super-chunks and wave w expands the
// w-th: its (at most SUPER) chunks are tested against the tile ball, four
// lanes per chunk (a quarter of the features each), all loads of the group
// issued together.  Each chunk's ball, position range and component range
// go to candidate slot SUPER w + step in LDS, flagged (bit 4 of gneed) when
// the chunk passed.  Every wave runs the super-chunk part identically, so
// all take the same decisions.
constexpr int GS = 4;                 // super-chunks per group (one per wave)
constexpr int GW = GS * SUPER;        // candidate slots per group
static_assert(GW == 64 && DMAX == 32, "one lane per slot; 4 lanes x 8 features per chunk");

template <bool TAB>
struct GroupGen {
    int ch_lo, ch_hi, start;         // chunk range of this split; the tile's own chunk
    int sc_lo, sc_hi, sc_start;      // super-chunk range; the tile's own super-chunk
    int ss;                          // next super-chunk step
    int sbase;                       // steps [sbase, sbase + 64) tested into smask
    unsigned long long smask;

    __device__ void init(const TileShared& sh, const CandArgs& a, const Item& it)
    {
        const int first_ch = chunk_first_of<TAB>(a, sh.col_lo);
        const int nch = chunk_end_of<TAB>(a, sh.col_hi) - first_ch;
        const int cps = (nch + it.nsp - 1) / it.nsp;
        ch_lo = first_ch + it.sp * cps;
        ch_hi = ch_lo + cps < first_ch + nch ? ch_lo + cps : first_ch + nch;
        if (ch_lo < ch_hi) {
            start = chunk_at<TAB>(a, sh.first_pos);
            start = start < ch_lo ? ch_lo : (start >= ch_hi ? ch_hi - 1 : start);
            sc_lo = super_of<TAB>(a, ch_lo);
            sc_hi = super_of<TAB>(a, ch_hi - 1) + 1;
            sc_start = super_of<TAB>(a, start);
        } else {
            start = ch_lo;
            sc_lo = sc_hi = sc_start = 0;    // nothing to visit
        }
        ss = 0;
        sbase = -64;
        smask = 0ull;
    }

    // The next (at most GS) super-chunks that pass the tile-level test
    // against the bound umax, into scl; returns how many.
    __device__ int take(const TileShared& sh, const CandArgs& a, int lo_r, int hi_r, float umax,
                        int (&scl)[GS])
    {
        const int lane = threadIdx.x & 63;
        const int nsc = sc_hi - sc_lo;
        int g = 0;
        while (g < GS && ss < nsc) {
            if (ss >= sbase + 64) {
                sbase = ss;
                const int step = ss + lane;
                bool pass = false;
                if (step < nsc) {
                    const int sc = zigzag(step, sc_start, sc_lo, sc_hi);
                    // a super-chunk entirely inside the tile's only component
                    bool own;
                    if constexpr (TAB) {
                        own = lo_r == hi_r && a.scomp[sc] == lo_r;
                    } else {
                        const int64_t s0 = (int64_t)sc * SUPER * CHUNK;
                        const int64_t s1 = chunk_end<TAB>(a, super_end<TAB>(a, sc) - 1) - 1;
                        own = lo_r == hi_r && a.compS[s0] == lo_r && a.compS[s1] == lo_r;
                    }
                    const float lb = a.prune ? ball_lb2(sh, a.sballs + (int64_t)sc * BALL_STRIDE) : 0.f;
                    pass = !own && lb <= umax;
                }
                smask = __ballot(pass);
            }
            const unsigned long long m = smask >> (ss - sbase);
            if (m == 0ull) {
                ss = sbase + 64;
                continue;
            }
            const int off = ss - sbase + (int)__builtin_ctzll(m);
            scl[g++] = zigzag(sbase + off, sc_start, sc_lo, sc_hi);
            ss = sbase + off + 1;
        }
        return g;
    }

    // Wave w expands super-chunk sc (-1: none) into slots [SUPER w, SUPER w + SUPER);
    // with gcm (super-chunk frames) also each chunk's column maxima of the
    // bound inputs, and the super-chunk itself into gsc[w].
    __device__ void expand(const TileShared& sh, const CandArgs& a, int lo_r, int hi_r, float umax,
                           int sc, int w, float (*gball)[BALL_STRIDE], int4* gpos, int32_t* gneed,
                           float4* gcm, int32_t* gsc)
    {
        const int lane = threadIdx.x & 63, step = lane & 15, part = lane >> 4;
        const int slot = SUPER * w + step;
        if (sc < 0) {
            if (part == 0) gneed[slot] = 0;
            return;
        }
        const int sf = super_first<TAB>(a, sc), se = super_end<TAB>(a, sc);
        const int lo = sf > ch_lo ? sf : ch_lo;
        const int hi = se < ch_hi ? se : ch_hi;
        const int first = (sc == sc_start) ? start : (sc > sc_start ? lo : hi - 1);
        const int nc = hi - lo;
        // steps past the end read the first chunk again; they are not candidates
        const int ci = zigzag(step < nc ? step : 0, first, lo, hi);
        const int64_t c0 = chunk_begin<TAB>(a, ci);
        const int64_t c1 = chunk_end<TAB>(a, ci);
        int clo, chi;
        if constexpr (TAB) {
            clo = chi = a.ccomp[ci];    // one component per chunk; no wait on c0
        } else {
            clo = a.compS[c0];
            chi = a.compS[c1 - 1];
        }
        const float* b = a.balls + (int64_t)ci * BALL_STRIDE;
        const float4 q0 = *reinterpret_cast<const float4*>(b + 8 * part);
        const float4 q1 = *reinterpret_cast<const float4*>(b + 8 * part + 4);
        const float rad = b[DMAX];
        // tile ball vs chunk ball: quarter sums of squares added across the
        // four lanes of a chunk (at most 12 roundings, within ball_lb2's margins)
        const float4* c4 = reinterpret_cast<const float4*>(sh.cen) + 2 * part;
        const float4 t0 = c4[0], t1 = c4[1];
        float s = 0.f;
        {
            const float d0 = t0.x - q0.x, d1 = t0.y - q0.y, d2 = t0.z - q0.z, d3 = t0.w - q0.w;
            const float e0 = t1.x - q1.x, e1 = t1.y - q1.y, e2 = t1.z - q1.z, e3 = t1.w - q1.w;
            s = __builtin_fmaf(d0, d0, s);
            s = __builtin_fmaf(d1, d1, s);
            s = __builtin_fmaf(d2, d2, s);
            s = __builtin_fmaf(d3, d3, s);
            s = __builtin_fmaf(e0, e0, s);
            s = __builtin_fmaf(e1, e1, s);
            s = __builtin_fmaf(e2, e2, s);
            s = __builtin_fmaf(e3, e3, s);
        }
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        const float lb = __builtin_sqrtf(s) * (1.0f - 0x1p-18f) - sh.rball - rad;
        const float lb2 = lb > 0.f ? lb * lb * (1.0f - 0x1p-20f) : 0.f;
        const bool pass = step < nc && !(lo_r == hi_r && clo == chi && lo_r == clo) &&
                          (!a.prune || lb2 <= umax);
        float4* gb = reinterpret_cast<float4*>(&gball[slot][8 * part]);
        gb[0] = q0;
        gb[1] = q1;
        if (part == 0) {
            gball[slot][DMAX] = rad;
            gpos[slot] = make_int4((int)c0, (int)c1, clo, chi);
            gneed[slot] = pass ? 16 : 0;
            if (gcm) {
                gcm[slot] = a.cmaxT[ci];
                if (step == 0) gsc[w] = sc;
            }
        }
    }
};

// Operand format helpers for the local frame (BF16 / FP16).
template <int OP> struct LpFmt;
template <> struct LpFmt<OP_BF16> {
    __device__ static uint16_t to(float f) { return f32_to_bf16_rn(f); }
    __device__ static float from(uint16_t h) { return bf16_to_f32(h); }
    static constexpr double alpha = 0x1p-8 + 0x1p-22;
    static constexpr double beta = 0x1p-125;
    static constexpr uint32_t inf_bits = 0x7F80u;
};
template <> struct LpFmt<OP_FP16> {
    __device__ static uint16_t to(float f) { return f32_to_f16_rn(f); }
    __device__ static float from(uint16_t h) { return f16_to_f32(h); }
    static constexpr double alpha = 0x1p-11 + 0x1p-22;
    static constexpr double beta = 0x1p-25 + 0x1p-149;
    static constexpr uint32_t inf_bits = 0x7C00u;
};
// Operands of one point in the frame centred at c (FP32) and scaled by the
// power of two sigma: q = lowp(sigma (x - c)); row form [q, n1,n2,n3, 1,1,1],
// column form [-2q, 1,1,1, n1,n2,n3] where n1+n2+n3 carries ||q||^2; plus
// the inputs of the error bound (Q, P, rho, eta) rounded up.
template <int OP>
__device__ __forceinline__ void local_operands(const float* x, const float* c, float sigma, int d,
                                               uint4 (&row)[4], uint4 (&col)[4], PointConst& pc)
{
    typedef LpFmt<OP> F;
    uint32_t rw[KSLOT / 2], cw[KSLOT / 2];
    float nrm = 0.f, vn = 0.f;
#pragma unroll
    for (int f2 = 0; f2 < KSLOT / 2; ++f2) {
        uint32_t rpk = 0, cpk = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int f = 2 * f2 + h;
            if (f < DMAX_MFMA && f < d) {
                const float u = (x[f] - c[f]) * sigma;
                const uint16_t q = F::to(u);
                const float qv = F::from(q);
                nrm = __builtin_fmaf(qv, qv, nrm);
                vn = __builtin_fmaf(u, u, vn);
                rpk |= (uint32_t)q << (16 * h);
                cpk |= (uint32_t)F::to(-2.0f * qv) << (16 * h);
            }
        }
        rw[f2] = rpk;
        cw[f2] = cpk;
    }
    // three-part split of ||q||^2; every residual is exact in FP32
    float r = nrm, psum = 0.f;
    uint16_t part[NORM_PARTS];
#pragma unroll
    for (int k = 0; k < NORM_PARTS; ++k) {
        part[k] = F::to(r);
        const float pv = F::from(part[k]);
        psum += __builtin_fabsf(pv);
        r -= pv;
    }
    const uint16_t one = F::to(1.0f);
    // slots 26..28: parts (row) / ones (col); slots 29..31: ones (row) / parts (col)
    rw[13] = (uint32_t)part[0] | ((uint32_t)part[1] << 16);
    rw[14] = (uint32_t)part[2] | ((uint32_t)one << 16);
    rw[15] = (uint32_t)one | ((uint32_t)one << 16);
    cw[13] = (uint32_t)one | ((uint32_t)one << 16);
    cw[14] = (uint32_t)one | ((uint32_t)part[0] << 16);
    cw[15] = (uint32_t)part[1] | ((uint32_t)part[2] << 16);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        row[w] = make_uint4(rw[4 * w], rw[4 * w + 1], rw[4 * w + 2], rw[4 * w + 3]);
        col[w] = make_uint4(cw[4 * w], cw[4 * w + 1], cw[4 * w + 2], cw[4 * w + 3]);
    }
    const double up = 1.0 + 0x1p-18;
    pc.Q = d2f_up((double)__builtin_sqrtf(nrm) * up);
    pc.P = d2f_up((double)psum * up);
    pc.rho = d2f_up(((double)__builtin_fabsf(r) + (double)nrm * 27.0 * 0x1p-24) * up);
    pc.eta = d2f_up((F::alpha * (double)__builtin_sqrtf(vn) * up + F::beta * __builtin_sqrt((double)d)) * up);
}

// Column operands of the super-chunk frames (BF16 on general data), once
// per round after the chunk tables and balls: workgroup ci writes the columns
// of chunk ci in the frame of its super-chunk (centre: that super-chunk's
// ball centre) to opC, and the maxima of their bound inputs (Q, P, rho, eta)
// to cmax[ci].  TAB: component-aligned tables; workgroups past the chunk
// count exit.
template <bool TAB, int OP>
__global__ __launch_bounds__(256) void k_split_columns(const float* __restrict__ xs, int64_t np, int d,
                                                       float sigma, const int32_t* __restrict__ cstart,
                                                       const int32_t* __restrict__ csup,
                                                       const int32_t* __restrict__ tabn,
                                                       const float* __restrict__ sballs,
                                                       uint4* __restrict__ opC, float4* __restrict__ cmax)
{
    __shared__ float4 red[4];
    const int ci = (int)blockIdx.x;
    int64_t c0, c1;
    int sc;
    if constexpr (TAB) {
        if (ci >= tabn[0]) return;
        c0 = cstart[ci];
        c1 = cstart[ci + 1];
        sc = csup[ci];
    } else {
        c0 = (int64_t)ci * CHUNK;
        c1 = c0 + CHUNK < np ? c0 + CHUNK : np;
        sc = ci / SUPER;
    }
    const int64_t p = c0 + threadIdx.x;
    float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
    if (p < c1) {
        float y[DMAX];
        const float4* src = reinterpret_cast<const float4*>(xs + p * DMAX);
#pragma unroll
        for (int q = 0; q < DMAX / 4; ++q) {
            const float4 v = src[q];
            y[4 * q + 0] = v.x; y[4 * q + 1] = v.y; y[4 * q + 2] = v.z; y[4 * q + 3] = v.w;
        }
        uint4 row[4], col[4];
        PointConst pc;
        local_operands<OP>(y, sballs + (int64_t)sc * BALL_STRIDE, sigma, d, row, col, pc);
#pragma unroll
        for (int q = 0; q < 4; ++q) opC[p * 4 + q] = col[q];
        m = make_float4(pc.Q, pc.P, pc.rho, pc.eta);
    }
    for (int off = 32; off > 0; off >>= 1) {
        m.x = fmaxf(m.x, __shfl_xor(m.x, off));
        m.y = fmaxf(m.y, __shfl_xor(m.y, off));
        m.z = fmaxf(m.z, __shfl_xor(m.z, off));
        m.w = fmaxf(m.w, __shfl_xor(m.w, off));
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float4 r = red[0];
        for (int w = 1; w < 4; ++w) {
            r.x = fmaxf(r.x, red[w].x);
            r.y = fmaxf(r.y, red[w].y);
            r.z = fmaxf(r.z, red[w].z);
            r.w = fmaxf(r.w, red[w].w);
        }
        cmax[ci] = r;
    }
}

// LOCAL: BF16 on general data in the super-chunk frames (see the top of the
// file); otherwise the precomputed global operands are used.
//
// Per-row state in LDS (thread t owns row t of the tile; the slow path of
// the wave holding the row touches it one lane group at a time), packed so
// that the slow path reads it with two vector loads:
//   rs[r][0] = (T, U, eps, eta): threshold on t, bound on the row's k-th key
//              (data units), the row's slack for the current chunk;
//   rs[r][1] = (survivor count, component) as integer bits;
//   topk[r][0..KP): the k smallest candidates, +inf padded (t, or for LOCAL
//              upper bounds on keys in data units, since the frame changes
//              per chunk).  KP is k rounded up to 8 or 32.
// One work item: row tile it.t against column split it.sp of its tile's
// column range.
template <int OP, bool LOCAL, bool SHARE, int KP, bool TAB>
__device__ __forceinline__ void cand_mfma_item(const CandArgs& a, const Item& it)
{
    typedef OpTraits<OP> Tr;
    typedef typename Tr::frag_t frag_t;
    constexpr int PF = Tr::BYTES / 16;                     // uint4s of one column's operand

    __shared__ __align__(16) frag_t colbuf[2][BN / 16 * 4 * 16];  // two chunks: one in use, one filling
    __shared__ __align__(16) int32_t colcomp[2][BN];
    __shared__ float4 gcm[LOCAL ? GW : 1];                 // LOCAL: column maxima per candidate chunk
    __shared__ int32_t gsc[GS];                            // LOCAL: super-chunk of each wave's slots
    __shared__ float4 rpc[LOCAL ? BM : 1];                 // LOCAL: rows' (Q, ||a||^2, eta) in the tile frame
    __shared__ float2 rpf[LOCAL ? BM : 1];                 // LOCAL: rows' (P, rho) in the current column frame
    __shared__ __align__(16) float dlt[LOCAL ? GS : 1][DMAX + 4];   // LOCAL: each wave's offset delta, ||delta|| at [DMAX]
    __shared__ float4 rs[BM][2];                           // per-row state, see above
    __shared__ float wmx[4];                               // per-wave max of U
    __shared__ __align__(16) float wcen[4][DMAX];          // per-wave ball of the rows
    __shared__ float wrad[4];
    // the current group of candidate chunks (see GroupGen).  The balls have
    // their own LDS: placed over the chunk buffers (free while they are
    // read) the k = 16 and k = 32 lists came out different from run to run,
    // cause not found; apart, every run is identical.
    __shared__ __align__(16) float gball[GW][BALL_STRIDE];
    __shared__ int4 gpos[GW];                              // [b0, b1), component range
    __shared__ int32_t gneed[GW];                          // bit w: wave w needs it; bit 4: candidate
    __shared__ TileShared sh;
    extern __shared__ float4 topk4[];                      // [BM][KP / 4]
    float* topk = reinterpret_cast<float*>(topk4);

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int grp = lane >> 4;
    const int k = a.k;
    const int4 tile = tile_of(a, BM, it);
    const int64_t row_base = tile.x;
    const int64_t row_end = tile.y;
    const int exact = a.bc.exact;
    const float s2 = a.bc.sigma2;                          // sigma^2, a power of two
    const double inv_s2 = 1.0 / (double)s2;
    const float sigma = __builtin_sqrtf(s2);               // exact

    // ---- per-row state ---------------------------------------------------
    const int64_t my_slot = row_base + tid;
    const bool my_valid = my_slot < row_end;
    const int my_rp = my_valid ? (a.rows ? a.rows[my_slot] : a.row0 + (int)my_slot) : 0;
    const int my_comp = my_valid ? a.compS[my_rp] : -2;
    float x[DMAX];
    {
        const float4* src = reinterpret_cast<const float4*>(a.xs + (int64_t)my_rp * DMAX);
#pragma unroll
        for (int q = 0; q < DMAX / 4; ++q) {
            const float4 v = my_valid ? src[q] : make_float4(0.f, 0.f, 0.f, 0.f);
            x[4 * q + 0] = v.x; x[4 * q + 1] = v.y; x[4 * q + 2] = v.z; x[4 * q + 3] = v.w;
        }
    }
    // kept for the per-row ball tests (LOCAL: reloaded per group instead,
    // which keeps them out of the registers of the chunk evaluation)
    float4 xq[LOCAL ? 1 : NQR];
#pragma unroll
    for (int q = 0; q < (LOCAL ? 1 : NQR); ++q) xq[q] = make_float4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
    float* my_tk = topk + tid * KP;
    for (int e = 0; e < KP; ++e) my_tk[e] = __builtin_huge_valf();
    float U = 0.f;
    if (my_valid) {
        U = __builtin_huge_valf();
        if (a.u0) {
            const double u0 = a.u0[my_rp];
            if (u0 >= 0.0) U = d2f_up(u0);
        }
        if (!(U < __builtin_huge_valf())) {
            // no bound yet: seed one from the row's 2 SEEDW neighbours in the
            // sorted order (distinct admissible columns, keys bounded from FP32)
            for (int o = -SEEDW; o <= SEEDW; ++o) {
                const int64_t q = (int64_t)my_rp + o;
                if (o == 0 || q < tile.z || q >= tile.w || q >= a.np || a.compS[q] == my_comp) continue;
                const float4* src = reinterpret_cast<const float4*>(a.xs + q * DMAX);
                float sq = 0.f;
#pragma unroll
                for (int f4 = 0; f4 < NQR; ++f4) {
                    const float4 y = src[f4];
                    const float d0 = x[4 * f4] - y.x, d1 = x[4 * f4 + 1] - y.y;
                    const float d2 = x[4 * f4 + 2] - y.z, d3 = x[4 * f4 + 3] - y.w;
                    sq = __builtin_fmaf(d0, d0, sq);
                    sq = __builtin_fmaf(d1, d1, sq);
                    sq = __builtin_fmaf(d2, d2, sq);
                    sq = __builtin_fmaf(d3, d3, sq);
                }
                const float ub = fp32_key_upper(sq, a.d);
                if (ub < my_tk[k - 1]) {
                    int p = k - 1;
                    while (p > 0 && my_tk[p - 1] > ub) { my_tk[p] = my_tk[p - 1]; --p; }
                    my_tk[p] = ub;
                }
            }
            U = my_tk[k - 1];
            for (int e = 0; e < KP; ++e) my_tk[e] = __builtin_huge_valf();
        }
    }
    rs[tid][0] = make_float4(-__builtin_huge_valf(), U, 0.f, 0.f);
    rs[tid][1] = make_float4(__int_as_float(0), __int_as_float(my_comp), 0.f, 0.f);
    if (a.prune || LOCAL) tile_ball<DMAX>(sh, x, my_valid, a.d);
    if (a.prune) wave_ball<DMAX>(&wcen[wave][0], &wrad[wave], x, my_valid, a.d);
    // row operand and its bound inputs (LOCAL: per super-chunk frame, below)
    PointConst mypc{0.f, 0.f, 0.f, 0.f};
    if constexpr (!LOCAL) {
        if (my_valid) mypc = a.pc[my_rp];
        // one frame for every pair: the row's slack is fixed
        rs[tid][0].z = global_eps(mypc, a.bc);
        rs[tid][0].w = global_eta(mypc, a.bc);
        rs[tid][0].x = my_valid ? thresh_from_U(U * s2, rs[tid][0].z, rs[tid][0].w, exact) : -__builtin_huge_valf();
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
    __syncthreads();                                       // the tile's shared fields are written
    // row fragments stay in registers for the whole sweep (LOCAL: both
    // halves in the tile's frame; a column frame only rewrites their norm
    // slots)
    // SPLIT: BF16 in the super-chunk frames keeps its rows as two halves
    constexpr bool SPLIT = LOCAL && OP == OP_BF16;
    static_assert(!LOCAL || OP != OP_FP8, "the super-chunk frames take BF16 or FP16 operands");
    frag_t bfrag[RB], bfl[SPLIT ? RB : 1];
    int32_t rprb[LOCAL ? RB : 1];
    int32_t rcomp[RB];
    uint32_t rvmask = 0;                                   // hit bits of valid rows
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int rl = wave * RB * 16 + rb * 16 + (lane & 15);
        const int64_t slot = row_base + rl;
        const bool ok = slot < row_end;
        const int rp = ok ? (a.rows ? a.rows[slot] : a.row0 + (int)slot) : 0;
        if constexpr (LOCAL) {
            rprb[rb] = rp;
        } else {
            bfrag[rb] = reinterpret_cast<const frag_t*>(a.opR)[(int64_t)rp * 4 + grp];
        }
        rcomp[rb] = ok ? a.compS[rp] : -2;
        if (ok) rvmask |= 0x000F000Fu << (4 * rb);
    }
    float Treg[RB];
    const int lo_r = sh.lo, hi_r = sh.hi;
    const bool one_comp = lo_r == hi_r;
    const int cl = sh.col_lo, ch = sh.col_hi;
    int frame = -1;                                        // LOCAL: the wave's current super-chunk frame

    // ---- column sweep: nearest chunks first, the next one in flight ---------
    unsigned long long pairs = 0;                          // per wave
    // Thread t carries column t of a chunk from global memory to LDS.
    uint4 pf[PF];
    int pf_cc = -1;
    // the bound the other column splits have found for this row, read with
    // each chunk's loads and used behind the next barrier (any older value is
    // still a valid bound)
    float pf_gU = __builtin_huge_valf();
    auto fetch = [&](int64_t c0, int64_t cend) {
        if (SHARE && my_valid) pf_gU = __uint_as_float(a.gU[my_slot]);
        const bool in = c0 + tid < cend;
        const uint4* src = reinterpret_cast<const uint4*>(a.opC) + (c0 + (in ? tid : 0)) * PF;
#pragma unroll
        for (int q = 0; q < PF; ++q) pf[q] = src[q];
        pf_cc = in ? a.compS[c0 + tid] : -1;
    };
    // registers -> LDS buffer b, in fragment order; columns this tile never
    // pairs with (beyond the data, outside its column range, or in the
    // component of a one-component tile) get t = +inf where the format has one
    //   LOCAL: a column's norm slots 29..31 are rewritten from ||p||^2 to
    //   C = ||p||^2 - 2 delta.p for the chunk's frame offset (FP32, three
    //   BF16 parts; see frame_rows)
    auto stash = [&](int64_t c0, int b, int slot) {
        // (pf_cc < 0: past the chunk's end; component ids are >= 0)
        const bool col_ok = pf_cc >= 0 && c0 + tid >= cl && c0 + tid < ch &&
                            !(one_comp && pf_cc == lo_r);
        colcomp[b][tid] = col_ok ? pf_cc : -1;
        if constexpr (LOCAL) {
            if (col_ok) {
                typedef LpFmt<OP> F;
                const float4* dv4 = reinterpret_cast<const float4*>(&dlt[slot / SUPER][0]);
                float dotp = 0.f;                          // (-2 p) . delta, eight features a quarter
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float4 da = dv4[2 * q], db = dv4[2 * q + 1];
                    const float dq[8] = {da.x, da.y, da.z, da.w, db.x, db.y, db.z, db.w};
                    const uint32_t wq[4] = {pf[q].x, pf[q].y, pf[q].z, pf[q].w};
#pragma unroll
                    for (int f = 0; f < 8; ++f) {
                        const int kf = 8 * q + f;
                        if (kf < DMAX_MFMA && kf < a.d) {
                            const uint32_t wv = wq[f >> 1];
                            const float m2p = F::from((uint16_t)((f & 1) ? (wv >> 16) : (wv & 0xFFFFu)));
                            dotp = __builtin_fmaf(m2p, dq[f], dotp);
                        }
                    }
                }
                // slots 29, 30, 31: the parts of ||p||^2
                const float normp = (F::from((uint16_t)(pf[3].z >> 16)) + F::from((uint16_t)(pf[3].w & 0xFFFFu))) +
                                    F::from((uint16_t)(pf[3].w >> 16));
                float r = normp + dotp;
                uint32_t part[NORM_PARTS];
#pragma unroll
                for (int k3 = 0; k3 < NORM_PARTS; ++k3) {
                    part[k3] = F::to(r);
                    r -= F::from((uint16_t)part[k3]);
                }
                pf[3].z = (pf[3].z & 0xFFFFu) | (part[0] << 16);
                pf[3].w = part[1] | (part[2] << 16);
            }
        }
        if constexpr (Tr::BYTES == 64) {
            uint4* cb4 = reinterpret_cast<uint4*>(&colbuf[b][0]);
            if (__ballot(!col_ok) == 0ull) {               // the usual case: copies only
#pragma unroll
                for (int q = 0; q < 4; ++q) cb4[((tid >> 4) * 4 + q) * 16 + (tid & 15)] = pf[q];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint4 v = pf[q];
                    if (!col_ok) {
                        v = make_uint4(0, 0, 0, 0);
                        // K slot 29: t = +inf; LOCAL: the largest finite BF16
                        // (the rows' low halves hold 0 there, and 0 x inf would
                        // be NaN); the slow path drops such a column anyway
                        if (q == 3) v.z = (SPLIT ? 0x7F7Fu : LpFmt<OP>::inf_bits) << 16;
                    }
                    cb4[((tid >> 4) * 4 + q) * 16 + (tid & 15)] = v;
                }
            }
        } else {
            // FP8 has no infinity: masked columns are zero and the slow path
            // drops them by their component entry
            uint2* cb2 = reinterpret_cast<uint2*>(&colbuf[b][0]);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint4 v = col_ok ? pf[h] : make_uint4(0, 0, 0, 0);
                cb2[((tid >> 4) * 4 + 2 * h) * 16 + (tid & 15)] = make_uint2(v.x, v.y);
                cb2[((tid >> 4) * 4 + 2 * h + 1) * 16 + (tid & 15)] = make_uint2(v.z, v.w);
            }
        }
    };

    // LOCAL: the rows in their tile's frame (centre c_T = the tile ball's
    // centre), split once.  Lane l builds, for every row block rb, K slots
    // 8g..8g+7 (g = l / 16) of row rb * 16 + l % 16 -- its own B fragments --
    // for both halves of a = ah + al: u = sigma (x - c_T) in FP32,
    // ah = bf16(u), al = bf16(u - ah) (the difference is exact in FP32, and
    // ah + al too).  The norm slots stay for the column frames (the high
    // half's ones are set here, its parts per frame; the low half holds
    // zeros there).  Per row, into rpc: Q = ||ah|| + ||al||, ||a||^2 (FP32),
    // and eta from |al - (u - ah)| <= 2^-8 |u - ah| <= 2^-16 |u| per feature,
    // plus the FP32 offset's rounding and BF16's subnormal floor.
    auto tile_split = [&](const int (&rp)[RB]) {
      if constexpr (LOCAL) {
        typedef LpFmt<OP> F;
        const float4* c4 = reinterpret_cast<const float4*>(sh.cen) + 2 * grp;
        const float4 ca = c4[0], cb = c4[1];
        const float cv[8] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
        const uint32_t one = F::to(1.0f);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const float4* x4 = reinterpret_cast<const float4*>(a.xs + (int64_t)rp[rb] * DMAX) + 2 * grp;
            const float4 xa = x4[0], xb = x4[1];
            const float xv[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
            uint32_t hw[4], lw[4];
            float nrm = 0.f, vn = 0.f, nh = 0.f, nl = 0.f;
#pragma unroll
            for (int f2 = 0; f2 < 4; ++f2) {
                uint32_t hp = 0, lp = 0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int f = 2 * f2 + h, kf = 8 * grp + f;
                    if (kf < DMAX_MFMA && kf < a.d) {
                        const float u = (xv[f] - cv[f]) * sigma;
                        const uint32_t qh = F::to(u);
                        const float qhv = F::from((uint16_t)qh);
                        uint32_t ql = 0;
                        float qlv = 0.f;
                        if constexpr (SPLIT) {
                            ql = F::to(u - qhv);
                            qlv = F::from((uint16_t)ql);
                        }
                        const float q = qhv + qlv;
                        nrm = __builtin_fmaf(q, q, nrm);
                        vn = __builtin_fmaf(u, u, vn);
                        nh = __builtin_fmaf(qhv, qhv, nh);
                        nl = __builtin_fmaf(qlv, qlv, nl);
                        hp |= qh << (16 * h);
                        lp |= ql << (16 * h);
                    }
                }
                hw[f2] = hp;
                lw[f2] = lp;
            }
            // the row's sums: the four lanes' quarter sums (the same value in each)
            nrm += __shfl_xor(nrm, 16);
            vn += __shfl_xor(vn, 16);
            nh += __shfl_xor(nh, 16);
            nl += __shfl_xor(nl, 16);
            nrm += __shfl_xor(nrm, 32);
            vn += __shfl_xor(vn, 32);
            nh += __shfl_xor(nh, 32);
            nl += __shfl_xor(nl, 32);
            if (grp == 3) {                                // slots 24..31: features 24, 25, norm slots
                hw[1] = 0;                                 // parts 1, 2: per frame
                hw[2] = one << 16;                         // part 3: per frame; slot 29: 1
                hw[3] = one | (one << 16);
            }
            bfrag[rb] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
            if constexpr (SPLIT) bfl[rb] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
            if (grp == 0) {
                const double up = 1.0 + 0x1p-18;
                const double sq = (double)__builtin_sqrtf(nh) + (double)__builtin_sqrtf(nl);
                // split rows: |a - u| <= 2^-16 |u|; one half: the format's roundoff
                const double alpha = SPLIT ? 0x1p-16 + 0x1p-22 : F::alpha;
                rpc[wave * RB * 16 + rb * 16 + lane] = make_float4(
                    d2f_up(sq * up), nrm,
                    d2f_up((alpha * (double)__builtin_sqrtf(vn) * up +
                            F::beta * __builtin_sqrt((double)a.d)) * up), 0.f);
            }
        }
      }
    };

    // LOCAL: the rows' norm slots in the frame of the column super-chunk
    // whose offset is dlt[w] (delta = sigma (c_T - c_S), FP32): with a the
    // row in its tile's frame and p a column in its super-chunk's, the pair's
    // t = ||a + delta||^2 + ||p||^2 - 2 a.p - 2 delta.p, so the row's slots
    // carry R = ||a||^2 + 2 a.delta + ||delta||^2 (FP32: each dot product
    // within 10 roundings, the sums within two more) as three BF16 parts and
    // the columns' slots carry ||p||^2 - 2 delta.p (rewritten when staged).
    // Per row into rpf: P = sum of |parts|, rho = residual + 30 2^-24 (||a||^2
    // + 2 Q ||delta|| + ||delta||^2); eta grows by 2^-22 ||delta|| (the FP32
    // rounding of delta moves the represented row).
    auto frame_rows = [&](int w) {
      if constexpr (LOCAL) {
        typedef LpFmt<OP> F;
        const float dn = dlt[w][DMAX];
        float dv[8];
#pragma unroll
        for (int f = 0; f < 8; ++f) dv[f] = dlt[w][8 * grp + f];   // zero beyond the data's features
        float dd = 0.f;
#pragma unroll
        for (int f = 0; f < 8; ++f) dd = __builtin_fmaf(dv[f], dv[f], dd);
        dd += __shfl_xor(dd, 16);
        dd += __shfl_xor(dd, 32);
        const uint32_t one = F::to(1.0f);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            // a . delta over the lane's eight features, read in place
            auto half = [](uint32_t w, int h) { return F::from((uint16_t)(h ? (w >> 16) : (w & 0xFFFFu))); };
            float dot = 0.f;
#pragma unroll
            for (int f = 0; f < 8; ++f) {
                const int kf = 8 * grp + f;
                if (kf < DMAX_MFMA && kf < a.d) {
                    const uint32_t wh = (f >> 1) == 0 ? bfrag[rb].x : (f >> 1) == 1 ? bfrag[rb].y
                                      : (f >> 1) == 2 ? bfrag[rb].z : bfrag[rb].w;
                    float av = half(wh, f & 1);
                    if constexpr (SPLIT) {
                        const uint32_t wl = (f >> 1) == 0 ? bfl[rb].x : (f >> 1) == 1 ? bfl[rb].y
                                          : (f >> 1) == 2 ? bfl[rb].z : bfl[rb].w;
                        av += half(wl, f & 1);
                    }
                    dot = __builtin_fmaf(av, dv[f], dot);
                }
            }
            dot += __shfl_xor(dot, 16);
            dot += __shfl_xor(dot, 32);
            const int row = wave * RB * 16 + rb * 16 + (lane & 15);
            const float4 rc = rpc[row];                    // Q, ||a||^2, eta
            const float R = (rc.y + 2.f * dot) + dd;
            float r = R, psum = 0.f;
            uint32_t part[NORM_PARTS];
#pragma unroll
            for (int k3 = 0; k3 < NORM_PARTS; ++k3) {
                part[k3] = F::to(r);
                const float pv = F::from((uint16_t)part[k3]);
                psum += __builtin_fabsf(pv);
                r -= pv;
            }
            if (grp == 3) {                                // slots 26, 27 and 28
                bfrag[rb].y = part[0] | (part[1] << 16);
                bfrag[rb].z = part[2] | (one << 16);
            }
            if (grp == 0) {
                const double up = 1.0 + 0x1p-18;
                rpf[row] = make_float2(
                    d2f_up((double)psum * up),
                    d2f_up(((double)__builtin_fabsf(r) +
                            30.0 * 0x1p-24 * ((double)rc.y + 2.0 * (double)rc.x * (double)dn + (double)dd)) * up));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const float4 rc = rpc[tid];
        const float2 rf = rpf[tid];
        mypc = PointConst{rc.x, rf.x, rf.y, d2f_up(((double)rc.z + 0x1p-22 * (double)dn) * (1.0 + 0x1p-18))};
      }
    };
    if constexpr (LOCAL) tile_split(rprb);

    // chunk [c0, cend) in LDS buffer b, components lo_c..hi_c, candidate slot
    // `slot`; wneed: some row of this wave passed its test for the chunk
    // (else nothing to do)
    auto process = [&](int b, int lo_c, int hi_c, int64_t c0, int64_t cend, bool wneed, int slot) {
        if (!wneed) return;
        const int ncols = (int)(cend - c0);
        const bool pure = lo_c == hi_c;                    // the chunk is one component
        // super-chunk frames: the rows in this chunk's frame, and this
        // chunk's slack and threshold for the row (the wave's rows are read
        // back by other lanes of the same wave only).  In the global frame
        // the slack is fixed and T follows U wherever U moves, so nothing is
        // recomputed per chunk.
        if constexpr (LOCAL) {
            const int fw = slot / SUPER;
            const int fsc = gsc[fw];
            if (fsc != frame) {                            // wave-uniform
                frame_rows(fw);
                frame = fsc;
            }
            // the chunk's columns: maxima of Q, (P), rho, eta in their own
            // frame; their rewritten norm slots carry |C| <= Q*^2 + rho* +
            // 2 Q* ||delta|| (P: parts within 2^-6 of it) with FP32 error
            // within 32 2^-24 of it beyond rho*
            const float4 cm = gcm[slot];
            const float mag = (cm.x * cm.x + cm.z + 2.f * cm.x * dlt[fw][DMAX]) * (1.f + 0x1p-18f);
            const float Ps = mag * (1.f + 0x1p-6f);
            const float rhoS = (cm.z + 32.f * 0x1p-24f * mag) * (1.f + 0x1p-18f);
            const float eps = (a.bc.gamma * (2.f * mypc.Q * cm.x + mypc.P + Ps) + mypc.rho + rhoS) *
                              (1.f + 0x1p-20f);
            const float eta = (mypc.eta + cm.w) * (1.f + 0x1p-22f);
            rs[tid][0].z = eps;
            rs[tid][0].w = eta;
            rs[tid][0].x = my_valid ? thresh_from_U(rs[tid][0].y * s2, eps, eta, exact) : -__builtin_huge_valf();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // rows of a one-component chunk's own component see no candidate
        bool own[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) own[rb] = pure && rcomp[rb] == lo_c;
        auto reload_T = [&]() {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                Treg[rb] = own[rb] ? -__builtin_huge_valf() : rs[wave * RB * 16 + rb * 16 + (lane & 15)][0].x;
        };
        reload_T();
        pairs += (unsigned long long)ncols;

        const frag_t* cbuf = &colbuf[b][0];
        const int32_t* ccomp = &colcomp[b][0];
        const int nblk = (ncols + 15) >> 4;
        // Slow path for the blocks cb (and cb + 1 if two): every lane first
        // collects its candidates below its rows' thresholds as bits
        // (b * 16 + rb * 4 + r), then walks only those, one per step.  The
        // four lanes lane & 15 + 16 g hold columns of the same rows: in a
        // step, a lane whose next candidate is in the same row block as that
        // of a lane of a lower group waits, so a row's LDS state is never
        // touched by two lanes at once, and lanes of different rows proceed
        // together.
        auto slow = [&](int cb, const f32x4_t (&acc0)[RB], const f32x4_t (&acc1)[RB], bool two) {
            uint32_t hm = 0;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    hm |= (uint32_t)(acc0[rb][r] <= Treg[rb]) << (rb * 4 + r);
                    if (two) hm |= (uint32_t)(acc1[rb][r] <= Treg[rb]) << (16 + rb * 4 + r);
                }
            }
            hm &= rvmask;
            while (__ballot(hm != 0u)) {
                const int e = hm ? (int)__builtin_ctz(hm) : 0;
                const int rbs = hm ? ((e >> 2) & 3) : -1;     // row block of the next candidate
                const int o1 = __shfl_xor(rbs, 16), o2 = __shfl_xor(rbs, 32), o3 = __shfl_xor(rbs, 48);
                const int g = grp;
                const bool wait = ((g ^ 1) < g && o1 == rbs) || ((g ^ 2) < g && o2 == rbs) ||
                                  ((g ^ 3) < g && o3 == rbs);
                if (rbs >= 0 && !wait) {
                    hm &= hm - 1;
                    do {
                        const float v = pick32(acc0, acc1, e);
                        const int rb = (e >> 2) & 3, r = e & 3;
                        const int rl = wave * RB * 16 + rb * 16 + (lane & 15);
                        // every LDS read this hit may need, issued together
                        const int cj = (cb + (e >> 4)) * 16 + 4 * g + r;
                        const float4 st = rs[rl][0];              // T, U, eps, eta
                        const float4 s1 = rs[rl][1];              // count, component
                        const int cc = ccomp[cj];
                        float4* tk4 = topk4 + rl * (KP / 4);
                        float4 tq[KP / 4];
#pragma unroll
                        for (int q = 0; q < KP / 4; ++q) tq[q] = tk4[q];
                        if (!(v <= st.x)) continue;
                        // same component, or a column this tile must not pair with
                        if (cc < 0 || cc == __float_as_int(s1.y)) continue;
                        const int64_t slot = row_base + rl;
                        int pos;
                        if (SHARE) {
                            pos = atomicAdd(&a.surv_cnt[slot], 1);
                        } else {
                            pos = __float_as_int(s1.x);
                            rs[rl][1].x = __int_as_float(pos + 1);
                        }
                        const float eps = st.z, eta = st.w;
                        // LOCAL: t + E(t) in this chunk's frame (kept for the
                        // error report) and the bound on the key in data units
                        const float upv = LOCAL ? upper_from_t(v, eps, eta, exact) : v;
                        if (pos < a.S) {
                            a.surv_j[slot * a.S + pos] = (int)(c0 + cj);
                            a.surv_t[slot * a.S + pos] = v;
                            if (LOCAL) a.surv_e[slot * a.S + pos] = upv;
                        }
                        const float key = LOCAL ? d2f_up((double)upv * inv_s2) : v;
                        // the row's list (read above), rewritten with vector stores
                        float kth_old = __builtin_huge_valf();
#pragma unroll
                        for (int q = 0; q < KP / 4; ++q) {
                            const float x4[4] = {tq[q].x, tq[q].y, tq[q].z, tq[q].w};
#pragma unroll
                            for (int h = 0; h < 4; ++h)
                                if (4 * q + h == k - 1) kth_old = x4[h];
                        }
                        if (key < kth_old) {
                            // insert into the sorted first k entries
                            float prev = -__builtin_huge_valf(), kth = 0.f;
#pragma unroll
                            for (int q = 0; q < KP / 4; ++q) {
                                float x4[4] = {tq[q].x, tq[q].y, tq[q].z, tq[q].w};
#pragma unroll
                                for (int h = 0; h < 4; ++h) {
                                    const int e2 = 4 * q + h;
                                    const float old = x4[h];
                                    if (e2 < k) x4[h] = old <= key ? old : (prev <= key ? key : prev);
                                    if (e2 == k - 1) kth = x4[h];
                                    prev = old;
                                }
                                tk4[q] = make_float4(x4[0], x4[1], x4[2], x4[3]);
                            }
                            if (kth < __builtin_huge_valf()) {
                                const float Usc = LOCAL ? kth * s2 : upper_from_t(kth, eps, eta, exact);
                                const float Us = LOCAL ? kth : d2f_up((double)Usc * inv_s2);
                                const float T = thresh_from_U(Usc, eps, eta, exact);
                                if (Us < st.y || T < st.x) {
                                    if (SHARE && Us < st.y) atomicMin(&a.gU[slot], __float_as_uint(Us));
                                    rs[rl][0] = make_float4(fminf(st.x, T), fminf(st.y, Us), eps, eta);
                                }
                            }
                        }
                    } while (false);
                }
                // this step's row-state writes before the next step's reads
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        };
        // two 16-column blocks per step: 8 MFMAs, then one min3 chain and
        // one compare per row block for 8 candidates
        auto step2 = [&](int cb, const frag_t& af0, const frag_t& af1) {
            f32x4_t acc0[RB], acc1[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc0[rb] = Tr::mma(af0, bfrag[rb]);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc1[rb] = Tr::mma(af1, bfrag[rb]);
            if constexpr (SPLIT) {                         // the rows' low halves
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) acc0[rb] = Tr::mma_acc(af0, bfl[rb], acc0[rb]);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) acc1[rb] = Tr::mma_acc(af1, bfl[rb], acc1[rb]);
            }
            // all eight MFMAs issue back to back; the epilogue then finds the
            // first results ready instead of stalling after each pair
            __builtin_amdgcn_sched_barrier(0);
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
                slow(cb, acc0, acc1, true);
                reload_T();
            }
        };
        auto frag = [&](int blk) { return cbuf[(blk * 4 + grp) * 16 + (lane & 15)]; };
        // unrolled by two steps with two fragment sets, so the fragments of
        // the next step are read while this step's MFMAs run, without copies
        int cb = 0;
        if (nblk >= 2) {
            frag_t fa0 = frag(0), fa1 = frag(1);
            for (; cb + 3 < nblk; cb += 4) {
                const frag_t fb0 = frag(cb + 2), fb1 = frag(cb + 3);
                step2(cb, fa0, fa1);
                if (cb + 5 < nblk) {
                    fa0 = frag(cb + 4);
                    fa1 = frag(cb + 5);
                }
                step2(cb + 2, fb0, fb1);
            }
            if (cb + 1 < nblk) {
                step2(cb, fa0, fa1);
                cb += 2;
            }
        }
        if (cb < nblk) {
            const frag_t af = cbuf[(cb * 4 + grp) * 16 + (lane & 15)];
            f32x4_t acc[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[rb] = Tr::mma(af, bfrag[rb]);
            if constexpr (SPLIT) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) acc[rb] = Tr::mma_acc(af, bfl[rb], acc[rb]);
            }
            bool hit = false;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const float m = fminf(fminf(acc[rb][0], acc[rb][1]), fminf(acc[rb][2], acc[rb][3]));
                hit |= (m <= Treg[rb]);
            }
            if (__ballot(hit)) {
                slow(cb, acc, acc, false);
                reload_T();
            }
        }
    };

    // Groups of candidate chunks, nearest super-chunks first.  Per group:
    // the tile's bound umax (max over its rows' U), the candidates of up to
    // GS passing super-chunks (tile-level tests), each row's test against
    // every candidate (bits per wave), then the chunks some wave needs, in
    // order, with the next one in flight.
    GroupGen<TAB> gen;
    gen.init(sh, a, it);
    float reach = __builtin_huge_valf(), reachU = __builtin_huge_valf();   // sqrt bound of U
    int buf = 0;
    for (;;) {
        float um = my_valid ? rs[tid][0].y : 0.f;
        for (int off = 32; off > 0; off >>= 1) um = fmaxf(um, __shfl_xor(um, off));
        if (lane == 0) wmx[wave] = um;
        __syncthreads();                                   // every wave done with the last group
        const float umax = fmaxf(fmaxf(wmx[0], wmx[1]), fmaxf(wmx[2], wmx[3]));
        int scl[GS];
        const int g = gen.take(sh, a, lo_r, hi_r, umax, scl);
        if (g == 0) break;                                 // the same decision in every wave
        float4 xg[LOCAL ? NQR : 1];                        // LOCAL: the row's coordinates for the tests
        if constexpr (LOCAL) {
            const float4* src = reinterpret_cast<const float4*>(a.xs + (int64_t)my_rp * DMAX);
#pragma unroll
            for (int q = 0; q < NQR; ++q) xg[q] = src[q];
        }
        gen.expand(sh, a, lo_r, hi_r, umax, wave < g ? scl[wave < GS ? wave : 0] : -1, wave, gball, gpos,
                   gneed, LOCAL ? gcm : nullptr, gsc);
        if constexpr (LOCAL) {
            // the offset delta = sigma (c_T - c_S) of this wave's super-chunk
            // (FP32; zero beyond the data's features) and ||delta|| rounded up
            const int scw = wave < g ? scl[wave < GS ? wave : 0] : -1;
            if (scw >= 0) {
                float dk = 0.f;
                if (lane < a.d && lane < DMAX_MFMA)
                    dk = (sh.cen[lane] - a.sballs[(int64_t)scw * BALL_STRIDE + lane]) * sigma;
                if (lane < DMAX) dlt[wave][lane] = dk;
                float sq = dk * dk;
                for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
                if (lane == 0) dlt[wave][DMAX] = d2f_up((double)__builtin_sqrtf(sq) * (1.0 + 0x1p-18));
            }
        }
        __syncthreads();                                   // candidates in LDS
        // candidates within reach of this wave's ball (one per lane), then
        // the rows' own tests for those
        bool wpass = (gneed[lane] & 16) != 0;
        if (a.prune && wpass) wpass = balls_lb2(&wcen[wave][0], wrad[wave], &gball[lane][0]) <= um;
        const unsigned long long vmask = __ballot(wpass);
        if (a.prune) {
            const float Ucur = rs[tid][0].y;
            if (Ucur != reachU) {                          // the root only when U moved
                reachU = Ucur;
                reach = reach_of(Ucur);
            }
        }
        for (unsigned long long m = vmask; m != 0ull; m &= m - 1ull) {
            const int slot = (int)__builtin_ctzll(m);
            const int4 gp = gpos[slot];
            // a row skips a chunk made only of its own component, or whose
            // ball lies farther than its bound
            bool need = my_valid && !(gp.z == gp.w && gp.z == my_comp);
            if (a.prune && need) {
                if constexpr (LOCAL) need = point_ball_reach(xg, &gball[slot][0], reach);
                else need = point_ball_reach(xq, &gball[slot][0], reach);
            }
            if (__ballot(need) != 0ull && lane == 0) atomicOr(&gneed[slot], 1 << wave);
        }
        __syncthreads();                                   // every wave's needs in LDS
        const int gn = gneed[lane];
        unsigned long long nmask = __ballot((gn & 15) != 0);
        int cur = nmask ? (int)__builtin_ctzll(nmask) : -1;
        if (cur >= 0) {
            nmask &= nmask - 1ull;
            fetch(gpos[cur].x, gpos[cur].y);
        }
        while (cur >= 0) {
            const int4 cp = gpos[cur];
            const bool wn = ((__builtin_amdgcn_readlane(gn, cur) >> wave) & 1) != 0;
            stash(cp.x, buf, cur);
            __syncthreads();    // chunk cur in LDS; every wave is done with buf ^ 1's last use
            // bounds found by the other column splits of the row (loaded with
            // the chunk now in LDS, so nothing waits here)
            if (SHARE && my_valid) {
                const float gu = pf_gU;
                if (gu < rs[tid][0].y) {
                    rs[tid][0].y = gu;
                    if (!LOCAL)
                        rs[tid][0].x = fminf(rs[tid][0].x, thresh_from_U(gu * s2, rs[tid][0].z, rs[tid][0].w, exact));
                }
            }
            const int nxt = nmask ? (int)__builtin_ctzll(nmask) : -1;
            if (nxt >= 0) {
                nmask &= nmask - 1ull;
                fetch(gpos[nxt].x, gpos[nxt].y);           // in flight while cur is processed
            }
            process(buf, cp.z, cp.w, cp.x, cp.y, wn, cur);
            cur = nxt;
            buf ^= 1;
        }
    }
    if (!SHARE && my_valid) a.surv_cnt[my_slot] = __float_as_int(rs[tid][1].x);
    // the row's final threshold (one frame for every pair): a survivor above
    // it has key > U >= the row's k-th key, so rescoring may drop it.  LOCAL
    // (the frame changes per chunk): the final bound U itself, in data units;
    // rescoring drops a survivor whose key is provably above it
    if (a.tfin && my_valid) {
        if constexpr (LOCAL) atomicMin(&a.tfin[my_slot], __float_as_uint(rs[tid][0].y));
        else atomicMin(&a.tfin[my_slot], __float_as_uint(fmaxf(rs[tid][0].x, 0.f)));
    }
    const int wrows = sh.rows - wave * 64;
    if (lane == 0 && a.pairs && wrows > 0)
        atomicAdd(&a.pairs[((blockIdx.x * 4 + wave) & (NSPREAD - 1)) * SPREAD_STRIDE],
                  pairs * (unsigned long long)(wrows < 64 ? wrows : 64));
}

template <int OP, bool LOCAL, bool SHARE, int KP, bool TAB>
__global__ __launch_bounds__(256, 2) void k_cand_mfma(CandArgs a)
{
    cand_mfma_item<OP, LOCAL, SHARE, KP, TAB>(a, grid_item(a));
}

// device-sized launch: a fixed grid pops (tile, split) items; the splits of
// a row always share their thresholds
template <int OP, bool LOCAL, int KP>
__global__ __launch_bounds__(256, 2) void k_cand_mfma_q(CandArgs a)
{
    __shared__ int slot;
    Item it;
    while (pop_item(a, slot, it)) cand_mfma_item<OP, LOCAL, true, KP, false>(a, it);
}

template <int OP, bool LOCAL, bool TAB>
void launch_tab(const CandArgs& a, dim3 grid, hipStream_t s)
{
    if (a.k <= 8) {
        const size_t shm = (size_t)BM * 8 * sizeof(float);
        if (a.share) k_cand_mfma<OP, LOCAL, true, 8, TAB><<<grid, 256, shm, s>>>(a);
        else k_cand_mfma<OP, LOCAL, false, 8, TAB><<<grid, 256, shm, s>>>(a);
    } else {
        const size_t shm = (size_t)BM * KMAX * sizeof(float);
        if (a.share) k_cand_mfma<OP, LOCAL, true, KMAX, TAB><<<grid, 256, shm, s>>>(a);
        else k_cand_mfma<OP, LOCAL, false, KMAX, TAB><<<grid, 256, shm, s>>>(a);
    }
}

template <int OP, bool LOCAL>
void launch_one(const CandArgs& a, dim3 grid, size_t, hipStream_t s)
{
    if (a.desc) {
        if (a.k <= 8) k_cand_mfma_q<OP, LOCAL, 8><<<QGRID, 256, (size_t)BM * 8 * sizeof(float), s>>>(a);
        else k_cand_mfma_q<OP, LOCAL, KMAX><<<QGRID, 256, (size_t)BM * KMAX * sizeof(float), s>>>(a);
    } else if (a.cstart) {
        launch_tab<OP, LOCAL, true>(a, grid, s);
    } else {
        launch_tab<OP, LOCAL, false>(a, grid, s);
    }
}

}  // namespace

template <int OP>
void split_columns_op(const float* xs, int64_t np, int d, float sigma, const int32_t* cstart,
                      const int32_t* csup, const int32_t* tabn, int64_t nch_bound, const float* sballs,
                      void* opC, float4* cmax, hipStream_t s)
{
    if (cstart) {
        k_split_columns<true, OP><<<(unsigned)nch_bound, 256, 0, s>>>(xs, np, d, sigma, cstart, csup, tabn,
                                                                      sballs, (uint4*)opC, cmax);
    } else {
        const unsigned nc = (unsigned)((np + CHUNK - 1) / CHUNK);
        k_split_columns<false, OP><<<nc, 256, 0, s>>>(xs, np, d, sigma, nullptr, nullptr, nullptr, sballs,
                                                      (uint4*)opC, cmax);
    }
}

hipError_t launch_split_columns(int opkind, const float* xs, int64_t np, int d, float sigma,
                                const int32_t* cstart, const int32_t* csup, const int32_t* tabn,
                                int64_t nch_bound, const float* sballs, void* opC, float4* cmax,
                                hipStream_t s)
{
    if (np <= 0) return hipSuccess;
    if (opkind != OP_BF16) return hipErrorInvalidValue;   // the super-chunk frames are BF16's
    split_columns_op<OP_BF16>(xs, np, d, sigma, cstart, csup, tabn, nch_bound, sballs, opC, cmax, s);
    return hipGetLastError();
}

hipError_t launch_cand_mfma(int opkind, const CandArgs& a, hipStream_t s)
{
    if (a.desc && a.cstart) return hipErrorInvalidValue;   // device-sized launches use fixed chunks
    const unsigned nt = a.desc ? 1u : a.tiles ? (unsigned)a.n_tiles : (unsigned)((a.n_rows + BM - 1) / BM);
    if (!a.desc && (a.n_rows <= 0 || nt == 0)) return hipSuccess;
    dim3 grid(nt, a.desc ? 1u : (unsigned)a.col_splits);
    size_t shm = (size_t)BM * a.k * sizeof(float);
    const bool local = a.local != 0;
    switch (opkind) {
    case OP_BF16:
        if (local) launch_one<OP_BF16, true>(a, grid, shm, s);
        else launch_one<OP_BF16, false>(a, grid, shm, s);
        break;
    case OP_FP16:
        // FP16 runs in the global frame: in the super-chunk frames (one MFMA
        // per block) it kept 2.7x fewer first-round survivors but the per-chunk
        // thresholds and slot rewrites cost more in the merge rounds (2M
        // workload: 114 against 96 ms)
        if (local) return hipErrorInvalidValue;
        launch_one<OP_FP16, false>(a, grid, shm, s);
        break;
    case OP_FP8:
        if (local) return hipErrorInvalidValue;   // FP8 is used on exact integer data only
        launch_one<OP_FP8, false>(a, grid, shm, s);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nnm
