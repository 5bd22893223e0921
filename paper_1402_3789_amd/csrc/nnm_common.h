// nnm_common.h -- definitions shared by the gfx950 kernels and the host
// driver of the nearest-neighbour clustering library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nnm.h"

namespace nnm {

// Operand slots per point for the matrix-core candidate pass: D features
// plus three (value, constant) slot pairs that fold both squared norms into
// the dot product, padded to the K = 32 of one 16x16x32 MFMA.
constexpr int KSLOT = 32;
constexpr int NORM_PARTS = 3;
constexpr int DMAX = 32;                         // FP32 path
constexpr int DMAX_MFMA = KSLOT - 2 * NORM_PARTS;  // 26
constexpr int KMAX = 32;                         // neighbour-cache depth
// A bounding ball: centre[DMAX] (zero beyond the data's features), radius
// at [DMAX], zero padding to a 16-byte multiple.
constexpr int BALL_STRIDE = DMAX + 4;
constexpr int NSPREAD = 64;           // slots of the spread event counters
constexpr int SPREAD_STRIDE = 16;     // u64 per slot: one 128-byte cache line each
constexpr int SMAX = 2048;                       // survivor cap
// Column chunk of the candidate sweep (at most CHUNK sorted positions; the
// bounding balls are built per chunk) and super-chunks of SUPER chunks.
constexpr int CHUNK = 256;
constexpr int SUPER = 16;

enum OpKind : int { OP_BF16 = 0, OP_FP16 = 1, OP_FP8 = 2, OP_FP32 = 3 };

// Inputs of the per-pair error bound of one point, in the scaled candidate
// domain, each rounded up:
//   Q   = ||q||_2 of the quantised vector
//   P   = sum of |value * constant| over its norm slots
//   rho = |exact squared norm of q - what the norm slots carry|
//   eta = bound on ||q - sigma * (x - c)||_2 (quantisation error)
struct PointConst {
    float Q, P, rho, eta;
};

// Per-run constants of the candidate pass.
struct BoundConst {
    float colQ, colP, colRho, colEta;  // maxima over all points
    float gamma;                       // FP32 accumulation factor
    float sigma2;                      // sigma^2: t = sigma^2 * s (+ error)
    int exact;                         // 1: t == sigma^2 * s exactly
    int pad_;
};

// Sort record used for both the component sort and the edge sort.
struct SortRec {
    uint64_t k0;  // edge: bits of s; component sort: 0
    uint32_t k1;  // edge: u;         component sort: component id
    uint32_t k2;  // edge: v;         component sort: point id
};

// ---- small device helpers ------------------------------------------------

__device__ __forceinline__ uint16_t f32_to_bf16_rn(float f)
{
    uint32_t u = __float_as_uint(f);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float(((uint32_t)h) << 16);
}

__device__ __forceinline__ uint16_t f32_to_f16_rn(float f)
{
    _Float16 h = (_Float16)f;
    return __builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ float f16_to_f32(uint16_t h)
{
    return (float)__builtin_bit_cast(_Float16, h);
}

// Round a double up to the nearest float that is >= it.
__device__ __forceinline__ float d2f_up(double x)
{
    float f = (float)x;
    if ((double)f < x) {
        const uint32_t u = __float_as_uint(f);
        if (f == 0.0f) f = __uint_as_float(1u);           // smallest subnormal
        else if (f > 0.0f) f = __uint_as_float(u + 1u);
        else f = __uint_as_float(u - 1u);
    }
    return f;
}

// Squared distance of eq. (1) in FP64: exact widening, one rounding for the
// difference, one for the square, left-to-right sum over features.
__device__ __forceinline__ double sqdist_fp64(const float* a, const float* b, int d)
{
    double s = 0.0;
    for (int f = 0; f < d; ++f) {
        double diff = __dsub_rn((double)a[f], (double)b[f]);
        double sq = __dmul_rn(diff, diff);
        s = (f == 0) ? sq : __dadd_rn(s, sq);
    }
    return s;
}

// The same key for two rows of the padded sorted copy ([DMAX] floats each,
// 16-byte aligned): vector loads, identical arithmetic and order.
__device__ __forceinline__ double sqdist_fp64_rows(const float* a, const float* b, int d)
{
    const float4* a4 = reinterpret_cast<const float4*>(a);
    const float4* b4 = reinterpret_cast<const float4*>(b);
    double s = 0.0;
    for (int q = 0; q * 4 < d; ++q) {
        const float4 u = a4[q], v = b4[q];
        const float au[4] = {u.x, u.y, u.z, u.w};
        const float bv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int f = 4 * q + h;
            if (f < d) {
                const double diff = __dsub_rn((double)au[h], (double)bv[h]);
                const double sq = __dmul_rn(diff, diff);
                s = (f == 0) ? sq : __dadd_rn(s, sq);
            }
        }
    }
    return s;
}

// Keys of the L1 and L-infinity metrics (nnm_metric) for two rows of the
// padded sorted copy: exact |differences| in FP64, summed left to right, or
// their maximum.  metric_key_rows(m, ...) picks the metric's key (the
// cosine metric runs as Euclidean on scaled rows).
__device__ __forceinline__ double metric_key_rows(int metric, const float* a, const float* b, int d)
{
    if (metric == NNM_METRIC_L1 || metric == NNM_METRIC_LINF) {
        const float4* a4 = reinterpret_cast<const float4*>(a);
        const float4* b4 = reinterpret_cast<const float4*>(b);
        double s = 0.0;
        for (int q = 0; q * 4 < d; ++q) {
            const float4 u = a4[q], v = b4[q];
            const float au[4] = {u.x, u.y, u.z, u.w};
            const float bv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int f = 4 * q + h;
                if (f < d) {
                    const double t = __builtin_fabs(__dsub_rn((double)au[h], (double)bv[h]));
                    if (metric == NNM_METRIC_L1) s = (f == 0) ? t : __dadd_rn(s, t);
                    else s = t > s ? t : s;
                }
            }
        }
        return s;
    }
    return sqdist_fp64_rows(a, b, d);
}

// The same for two rows of an FP32 input (row-major, any stride).
__device__ __forceinline__ double metric_key(int metric, const float* a, const float* b, int d)
{
    if (metric == NNM_METRIC_L1 || metric == NNM_METRIC_LINF) {
        double s = 0.0;
        for (int f = 0; f < d; ++f) {
            const double t = __builtin_fabs(__dsub_rn((double)a[f], (double)b[f]));
            if (metric == NNM_METRIC_L1) s = (f == 0) ? t : __dadd_rn(s, t);
            else s = t > s ? t : s;
        }
        return s;
    }
    return sqdist_fp64(a, b, d);
}

// The reported distance of a key.
__host__ __device__ __forceinline__ bool metric_key_is_distance(int metric)
{
    return metric == NNM_METRIC_L1 || metric == NNM_METRIC_LINF;
}

// (s, j) order for one row: smaller s, then smaller j.
__device__ __forceinline__ bool sj_less(double s1, int j1, double s2, int j2)
{
    return s1 < s2 || (s1 == s2 && j1 < j2);
}

}  // namespace nnm

// ---- host-side launch interface (implemented in the .hip files) ----------

namespace nnm {

struct StageStats {
    uint32_t fmin[DMAX];   // ordered-float encodings
    uint32_t fmax[DMAX];
    int32_t nonfinite;
    int32_t nonint;        // a feature that is not an integer in [-16, 16]
    uint32_t colmax[4];    // float bits of max Q, P, rho, eta
    int32_t pad_[2];
};

hipError_t launch_stage_stats(const float* X, int64_t n, int d, int64_t ld,
                              StageStats* st, hipStream_t s);
hipError_t launch_stage_operands(const float* X, int64_t n, int d, int64_t ld,
                                 int opkind, int exact, const float* centre,
                                 float sigma, void* opR, void* opC,
                                 PointConst* pc, StageStats* st, hipStream_t s);
hipError_t launch_gather_points(int64_t n, int opkind, const int32_t* perm,
                                const void* opR, const void* opC,
                                const PointConst* pc, const float* X, int d,
                                int64_t ld, const int32_t* comp, void* opRs,
                                void* opCs, PointConst* pcs, float* xs,
                                int32_t* compS, hipStream_t s);

// Rounds replayed from a captured hipGraph take the size of each launch
// from the device: one descriptor per launch site, written by a one-thread
// kernel just before the launch.  The kernels of such a launch run a fixed
// grid that loops over the work; the candidate passes pop their (tile,
// column split) items from `queue`.
struct LaunchDesc {
    int32_t n_rows;    // rows of the launch
    int32_t n_tiles;   // row tiles (256 consecutive slots, or tile descriptors)
    int32_t splits;    // column splits per tile
    int32_t queue;     // next work item; zero before the candidate launch
    int32_t over;      // rows whose survivor list overflowed (rescoring)
    int32_t pad_[3];
};

// Candidate pass over a list of rows (sorted positions) against all columns.
struct CandArgs {
    const void* opR;          // row-form operands, sorted order
    const void* opC;          // column-form operands, sorted order
    const float* xs;          // [np][DMAX] FP32 coordinates in sorted order
    const PointConst* pc;     // per sorted position
    const int32_t* compS;     // component of each sorted position
    const int32_t* rows;      // row list (sorted positions), NULL = row0 + slot
    const double* u0;         // per sorted position: bound on the key, or NULL
    int32_t row0;
    int32_t n_rows;
    // optional tile descriptors (one per workgroup): x = first row slot,
    // y = end row slot, z = first column, w = end column (sorted positions);
    // NULL = tiles of 256 consecutive slots, columns [0, np)
    const int4* tiles;
    int32_t n_tiles;
    int32_t np;
    int32_t d;
    int32_t k;                // top-k depth
    int32_t S;                // survivor cap per row
    int32_t col_splits;
    BoundConst bc;
    int32_t* surv_cnt;        // [n_rows]
    int32_t* surv_j;          // [n_rows][S] sorted column positions
    float* surv_t;            // [n_rows][S] candidate values
    float* surv_e;            // [n_rows][S] super-chunk frames only: t + E(t) as applied
    unsigned long long* pairs;// [NSPREAD * SPREAD_STRIDE] count of evaluated pairs
    // chunk pruning and near-first order
    const float* X;           // original features (row-tile balls)
    int64_t ld;
    const int32_t* perm;      // sorted position -> point
    const float* balls;       // [chunks][BALL_STRIDE]
    const float* sballs;      // [super-chunks][BALL_STRIDE]
    // component-aligned column chunks (NULL: chunks of CHUNK consecutive
    // sorted positions, super-chunks of SUPER consecutive chunks): chunk c is
    // [cstart[c], cstart[c + 1]), in super-chunk csup[c]; super-chunk q is
    // chunks [sfirst[q], sfirst[q + 1]); pos2chunk[p] is the chunk holding
    // sorted position p; tabn = {chunks, super-chunks}
    const int32_t* cstart;
    const int32_t* csup;
    const int32_t* sfirst;
    const int32_t* pos2chunk;
    const int32_t* tabn;
    const int32_t* spos;      // [super-chunks + 1] first sorted position of each super-chunk
    const int32_t* ccomp;     // [chunks] the component of each chunk (each holds one)
    const int32_t* scomp;     // [super-chunks] and of each super-chunk
    int32_t prune;
    int32_t local;            // BF16 on general data: super-chunk frames (opC from
                              // launch_split_columns, rows split in-kernel from xs)
    const float4* cmaxT;      // [chunks] LOCAL: maxima of the columns' (Q, P, rho, eta)
    // thresholds shared by the column splits of one row (float bits)
    int32_t share;
    uint32_t* gT;             // [n_rows] candidate-domain threshold
    uint32_t* tfin;           // [n_rows] or NULL: each row's final threshold (FP32
                              // bits, clamped at 0; min over column splits); LOCAL:
                              // its final bound U on the k-th key (data units)
    uint32_t* gU;             // [n_rows] bound on the key of the k-th neighbour
    // device-sized launch (NULL: n_rows, n_tiles and col_splits above)
    LaunchDesc* desc;
    int32_t metric;           // nnm_metric (the FP32 path; the matrix cores: Euclidean)
};

hipError_t launch_cand_mfma(int opkind, const CandArgs& a, hipStream_t s);
// BF16 column operands in the frame of each column's super-chunk (centre:
// the super-chunk's ball centre) and each chunk's maxima of their bound
// inputs; cstart/csup/tabn: the component-aligned tables (NULL: fixed
// chunks), nch_bound: at least their chunk count.
hipError_t launch_split_columns(int opkind, const float* xs, int64_t np, int d, float sigma,
                                const int32_t* cstart, const int32_t* csup, const int32_t* tabn,
                                int64_t nch_bound, const float* sballs, void* opC, float4* cmax,
                                hipStream_t s);
hipError_t launch_cand_fp32(const CandArgs& a, hipStream_t s);

// FP64 rescoring of survivors into exact top-k lists.
struct RescoreArgs {
    const float* X;
    const float* xs;          // [np][DMAX] sorted FP32 copy (same values as X)
    int64_t ld;
    int32_t d;
    int32_t n_rows;
    int32_t k;                // neighbours sought (<= kstride)
    int32_t kstride;          // row stride of the neighbour cache
    int32_t S;
    const int32_t* rows;      // row list (sorted positions), NULL = row0 + slot
    int32_t row0;
    const int32_t* perm;      // sorted position -> point
    const uint32_t* tfin;     // NULL or the candidate pass's final threshold per row
                              // (super-chunk frames: its final bound on the k-th key)
    const int32_t* comp;      // component of each point
    const int32_t* surv_cnt;
    const int32_t* surv_j;
    const float* surv_t;
    const double* u0;         // per sorted position: bound on the key, or NULL
    double inv_sigma2;        // 1 / sigma^2, for the error report
    float sigma2;
    int32_t force_fallback;
    int64_t np;
    const int32_t* inst_off;  // [ninst + 1] instance offsets in point order (ninst > 1)
    int32_t ninst;            // instances; the exact scan stays inside the row's own
    // outputs, indexed by point id
    int32_t* cidx;            // [n][k]
    double* cs;               // [n][k]
    int32_t* clen;            // [n]
    int32_t* ccur;            // [n]
    double* clb;              // [n] lower bound for rows past the list
    int32_t* cflag;           // [n] bit0: list holds every outside point
    int32_t* overflow_rows;   // counter
    int32_t level;            // 1: overflowed rows get a bound and a re-scan; 2: full scan
    int32_t kb;               // level 1 bound: the kb-th key of the first S survivors
    double* u0b;              // [n] by sorted position: bound for the re-scan (level 1)
    int32_t* oflag;           // [n] by sorted position: row overflowed (level 1)
    unsigned long long* survivors; // [NSPREAD * SPREAD_STRIDE] counter
    // error report: max |t - s|, max |t - s| / s, the largest bound E(t)
    // applied to a rescored survivor and max |t - s| / E(t) (double bits)
    unsigned long long* err_bits;  // [4]
    int32_t bound_mode;       // BoundMode of the candidate pass that ran
    const PointConst* pcs;    // BOUND_GLOBAL: per sorted position
    BoundConst bc;            // BOUND_GLOBAL: column maxima
    const float* surv_e;      // BOUND_LOCAL: [n_rows][S] t + E(t)
    const LaunchDesc* desc;   // device-sized launch (NULL: n_rows above)
    int32_t metric;           // nnm_metric of the keys (cosine: Euclidean on scaled rows)
};

hipError_t launch_rescore(const RescoreArgs& a, int32_t* overflow_list, hipStream_t s);
hipError_t launch_fallback(const RescoreArgs& a, const int32_t* overflow_list, int n_over,
                           hipStream_t s);
// the exact scan of the rows counted in *n_over (device-sized launch)
hipError_t launch_fallback_dev(const RescoreArgs& a, const int32_t* overflow_list,
                               const int32_t* n_over, hipStream_t s);

// Descriptor of a device-sized launch over rows [off, off + cap) of a list
// of *count rows: n_rows = clamp(*count - off, 0, cap), tiles of 256 rows,
// column splits as the host would pick them (fixed_splits > 0: that many),
// queue and overflow count cleared.
hipError_t launch_desc_rows(LaunchDesc* d, const int32_t* count, int32_t off, int32_t cap,
                            int64_t np, int32_t target, int32_t fixed_splits, hipStream_t s);
// launch_desc_rows, and the first n_rows entries of surv_cnt (0) and of
// tfin (if not NULL), gT and gU (+inf) set, in one launch
hipError_t launch_prep_launch(LaunchDesc* d, const int32_t* count, int32_t off, int32_t cap,
                              int64_t np, int32_t target, int32_t fixed_splits, int32_t* surv_cnt,
                              uint32_t* tfin, uint32_t* gT, uint32_t* gU, hipStream_t s);
// After tile descriptors were built: splits from d->n_tiles.
hipError_t launch_desc_splits(LaunchDesc* d, int64_t np, int32_t target, int32_t fixed_splits,
                              hipStream_t s);
// p[0 .. d->n_rows) = v
hipError_t launch_fill_i32_desc(int32_t* p, int32_t v, const LaunchDesc* d, hipStream_t s);

// Merge-round kernels.
struct MergeArgs {
    int64_t n;
    int32_t k;
    int32_t* comp;            // [n] component root of each point
    int32_t* parent;          // [n] by root id
    const int32_t* cidx;
    const double* cs;
    int32_t* clen;
    int32_t* ccur;
    double* clb;
    int32_t* cflag;
    double* rbest_s;          // [n] row best (valid rows)
    int32_t* rbest_j;         // [n]
    int32_t* rstat;           // [n] 0 none, 1 valid, 2 exhausted
    unsigned long long* cbest_s;  // [n] by root id
    unsigned long long* cbest_p;  // [n]
    const int32_t* perm;      // sorted position -> point
    int32_t* rflag;           // [n] by sorted position
    double* u0s;              // [n] by sorted position: bound for the rescan
    float sigma2;
    int32_t disable_prune;
    SortRec* edges;           // round edges appended here
    int32_t* counters;        // [0] edges, [1] roots, [2] jump changes
};

hipError_t launch_cursor(const MergeArgs& a, hipStream_t s);
hipError_t launch_compmin1(const MergeArgs& a, hipStream_t s);
hipError_t launch_flag_rescan(const MergeArgs& a, hipStream_t s);
hipError_t launch_compmin2(const MergeArgs& a, hipStream_t s);
hipError_t launch_hook(const MergeArgs& a, hipStream_t s);
hipError_t launch_jump(const MergeArgs& a, int iters, hipStream_t s);
hipError_t launch_jump_check(const MergeArgs& a, hipStream_t s);
hipError_t launch_pick_reps(const MergeArgs& a, const int32_t* seg, int32_t* segstart,
                            int64_t nseg, int32_t* flag2, hipStream_t s);
// the same with the segment count on the device
hipError_t launch_pick_reps_dev(const MergeArgs& a, const int32_t* seg, int32_t* segstart,
                                const int32_t* nseg, int32_t* flag2, hipStream_t s);
// P-minimal-pairs pass: thr[0..1] (set to all ones before) receives the pass
// threshold over the rows' lists; out[0 .. *count) the listed pairs below
// it as (s bits, lo, hi), each once from each of its rows (at most cap kept;
// *count may exceed cap).
hipError_t launch_pm_candidates(const MergeArgs& a, unsigned long long* thr, SortRec* out,
                                int32_t* count, int64_t cap, hipStream_t s);
// *eff = *nrep when 0 < *nrep < *rcount, else 0 (the representatives are
// scanned first only when they are fewer than the rows to scan)
hipError_t launch_rep_select(const int32_t* nrep, const int32_t* rcount, int32_t* eff, hipStream_t s);
// dst[0 .. *count) = src[0 .. *count), *count <= cap
hipError_t launch_copy_i32_dev(int32_t* dst, const int32_t* src, const int32_t* count, int64_t cap,
                               hipStream_t s);
hipError_t launch_export_knn(int64_t n, int k, const int32_t* cidx, const double* cs,
                             const int32_t* clen, int32_t* idx, double* sd, int32_t* len,
                             hipStream_t s);
hipError_t launch_relabel(const MergeArgs& a, hipStream_t s);
hipError_t launch_reset_comp(const MergeArgs& a, hipStream_t s);
hipError_t launch_init_points(const MergeArgs& a, hipStream_t s);

// Scans and sorts.
size_t scan_temp_bytes(int64_t n);
hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n,
                                 void* temp, int32_t* total, hipStream_t s);
hipError_t launch_compact(const int32_t* flags, int64_t n, int32_t* out_list,
                          int32_t* out_count, void* temp, hipStream_t s);
// the same, leaving every flag zero
hipError_t launch_compact_clear(int32_t* flags, int64_t n, int32_t* out_list,
                                int32_t* out_count, void* temp, hipStream_t s);
size_t radix_temp_bytes(int64_t n);
// Stable LSD sort of records by the listed key fields (0: k0, 1: k1, 2: k2),
// least significant first; bits = significant bits of each field.
hipError_t launch_radix_sort(SortRec* a, SortRec* b, int64_t n,
                             const int* fields, const int* bits, int nfields,
                             void* temp, SortRec** result, hipStream_t s);
hipError_t launch_comp_records(const int32_t* comp, int64_t n, SortRec* rec,
                               hipStream_t s);
hipError_t launch_perm_from_records(const SortRec* rec, int64_t n,
                                    int32_t* perm, hipStream_t s);
// w = sqrt(s), or w = s for a metric whose key is the distance
hipError_t launch_write_edges(const SortRec* rec, int64_t ne, nnm_edge* out, int metric,
                              hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);

// Spatial order, component order and chunk balls (spatial.hip).
size_t spatial_temp_bytes(int64_t n, int L1, int L2);
hipError_t launch_spatial_order(const float* X, int64_t n, int d, int64_t ld, int L1, int L2,
                                int32_t* perm0, int32_t* rank0, SortRec* recA, SortRec* recB,
                                void* temp, hipStream_t s);
hipError_t launch_component_order(const int32_t* comp, const int32_t* perm0, const int32_t* rank0,
                                  int64_t n, int32_t* ckey, SortRec* recA, SortRec* recB,
                                  int32_t* perm, int32_t* seg, int32_t* flag, int32_t* excl,
                                  void* radix_temp, void* scan_temp, hipStream_t s);
// balls of the chunks of bn rows of the sorted FP32 copy xs ([n][DMAX], zero
// beyond the data's features)
hipError_t launch_chunk_balls(const float* xs, int64_t n, int bn, float* balls, hipStream_t s);

// Component-aligned chunk tables of the sorted order (see CandArgs) and the
// bounding balls of their chunks and super-chunks.
struct ChunkTabs {
    int32_t* segstart;   // [n + 1]
    int32_t* ccnt;       // [n] chunks per segment
    int32_t* scnt;       // [n] super-chunks per segment
    int32_t* cbase;      // [n] first chunk of each segment
    int32_t* sbase;      // [n] first super-chunk of each segment
    int32_t* cstart;     // [n + 1]
    int32_t* csup;       // [n]
    int32_t* sfirst;     // [n + 1]
    int32_t* spos;       // [n + 1] first sorted position of each super-chunk
    int32_t* pos2chunk;  // [n]
    int32_t* tabn;       // [2]
    int32_t* ccomp;      // [n] component (segment) of each chunk
    int32_t* scomp;      // [n] and of each super-chunk
};
hipError_t launch_chunk_tables(const int32_t* seg, int64_t n, int64_t nseg, const ChunkTabs& t,
                               const float* xs, float* balls, float* sballs, void* scan_temp,
                               hipStream_t s);

// Many instances in one point set (spatial.hip).
struct InstDev {
    const float* X;
    int64_t ld;
    int32_t d;
    int32_t pad_;
};
hipError_t launch_concat(const InstDev* inst, const int32_t* off, int ninst, int64_t n, int dmax,
                         float* Xc, hipStream_t s);
hipError_t launch_instance_major(int32_t* perm0, int32_t* rank0, const int32_t* off, int ninst,
                                 int64_t n, SortRec* recA, SortRec* recB, void* radix_temp,
                                 hipStream_t s);
hipError_t launch_tiles(const int32_t* rows, int32_t row0, int64_t nb, const int32_t* off, int ninst,
                        int bm, int32_t* flag, int32_t* tstart, int32_t* ntiles_dev, void* scan_temp,
                        hipStream_t s);
hipError_t launch_tile_desc(const int32_t* tstart, int ntiles, const int32_t* rows, int32_t row0,
                            int64_t nb, const int32_t* off, int ninst, int bm, int4* tiles,
                            hipStream_t s);
// Device-sized forms: the rows are the first d->n_rows of the list (at most
// cap); the tile count goes to d->n_tiles (at most max_tiles).
hipError_t launch_tiles_dev(const int32_t* rows, int64_t cap, const int32_t* off, int ninst, int bm,
                            int32_t* flag, int32_t* tstart, LaunchDesc* d, void* scan_temp,
                            hipStream_t s);
hipError_t launch_tile_desc_dev(const int32_t* tstart, int max_tiles, const int32_t* rows,
                                const int32_t* off, int ninst, int bm, int4* tiles,
                                const LaunchDesc* d, hipStream_t s);
hipError_t launch_write_edges_batched(const SortRec* sorted, int64_t ne, const int32_t* off, int ninst,
                                      SortRec* recA, SortRec* recB, void* radix_temp,
                                      nnm_edge* const* out, int metric, hipStream_t s);
// rows scaled to unit Euclidean length (the cosine metric), out [n][d]
hipError_t launch_normalize_rows(const float* X, int64_t n, int d, int64_t ld, float* out,
                                 hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v,
                           int64_t n, hipStream_t s);

}  // namespace nnm
