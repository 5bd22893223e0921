// driver.hip -- host orchestration behind knn_build and mst_build.
//
// mst_build runs merge rounds until one component is left:
//   round 0   every row is scanned (candidate pass with depth k, FP64
//             rescoring) -> exact k-nearest-neighbour prefix of every point;
//   round r   cursors skip list entries now inside the point's component;
//             components take the minimum over their rows; rows whose list
//             is used up are rescanned only if their lower bound can still
//             beat their component's best (the rescan only looks below that
//             best); components hook to their partners, mutual pairs are
//             resolved, trees collapse by pointer jumping; points are then
//             re-sorted by component so tiles of rows and chunks of columns
//             rarely share a component.
// The N-1 edges collected on the way are sorted by key at the end.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <mutex>
#include <vector>

#include "cand_common.h"

namespace nnm {
namespace {

struct Counters {
    int32_t ctr[8];                 // [0] edges [1] roots [2] jump misses
    int32_t rcount;                 // rows to rescan
    int32_t over;                   // overflowed rows in the last batch
    int32_t tcount;                 // tiles of the last batch
    int32_t pad_[5];
    // graph-replayed rounds: row counts kept on the device
    int32_t dc[8];                  // [0] rows to scan [1] representatives
                                    // [2] representatives scanned [3] overflowed rows
    int32_t pad2_[8];
    // totals spread over NSPREAD slots on separate cache lines (slot =
    // workgroup mod NSPREAD), so that no address or line takes an atomic
    // from every workgroup
    unsigned long long pairs[NSPREAD * SPREAD_STRIDE];
    unsigned long long survivors[NSPREAD * SPREAD_STRIDE];
    unsigned long long err_bits[4];
};

unsigned long long spread_sum(const unsigned long long* v)
{
    unsigned long long t = 0;
    for (int i = 0; i < NSPREAD; ++i) t += v[i * SPREAD_STRIDE];
    return t;
}

// Component-aligned column chunks are used in the merge rounds whose
// components hold ALIGN_AVG points or more on average (fewer, larger
// components: few partly filled chunks).
constexpr int64_t ALIGN_AVG = 512;

struct Plan {
    int64_t n = 0;
    int d = 0;
    int64_t ld = 0;
    int opkind = OP_FP32;
    int exact = 0;
    int k = 6;
    int S = 256;
    int64_t rmax = 0;               // rows per candidate launch
    int op_bytes = 64;
    bool mst = true;
    int S_global = 256;             // survivor cap of the global frame
    int L1 = 1, L2 = 1;             // fine / coarse landmarks of the spatial order
    int ninst = 1;                  // instances in the point set (batched calls)
    bool local = false;             // BF16 in the super-chunk frames (not exact data)
    bool keep_e = false;            // workspace holds t + E(t) per survivor (BF16 asked for)
    int metric = NNM_METRIC_EUCLIDEAN;  // nnm_metric asked for
    // the metric of the keys the kernels compute: the cosine metric runs as
    // the Euclidean one on rows scaled to unit length
    int key_metric() const { return metric == NNM_METRIC_COSINE ? NNM_METRIC_EUCLIDEAN : metric; }
};

struct WS {
    StageStats* stats;
    Counters* ctr;
    float* centre;
    void* opR; void* opC; PointConst* pc;
    void* opRs; void* opCs; PointConst* pcs;
    float* xs;
    int32_t* compS; int32_t* perm; int32_t* comp; int32_t* parent;
    int32_t* cidx; double* cs; int32_t* clen; int32_t* ccur; double* clb; int32_t* cflag;
    double* rbest_s; int32_t* rbest_j; int32_t* rstat;
    unsigned long long* cbest_s; unsigned long long* cbest_p;
    int32_t* rflag; int32_t* rlist; double* u0s;
    int32_t* surv_cnt; int32_t* surv_j; float* surv_t; float* surv_e;
    int32_t* overflow_list;
    SortRec* edges; SortRec* srtA; SortRec* srtB;
    void* scan_temp; void* radix_temp;
    int32_t* perm0; int32_t* rank0; int32_t* ckey; int32_t* flag; int32_t* excl;
    float* balls;
    float* sballs;
    float4* cmaxT;                  // BF16 super-chunk frames: per-chunk column maxima
    ChunkTabs tabs;
    uint32_t* gT; uint32_t* gU;
    uint32_t* tfin;
    void* spatial_temp;
    double* u0b; int32_t* oflag; int32_t* olist; int32_t* rep_pos; int32_t* rflag2;
    int4* tiles; int32_t* tflag; int32_t* tstart;
    float* Xcat; int32_t* inst_off; InstDev* inst; nnm_edge** outp;
    LaunchDesc* desc;
    float* Xn;                      // cosine metric, one instance: the scaled rows [n][d]
};

struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

size_t carve(const Plan& p, void* base, WS* w)
{
    Carver c{(char*)base};
    const size_t n = (size_t)p.n;
    const bool mfma = p.opkind != OP_FP32;
    w->stats = c.take<StageStats>(1);
    w->ctr = c.take<Counters>(1);
    w->centre = c.take<float>(DMAX);
    w->opR = mfma ? c.take<char>(n * p.op_bytes) : nullptr;
    w->opC = mfma ? c.take<char>(n * p.op_bytes) : nullptr;
    w->pc = c.take<PointConst>(n);
    w->opRs = mfma ? c.take<char>(n * p.op_bytes) : nullptr;
    w->opCs = mfma ? c.take<char>(n * p.op_bytes) : nullptr;
    w->pcs = c.take<PointConst>(n);
    w->xs = c.take<float>(n * DMAX);   // also the source of the BF16 super-chunk operands
    w->compS = c.take<int32_t>(n);
    w->perm = c.take<int32_t>(n);
    w->comp = c.take<int32_t>(n);
    w->parent = c.take<int32_t>(n);
    w->cidx = c.take<int32_t>(n * p.k);
    w->cs = c.take<double>(n * p.k);
    w->clen = c.take<int32_t>(n);
    w->ccur = c.take<int32_t>(n);
    w->clb = c.take<double>(n);
    w->cflag = c.take<int32_t>(n);
    w->rbest_s = c.take<double>(n);
    w->rbest_j = c.take<int32_t>(n);
    w->rstat = c.take<int32_t>(n);
    w->cbest_s = c.take<unsigned long long>(n);
    w->cbest_p = c.take<unsigned long long>(n);
    w->rflag = c.take<int32_t>(n);
    w->rlist = c.take<int32_t>(n);
    w->u0s = c.take<double>(n);
    w->surv_cnt = c.take<int32_t>((size_t)p.rmax);
    w->surv_j = c.take<int32_t>((size_t)p.rmax * p.S);
    w->surv_t = c.take<float>((size_t)p.rmax * p.S);
    w->surv_e = p.keep_e ? c.take<float>((size_t)p.rmax * p.S) : nullptr;
    w->overflow_list = c.take<int32_t>((size_t)p.rmax);
    w->edges = c.take<SortRec>(n);
    w->srtA = c.take<SortRec>(n);
    w->srtB = c.take<SortRec>(n);
    w->scan_temp = c.take<char>(scan_temp_bytes((int64_t)n));
    w->radix_temp = c.take<char>(radix_temp_bytes((int64_t)n));
    w->perm0 = c.take<int32_t>(n);
    w->rank0 = c.take<int32_t>(n);
    w->ckey = c.take<int32_t>(n);
    w->flag = c.take<int32_t>(n);
    w->excl = c.take<int32_t>(n);
    // fixed chunks, or component-aligned ones (at most n / ALIGN_AVG
    // components, each adding at most one chunk and one super-chunk)
    const size_t nseg_max = n / ALIGN_AVG + 1;
    const size_t nch_max = (n + CHUNK - 1) / CHUNK + nseg_max;
    const size_t nsc_max = (n + CHUNK * SUPER - 1) / (CHUNK * SUPER) + nseg_max;
    w->balls = c.take<float>(nch_max * BALL_STRIDE);
    w->sballs = c.take<float>(nsc_max * BALL_STRIDE);
    w->cmaxT = c.take<float4>(nch_max);
    w->tabs.segstart = c.take<int32_t>(nseg_max + 1);
    w->tabs.ccnt = c.take<int32_t>(nseg_max);
    w->tabs.scnt = c.take<int32_t>(nseg_max);
    w->tabs.cbase = c.take<int32_t>(nseg_max);
    w->tabs.sbase = c.take<int32_t>(nseg_max);
    w->tabs.cstart = c.take<int32_t>(nch_max + 1);
    w->tabs.csup = c.take<int32_t>(nch_max);
    w->tabs.sfirst = c.take<int32_t>(nsc_max + 1);
    w->tabs.spos = c.take<int32_t>(nsc_max + 1);
    w->tabs.pos2chunk = c.take<int32_t>(n);
    w->tabs.tabn = c.take<int32_t>(2);
    w->tabs.ccomp = c.take<int32_t>(nch_max);
    w->tabs.scomp = c.take<int32_t>(nsc_max);
    w->gT = c.take<uint32_t>((size_t)p.rmax);
    w->gU = c.take<uint32_t>((size_t)p.rmax);
    w->tfin = c.take<uint32_t>((size_t)p.rmax);
    w->spatial_temp = c.take<char>(spatial_temp_bytes((int64_t)n, p.L1, p.L2));
    w->u0b = c.take<double>(n);
    w->oflag = c.take<int32_t>(n);
    w->olist = c.take<int32_t>(n);
    w->rep_pos = c.take<int32_t>(n);
    w->rflag2 = c.take<int32_t>(n);
    w->tiles = c.take<int4>((size_t)p.rmax);
    w->tflag = c.take<int32_t>((size_t)p.rmax);
    w->tstart = c.take<int32_t>((size_t)p.rmax);
    const bool multi = p.ninst > 1;
    w->Xcat = multi ? c.take<float>(n * (size_t)p.d) : nullptr;
    w->inst_off = c.take<int32_t>((size_t)p.ninst + 1);
    w->inst = multi ? c.take<InstDev>((size_t)p.ninst) : nullptr;
    w->outp = multi ? c.take<nnm_edge*>((size_t)p.ninst) : nullptr;
    w->desc = c.take<LaunchDesc>(1);
    w->Xn = (p.metric == NNM_METRIC_COSINE && !multi) ? c.take<float>(n * (size_t)p.d) : nullptr;
    return c.off + 256;
}

int pow2_at_least(int64_t v)
{
    int r = 64;
    while (r < v && r < SMAX) r <<= 1;
    return r;
}

nnm_status plan_common(int64_t n, int32_t d, int32_t k, const nnm_options* opt, bool mst, Plan* p)
{
    if (n < 1 || n > (int64_t)0x7FFFFFF0 || d < 1 || d > DMAX) return NNM_EINVAL;
    nnm_options o;
    nnm_default_options(&o);
    if (opt) o = *opt;
    p->n = n;
    p->d = d;
    p->mst = mst;
    if (o.metric < NNM_METRIC_EUCLIDEAN || o.metric > NNM_METRIC_COSINE) return NNM_EINVAL;
    p->metric = o.metric;
    // L1 and L-infinity have no dot-product form: the FP32 vector path only
    const bool vec_only = o.metric == NNM_METRIC_L1 || o.metric == NNM_METRIC_LINF;
    if (vec_only && o.precision != NNM_PREC_FP32 && o.precision != NNM_PREC_AUTO)
        return NNM_EUNSUPPORTED;
    // workspace is sized for the widest operand so the precision can be
    // settled after the data have been inspected
    p->opkind = (o.precision == NNM_PREC_FP32 || vec_only) ? OP_FP32 : OP_FP16;
    if (o.precision == NNM_PREC_AUTO && d > DMAX_MFMA) p->opkind = OP_FP32;
    // cache depth: the matrix-core paths' survivor band grows with k, so
    // they keep fewer neighbours than the FP32 path (measured best on the 2M
    // workload: 6, and 8)
    const bool deep = p->opkind == OP_FP32;
    p->k = k > 0 ? k : (o.knn_k > 0 ? o.knn_k : (deep ? 8 : 6));
    if (p->k < 1 || p->k > KMAX) return NNM_EINVAL;
    if (o.precision != NNM_PREC_FP32 && o.precision != NNM_PREC_AUTO && d > DMAX_MFMA)
        return NNM_EUNSUPPORTED;
    p->op_bytes = 64;
    // the super-chunk frames (BF16 on data that is not an integer grid)
    // keep the bound they applied to each survivor for the error report
    p->keep_e = o.precision == NNM_PREC_BF16;
    int S = o.survivor_cap;
    if (S <= 0) {
        const double lnr = log((double)std::max<int64_t>(n / std::max(p->k, 1), 2));
        S = pow2_at_least((int64_t)(p->k * (4.0 + lnr) + 32));
    }
    if (S < 64) S = 64;
    if (S > SMAX) S = SMAX;
    S = pow2_at_least(S);
    p->S_global = S;
    // BF16 on data that is not an integer grid works in the super-chunk
    // frames (see stage); its margin is wider, so it keeps 2x the survivors
    // per row (measured best on the 2M workload)
    if (o.precision == NNM_PREC_BF16 && o.survivor_cap <= 0) S = S * 2 < SMAX ? S * 2 : SMAX;
    p->S = S;
    // survivor buffers of at most 2^30 entries (8 GB; 12 GB with the BF16
    // bounds): 4M rows at S = 256 in one launch (a split launch pays two
    // tails and narrower column splits)
    int64_t rmax = ((int64_t)1 << 30) / S;
    if (rmax > n) rmax = n;
    if (rmax < 1) rmax = 1;
    p->rmax = rmax;
    int64_t l1 = n / 384;
    if (l1 < 1) l1 = 1;
    if (l1 > 16384) l1 = 16384;
    int64_t l2 = (int64_t)llround(sqrt((double)l1));
    if (l2 < 1) l2 = 1;
    if (l2 > 256) l2 = 256;
    p->L1 = (int)l1;
    p->L2 = (int)l2;
    return NNM_OK;
}

struct Timer {
    bool on;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    double* acc;
    Timer(bool on_, hipStream_t s_, double* acc_) : on(on_), s(s_), acc(acc_)
    {
        if (on) {
            hipEventCreate(&a);
            hipEventCreate(&b);
            hipEventRecord(a, s);
        }
    }
    ~Timer()
    {
        if (on) {
            hipEventRecord(b, s);
            hipEventSynchronize(b);
            float ms = 0.f;
            hipEventElapsedTime(&ms, a, b);
            *acc += ms;
            hipEventDestroy(a);
            hipEventDestroy(b);
        }
    }
};

#define HIP_TRY(x)                                 \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return NNM_EDEVICE;  \
    } while (0)

struct Run {
    Plan p;
    WS w;
    hipStream_t s;
    nnm_report* rep;
    bool timers = false;    // HIP-event phase timers (with a report, unless the caller can't allocate)
    nnm_options o;
    BoundConst bc;
    float sigma = 1.f;
    int splits_opt = 0;
    int round = 0;          // current merge round (per-round report entries)
    int kk = 0;             // neighbours sought by the current scan (0 = the cache depth)
    bool fp32_scan = false; // the current scan uses the FP32 kernel whatever the precision
    bool aligned = false;   // this round's column chunks follow the components (w.tabs)
    int64_t max_inst = 0;   // points of the largest instance
};

int ceil_log2(int64_t v)
{
    int r = 0;
    while (((int64_t)1 << r) < v) ++r;
    return r;
}

// Inspect the data (finite, ranges, integer grid), settle the precision and
// write the operands.
nnm_status stage(Run& R, const float* X)
{
    Plan& p = R.p;
    WS& w = R.w;
    StageStats init;
    for (int f = 0; f < DMAX; ++f) { init.fmin[f] = 0xFFFFFFFFu; init.fmax[f] = 0u; }
    init.nonfinite = 0;
    init.nonint = 0;
    for (int e = 0; e < 4; ++e) init.colmax[e] = 0u;
    init.pad_[0] = init.pad_[1] = 0;
    HIP_TRY(hipMemcpyAsync(w.stats, &init, sizeof(init), hipMemcpyHostToDevice, R.s));
    HIP_TRY(hipMemsetAsync(w.ctr, 0, sizeof(Counters), R.s));
    HIP_TRY(launch_stage_stats(X, p.n, p.d, p.ld, w.stats, R.s));
    StageStats st;
    HIP_TRY(hipMemcpyAsync(&st, w.stats, sizeof(st), hipMemcpyDeviceToHost, R.s));
    HIP_TRY(hipStreamSynchronize(R.s));
    if (st.nonfinite) return NNM_ENONFINITE;
    const bool intgrid = !st.nonint && p.d <= DMAX_MFMA;
    const int prec = (p.metric == NNM_METRIC_L1 || p.metric == NNM_METRIC_LINF) ? NNM_PREC_FP32
                                                                               : R.o.precision;
    switch (prec) {
    case NNM_PREC_FP32: p.opkind = OP_FP32; break;
    case NNM_PREC_BF16: p.opkind = OP_BF16; break;
    case NNM_PREC_FP16: p.opkind = OP_FP16; break;
    case NNM_PREC_FP8:
        if (!intgrid) return NNM_EUNSUPPORTED;
        p.opkind = OP_FP8;
        break;
    case NNM_PREC_AUTO:
    default:
        p.opkind = intgrid ? OP_FP8 : (p.d <= DMAX_MFMA ? OP_FP16 : OP_FP32);
        break;
    }
    p.exact = (p.opkind != OP_FP32 && intgrid) ? 1 : 0;
    // BF16 keeps 8 bits: relative to the data's centre its error would swamp
    // nearest-neighbour distances, so it works in the frames of the column
    // super-chunks, with the rows split into two BF16 halves
    p.local = p.opkind == OP_BF16 && !p.exact;
    // BF16 on an integer grid is exact in the global frame: the global cap
    // (the buffers were sized for the larger BF16 one)
    if (!p.local) p.S = p.S_global;
    p.op_bytes = (p.opkind == OP_FP8) ? 32 : 64;
    R.bc = BoundConst{};
    R.sigma = 1.f;
    if (p.opkind == OP_FP32) {
        R.bc.sigma2 = 1.f;
        return NNM_OK;
    }
    float centre[DMAX] = {0};
    float sigma = 1.f;
    if (!p.exact) {
        double span = 0.0;
        for (int f = 0; f < p.d; ++f) {
            auto dec = [](uint32_t e) {
                uint32_t u = (e & 0x80000000u) ? (e & 0x7FFFFFFFu) : ~e;
                float v;
                memcpy(&v, &u, 4);
                return v;
            };
            const float lo = dec(st.fmin[f]), hi = dec(st.fmax[f]);
            centre[f] = (float)(0.5 * ((double)lo + (double)hi));
            span = std::max(span, std::max(fabs((double)hi - centre[f]), fabs((double)lo - centre[f])));
        }
        if (span > 0.0) {
            int e = 0;
            frexp(span, &e);     // span = m * 2^e, m in [0.5, 1)
            if (e < -60 || e > 60) {
                // sigma^2 would leave the normal FP32 range: the matrix-core
                // formats cannot carry such data faithfully
                if (R.o.precision != NNM_PREC_AUTO) return NNM_EUNSUPPORTED;
                p.opkind = OP_FP32;
                p.exact = 0;
                p.local = false;
                R.bc.sigma2 = 1.f;
                return NNM_OK;
            }
            sigma = (float)ldexp(1.0, -e);
        }
    }
    R.sigma = sigma;
    if (!p.local) {
        // global operands (exact integer data): one frame for every pair
        HIP_TRY(hipMemcpyAsync(w.centre, centre, sizeof(centre), hipMemcpyHostToDevice, R.s));
        HIP_TRY(launch_stage_operands(X, p.n, p.d, p.ld, p.opkind, p.exact, w.centre, sigma, w.opR,
                                      w.opC, w.pc, w.stats, R.s));
        HIP_TRY(hipMemcpyAsync(&st, w.stats, sizeof(st), hipMemcpyDeviceToHost, R.s));
        HIP_TRY(hipStreamSynchronize(R.s));
        float cm[4];
        memcpy(cm, st.colmax, sizeof(cm));
        R.bc.colQ = cm[0];
        R.bc.colP = cm[1];
        R.bc.colRho = cm[2];
        R.bc.colEta = cm[3];
    }
    // FP32 accumulation of 32 exact products (one MFMA), or of 64 in two
    // chained MFMAs (the split rows): any order, even truncating
    R.bc.gamma = p.exact ? 0.f : (float)((p.local && p.opkind == OP_BF16 ? 67.0 : 33.0) * 0x1p-23);
    R.bc.sigma2 = sigma * sigma;
    R.bc.exact = p.exact;
    return NNM_OK;
}

MergeArgs merge_args(Run& R)
{
    MergeArgs m{};
    m.n = R.p.n;
    m.k = R.p.k;
    m.comp = R.w.comp;
    m.parent = R.w.parent;
    m.cidx = R.w.cidx;
    m.cs = R.w.cs;
    m.clen = R.w.clen;
    m.ccur = R.w.ccur;
    m.clb = R.w.clb;
    m.cflag = R.w.cflag;
    m.rbest_s = R.w.rbest_s;
    m.rbest_j = R.w.rbest_j;
    m.rstat = R.w.rstat;
    m.cbest_s = R.w.cbest_s;
    m.cbest_p = R.w.cbest_p;
    m.perm = R.w.perm;
    m.rflag = R.w.rflag;
    m.u0s = R.w.u0s;
    m.sigma2 = R.bc.sigma2;
    m.disable_prune = R.o.disable_prune;
    m.edges = R.w.edges;
    m.counters = R.w.ctr->ctr;
    return m;
}

// Order points by component (components by their earliest spatial position,
// members by spatial position); gather the operands in that order and
// compute the bounding ball of every chunk.
nnm_status sort_points(Run& R, const float* X, int64_t ncomp)
{
    Plan& p = R.p;
    WS& w = R.w;
    HIP_TRY(launch_component_order(w.comp, w.perm0, w.rank0, p.n, w.ckey, w.srtA, w.srtB, w.perm,
                                   w.compS, w.flag, w.excl, w.radix_temp, w.scan_temp, R.s));
    // the sorted FP32 copy (tile balls; the BF16 super-chunk operands) ...
    HIP_TRY(launch_gather_points(p.n, OP_FP32, w.perm, w.opR, w.opC, w.pc, X, p.d, p.ld, w.comp,
                                 w.opRs, w.opCs, w.pcs, w.xs, w.compS, R.s));
    // ... and the precomputed operands where one global frame is used
    if (p.opkind != OP_FP32 && !p.local)
        HIP_TRY(launch_gather_points(p.n, p.opkind, w.perm, w.opR, w.opC, w.pc, X, p.d, p.ld, w.comp,
                                     w.opRs, w.opCs, w.pcs, w.xs, w.compS, R.s));
    // balls from the sorted FP32 copy (the same values, contiguous rows)
    if (R.aligned) {
        HIP_TRY(launch_chunk_tables(w.compS, p.n, ncomp, w.tabs, w.xs, w.balls, w.sballs, w.scan_temp,
                                    R.s));
    } else {
        HIP_TRY(launch_chunk_balls(w.xs, p.n, CHUNK, w.balls, R.s));
        HIP_TRY(launch_chunk_balls(w.xs, p.n, CHUNK * SUPER, w.sballs, R.s));
    }
    // BF16: the column operands in the frames of this order's super-chunks
    if (p.local) {
        const int64_t nch_bound = R.aligned ? (p.n + CHUNK - 1) / CHUNK + ncomp : 0;
        HIP_TRY(launch_split_columns(p.opkind, w.xs, p.n, p.d, R.sigma, R.aligned ? w.tabs.cstart : nullptr,
                                     w.tabs.csup, w.tabs.tabn, nch_bound, w.sballs, w.opCs, w.cmaxT, R.s));
    }
    return NNM_OK;
}

nnm_status spatial_order(Run& R, const float* X)
{
    Plan& p = R.p;
    WS& w = R.w;
    HIP_TRY(launch_spatial_order(X, p.n, p.d, p.ld, p.L1, p.L2, w.perm0, w.rank0, w.srtA, w.srtB,
                                 w.spatial_temp, R.s));
    if (p.ninst > 1)
        HIP_TRY(launch_instance_major(w.perm0, w.rank0, w.inst_off, p.ninst, p.n, w.srtA, w.srtB,
                                      w.radix_temp, R.s));
    return NNM_OK;
}

// Column splits per row tile: enough workgroups to fill the chip twice
// over for the bounded scans of the merge rounds; the first round (every
// row's k nearest, hit-heavy) does better with half as many (measured on the
// 2M workload).
int pick_splits(const Run& R, int64_t rows, bool bounded)
{
    if (R.o.col_splits > 0) return R.o.col_splits;
    const int64_t bm = 256;
    const int64_t tiles = (rows + bm - 1) / bm;
    const int64_t target = bounded ? (R.o.split_target > 0 ? R.o.split_target : 8192)
                                   : (R.o.split_target0 > 0 ? R.o.split_target0 : 4096);
    int64_t want = (target + tiles - 1) / tiles;
    int64_t cap = R.p.n / 65536;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    if (want > 64) want = 64;
    return (int)want;
}

// One candidate launch + FP64 rescoring for nb rows (a row list of sorted
// positions, or row0 + slot).  level 1: overflowed rows are flagged in
// w.oflag with a bound in w.u0b; level 2: they get the exact full scan.
nnm_status scan_batch(Run& R, const float* X, const int32_t* rows, int32_t row0, int64_t nb,
                      const double* u0, bool final_pass, int32_t* n_over)
{
    Plan& p = R.p;
    WS& w = R.w;
    HIP_TRY(hipMemsetAsync(w.surv_cnt, 0, sizeof(int32_t) * (size_t)nb, R.s));
    const bool use32 = p.opkind == OP_FP32 || R.fp32_scan;
    CandArgs a{};
    a.opR = w.opRs;
    a.opC = w.opCs;
    a.xs = w.xs;
    a.pc = w.pcs;
    a.compS = w.compS;
    a.rows = rows;
    a.row0 = row0;
    a.u0 = u0;
    a.n_rows = (int32_t)nb;
    a.np = (int32_t)p.n;
    a.d = p.d;
    const int kk = R.kk > 0 ? R.kk : p.k;
    a.k = kk;
    a.S = p.S;
    a.col_splits = pick_splits(R, nb, u0 != nullptr && R.round > 0);
    if (p.ninst > 1) {
        // tiles never mix instances; each pairs only with its own instance
        int32_t nt = 0;
        HIP_TRY(launch_tiles(rows, row0, nb, w.inst_off, p.ninst, 256, w.tflag, w.tstart,
                             &w.ctr->tcount, w.scan_temp, R.s));
        HIP_TRY(hipMemcpyAsync(&nt, &w.ctr->tcount, sizeof(int32_t), hipMemcpyDeviceToHost, R.s));
        HIP_TRY(hipStreamSynchronize(R.s));
        HIP_TRY(launch_tile_desc(w.tstart, nt, rows, row0, nb, w.inst_off, p.ninst, 256, w.tiles, R.s));
        a.tiles = w.tiles;
        a.n_tiles = nt;
        a.col_splits = pick_splits(R, (int64_t)nt * 256, u0 != nullptr && R.round > 0);
    }
    a.bc = R.bc;
    a.metric = p.key_metric();
    a.surv_cnt = w.surv_cnt;
    a.surv_j = w.surv_j;
    a.surv_t = w.surv_t;
    a.surv_e = w.surv_e;
    a.pairs = w.ctr->pairs;
    a.X = X;
    a.ld = p.ld;
    a.perm = w.perm;
    a.balls = w.balls;
    a.sballs = w.sballs;
    a.cmaxT = w.cmaxT;
    if (R.aligned) {
        a.cstart = w.tabs.cstart;
        a.csup = w.tabs.csup;
        a.sfirst = w.tabs.sfirst;
        a.pos2chunk = w.tabs.pos2chunk;
        a.tabn = w.tabs.tabn;
        a.spos = w.tabs.spos;
        a.ccomp = w.tabs.ccomp;
        a.scomp = w.tabs.scomp;
    }
    a.prune = R.o.disable_prune ? 0 : 1;
    a.local = (p.local && !use32) ? 1 : 0;
    a.share = a.col_splits > 1 ? 1 : 0;
    a.gT = w.gT;
    // final thresholds (global frame) or final key bounds (super-chunk frames)
    const bool use_tfin = !use32;
    a.tfin = use_tfin ? w.tfin : nullptr;
    if (use_tfin) HIP_TRY(launch_fill_i32((int32_t*)w.tfin, 0x7F800000, nb, R.s));
    a.gU = w.gU;
    if (a.share) {
        HIP_TRY(launch_fill_i32((int32_t*)w.gT, 0x7F800000, nb, R.s));
        HIP_TRY(launch_fill_i32((int32_t*)w.gU, 0x7F800000, nb, R.s));
    }
    {
        double ms = 0.0;
        {
            Timer t(R.timers, R.s, &ms);
            if (use32) HIP_TRY(launch_cand_fp32(a, R.s));
            else HIP_TRY(launch_cand_mfma(p.opkind, a, R.s));
        }
        if (R.rep) {
            R.rep->ms_candidates += ms;
            R.rep->cand_ms_per_round[R.round < 32 ? R.round : 31] += ms;
        }
    }
    RescoreArgs r{};
    r.X = X;
    r.xs = w.xs;
    r.ld = p.ld;
    r.d = p.d;
    r.n_rows = (int32_t)nb;
    r.k = kk;
    r.kstride = p.k;
    r.S = p.S;
    r.rows = rows;
    r.row0 = row0;
    r.perm = w.perm;
    r.tfin = a.tfin;
    r.comp = w.comp;
    r.surv_cnt = w.surv_cnt;
    r.surv_j = w.surv_j;
    r.surv_t = w.surv_t;
    r.u0 = u0;
    // FP32 candidates are in data units
    r.inv_sigma2 = use32 ? 1.0 : 1.0 / (double)R.bc.sigma2;
    r.sigma2 = use32 ? 1.f : R.bc.sigma2;
    r.force_fallback = R.o.force_fallback;
    r.np = p.n;
    r.inst_off = w.inst_off;
    r.ninst = (int32_t)p.ninst;
    r.cidx = w.cidx;
    r.cs = w.cs;
    r.clen = w.clen;
    r.ccur = w.ccur;
    r.clb = w.clb;
    r.cflag = w.cflag;
    r.overflow_rows = &w.ctr->over;
    r.level = final_pass ? 2 : 1;
    // the tree only needs exact prefixes, so an overflowed row is re-scanned
    // below its 4th key; knn_build needs all k
    r.kb = p.mst ? std::min(kk, 4) : kk;
    r.u0b = w.u0b;
    r.oflag = w.oflag;
    r.survivors = w.ctr->survivors;
    r.err_bits = w.ctr->err_bits;
    r.bound_mode = use32 ? BOUND_FP32 : (p.exact ? BOUND_EXACT : (a.local ? BOUND_LOCAL : BOUND_GLOBAL));
    r.pcs = w.pcs;
    r.bc = R.bc;
    r.surv_e = w.surv_e;
    r.metric = p.key_metric();
    int32_t over = 0;
    {
        Timer t(R.timers, R.s, R.rep ? &R.rep->ms_rescore : nullptr);
        HIP_TRY(hipMemsetAsync(&w.ctr->over, 0, sizeof(int32_t), R.s));
        HIP_TRY(launch_rescore(r, w.overflow_list, R.s));
        HIP_TRY(hipMemcpyAsync(&over, &w.ctr->over, sizeof(int32_t), hipMemcpyDeviceToHost, R.s));
        HIP_TRY(hipStreamSynchronize(R.s));
        // rows sent straight to the exact scan
        if (over > 0 && (final_pass || R.o.force_fallback))
            HIP_TRY(launch_fallback(r, w.overflow_list, over, R.s));
    }
    if (R.rep) {
        R.rep->rows_scanned += nb;
        R.rep->cand_launches += 1;
        const int rd = R.round < 32 ? R.round : 31;
        if (final_pass || R.o.force_fallback) {
            R.rep->overflow_rows += over;
            R.rep->exact_per_round[rd] += over;
        } else {
            R.rep->over_per_round[rd] += over;
        }
    }
    *n_over = over;
    return NNM_OK;
}

// Candidate pass + FP64 rescoring for rows rows[0..count) (sorted positions,
// ascending) or, with rows == NULL, for positions 0..count-1.  Rows whose
// survivor list overflows are scanned again below the bound their first
// survivors give (each pass tightens it); after OVER_PASSES such passes the
// rest get the exact full-row scan.
constexpr int OVER_PASSES = 4;

nnm_status scan_rows(Run& R, const float* X, const int32_t* rows, int64_t count, bool use_u0)
{
    Plan& p = R.p;
    WS& w = R.w;
    for (int64_t b0 = 0; b0 < count; b0 += p.rmax) {
        const int64_t nb = std::min<int64_t>(p.rmax, count - b0);
        HIP_TRY(launch_fill_i32(w.oflag, 0, p.n, R.s));
        int32_t over = 0;
        nnm_status st = scan_batch(R, X, rows ? rows + b0 : nullptr, rows ? 0 : (int32_t)b0, nb,
                                   use_u0 ? w.u0s : nullptr, false, &over);
        if (st != NNM_OK) return st;
        for (int pass = 1; over > 0 && !R.o.force_fallback; ++pass) {
            // overflowed rows (flagged in oflag, bound in u0b): scan again
            int32_t on = 0;
            HIP_TRY(launch_compact(w.oflag, p.n, w.olist, &w.ctr->rcount, w.scan_temp, R.s));
            HIP_TRY(hipMemcpyAsync(&on, &w.ctr->rcount, sizeof(int32_t), hipMemcpyDeviceToHost, R.s));
            HIP_TRY(hipStreamSynchronize(R.s));
            HIP_TRY(launch_fill_i32(w.oflag, 0, p.n, R.s));
            if (R.rep) R.rep->rescanned_bounded += on;
            const bool final_pass = pass >= OVER_PASSES;
            // rows whose matrix-core survivors keep overflowing are
            // rescanned with the FP32 kernel: its margin is a few units in
            // the last place, where the low-precision margin may hold
            // thousands of columns (points clustered far tighter than the
            // data's extent).  The first rescan stays on the matrix cores,
            // which settle milder overflows faster, and so does a second one
            // of a few rows (too few tiles to hide the slower kernel's
            // sweep).  Exact integer data has no margin; there only ties
            // overflow.
            R.fp32_scan = p.opkind != OP_FP32 && !p.exact && (pass >= 3 || (pass == 2 && on >= 4096));
            over = 0;
            for (int64_t c0 = 0; c0 < on; c0 += p.rmax) {
                const int64_t nc = std::min<int64_t>(p.rmax, on - c0);
                int32_t o2 = 0;
                st = scan_batch(R, X, w.olist + c0, 0, nc, w.u0b, final_pass, &o2);
                if (st != NNM_OK) { R.fp32_scan = false; return st; }
                if (!final_pass) over += o2;
            }
        }
        R.fp32_scan = false;
    }
    return NNM_OK;
}

// ---- device-sized scans (rounds replayed from a captured graph) ----------
//
// The same steps as scan_batch / scan_rows, sized on the device: each
// launch covers rows [off, off + rmax) of a row list whose length is a
// device count, and the overflow passes run a fixed number of times (empty
// passes do no work).  No host read, no memset: everything here may be
// captured.

// overflow passes after the first scan: bounded re-scans on the matrix
// cores, then the FP32 kernel, the last one with the exact scan for rows
// that overflow again (exact data: matrix cores throughout)
constexpr int DEV_PASSES = 3;

nnm_status scan_batch_dev(Run& R, const float* X, const int32_t* rows, const int32_t* count,
                          int32_t off, int kk, const double* u0, bool use32, int level)
{
    Plan& p = R.p;
    WS& w = R.w;
    LaunchDesc* D = w.desc;
    const int32_t cap = (int32_t)p.rmax;
    const int32_t target = u0 ? (R.o.split_target > 0 ? R.o.split_target : 8192)
                              : (R.o.split_target0 > 0 ? R.o.split_target0 : 4096);
    const bool use_tfin = !use32;
    HIP_TRY(launch_prep_launch(D, count, off, cap, p.n, target, R.o.col_splits, w.surv_cnt,
                               use_tfin ? w.tfin : nullptr, w.gT, w.gU, R.s));
    const int32_t* lrows = rows + off;
    CandArgs a{};
    a.opR = w.opRs;
    a.opC = w.opCs;
    a.xs = w.xs;
    a.pc = w.pcs;
    a.compS = w.compS;
    a.rows = lrows;
    a.row0 = 0;
    a.u0 = u0;
    a.n_rows = cap;
    a.np = (int32_t)p.n;
    a.d = p.d;
    a.k = kk;
    a.S = p.S;
    a.col_splits = 0;
    a.desc = D;
    if (p.ninst > 1) {
        const int64_t max_tiles = std::min<int64_t>(p.rmax, (int64_t)cap / 256 + p.ninst + 1);
        HIP_TRY(launch_tiles_dev(lrows, cap, w.inst_off, p.ninst, 256, w.tflag, w.tstart, D,
                                 w.scan_temp, R.s));
        HIP_TRY(launch_tile_desc_dev(w.tstart, (int)max_tiles, lrows, w.inst_off, p.ninst, 256,
                                     w.tiles, D, R.s));
        HIP_TRY(launch_desc_splits(D, p.n, target, R.o.col_splits, R.s));
        a.tiles = w.tiles;
    }
    a.bc = R.bc;
    a.metric = p.key_metric();
    a.surv_cnt = w.surv_cnt;
    a.surv_j = w.surv_j;
    a.surv_t = w.surv_t;
    a.surv_e = w.surv_e;
    a.pairs = w.ctr->pairs;
    a.X = X;
    a.ld = p.ld;
    a.perm = w.perm;
    a.balls = w.balls;
    a.sballs = w.sballs;
    a.cmaxT = w.cmaxT;
    a.prune = R.o.disable_prune ? 0 : 1;
    a.local = (p.local && !use32) ? 1 : 0;
    a.share = 1;
    a.gT = w.gT;
    a.gU = w.gU;
    a.tfin = use_tfin ? w.tfin : nullptr;
    if (use32) HIP_TRY(launch_cand_fp32(a, R.s));
    else HIP_TRY(launch_cand_mfma(p.opkind, a, R.s));
    RescoreArgs r{};
    r.X = X;
    r.xs = w.xs;
    r.ld = p.ld;
    r.d = p.d;
    r.n_rows = cap;
    r.k = kk;
    r.kstride = p.k;
    r.S = p.S;
    r.rows = lrows;
    r.row0 = 0;
    r.perm = w.perm;
    r.tfin = a.tfin;
    r.comp = w.comp;
    r.surv_cnt = w.surv_cnt;
    r.surv_j = w.surv_j;
    r.surv_t = w.surv_t;
    r.u0 = u0;
    r.inv_sigma2 = use32 ? 1.0 : 1.0 / (double)R.bc.sigma2;
    r.sigma2 = use32 ? 1.f : R.bc.sigma2;
    r.force_fallback = R.o.force_fallback;
    r.np = p.n;
    r.inst_off = w.inst_off;
    r.ninst = (int32_t)p.ninst;
    r.cidx = w.cidx;
    r.cs = w.cs;
    r.clen = w.clen;
    r.ccur = w.ccur;
    r.clb = w.clb;
    r.cflag = w.cflag;
    r.overflow_rows = &D->over;
    r.level = level;
    r.kb = p.mst ? std::min(kk, 4) : kk;
    r.u0b = w.u0b;
    r.oflag = w.oflag;
    r.survivors = w.ctr->survivors;
    r.err_bits = w.ctr->err_bits;
    r.bound_mode = use32 ? BOUND_FP32 : (p.exact ? BOUND_EXACT : (a.local ? BOUND_LOCAL : BOUND_GLOBAL));
    r.pcs = w.pcs;
    r.bc = R.bc;
    r.surv_e = w.surv_e;
    r.metric = p.key_metric();
    r.desc = D;
    HIP_TRY(launch_rescore(r, w.overflow_list, R.s));
    if (level == 2 || R.o.force_fallback)
        HIP_TRY(launch_fallback_dev(r, w.overflow_list, &D->over, R.s));
    return NNM_OK;
}

// scan_rows for the first *count entries of rows (at most n)
nnm_status scan_rows_dev(Run& R, const float* X, const int32_t* rows, const int32_t* count,
                         bool use_u0, int kk)
{
    Plan& p = R.p;
    WS& w = R.w;
    int32_t* on = &w.ctr->dc[3];
    // oflag is all zero here and after every compaction below
    for (int64_t b0 = 0; b0 < p.n; b0 += p.rmax) {
        nnm_status st = scan_batch_dev(R, X, rows, count, (int32_t)b0, kk, use_u0 ? w.u0s : nullptr,
                                       p.opkind == OP_FP32, 1);
        if (st != NNM_OK) return st;
        if (R.o.force_fallback) continue;
        for (int pass = 1; pass <= DEV_PASSES; ++pass) {
            HIP_TRY(launch_compact_clear(w.oflag, p.n, w.olist, on, w.scan_temp, R.s));
            // the rows overflowed in this batch: at most rmax of them
            const bool use32 = p.opkind == OP_FP32 || (!p.exact && pass >= 2);
            st = scan_batch_dev(R, X, w.olist, on, 0, kk, w.u0b, use32, pass == DEV_PASSES ? 2 : 1);
            if (st != NNM_OK) return st;
        }
    }
    return NNM_OK;
}

// One merge round (not the first) with every size on the device: the
// body of the round graph.
nnm_status round_dev(Run& R, const float* X)
{
    Plan& p = R.p;
    WS& w = R.w;
    const int64_t n = p.n;
    MergeArgs m = merge_args(R);
    int32_t* dc = w.ctr->dc;
    R.aligned = false;
    nnm_status st = sort_points(R, X, 0);
    if (st != NNM_OK) return st;
    HIP_TRY(launch_reset_comp(m, R.s));
    HIP_TRY(launch_cursor(m, R.s));
    HIP_TRY(launch_compmin1(m, R.s));
    HIP_TRY(launch_flag_rescan(m, R.s));
    HIP_TRY(launch_compact(w.rflag, n, w.rlist, &dc[0], w.scan_temp, R.s));
    if (!R.o.disable_prune) {
        // representatives of the components without a bound go first (their
        // nearest outside point), when they are fewer than the rows to scan
        HIP_TRY(launch_pick_reps_dev(m, w.compS, w.rep_pos, &w.ctr->ctr[1], w.rflag2, R.s));
        HIP_TRY(launch_compact(w.rflag2, n, w.olist, &dc[1], w.scan_temp, R.s));
        HIP_TRY(launch_rep_select(&dc[1], &dc[0], &dc[2], R.s));
        HIP_TRY(launch_copy_i32_dev(w.rlist, w.olist, &dc[2], n, R.s));
        st = scan_rows_dev(R, X, w.rlist, &dc[2], false, 1);
        if (st != NNM_OK) return st;
        HIP_TRY(launch_cursor(m, R.s));
        HIP_TRY(launch_compmin1(m, R.s));
        HIP_TRY(launch_flag_rescan(m, R.s));
        HIP_TRY(launch_compact(w.rflag, n, w.rlist, &dc[0], w.scan_temp, R.s));
    }
    st = scan_rows_dev(R, X, w.rlist, &dc[0], true, p.k);
    if (st != NNM_OK) return st;
    HIP_TRY(launch_cursor(m, R.s));
    HIP_TRY(launch_compmin1(m, R.s));
    HIP_TRY(launch_compmin2(m, R.s));
    HIP_TRY(launch_hook(m, R.s));
    // a hook chain has at most as many links as the largest instance has
    // points; each jump launch at least doubles every pointer's reach
    HIP_TRY(launch_jump(m, ceil_log2(std::max<int64_t>(R.max_inst, 2)) + 1, R.s));
    HIP_TRY(launch_fill_i32(&w.ctr->ctr[1], 0, 2, R.s));
    HIP_TRY(launch_jump_check(m, R.s));
    HIP_TRY(launch_relabel(m, R.s));
    return NNM_OK;
}

// Executable round graphs kept for later calls: the kernels' arguments are
// fixed by the workspace address, the input address, the plan, the options
// and the frame, so a call with the same values replays the same graph.
struct RoundGraph {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int nodes = 0;
    ~RoundGraph()
    {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
    }
};

constexpr size_t GRAPH_CACHE = 8;
std::mutex g_graph_mu;
std::vector<std::shared_ptr<RoundGraph>> g_graphs;     // most recent last
hipStream_t g_capture_stream[64] = {};

template <typename T>
void key_bytes(std::vector<uint64_t>& k, const T& v)
{
    uint64_t buf[(sizeof(T) + 7) / 8] = {};
    memcpy(buf, &v, sizeof(T));
    for (uint64_t x : buf) k.push_back(x);
}

std::vector<uint64_t> graph_key(const Run& R, const float* X, int dev)
{
    std::vector<uint64_t> k;
    k.push_back((uint64_t)dev);
    k.push_back((uint64_t)(uintptr_t)R.w.stats);      // workspace base
    k.push_back((uint64_t)(uintptr_t)X);
    const Plan& p = R.p;
    const int64_t f[] = {p.n, p.d, p.ld, p.opkind, p.exact, p.k, p.S, p.rmax, p.mst, p.L1, p.L2,
                         p.ninst, p.local, p.keep_e, R.max_inst};
    for (int64_t x : f) k.push_back((uint64_t)x);
    key_bytes(k, R.o);
    key_bytes(k, R.bc);
    return k;
}

// The round graph for this call: a kept one, or captured now (on a stream
// of the library's; the graph is then launched on the caller's stream).
nnm_status round_graph(Run& R, const float* X, std::shared_ptr<RoundGraph>* out, bool* captured)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return NNM_EDEVICE;
    std::vector<uint64_t> key = graph_key(R, X, dev);
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (size_t i = 0; i < g_graphs.size(); ++i) {
        if (g_graphs[i]->key == key) {
            std::shared_ptr<RoundGraph> g = g_graphs[i];
            g_graphs.erase(g_graphs.begin() + (long)i);
            g_graphs.push_back(g);
            *out = g;
            *captured = false;
            return NNM_OK;
        }
    }
    if (!g_capture_stream[dev])
        HIP_TRY(hipStreamCreateWithFlags(&g_capture_stream[dev], hipStreamNonBlocking));
    auto g = std::make_shared<RoundGraph>();
    g->key = std::move(key);
    hipStream_t caller = R.s;
    R.s = g_capture_stream[dev];
    HIP_TRY(hipStreamBeginCapture(R.s, hipStreamCaptureModeThreadLocal));
    nnm_status st = round_dev(R, X);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(R.s, &graph);
    R.s = caller;
    g->graph = graph;
    if (st != NNM_OK) return st;
    if (e != hipSuccess || !graph) return NNM_EDEVICE;
    size_t nn = 0;
    HIP_TRY(hipGraphGetNodes(graph, nullptr, &nn));
    g->nodes = (int)nn;
    HIP_TRY(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0));
    g_graphs.push_back(g);
    if (g_graphs.size() > GRAPH_CACHE) g_graphs.erase(g_graphs.begin());
    *out = g;
    *captured = true;
    return NNM_OK;
}

nnm_status finish_report(Run& R, std::chrono::steady_clock::time_point t0)
{
    if (!R.rep) return NNM_OK;
    Counters c;
    HIP_TRY(hipMemcpyAsync(&c, R.w.ctr, sizeof(c), hipMemcpyDeviceToHost, R.s));
    HIP_TRY(hipStreamSynchronize(R.s));
    R.rep->pairs_evaluated = (int64_t)spread_sum(c.pairs);
    R.rep->survivors = (int64_t)spread_sum(c.survivors);
    double e0, e1;
    memcpy(&e0, &c.err_bits[0], 8);
    memcpy(&e1, &c.err_bits[1], 8);
    R.rep->max_abs_err = e0;
    R.rep->max_rel_err = e1;
    R.rep->precision_used = R.p.opkind == OP_FP32 ? NNM_PREC_FP32
                            : R.p.opkind == OP_BF16 ? NNM_PREC_BF16
                            : R.p.opkind == OP_FP16 ? NNM_PREC_FP16 : NNM_PREC_FP8;
    R.rep->integer_mode = R.p.exact;
    R.rep->knn_k = R.p.k;
    // the largest bound E(t) the candidate pass applied to a rescored
    // survivor, and the largest ratio of the observed error to it
    double e2, e3;
    memcpy(&e2, &c.err_bits[2], 8);
    memcpy(&e3, &c.err_bits[3], 8);
    R.rep->max_bound = e2;
    R.rep->max_err_ratio = e3;
    R.rep->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return NNM_OK;
}

nnm_status validate(const float* X, int64_t n, int32_t d, int64_t ld, void* ws)
{
    if (!X || !ws || n < 1 || d < 1 || d > DMAX || ld < d) return NNM_EINVAL;
    if (n > (int64_t)0x7FFFFFF0) return NNM_EINVAL;
    return NNM_OK;
}

}  // namespace
}  // namespace nnm

using namespace nnm;

extern "C" nnm_status mst_workspace_size(int64_t n, int32_t d, const nnm_options* opt, size_t* bytes)
{
    if (!bytes) return NNM_EINVAL;
    Plan p;
    nnm_status st = plan_common(n, d, 0, opt, true, &p);
    if (st != NNM_OK) return st;
    WS w;
    *bytes = carve(p, nullptr, &w);
    return NNM_OK;
}

extern "C" nnm_status knn_workspace_size(int64_t n, int32_t d, int32_t k, const nnm_options* opt,
                                         size_t* bytes)
{
    if (!bytes || k < 1 || k > KMAX) return NNM_EINVAL;
    Plan p;
    nnm_status st = plan_common(n, d, k, opt, false, &p);
    if (st != NNM_OK) return st;
    WS w;
    *bytes = carve(p, nullptr, &w);
    return NNM_OK;
}

namespace {

nnm_status begin(Run& R, const float* X, int64_t n, int32_t d, int64_t ld, int32_t k,
                 const nnm_options* opt, void* ws, size_t ws_bytes, void* stream, nnm_report* rep,
                 bool mst)
{
    nnm_status st = validate(X, n, d, ld, ws);
    if (st != NNM_OK) return st;
    st = plan_common(n, d, k, opt, mst, &R.p);
    if (st != NNM_OK) return st;
    R.p.ld = ld;
    nnm_default_options(&R.o);
    if (opt) R.o = *opt;
    const size_t need = carve(R.p, nullptr, &R.w);
    if (ws_bytes < need) return NNM_EINVAL;
    carve(R.p, ws, &R.w);
    R.s = (hipStream_t)stream;
    R.rep = rep;
    R.timers = rep != nullptr;
    if (rep) memset(rep, 0, sizeof(*rep));
    return NNM_OK;
}

nnm_status knn_round(Run& R, const float* X)
{
    MergeArgs m = merge_args(R);
    HIP_TRY(launch_init_points(m, R.s));
    nnm_status st = spatial_order(R, X);
    if (st != NNM_OK) return st;
    R.aligned = false;
    st = sort_points(R, X, R.p.n);
    if (st != NNM_OK) return st;
    // every row, no bound: exact k-nearest-neighbour prefixes
    return scan_rows(R, X, nullptr, R.p.n, false);
}

}  // namespace

extern "C" nnm_status knn_build(const float* X_dev, int64_t n, int32_t d, int64_t ld, int32_t k,
                                const nnm_options* opt, void* ws_dev, size_t ws_bytes,
                                int32_t* idx_dev, double* s_dev, int32_t* len_dev, void* stream,
                                nnm_report* rep)
{
    auto t0 = std::chrono::steady_clock::now();
    if (k < 1 || k > KMAX || !idx_dev || !s_dev || !len_dev) return NNM_EINVAL;
    Run R;
    nnm_status st = begin(R, X_dev, n, d, ld, k, opt, ws_dev, ws_bytes, stream, rep, false);
    if (st != NNM_OK) return st;
    if (R.p.metric == NNM_METRIC_COSINE) {
        HIP_TRY(launch_normalize_rows(X_dev, n, d, ld, R.w.Xn, R.s));
        X_dev = R.w.Xn;
        R.p.ld = d;
    }
    st = stage(R, X_dev);
    if (st != NNM_OK) return st;
    if (n > 1) {
        st = knn_round(R, X_dev);
        if (st != NNM_OK) return st;
    } else {
        HIP_TRY(launch_fill_i32(R.w.clen, 0, n, R.s));
    }
    // copy the lists out, padded past len with (-1, +inf)
    HIP_TRY(launch_export_knn(n, k, R.w.cidx, R.w.cs, R.w.clen, idx_dev, s_dev, len_dev, R.s));
    HIP_TRY(hipStreamSynchronize(R.s));
    return finish_report(R, t0);
}

namespace {

// Merge rounds until every instance is one component; the n - ninst tree
// edges are left (unsorted) in w.edges.
nnm_status mst_rounds(Run& R, const float* X)
{
    Plan& p = R.p;
    WS& w = R.w;
    nnm_report* rep = R.rep;
    const int64_t n = p.n;
    nnm_status st;
    MergeArgs m = merge_args(R);
    {
        Timer t(R.timers, R.s, rep ? &rep->ms_merge : nullptr);
        HIP_TRY(launch_init_points(m, R.s));
    }
    {
        Timer t(R.timers, R.s, rep ? &rep->ms_sort : nullptr);
        st = spatial_order(R, X);
        if (st != NNM_OK) return st;
    }
    int64_t ncomp = n;
    int round = 0;
    Counters hc;
    memset(&hc, 0, sizeof(hc));
    unsigned long long pairs_before = 0, surv_before = 0;
    std::shared_ptr<RoundGraph> rg;
    for (; ncomp > p.ninst; ++round) {
        if (round >= 64) return NNM_EDEVICE;   // cannot happen: components at least halve
        R.round = round;
        if (rep && round < 32) rep->comps_per_round[round] = ncomp;
        if (R.o.graph && round >= 1) {
            // replay the round graph; one read of the counters per round
            if (!rg) {
                bool captured = false;
                st = round_graph(R, X, &rg, &captured);
                if (st != NNM_OK) return st;
                if (rep) {
                    rep->graph_nodes = rg->nodes;
                    rep->graph_captured = captured ? 1 : 0;
                }
            }
            {
                Timer t(R.timers, R.s, rep ? &rep->ms_graph : nullptr);
                HIP_TRY(hipGraphLaunch(rg->exec, R.s));
            }
            HIP_TRY(hipMemcpyAsync(&hc, w.ctr, sizeof(hc), hipMemcpyDeviceToHost, R.s));
            HIP_TRY(hipStreamSynchronize(R.s));
            if (hc.ctr[2] != 0) return NNM_EDEVICE;   // cannot happen: enough jumps
            const int64_t next = hc.ctr[1];
            if (next >= ncomp) return NNM_EDEVICE;
            ncomp = next;
            if (rep) {
                rep->graph_rounds += 1;
                rep->rows_scanned += hc.dc[0] + hc.dc[2];
                if (round < 32) {
                    rep->rows_per_round[round] = hc.dc[0] + hc.dc[2];
                    const unsigned long long pairs_now = spread_sum(hc.pairs);
                    const unsigned long long surv_now = spread_sum(hc.survivors);
                    rep->pairs_per_round[round] = (int64_t)(pairs_now - pairs_before);
                    rep->surv_per_round[round] = (int64_t)(surv_now - surv_before);
                    pairs_before = pairs_now;
                    surv_before = surv_now;
                }
            }
            continue;
        }
        {
            Timer t(R.timers, R.s, rep ? &rep->ms_sort : nullptr);
            R.aligned = round > 0 && ncomp * ALIGN_AVG <= n && !R.o.fixed_chunks;
            st = sort_points(R, X, ncomp);
            if (st != NNM_OK) return st;
        }
        int32_t rcount = 0;
        {
            Timer t(R.timers, R.s, rep ? &rep->ms_merge : nullptr);
            HIP_TRY(launch_reset_comp(m, R.s));
            HIP_TRY(launch_cursor(m, R.s));
            HIP_TRY(launch_compmin1(m, R.s));
            HIP_TRY(launch_flag_rescan(m, R.s));
            HIP_TRY(launch_compact(w.rflag, n, w.rlist, &w.ctr->rcount, w.scan_temp, R.s));
            HIP_TRY(hipMemcpyAsync(&rcount, &w.ctr->rcount, sizeof(int32_t), hipMemcpyDeviceToHost, R.s));
            HIP_TRY(hipStreamSynchronize(R.s));
        }
        if (rcount > 0 && !R.o.disable_prune) {
            // components without any cached candidate: scan a few spread-out
            // rows of each first, so that every other row is scanned below a
            // known bound
            int32_t nrep = 0;
            {
                Timer t(R.timers, R.s, rep ? &rep->ms_merge : nullptr);
                HIP_TRY(launch_pick_reps(m, w.compS, w.rep_pos, ncomp, w.rflag2, R.s));
                HIP_TRY(launch_compact(w.rflag2, n, w.olist, &w.ctr->rcount, w.scan_temp, R.s));
                HIP_TRY(hipMemcpyAsync(&nrep, &w.ctr->rcount, sizeof(int32_t), hipMemcpyDeviceToHost, R.s));
                HIP_TRY(hipStreamSynchronize(R.s));
            }
            if (nrep > 0 && nrep < rcount) {
                HIP_TRY(hipMemcpyAsync(w.rlist, w.olist, sizeof(int32_t) * (size_t)nrep,
                                       hipMemcpyDeviceToDevice, R.s));
                // a representative only has to bound its component's
                // smallest outgoing key: its nearest outside point will do
                R.kk = 1;
                st = scan_rows(R, X, w.rlist, nrep, false);
                R.kk = 0;
                if (st != NNM_OK) return st;
                if (rep && round < 32) rep->rows_per_round[round] += nrep;
                Timer t(R.timers, R.s, rep ? &rep->ms_merge : nullptr);
                HIP_TRY(launch_cursor(m, R.s));
                HIP_TRY(launch_compmin1(m, R.s));
                HIP_TRY(launch_flag_rescan(m, R.s));
                HIP_TRY(launch_compact(w.rflag, n, w.rlist, &w.ctr->rcount, w.scan_temp, R.s));
                HIP_TRY(hipMemcpyAsync(&rcount, &w.ctr->rcount, sizeof(int32_t), hipMemcpyDeviceToHost, R.s));
                HIP_TRY(hipStreamSynchronize(R.s));
            }
        }
        if (rep && round < 32) rep->rows_per_round[round] += rcount;
        if (rcount > 0) {
            st = scan_rows(R, X, w.rlist, rcount, true);
            if (st != NNM_OK) return st;
        }
        {
            Timer t(R.timers, R.s, rep ? &rep->ms_merge : nullptr);
            if (rcount > 0) {
                HIP_TRY(launch_cursor(m, R.s));
                HIP_TRY(launch_compmin1(m, R.s));
            }
            HIP_TRY(launch_compmin2(m, R.s));
            HIP_TRY(launch_hook(m, R.s));
            int iters = ceil_log2(ncomp) + 1;
            for (int extra = 0;; ++extra) {
                if (extra > 64) return NNM_EDEVICE;   // cannot happen: hooks form a forest
                HIP_TRY(launch_jump(m, iters, R.s));
                HIP_TRY(hipMemsetAsync(&w.ctr->ctr[1], 0, 2 * sizeof(int32_t), R.s));
                HIP_TRY(launch_jump_check(m, R.s));
                HIP_TRY(hipMemcpyAsync(&hc, w.ctr, sizeof(hc), hipMemcpyDeviceToHost, R.s));
                HIP_TRY(hipStreamSynchronize(R.s));
                if (hc.ctr[2] == 0) break;
                iters = 2;
            }
            HIP_TRY(launch_relabel(m, R.s));
        }
        const int64_t next = hc.ctr[1];
        if (next >= ncomp) return NNM_EDEVICE;   // no progress: cannot happen
        ncomp = next;
        if (rep && round < 32) {
            const unsigned long long pairs_now = spread_sum(hc.pairs);
            const unsigned long long surv_now = spread_sum(hc.survivors);
            rep->pairs_per_round[round] = (int64_t)(pairs_now - pairs_before);
            rep->surv_per_round[round] = (int64_t)(surv_now - surv_before);
            pairs_before = pairs_now;
            surv_before = surv_now;
        }
    }
    if (ncomp != p.ninst || (int64_t)hc.ctr[0] != n - p.ninst) return NNM_EDEVICE;
    if (rep) rep->rounds = round;
    return NNM_OK;
}

// Sort the n - ninst collected edges by key (s, u, v); returns the sorted buffer.
nnm_status sort_edges(Run& R, SortRec** res)
{
    const int64_t ne = R.p.n - R.p.ninst;
    const int lg = std::max(ceil_log2(R.p.n), 1);
    const int fields[3] = {2, 1, 0};
    const int bits[3] = {lg, lg, 64};
    HIP_TRY(launch_radix_sort(R.w.edges, R.w.srtA, ne, fields, bits, 3, R.w.radix_temp, res, R.s));
    return NNM_OK;
}

}  // namespace

namespace {

nnm_status mst_build_in(const float* X_dev, int64_t n, int32_t d, int64_t ld, const nnm_options* opt,
                        void* ws_dev, size_t ws_bytes, nnm_edge* edges_dev, void* stream,
                        nnm_report* rep, bool timers)
{
    auto t0 = std::chrono::steady_clock::now();
    if (n > 1 && !edges_dev) return NNM_EINVAL;
    Run R;
    nnm_status st = begin(R, X_dev, n, d, ld, 0, opt, ws_dev, ws_bytes, stream, rep, true);
    if (st != NNM_OK) return st;
    R.timers = R.timers && timers;
    R.max_inst = n;
    if (R.p.metric == NNM_METRIC_COSINE) {
        HIP_TRY(launch_normalize_rows(X_dev, n, d, ld, R.w.Xn, R.s));
        X_dev = R.w.Xn;
        R.p.ld = d;
    }
    st = stage(R, X_dev);
    if (st != NNM_OK) return st;
    if (n == 1) return finish_report(R, t0);
    const int32_t off[2] = {0, (int32_t)n};
    HIP_TRY(hipMemcpyAsync(R.w.inst_off, off, sizeof(off), hipMemcpyHostToDevice, R.s));
    st = mst_rounds(R, X_dev);
    if (st != NNM_OK) return st;
    {
        Timer t(R.timers, R.s, rep ? &rep->ms_sort : nullptr);
        SortRec* res = nullptr;
        st = sort_edges(R, &res);
        if (st != NNM_OK) return st;
        HIP_TRY(launch_write_edges(res, n - 1, edges_dev, R.p.key_metric(), R.s));
        HIP_TRY(hipStreamSynchronize(R.s));
    }
    return finish_report(R, t0);
}

// ---- the paper's P-minimal-pairs pipeline --------------------------------
//
// The section "General description of the algorithm for constructing the
// set of minimum distances": each pass selects the P smallest pairs of
// points that are not inside one cluster, sorts them by key and unites
// clusters along them in that order (pairs that fall inside a cluster by
// then are skipped), until one cluster is left.  Here a pass is: every
// row's k smallest pairs to points outside its cluster (the same candidate
// and rescoring kernels as the merge rounds), the threshold below which
// those lists hold every such pair, the pairs under it sorted by key, and
// the first P of them taken on the host.  The unions are the key-ordered
// minimum spanning tree, the same as mst_build's.

struct PmWS {
    SortRec* candA;
    SortRec* candB;
    void* rtemp;
    unsigned long long* thr;
    int32_t* count;
};

size_t pm_carve(size_t base_bytes, int64_t cap, char* base, PmWS* w)
{
    size_t off = (base_bytes + 255) & ~(size_t)255;
    auto take = [&](size_t bytes) -> void* {
        off = (off + 255) & ~(size_t)255;
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    w->candA = (SortRec*)take((size_t)cap * sizeof(SortRec));
    w->candB = (SortRec*)take((size_t)cap * sizeof(SortRec));
    w->rtemp = take(radix_temp_bytes(cap));
    w->thr = (unsigned long long*)take(2 * sizeof(unsigned long long));
    w->count = (int32_t*)take(sizeof(int32_t));
    return off + 256;
}

nnm_status pm_sizes(int64_t n, int32_t d, const nnm_options* opt, size_t* base, int64_t* cap,
                    size_t* total)
{
    nnm_status st = mst_workspace_size(n, d, opt, base);
    if (st != NNM_OK) return st;
    Plan p;
    st = plan_common(n, d, 0, opt, true, &p);
    if (st != NNM_OK) return st;
    *cap = std::max<int64_t>(n * p.k, 1);
    PmWS w;
    *total = pm_carve(*base, *cap, nullptr, &w);
    return NNM_OK;
}

// Fixed scratch of mst_build_noalloc: a file-scope device array, so the
// entry point needs no allocation.  Every GPU the library runs on holds its
// own copy from the time the library's code is loaded there until the
// process ends.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = NNM_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_MAX_DEVICES = 64;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The current device's copy of `scratch` (looked up on the first call on
// that device, with that device current).
nnm_status scratch_of_current_device(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return NNM_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NNM_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NNM_OK;
}

}  // namespace

extern "C" nnm_status mst_build(const float* X_dev, int64_t n, int32_t d, int64_t ld,
                                const nnm_options* opt, void* ws_dev, size_t ws_bytes,
                                nnm_edge* edges_dev, void* stream, nnm_report* rep)
{
    return mst_build_in(X_dev, n, d, ld, opt, ws_dev, ws_bytes, edges_dev, stream, rep, true);
}

extern "C" nnm_status mst_build_noalloc(const float* X_dev, int64_t n, int32_t d, int64_t ld,
                                        const nnm_options* opt, nnm_edge* edges_dev, void* stream,
                                        nnm_report* rep)
{
    // every argument and size check comes before the first device call
    if (!X_dev || n < 1 || d < 1 || d > DMAX || ld < d || (n > 1 && !edges_dev)) return NNM_EINVAL;
    size_t need = 0;
    nnm_status st = mst_workspace_size(n, d, opt, &need);
    if (st != NNM_OK) return st;
    if (need > NOALLOC_SCRATCH_BYTES) return NNM_ETOOLARGE;
    void* ws = nullptr;
    st = scratch_of_current_device(&ws);
    if (st != NNM_OK) return st;
    // no HIP events either: the phase times of the report stay 0; and no
    // graph (instantiating one allocates)
    nnm_options o;
    nnm_default_options(&o);
    if (opt) o = *opt;
    o.graph = 0;
    return mst_build_in(X_dev, n, d, ld, &o, ws, NOALLOC_SCRATCH_BYTES, edges_dev, stream, rep, false);
}

extern "C" nnm_status pminimal_workspace_size(int64_t n, int32_t d, const nnm_options* opt,
                                              size_t* bytes)
{
    if (!bytes) return NNM_EINVAL;
    size_t base = 0;
    int64_t cap = 0;
    return pm_sizes(n, d, opt, &base, &cap, bytes);
}

extern "C" nnm_status mst_build_pminimal(const float* X_dev, int64_t n, int32_t d, int64_t ld,
                                         int64_t P, const nnm_options* opt, void* ws_dev,
                                         size_t ws_bytes, nnm_edge* edges_dev, void* stream,
                                         nnm_report* rep)
{
    auto t0 = std::chrono::steady_clock::now();
    if (P < 0 || (n > 1 && !edges_dev)) return NNM_EINVAL;
    if (!X_dev || !ws_dev || n < 1 || d < 1 || d > DMAX || ld < d) return NNM_EINVAL;
    size_t base = 0, total = 0;
    int64_t cap = 0;
    nnm_status st = pm_sizes(n, d, opt, &base, &cap, &total);
    if (st != NNM_OK) return st;
    if (ws_bytes < total) return NNM_EINVAL;
    Run R;
    st = begin(R, X_dev, n, d, ld, 0, opt, ws_dev, base, stream, rep, true);
    if (st != NNM_OK) return st;
    PmWS pw;
    pm_carve(base, cap, (char*)ws_dev, &pw);
    R.max_inst = n;
    if (R.p.metric == NNM_METRIC_COSINE) {
        HIP_TRY(launch_normalize_rows(X_dev, n, d, ld, R.w.Xn, R.s));
        X_dev = R.w.Xn;
        R.p.ld = d;
    }
    st = stage(R, X_dev);
    if (st != NNM_OK) return st;
    if (n == 1) return finish_report(R, t0);
    const int32_t off[2] = {0, (int32_t)n};
    HIP_TRY(hipMemcpyAsync(R.w.inst_off, off, sizeof(off), hipMemcpyHostToDevice, R.s));
    MergeArgs m = merge_args(R);
    HIP_TRY(launch_init_points(m, R.s));
    st = spatial_order(R, X_dev);
    if (st != NNM_OK) return st;
    const int64_t take = P > 0 ? P : std::max<int64_t>(n / 2, 1);
    std::vector<int32_t> par((size_t)n), comp((size_t)n);
    std::vector<int64_t> sz((size_t)n, 1);
    for (int64_t i = 0; i < n; ++i) par[(size_t)i] = (int32_t)i;
    auto find = [&](int32_t x) {
        while (par[(size_t)x] != x) {
            par[(size_t)x] = par[(size_t)par[(size_t)x]];
            x = par[(size_t)x];
        }
        return x;
    };
    std::vector<nnm_edge> edges;
    edges.reserve((size_t)n - 1);
    std::vector<SortRec> host;
    const int lg = std::max(ceil_log2(n), 1);
    const int fields[3] = {2, 1, 0};
    const int bits[3] = {lg, lg, 64};
    const int km = R.p.key_metric();
    int64_t ncomp = n;
    int pass = 0;
    while (ncomp > 1) {
        if (pass >= 1 << 20) return NNM_EDEVICE;        // cannot happen: every pass unites
        R.round = pass;
        if (rep && pass < 32) rep->comps_per_round[pass] = ncomp;
        R.aligned = pass > 0 && ncomp * ALIGN_AVG <= n && !R.o.fixed_chunks;
        st = sort_points(R, X_dev, ncomp);
        if (st != NNM_OK) return st;
        // every row: its k smallest pairs leaving its cluster
        st = scan_rows(R, X_dev, nullptr, n, false);
        if (st != NNM_OK) return st;
        HIP_TRY(launch_fill_u64(pw.thr, ~0ull, 2, R.s));
        HIP_TRY(launch_fill_i32(pw.count, 0, 1, R.s));
        HIP_TRY(launch_pm_candidates(m, pw.thr, pw.candA, pw.count, cap, R.s));
        int32_t cnt = 0;
        HIP_TRY(hipMemcpyAsync(&cnt, pw.count, sizeof(cnt), hipMemcpyDeviceToHost, R.s));
        HIP_TRY(hipStreamSynchronize(R.s));
        const int64_t C = std::min<int64_t>(cnt, cap);
        if (C <= 0) return NNM_EDEVICE;                 // cannot happen: the smallest pair is below
        SortRec* res = nullptr;
        HIP_TRY(launch_radix_sort(pw.candA, pw.candB, C, fields, bits, 3, pw.rtemp, &res, R.s));
        // each pair is listed at most twice: 2P records hold the first P pairs
        const int64_t need = std::min<int64_t>(C, 2 * take);
        host.resize((size_t)need);
        HIP_TRY(hipMemcpyAsync(host.data(), res, sizeof(SortRec) * (size_t)need, hipMemcpyDeviceToHost,
                               R.s));
        HIP_TRY(hipStreamSynchronize(R.s));
        int64_t taken = 0, united = 0;
        for (int64_t q = 0; q < need && taken < take; ++q) {
            const SortRec& r = host[(size_t)q];
            if (q > 0 && r.k0 == host[(size_t)q - 1].k0 && r.k1 == host[(size_t)q - 1].k1 &&
                r.k2 == host[(size_t)q - 1].k2)
                continue;
            ++taken;
            int32_t a = find((int32_t)r.k1), b = find((int32_t)r.k2);
            if (a == b) continue;                        // inside one cluster by now
            if (sz[(size_t)a] < sz[(size_t)b]) std::swap(a, b);
            par[(size_t)b] = a;
            sz[(size_t)a] += sz[(size_t)b];
            nnm_edge e;
            e.u = (int32_t)r.k1;
            e.v = (int32_t)r.k2;
            memcpy(&e.s, &r.k0, 8);
            e.w = metric_key_is_distance(km) ? e.s : sqrt(e.s);
            edges.push_back(e);
            ++united;
            --ncomp;
        }
        if (united == 0) return NNM_EDEVICE;             // cannot happen: the smallest pair unites
        if (rep && pass < 32) {
            rep->rows_per_round[pass] = taken;
            rep->surv_per_round[pass] = united;
        }
        for (int64_t i = 0; i < n; ++i) comp[(size_t)i] = find((int32_t)i);
        HIP_TRY(hipMemcpyAsync(R.w.comp, comp.data(), sizeof(int32_t) * (size_t)n,
                               hipMemcpyHostToDevice, R.s));
        ++pass;
    }
    if ((int64_t)edges.size() != n - 1) return NNM_EDEVICE;
    HIP_TRY(hipMemcpyAsync(edges_dev, edges.data(), sizeof(nnm_edge) * edges.size(),
                           hipMemcpyHostToDevice, R.s));
    HIP_TRY(hipStreamSynchronize(R.s));
    if (rep) rep->rounds = pass;
    return finish_report(R, t0);
}

namespace {

nnm_status batched_plan(const nnm_instance* inst, int32_t count, const nnm_options* opt,
                        Plan* p, int64_t* ntot, int32_t* dmax)
{
    if (!inst || count < 1) return NNM_EINVAL;
    int64_t tot = 0;
    int32_t dm = 1;
    for (int32_t b = 0; b < count; ++b) {
        if (inst[b].n < 1 || inst[b].d < 1 || inst[b].d > DMAX || inst[b].ld < inst[b].d) return NNM_EINVAL;
        if (!inst[b].X_dev || (inst[b].n > 1 && !inst[b].edges_dev)) return NNM_EINVAL;
        tot += inst[b].n;
        dm = std::max(dm, inst[b].d);
    }
    if (tot > (int64_t)0x7FFFFFF0) return NNM_EINVAL;
    nnm_status st = plan_common(tot, dm, 0, opt, true, p);
    if (st != NNM_OK) return st;
    p->ninst = count;
    p->ld = dm;
    *ntot = tot;
    *dmax = dm;
    return NNM_OK;
}

}  // namespace

extern "C" nnm_status mst_batched_workspace_size(const nnm_instance* inst, int32_t count,
                                                 const nnm_options* opt, size_t* bytes)
{
    if (!bytes) return NNM_EINVAL;
    if (count == 0) { *bytes = 0; return NNM_OK; }
    Plan p;
    int64_t tot;
    int32_t dm;
    nnm_status st = batched_plan(inst, count, opt, &p, &tot, &dm);
    if (st != NNM_OK) return st;
    WS w;
    *bytes = carve(p, nullptr, &w);
    return NNM_OK;
}

// All instances are concatenated into one point set (features zero-padded to
// the widest instance, which leaves every FP64 key bit-identical), kept
// contiguous in every order the rounds use, and every tile of rows pairs only
// with its own instance's columns.  One launch per phase serves all
// instances; the rounds stop when every instance is a single tree.
extern "C" nnm_status mst_build_batched(const nnm_instance* inst, int32_t count,
                                        const nnm_options* opt, void* ws_dev, size_t ws_bytes,
                                        void* stream, nnm_report* reps)
{
    auto t0 = std::chrono::steady_clock::now();
    if (count == 0) return NNM_OK;
    if (!ws_dev) return NNM_EINVAL;
    Run R;
    int64_t tot;
    int32_t dm;
    nnm_status st = batched_plan(inst, count, opt, &R.p, &tot, &dm);
    if (st != NNM_OK) return st;
    nnm_default_options(&R.o);
    if (opt) R.o = *opt;
    const size_t need = carve(R.p, nullptr, &R.w);
    if (ws_bytes < need) return NNM_EINVAL;
    carve(R.p, ws_dev, &R.w);
    R.s = (hipStream_t)stream;
    nnm_report rep0;
    memset(&rep0, 0, sizeof(rep0));
    R.rep = reps ? &rep0 : nullptr;
    R.timers = R.rep != nullptr;
    std::vector<int32_t> off(count + 1, 0);
    std::vector<InstDev> hin(count);
    std::vector<nnm_edge*> outp(count);
    for (int32_t b = 0; b < count; ++b) {
        off[b + 1] = off[b] + (int32_t)inst[b].n;
        R.max_inst = std::max<int64_t>(R.max_inst, inst[b].n);
        hin[b].X = inst[b].X_dev;
        hin[b].ld = inst[b].ld;
        hin[b].d = inst[b].d;
        hin[b].pad_ = 0;
        outp[b] = inst[b].edges_dev;
    }
    HIP_TRY(hipMemcpyAsync(R.w.inst_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, R.s));
    HIP_TRY(hipMemcpyAsync(R.w.inst, hin.data(), sizeof(InstDev) * hin.size(), hipMemcpyHostToDevice, R.s));
    HIP_TRY(hipMemcpyAsync(R.w.outp, outp.data(), sizeof(nnm_edge*) * outp.size(), hipMemcpyHostToDevice, R.s));
    HIP_TRY(launch_concat(R.w.inst, R.w.inst_off, count, tot, dm, R.w.Xcat, R.s));
    // the zero padding leaves every row's norm as it is
    if (R.p.metric == NNM_METRIC_COSINE)
        HIP_TRY(launch_normalize_rows(R.w.Xcat, tot, dm, dm, R.w.Xcat, R.s));
    const float* X = R.w.Xcat;
    st = stage(R, X);
    if (st != NNM_OK) return st;
    if (tot > count) {
        st = mst_rounds(R, X);
        if (st != NNM_OK) return st;
        Timer t(R.timers, R.s, R.rep ? &R.rep->ms_sort : nullptr);
        SortRec* res = nullptr;
        st = sort_edges(R, &res);
        if (st != NNM_OK) return st;
        SortRec* other = (res == R.w.srtA) ? R.w.edges : R.w.srtA;
        HIP_TRY(launch_write_edges_batched(res, tot - count, R.w.inst_off, count, other, R.w.srtB,
                                           R.w.radix_temp, R.w.outp, R.p.key_metric(), R.s));
    }
    HIP_TRY(hipStreamSynchronize(R.s));
    st = finish_report(R, t0);
    if (st != NNM_OK) return st;
    if (reps)
        for (int32_t b = 0; b < count; ++b) reps[b] = rep0;
    return NNM_OK;
}
