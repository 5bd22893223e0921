// rescore.hip -- exact FP64 rescoring of the candidate survivors.
//
// Every survivor of the candidate pass is re-evaluated with the FP64 key of
// eq. (1) (exact widening, one rounding per difference and per square, sum
// in feature order) and the k smallest keys (s, j) of the row are written to
// the row's neighbour list.  Rows whose survivor list overflowed are handled
// by an exact FP64 scan of the whole row instead.  These are the only places
// besides the final edge sort where the GPU computes in FP64.
#include "bound.h"
#include "nnm_common.h"

namespace nnm {
namespace {

// Running maximum of positive doubles kept as their bits; the plain read
// first skips the atomic whenever the value cannot raise the maximum (the
// common case once a few rows are in), so rows do not queue on one address.
__device__ __forceinline__ void atomic_max_pos_double(unsigned long long* p, double v)
{
    if (!(v > 0.0)) return;
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b <= __atomic_load_n(p, __ATOMIC_RELAXED)) return;
    atomicMax(p, b);
}

// A row whose survivor list overflowed keeps its first S survivors, all real
// columns outside its component: the kb-th smallest exact key among them
// (kb <= k) bounds the row's kb-th key from above, so the row is
// scanned again below that bound and gets an exact prefix of at least kb
// neighbours (level 1).  A row that overflows again goes to the exact scan.
// W lanes serve the row (64: a wave; 32: half a wave, two rows a wave),
// E slots each (E * W >= S).
template <int E, int W>
__device__ __forceinline__ void rescore_row(const RescoreArgs& a, int64_t slot, int32_t* overflow_list)
{
    const int lane = threadIdx.x & (W - 1);
    const int rp = a.rows ? a.rows[slot] : a.row0 + (int)slot;
    const int i = a.perm[rp];
    const int cnt = a.surv_cnt[slot];
    const bool over = cnt > a.S;
    if (a.force_fallback || (over && a.level == 2)) {   // final pass: exact scan
        if (lane == 0) {
            const int pos = atomicAdd(a.overflow_rows, 1);
            overflow_list[pos] = (int)slot;
        }
        return;
    }
    const int m = over ? a.S : cnt;
    const double u0s = a.u0 ? a.u0[rp] : -1.0;
    const float* xi = a.xs + (int64_t)rp * DMAX;
    // survivors above the row's final threshold cannot be among its k
    // nearest (their key exceeds the final bound U); an overflowed row keeps
    // all of its first S for the bound it passes on.  Super-chunk frames:
    // tfin is U itself (data units) and a survivor goes when its key's lower
    // bound t - E(t) >= 2t - (t + E(t) as stored), scaled, exceeds it
    const float tf = (a.tfin && !over) ? __uint_as_float(a.tfin[slot]) : __builtin_huge_valf();
    const bool key_bound = a.bound_mode == BOUND_LOCAL;
    double sv[E];
    int jv[E];
    double emax = 0.0, rmax = 0.0, bmax = 0.0, qmax = 0.0;
    int nsurv = 0;
    // the bound the candidate pass applied to this row's survivors
    float eps_r = 0.f, eta_r = 0.f;
    if (a.bound_mode == BOUND_GLOBAL) {
        const PointConst pr = a.pcs[rp];
        eps_r = global_eps(pr, a.bc);
        eta_r = global_eta(pr, a.bc);
    }
    const double crel = fp32_crel(a.d), a0 = fp32_a0(a.d);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        sv[e] = __builtin_huge_val();
        jv[e] = 0x7FFFFFFF;
        const int idx = e * W + lane;
        const float tv = idx < m ? a.surv_t[slot * a.S + idx] : 0.f;
        const float te = (idx < m && key_bound) ? a.surv_e[slot * a.S + idx] : 0.f;
        const bool drop = key_bound ? ((double)tv - ((double)te - (double)tv)) * a.inv_sigma2 > (double)tf
                                    : tv > tf;
        if (idx < m && !drop) {
            const int jp = a.surv_j[slot * a.S + idx];
            const int j = a.perm[jp];
            const double s = metric_key_rows(a.metric, xi, a.xs + (int64_t)jp * DMAX, a.d);
            const double t = (double)tv * a.inv_sigma2;
            const double err = __builtin_fabs(t - s);
            emax = err > emax ? err : emax;
            if (s > 0.0) {
                const double rel = err / s;
                rmax = rel > rmax ? rel : rmax;
            }
            // E(t), data units: what the candidate pass took |t - s| to be at most
            double eb = 0.0;
            if (a.bound_mode == BOUND_FP32)
                eb = fp32_upper_from_t((double)tv, crel, a0) - (double)tv;
            else if (a.bound_mode == BOUND_GLOBAL)
                eb = ((double)upper_from_t(tv, eps_r, eta_r, 0) - (double)tv) * a.inv_sigma2;
            else if (a.bound_mode == BOUND_LOCAL)
                eb = ((double)te - (double)tv) * a.inv_sigma2;
            bmax = eb > bmax ? eb : bmax;
            const double q = err > 0.0 ? (eb > 0.0 ? err / eb : __builtin_huge_val()) : 0.0;
            qmax = q > qmax ? q : qmax;
            ++nsurv;
            if (over || u0s < 0.0 || s <= u0s) {
                sv[e] = s;
                jv[e] = j;
            }
        }
    }
    int kept = 0;
    double last = __builtin_huge_val();
    // an overflowed row is scanned again below its kb-th key: that still
    // yields an exact prefix of its neighbour list (at least kb entries)
    const int kb = a.kb < a.k ? a.kb : a.k;
    double bound = __builtin_huge_val();
    for (int r = 0; r < a.k; ++r) {
        double bs = __builtin_huge_val();
        int bj = 0x7FFFFFFF;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (sj_less(sv[e], jv[e], bs, bj)) { bs = sv[e]; bj = jv[e]; }
        double ws = bs;
        int wj = bj;
#pragma unroll
        for (int off = W / 2; off > 0; off >>= 1) {
            const double os = __shfl_xor(ws, off);
            const int oj = __shfl_xor(wj, off);
            if (sj_less(os, oj, ws, wj)) { ws = os; wj = oj; }
        }
        if (!(ws < __builtin_huge_val())) break;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (sv[e] == ws && jv[e] == wj) { sv[e] = __builtin_huge_val(); jv[e] = 0x7FFFFFFF; }
        if (!over && lane == 0) {
            a.cidx[(int64_t)i * a.kstride + r] = wj;
            a.cs[(int64_t)i * a.kstride + r] = ws;
        }
        last = ws;
        ++kept;
        if (kept == kb) bound = ws;
    }
    for (int off = W / 2; off > 0; off >>= 1) {
        const double o1 = __shfl_xor(emax, off);
        const double o2 = __shfl_xor(rmax, off);
        const double o3 = __shfl_xor(bmax, off);
        const double o4 = __shfl_xor(qmax, off);
        emax = o1 > emax ? o1 : emax;
        rmax = o2 > rmax ? o2 : rmax;
        bmax = o3 > bmax ? o3 : bmax;
        qmax = o4 > qmax ? o4 : qmax;
        nsurv += __shfl_xor(nsurv, off);
    }
    if (lane != 0) return;
    atomic_max_pos_double(&a.err_bits[0], emax);
    atomic_max_pos_double(&a.err_bits[1], rmax);
    atomic_max_pos_double(&a.err_bits[2], bmax);
    atomic_max_pos_double(&a.err_bits[3], qmax);
    if (over) {
        double b = kept >= kb ? bound : -1.0;
        if (u0s >= 0.0 && (b < 0.0 || u0s < b)) b = u0s;
        a.u0b[rp] = b;
        a.oflag[rp] = 1;
        atomicAdd(a.overflow_rows, 1);
        return;
    }
    a.clen[i] = kept;
    a.ccur[i] = 0;
    if (kept == a.k) {
        a.clb[i] = a.cs[(int64_t)i * a.kstride + a.k - 1];
        a.cflag[i] = 0;
    } else if (u0s >= 0.0) {
        a.clb[i] = u0s;
        a.cflag[i] = 0;
    } else {
        a.clb[i] = __builtin_huge_val();
        a.cflag[i] = 1;
    }
    atomicAdd(&a.survivors[(slot & (NSPREAD - 1)) * SPREAD_STRIDE], (unsigned long long)nsurv);
}

// one wave per row
template <int E, int W>
__global__ __launch_bounds__(256) void k_rescore(RescoreArgs a, int32_t* overflow_list)
{
    const int64_t slot = (int64_t)blockIdx.x * (256 / W) + (threadIdx.x / W);
    if (slot < a.n_rows) rescore_row<E, W>(a, slot, overflow_list);
}

// device-sized: a fixed grid of waves strides over the launch's rows
template <int E, int W>
__global__ __launch_bounds__(256) void k_rescore_dev(RescoreArgs a, int32_t* overflow_list)
{
    const int64_t n = a.desc->n_rows;
    for (int64_t slot = (int64_t)blockIdx.x * (256 / W) + (threadIdx.x / W); slot < n;
         slot += (int64_t)gridDim.x * (256 / W))
        rescore_row<E, W>(a, slot, overflow_list);
}

// Exact top-k of one row over every point of its instance outside its
// component, by a full FP64 scan (one workgroup per overflowed row).
__device__ __forceinline__ void fallback_row(const RescoreArgs& a, int64_t slot)
{
    __shared__ double ws_s[4];
    __shared__ int ws_j[4], ws_t[4];
    __shared__ int winner;
    const int rp = a.rows ? a.rows[slot] : a.row0 + (int)slot;
    const int i = a.perm[rp];
    const int ci = a.comp[i];
    const float* xi = a.X + (int64_t)i * a.ld;
    const int tid = threadIdx.x;
    double ls[KMAX];
    int lj[KMAX];
    for (int e = 0; e < KMAX; ++e) { ls[e] = __builtin_huge_val(); lj[e] = 0x7FFFFFFF; }
    const int k = a.k;
    // the row's instance: the last b with inst_off[b] <= i
    int64_t jlo = 0, jhi = a.np;
    if (a.ninst > 1) {
        int lo = 0, hi = a.ninst;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.inst_off[mid] <= i) lo = mid;
            else hi = mid;
        }
        jlo = a.inst_off[lo];
        jhi = a.inst_off[lo + 1];
    }
    for (int64_t j = jlo + tid; j < jhi; j += 256) {
        if (j == i || a.comp[j] == ci) continue;
        const double s = metric_key(a.metric, xi, a.X + j * a.ld, a.d);
        if (!sj_less(s, (int)j, ls[k - 1], lj[k - 1])) continue;
        int p = k - 1;
        while (p > 0 && sj_less(s, (int)j, ls[p - 1], lj[p - 1])) {
            ls[p] = ls[p - 1];
            lj[p] = lj[p - 1];
            --p;
        }
        ls[p] = s;
        lj[p] = (int)j;
    }
    int head = 0;
    int kept = 0;
    for (int r = 0; r < k; ++r) {
        double bs = head < k ? ls[head] : __builtin_huge_val();
        int bj = head < k ? lj[head] : 0x7FFFFFFF;
        int bt = tid;
        for (int off = 32; off > 0; off >>= 1) {
            const double os = __shfl_xor(bs, off);
            const int oj = __shfl_xor(bj, off);
            const int ot = __shfl_xor(bt, off);
            if (sj_less(os, oj, bs, bj)) { bs = os; bj = oj; bt = ot; }
        }
        if ((tid & 63) == 0) { ws_s[tid >> 6] = bs; ws_j[tid >> 6] = bj; ws_t[tid >> 6] = bt; }
        __syncthreads();
        if (tid == 0) {
            double s0 = ws_s[0];
            int j0 = ws_j[0], t0 = ws_t[0];
            for (int w = 1; w < 4; ++w)
                if (sj_less(ws_s[w], ws_j[w], s0, j0)) { s0 = ws_s[w]; j0 = ws_j[w]; t0 = ws_t[w]; }
            winner = (s0 < __builtin_huge_val()) ? t0 : -1;
            if (winner >= 0) {
                a.cidx[(int64_t)i * a.kstride + r] = j0;
                a.cs[(int64_t)i * a.kstride + r] = s0;
            }
        }
        __syncthreads();
        const int wt = winner;
        __syncthreads();
        if (wt < 0) break;
        if (tid == wt) ++head;
        ++kept;
    }
    if (tid == 0) {
        a.clen[i] = kept;
        a.ccur[i] = 0;
        if (kept == k) {
            a.clb[i] = a.cs[(int64_t)i * a.kstride + k - 1];
            a.cflag[i] = 0;
        } else {
            a.clb[i] = __builtin_huge_val();
            a.cflag[i] = 1;
        }
    }
}

__global__ __launch_bounds__(256) void k_fallback(RescoreArgs a, const int32_t* overflow_list,
                                                  int n_over)
{
    if ((int)blockIdx.x < n_over) fallback_row(a, overflow_list[blockIdx.x]);
}

// device-sized: a fixed grid strides over the *n_over rows
__global__ __launch_bounds__(256) void k_fallback_dev(RescoreArgs a, const int32_t* overflow_list,
                                                      const int32_t* n_over)
{
    const int n = *n_over;
    for (int b = blockIdx.x; b < n; b += gridDim.x) {
        __syncthreads();   // the previous row's reads of the shared winner are done
        fallback_row(a, overflow_list[b]);
    }
}

}  // namespace

// Survivor lists of up to 256 (the global frame's cap at 2M points) are
// served by half a wave each: most rows of the merge rounds hold a survivor
// or two, and the row's dependent gathers, not its arithmetic, set the time,
// so two rows a wave halve the waves that wait.
template <int E>
void rescore_e(const RescoreArgs& a, int32_t* overflow_list, hipStream_t s)
{
    constexpr int W = E <= 4 ? 32 : 64;
    constexpr int EW = E * 64 / W;
    constexpr int RPB = 256 / W;
    if (a.desc) k_rescore_dev<EW, W><<<2048, 256, 0, s>>>(a, overflow_list);
    else k_rescore<EW, W><<<(unsigned)((a.n_rows + RPB - 1) / RPB), 256, 0, s>>>(a, overflow_list);
}

hipError_t launch_rescore(const RescoreArgs& a, int32_t* overflow_list, hipStream_t s)
{
    if (!a.desc && a.n_rows <= 0) return hipSuccess;
    switch (a.S / 64) {
    case 1: rescore_e<1>(a, overflow_list, s); break;
    case 2: rescore_e<2>(a, overflow_list, s); break;
    case 4: rescore_e<4>(a, overflow_list, s); break;
    case 8: rescore_e<8>(a, overflow_list, s); break;
    case 16: rescore_e<16>(a, overflow_list, s); break;
    case 32: rescore_e<32>(a, overflow_list, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fallback(const RescoreArgs& a, const int32_t* overflow_list, int n_over,
                           hipStream_t s)
{
    if (n_over <= 0) return hipSuccess;
    k_fallback<<<(unsigned)n_over, 256, 0, s>>>(a, overflow_list, n_over);
    return hipGetLastError();
}

hipError_t launch_fallback_dev(const RescoreArgs& a, const int32_t* overflow_list,
                               const int32_t* n_over, hipStream_t s)
{
    k_fallback_dev<<<1024, 256, 0, s>>>(a, overflow_list, n_over);
    return hipGetLastError();
}

}  // namespace nnm
