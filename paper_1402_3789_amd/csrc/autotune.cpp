// autotune.cpp -- the run-option autotuner (host code over the C ABI).
//
// How the merge rounds cut their work (cache depth k, how many workgroups
// the column splits aim at, graph replay of the rounds) decides how fully
// the GPU is loaded, and the best cut depends on the size and shape of the
// task and on the chip.  The tuner measures it on the caller's data:
// coordinate descent over a small grid, one knob at a time, every trial's
// trees checked against the first trial's.
#include <hip/hip_runtime_api.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "nnm.h"

namespace {

constexpr int32_t K_VALUES[] = {4, 6, 8, 12};
constexpr int32_t T0_VALUES[] = {2048, 4096, 8192};
constexpr int32_t T_VALUES[] = {4096, 8192, 16384};
constexpr int32_t G_VALUES[] = {0, 1};

nnm_status run_once(const nnm_instance* inst, int32_t count, const nnm_options* o, void* ws,
                    size_t ws_bytes, void* stream)
{
    if (count == 1)
        return mst_build(inst[0].X_dev, inst[0].n, inst[0].d, inst[0].ld, o, ws, ws_bytes,
                         inst[0].edges_dev, stream, nullptr);
    return mst_build_batched(inst, count, o, ws, ws_bytes, stream, nullptr);
}

nnm_status need_bytes(const nnm_instance* inst, int32_t count, const nnm_options* o, size_t* b)
{
    if (count == 1) return mst_workspace_size(inst[0].n, inst[0].d, o, b);
    return mst_batched_workspace_size(inst, count, o, b);
}

// the trees of every instance, copied to the host
nnm_status fetch_trees(const nnm_instance* inst, int32_t count, std::vector<char>* out)
{
    size_t tot = 0;
    for (int32_t b = 0; b < count; ++b) tot += (size_t)std::max<int64_t>(inst[b].n - 1, 0) * sizeof(nnm_edge);
    out->resize(tot);
    size_t off = 0;
    for (int32_t b = 0; b < count; ++b) {
        const size_t nb = (size_t)std::max<int64_t>(inst[b].n - 1, 0) * sizeof(nnm_edge);
        if (nb && hipMemcpy(out->data() + off, inst[b].edges_dev, nb, hipMemcpyDeviceToHost) != hipSuccess)
            return NNM_EDEVICE;
        off += nb;
    }
    return NNM_OK;
}

}  // namespace

extern "C" nnm_status mst_autotune_workspace_size(const nnm_instance* inst, int32_t count,
                                                  const nnm_options* base, size_t* bytes)
{
    if (!inst || count < 1 || !bytes) return NNM_EINVAL;
    nnm_options o0;
    nnm_default_options(&o0);
    if (base) o0 = *base;
    // only the cache depth changes the workspace
    size_t most = 0;
    nnm_status st = need_bytes(inst, count, &o0, &most);
    if (st != NNM_OK) return st;
    for (int32_t k : K_VALUES) {
        nnm_options o = o0;
        o.knn_k = k;
        size_t b = 0;
        st = need_bytes(inst, count, &o, &b);
        if (st != NNM_OK) return st;
        most = std::max(most, b);
    }
    *bytes = most;
    return NNM_OK;
}

extern "C" nnm_status mst_autotune(const nnm_instance* inst, int32_t count, const nnm_options* base,
                                   void* ws_dev, size_t ws_bytes, void* stream, int32_t reps,
                                   nnm_options* best, double* trial_ms, int32_t* n_trials)
{
    if (!inst || count < 1 || !ws_dev || !best || reps < 1 || reps > 16) return NNM_EINVAL;
    size_t need = 0;
    nnm_status st = mst_autotune_workspace_size(inst, count, base, &need);
    if (st != NNM_OK) return st;
    if (ws_bytes < need) return NNM_EINVAL;
    nnm_options cur;
    nnm_default_options(&cur);
    if (base) cur = *base;
    std::vector<char> ref, got;
    int32_t trials = 0;
    auto timed = [&](const nnm_options& o, double* ms) -> nnm_status {
        nnm_status s2 = run_once(inst, count, &o, ws_dev, ws_bytes, stream);   // untimed
        if (s2 != NNM_OK) return s2;
        double bestms = 1e300;
        for (int r = 0; r < reps; ++r) {
            const auto t0 = std::chrono::steady_clock::now();
            s2 = run_once(inst, count, &o, ws_dev, ws_bytes, stream);
            if (s2 != NNM_OK) return s2;
            if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return NNM_EDEVICE;
            bestms = std::min(bestms, std::chrono::duration<double, std::milli>(
                                          std::chrono::steady_clock::now() - t0).count());
        }
        s2 = fetch_trees(inst, count, trials == 0 ? &ref : &got);
        if (s2 != NNM_OK) return s2;
        if (trials > 0 && got != ref) return NNM_EDEVICE;   // cannot happen: results are exact
        if (trial_ms && trials < NNM_TUNE_MAX_TRIALS) trial_ms[trials] = bestms;
        ++trials;
        *ms = bestms;
        return NNM_OK;
    };
    double cur_ms = 0.0;
    st = timed(cur, &cur_ms);
    if (st != NNM_OK) return st;
    auto sweep = [&](int32_t nnm_options::*field, const int32_t* vals, int nv) -> nnm_status {
        for (int i = 0; i < nv; ++i) {
            if (cur.*field == vals[i]) continue;
            nnm_options o = cur;
            o.*field = vals[i];
            double ms = 0.0;
            nnm_status s2 = timed(o, &ms);
            if (s2 != NNM_OK) return s2;
            if (ms < cur_ms) {
                cur = o;
                cur_ms = ms;
            }
        }
        return NNM_OK;
    };
    st = sweep(&nnm_options::knn_k, K_VALUES, 4);
    if (st == NNM_OK) st = sweep(&nnm_options::split_target0, T0_VALUES, 3);
    if (st == NNM_OK) st = sweep(&nnm_options::split_target, T_VALUES, 3);
    if (st == NNM_OK) st = sweep(&nnm_options::graph, G_VALUES, 2);
    if (st != NNM_OK) return st;
    *best = cur;
    if (n_trials) *n_trials = trials;
    return NNM_OK;
}
