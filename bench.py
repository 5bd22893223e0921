"""Benchmark: exact single-linkage tree + constrained cut at N = 2,000,000, D = 25.

One step = mst_build (exact key-ordered minimum spanning tree on the GPU)
+ cluster_cut_device (the KL1 = 500 cut of that tree on the GPU; the tree
stays in device memory) + copy of the N labels to the host.  The input is
already resident in GPU memory when timing starts.  The same cut on the
host (edges copied out, cluster_cut) is timed once beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints ONE JSON line with the headline metric (effective pair-distances/s =
N(N-1)/2 / wall time per step) for the mixed-precision path, the plain FP32
path's wall time on the same data, the roofline of the dominant kernel (the
candidate pass, from HIP-event timings recorded on the library's stream)
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_PEAK_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "fp8": 5000.0}
FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash(name):
    p = os.path.join(ROOT, "paper_1402_3789_amd", "csrc", name)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(precision, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_cand_{precision}_{workload}.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash("cand_mfma.hip"):
        return None
    return t.get("bytes_per_launch")


def oracle_digest_match(tree, n, labels):
    """Compare the tree and the KL1 = 500 cut with the oracle's digests of the
    same workload (tests/golden/aniso500_oracle.json, written from the oracle
    alone); None when that file is absent or covers other data."""
    p = os.path.join(ROOT, "tests", "golden", "aniso500_oracle.json")
    if not os.path.exists(p):
        return None
    want = json.load(open(p))
    if want.get("n") != n:
        return None
    import numpy as np
    u, v, s, w = tree.to_numpy()
    h = hashlib.sha256()
    for a, t in ((u, "<i4"), (v, "<i4"), (s, "<f8"), (w, "<f8")):
        h.update(np.ascontiguousarray(a, dtype=t).tobytes())
    same_tree = h.hexdigest() == want["tree_sha256"]
    cut = [c for c in want["cuts"] if set(c) == {"kl1", "clusters", "labels_sha256"} and c["kl1"] == 500]
    lab = hashlib.sha256(np.ascontiguousarray(labels, "<i4").tobytes()).hexdigest()
    same_cut = bool(cut) and lab == cut[0]["labels_sha256"]
    return bool(same_tree and same_cut)


def cpu_baseline(X, seconds):
    """Dense FP64 Prim (the oracle) on the first n_s points of the workload."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        cores = min(cores, int(env))
    # size the sample so that one run takes about `seconds` (O(n^2) work;
    # small runs underestimate, so re-aim once more from a larger one)
    ns = min(20000, X.shape[0])
    t1 = 0.0
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.prim_mst(X[:ns], threads=cores)
        t1 = time.perf_counter() - t0
        if t1 >= 0.5 * seconds or ns >= X.shape[0]:
            break
        ns = max(ns, min(int(ns * (seconds / max(t1, 1e-3)) ** 0.5), X.shape[0]))
    pairs = ns * (ns - 1) / 2.0
    out = {"value": pairs / t1, "unit": "pair-distances/s", "cores": cores, "kind": "oracle",
           "sample": f"first {ns} of the {X.shape[0]} points (dense FP64 Prim, every pair "
                     f"evaluated once), {t1:.1f} s"}
    # one thread, on a sample of about a quarter of the time budget
    n1 = max(2000, int(ns * 0.5 / max(cores, 1) ** 0.5))
    n1 = min(n1, X.shape[0])
    t0 = time.perf_counter()
    oracle.prim_mst(X[:n1], threads=1)
    t2 = time.perf_counter() - t0
    r1 = n1 * (n1 - 1) / 2.0 / t2
    out["single_thread"] = {"value": r1, "cores": 1, "sample": f"first {n1} points, {t2:.1f} s",
                            "n262144_seconds_at_this_rate": round(262144 * 262143 / 2.0 / r1, 1)}
    # the whole workload, as run once by the script that wrote the oracle's digests
    gp = os.path.join(ROOT, "tests", "golden", "aniso500_oracle.json")
    if os.path.exists(gp):
        g = json.load(open(gp))
        if g.get("n") == X.shape[0] and g.get("oracle_seconds"):
            out["full_workload"] = {"seconds": g["oracle_seconds"], "threads": g.get("oracle_threads"),
                                    "value": X.shape[0] * (X.shape[0] - 1) / 2.0 / g["oracle_seconds"],
                                    "source": "tests/golden/aniso500_oracle.json (oracle_seconds, "
                                              "measured on the 8-core build container)"}
    return out


def batch_section(nnm, torch, steps):
    """The batching workload: 256 instances (N log-uniform in [1024, 65536],
    D in 4..25) in one mst_build_batched call, trees left in HBM; default
    options and the autotuner's entries (cache, else the shipped table), each
    compared with the oracle's per-instance tree digests."""
    import numpy as np
    from workloads import batch256
    from paper_1402_3789_amd import autotune
    Xs = batch256(0)
    Xd = [torch.from_numpy(x).to("cuda:0") for x in Xs]
    pairs = sum(x.shape[0] * (x.shape[0] - 1) / 2.0 for x in Xs)
    gp = os.path.join(ROOT, "tests", "golden", "batch256_oracle.json")
    want = json.load(open(gp))["instances"] if os.path.exists(gp) else None
    ntot = sum(x.shape[0] for x in Xs)
    dmax = max(x.shape[1] for x in Xs)
    out = {"workload": "batch256 seed 0", "instances": len(Xs), "points": ntot,
           "timed": "mst_build_batched (all 256 trees, in HBM)"}
    for prec, tuned in (("fp16", False), ("fp16", True), ("bf16", False), ("bf16", True)):
        def run():
            return nnm.mst_build_batched(Xd, precision=prec, tuned=tuned)
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            trees = run()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        match = None
        if want is not None:
            match = True
            for t, w in zip(trees, want):
                u, v, s_, w_ = t.to_numpy()
                h = hashlib.sha256()
                for a, ty in ((u, "<i4"), (v, "<i4"), (s_, "<f8"), (w_, "<f8")):
                    h.update(np.ascontiguousarray(a, dtype=ty).tobytes())
                match = match and h.hexdigest() == w["tree_sha256"]
        ent = autotune.lookup(ntot, dmax, prec, count=len(Xs)) if tuned else None
        name = prec + ("_tuned" if tuned else "")
        out[name] = {"ms_per_step": round(ms, 3), "value": pairs / (ms * 1e-3),
                     "unit": "pair-distances/s", "oracle_match": match,
                     "options": {k: ent[k] for k in autotune.KNOBS} if ent else None}
        log(f"[bench] batch256 {name}: {ms:.1f} ms/step, oracle digests match: {match}")
    return out


def grid_section(nnm, torch, steps, n):
    """The tie-stress workload: integer features 0..15 (FP8 exact on the
    matrix cores, AUTO), tree + KL1 = 64 cut, against the oracle's digests
    when they exist."""
    import numpy as np
    from workloads import int16grid
    X = int16grid(0, n=n)
    Xd = torch.from_numpy(X).to("cuda:0")

    def gstep():
        t = nnm.mst_build(Xd, precision="auto")
        lab, k = nnm.cluster_cut_device(t, kl1=64)
        return t, lab, k
    gstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t, lab, k = gstep()
    torch.cuda.synchronize()
    gms = 1e3 * (time.perf_counter() - t0) / steps
    out = {"workload": f"int16grid n={n} d=25 seed 0", "ms_per_step": round(gms, 3),
           "value": n * (n - 1) / 2.0 / (gms * 1e-3), "unit": "pair-distances/s",
           "precision_used": t.report["precision_used"], "integer_mode": t.report["integer_mode"],
           "max_abs_err": t.report["max_abs_err"], "clusters": k, "oracle_match": None}
    gp = os.path.join(ROOT, "tests", "golden", "int16grid_oracle.json")
    if os.path.exists(gp):
        want = json.load(open(gp))
        if want.get("n") == n:
            u, v, s_, w_ = t.to_numpy()
            h = hashlib.sha256()
            for a, ty in ((u, "<i4"), (v, "<i4"), (s_, "<f8"), (w_, "<f8")):
                h.update(np.ascontiguousarray(a, dtype=ty).tobytes())
            cut = [c for c in want["cuts"] if set(c) == {"kl1", "clusters", "labels_sha256"}
                   and c["kl1"] == 64]
            lh = hashlib.sha256(np.ascontiguousarray(lab, "<i4").tobytes()).hexdigest()
            out["oracle_match"] = bool(h.hexdigest() == want["tree_sha256"] and cut
                                       and lh == cut[0]["labels_sha256"])
    log(f"[bench] int16grid: {gms:.1f} ms/step ({out['precision_used']}), oracle digests match: "
        f"{out['oracle_match']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--precision", default="fp16")
    ap.add_argument("--fp32-steps", type=int, default=1,
                    help="timed steps of each comparison path (0 = none)")
    ap.add_argument("--compare", default="fp32,bf16",
                    help="other candidate precisions timed on the same data")
    ap.add_argument("--pipeline-steps", type=int, default=1,
                    help="timed steps of the P-minimal-pairs pipeline on the same data (0 = none)")
    ap.add_argument("--grid-steps", type=int, default=1,
                    help="timed steps of the integer-grid workload (FP8 exact, 0 = none)")
    ap.add_argument("--batch-steps", type=int, default=2,
                    help="timed steps of the 256-instance batched call (0 = none)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "launches": 3}), flush=True)
        return

    import numpy as np
    import paper_1402_3789_amd as nnm
    from workloads import aniso500

    t0 = time.perf_counter()
    X, _ = aniso500(0, n=args.n)
    log(f"[bench] workload aniso500 n={args.n} d=25 generated in {time.perf_counter() - t0:.1f}s")
    n, d = X.shape
    Xd = torch.from_numpy(X).to("cuda:0")
    torch.cuda.synchronize()

    last_labels = {}

    def step(precision):
        tree = nnm.mst_build(Xd, precision=precision)
        # the cut on the device; the labels come back to the host
        labels, k = nnm.cluster_cut_device(tree, kl1=500)
        last_labels[precision] = labels
        return tree, k

    for i in range(args.warmup):
        step(args.precision)
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        tree, k = step(args.precision)
        reps.append(tree.report)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / args.steps
    log(f"[bench] {args.precision}: {ms:.1f} ms/step over {args.steps} steps, {k} clusters")
    pairs = n * (n - 1) / 2.0

    # roofline of the candidate pass (dominant kernel)
    cand_ms = sum(r["ms_candidates"] for r in reps)
    launches = sum(r["cand_launches"] for r in reps)
    evaluated = sum(r["pairs_evaluated"] for r in reps)
    flops = evaluated * (2 * d + 1)              # x.y form: 2D + 1 flops per ordered pair
    achieved = flops / (cand_ms * 1e-3) / 1e12 if cand_ms > 0 else 0.0
    peak = MFMA_PEAK_TFLOPS.get(args.precision, FP32_VECTOR_PEAK_TFLOPS)
    bound = "mfma" if args.precision in MFMA_PEAK_TFLOPS else "alu"
    traffic = load_traffic(args.precision, "aniso500")
    roof = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 5), "traffic": traffic,
            "kernel": f"k_cand_mfma<{args.precision}>", "launches_per_step": launches / args.steps,
            "avg_launch_ms": cand_ms / max(launches, 1),
            "pairs_evaluated_per_step": evaluated / args.steps,
            "executed_pairs_per_s": evaluated / (cand_ms * 1e-3) if cand_ms > 0 else 0.0,
            "flops_per_pair": 2 * d + 1}
    if traffic and cand_ms > 0:
        roof["hbm_frac"] = round(traffic / (cand_ms * 1e-3 / max(launches, 1)) / 8e12, 5)

    # the plain FP32 path (and other precisions) on the same data
    others = {}
    if args.fp32_steps > 0:
        for prec in [p for p in args.compare.split(",") if p and p != args.precision]:
            step(prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.fp32_steps):
                tr2, _ = step(prec)
            torch.cuda.synchronize()
            ms2 = 1e3 * (time.perf_counter() - t0) / args.fp32_steps
            same = np.array_equal(tr2.host_bytes(), tree.host_bytes())
            r2 = tr2.report
            others[prec] = {"ms_per_step": round(ms2, 3), "value": pairs / (ms2 * 1e-3),
                            "speedup_of_" + args.precision: round(ms2 / ms, 3),
                            "identical_tree": bool(same),
                            "oracle_match": oracle_digest_match(tr2, n, last_labels[prec]),
                            "ms_candidates": round(r2["ms_candidates"], 3),
                            "max_err_ratio": r2["max_err_ratio"]}
            if r2["ms_candidates"] > 0:
                # that path's own candidate kernel against its own peak
                ev = r2["pairs_evaluated"]
                if prec == "fp32":
                    fl, pk, un = 3 * d, FP32_VECTOR_PEAK_TFLOPS, "alu"
                else:
                    fl, pk, un = 2 * d + 1, MFMA_PEAK_TFLOPS.get(prec, 2500.0), "mfma"
                ach = ev * fl / (r2["ms_candidates"] * 1e-3) / 1e12
                others[prec]["roofline"] = {"bound": un, "achieved": round(ach, 3), "peak": pk,
                                            "unit": "TFLOP/s", "frac": round(ach / pk, 5),
                                            "flops_per_pair": fl}
            log(f"[bench] {prec}: {ms2:.1f} ms/step, identical tree: {same}")

    # the paper's own pipeline (P minimal pairs per pass) on the same data and kernels
    pipeline = None
    if args.pipeline_steps > 0:
        def pstep():
            return nnm.mst_build_pminimal(Xd, P=args.n // 2, precision=args.precision)
        pstep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.pipeline_steps):
            pt = pstep()
        torch.cuda.synchronize()
        pms = 1e3 * (time.perf_counter() - t0) / args.pipeline_steps
        pipeline = {"ms_per_step": round(pms, 3), "P": args.n // 2, "passes": pt.report["rounds"],
                    "timed": "mst_build_pminimal (tree only, no cut)",
                    "identical_tree": bool(np.array_equal(pt.host_bytes(), tree.host_bytes())),
                    "vs_merge_rounds_ms": round(ms, 3)}
        log(f"[bench] P-minimal-pairs pipeline: {pms:.1f} ms, {pt.report['rounds']} passes, "
            f"identical tree: {pipeline['identical_tree']}")

    batch = batch_section(nnm, torch, args.batch_steps) if args.batch_steps > 0 else None
    grid = grid_section(nnm, torch, args.grid_steps, args.n) if args.grid_steps > 0 else None

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(X, args.cpu_seconds)
        log(f"[bench] cpu oracle: {cpu['value']:.3g} pair-distances/s ({cpu['sample']})")

    last = reps[-1]
    # the same cut on the host, for reference: edges to the host + cluster_cut
    cut_ms = {"same_labels": True}
    for where in ("device", "host"):
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if where == "device":
                lab_c, k_c = nnm.cluster_cut_device(tree, kl1=500)
            else:
                lab_c, k_c = nnm.cluster_cut(tree, n, kl1=500)
            dt = 1e3 * (time.perf_counter() - t1)
            best = dt if best is None else min(best, dt)
        same = bool(k_c == 500 and np.array_equal(lab_c, last_labels[args.precision]))
        cut_ms["same_labels"] = cut_ms["same_labels"] and same
        cut_ms[where] = round(best, 3)
    log(f"[bench] KL1 = 500 cut: device {cut_ms['device']:.2f} ms (labels to host), "
        f"host {cut_ms['host']:.2f} ms (edges to host + cluster_cut), "
        f"same labels as the timed steps: {cut_ms['same_labels']}")
    match = oracle_digest_match(tree, n, last_labels[args.precision])
    log(f"[bench] {args.precision} tree and cut vs the oracle's digests: {match}")
    out = {
        "metric": "MST+cut wall-time at N=2M,D=25; pair-distances/s, mixed-prec vs FP32",
        "value": pairs / (ms * 1e-3),
        "unit": "pair-distances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp16": "f16", "bf16": "bf16", "fp8": "fp8"}.get(args.precision, "f32"),
        "data": "synthetic",
        "config": {"workload": "aniso500", "n": n, "d": d, "clusters": 500,
                   "precision": args.precision, "cut": "kl1=500", "seed": 0},
        "roofline": roof,
        "cpu_baseline": cpu,
        "oracle_match": match,
        "cut_ms": cut_ms,
        "fp32_path": others.get("fp32"),
        "batch256": batch,
        "int16grid": grid,
        "p_minimal_pipeline": pipeline,
        "other_paths": {k2: v2 for k2, v2 in others.items() if k2 != "fp32"},
        "report": {k2: last[k2] for k2 in ("rounds", "rows_scanned", "pairs_evaluated",
                                            "survivors", "overflow_rows", "max_abs_err",
                                            "max_rel_err", "max_bound", "max_err_ratio",
                                            "ms_candidates", "ms_rescore",
                                            "ms_merge", "ms_sort", "rows_per_round",
                                            "comps_per_round")},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
