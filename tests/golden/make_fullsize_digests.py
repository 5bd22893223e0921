"""Write the oracle's SHA-256 digests for the full-size workloads.

    python tests/golden/make_fullsize_digests.py aniso500    # ~2 h on 8 cores
    python tests/golden/make_fullsize_digests.py int16grid   # ~2 h on 8 cores
    python tests/golden/make_fullsize_digests.py batch256    # minutes

* ``aniso500``: 2,000,000 points, D = 25, 500 anisotropic Gaussians, seed 0;
  the tree, the cut at KL1 = 500 (the benchmark's cut) and a cut with the
  KL4 priority and a distance threshold (heap path of the cut).
* ``int16grid``: 2,000,000 points, D = 25, integers 0..15, seed 0; the tree
  and the cut at KL1 = 64, whose stop lands inside groups of equal keys,
  plus a KL4 cut.
* ``batch256``: the 256 instances of seed 0; every instance's tree and its
  cut at KL1 = the number of mixture components it was drawn from.

Only the oracle (dense Prim, every pair evaluated once, and the oracle cut)
and the seeded generator run here; nothing comes from the GPU library.  The
GPU tests and the benchmark hash their own trees and labels the same way
and compare.  Each file also records how long the oracle took and on how
many threads.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CUTS = {
    "aniso500": [dict(kl1=500), dict(kl1=500, kl4=50, dmax=0.05)],
    "int16grid": [dict(kl1=64), dict(kl1=64, kl4=1000)],
}


def tree_digest(u, v, s, w):
    h = hashlib.sha256()
    for a, t in ((u, "<i4"), (v, "<i4"), (s, "<f8"), (w, "<f8")):
        h.update(np.ascontiguousarray(a, dtype=t).tobytes())
    return h.hexdigest()


def labels_digest(labels):
    return hashlib.sha256(np.ascontiguousarray(labels, dtype="<i4").tobytes()).hexdigest()


def _threads():
    return len(os.sched_getaffinity(0))


def one_workload(name):
    X = W.aniso500(0)[0] if name == "aniso500" else W.int16grid(0)
    n = int(X.shape[0])
    print(f"[{name}] X {X.shape} sha256 {W.sha256(X)}; oracle Prim on {_threads()} threads",
          flush=True)
    t0 = time.time()
    tree = oracle.prim_mst(X)
    t_prim = time.time() - t0
    print(f"[{name}] Prim {t_prim:.0f} s", flush=True)
    cuts = []
    for c in CUTS[name]:
        labels, k = oracle.cut(*tree, n, **c)
        cuts.append(dict(c, clusters=int(k), labels_sha256=labels_digest(labels)))
    u, v, s, w = tree
    out = {
        "workload": f"{name} seed 0",
        "n": n,
        "d": int(X.shape[1]),
        "x_sha256": W.sha256(X),
        "tree_sha256": tree_digest(*tree),
        "weight_sum": float(np.sum(w)),
        "max_s": float(s[-1]),
        "cuts": cuts,
        "oracle_seconds": round(t_prim, 1),
        "oracle_threads": _threads(),
        "made_by": f"python tests/golden/make_fullsize_digests.py {name} "
                   "(oracle dense Prim + oracle cut)",
    }
    return out


def batch():
    Xs, ks = W.batch256(0, with_components=True)
    t0 = time.time()
    inst = []
    for i, (X, k) in enumerate(zip(Xs, ks)):
        n = int(X.shape[0])
        tree = oracle.prim_mst(X)
        labels, kk = oracle.cut(*tree, n, kl1=k)
        inst.append(dict(n=n, d=int(X.shape[1]), components=int(k), x_sha256=W.sha256(X),
                         tree_sha256=tree_digest(*tree),
                         cut=dict(kl1=int(k), clusters=int(kk),
                                  labels_sha256=labels_digest(labels))))
        if i % 32 == 31:
            print(f"[batch256] {i + 1} instances, {time.time() - t0:.0f} s", flush=True)
    return {
        "workload": "batch256 seed 0",
        "count": len(inst),
        "instances": inst,
        "oracle_seconds": round(time.time() - t0, 1),
        "oracle_threads": _threads(),
        "made_by": "python tests/golden/make_fullsize_digests.py batch256 "
                   "(oracle dense Prim + oracle cut, one instance at a time)",
    }


def main():
    names = sys.argv[1:] or ["batch256", "aniso500", "int16grid"]
    for name in names:
        out = batch() if name == "batch256" else one_workload(name)
        path = os.path.join(HERE, f"{name}_oracle.json")
        with open(path + ".tmp", "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        os.replace(path + ".tmp", path)
        print(f"[{name}] wrote {path}", flush=True)


if __name__ == "__main__":
    main()
