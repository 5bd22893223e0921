"""Write mixture64_oracle.json: SHA-256 digests of the oracle's tree and cut
of the mixture64 workload (N = 262,144, D = 25, seed 0).

Only the oracle and the seeded generator run here; the GPU test compares the
digests of its own tree and cut with these.  Takes a few minutes on 8 cores:

    python tests/golden/make_mixture64_digest.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CUT = dict(kl1=64, kl4=50, dmax=0.2)


def tree_digest(u, v, s, w):
    h = hashlib.sha256()
    for a, t in ((u, "<i4"), (v, "<i4"), (s, "<f8"), (w, "<f8")):
        h.update(np.ascontiguousarray(a, dtype=t).tobytes())
    return h.hexdigest()


def labels_digest(labels):
    return hashlib.sha256(np.ascontiguousarray(labels, dtype="<i4").tobytes()).hexdigest()


def main():
    X, _ = W.mixture64(0)
    tree = oracle.prim_mst(X)
    labels, k = oracle.cut(*tree, X.shape[0], **CUT)
    out = {
        "workload": "mixture64 seed 0",
        "n": int(X.shape[0]),
        "d": int(X.shape[1]),
        "x_sha256": W.sha256(X),
        "tree_sha256": tree_digest(*tree),
        "cut": dict(CUT, clusters=int(k), labels_sha256=labels_digest(labels)),
        "made_by": "python tests/golden/make_mixture64_digest.py (oracle dense Prim + oracle cut)",
    }
    with open(os.path.join(HERE, "mixture64_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
