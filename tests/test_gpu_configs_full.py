"""Full-size parity on the two other benchmark workloads.

* mixture64 (N = 262,144, D = 25: 64 isotropic Gaussians plus 5 % uniform
  noise): the whole tree is compared bit for bit with the oracle's, for every
  candidate precision, and so is the constrained cut (KL1 = 64, KL4 = 50,
  dmax = 0.2), through SHA-256 digests of the oracle's tree and labels that
  tests/golden/make_mixture64_digest.py wrote (oracle dense Prim and oracle
  cut; minutes of CPU time, so not repeated here).
* batch256 (256 independent instances, N log-uniform in [1024, 65536], D in
  4..25), built in one batched call in each candidate precision: every
  instance's tree and its cut at KL1 = its own component count must match,
  bit for bit, the oracle's digests (tests/golden/batch256_oracle.json,
  written by tests/golden/make_fullsize_digests.py: oracle dense Prim and
  oracle cut, one instance at a time); structure and the nearest-neighbour
  edges of sampled points of the largest instance are checked as well.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def nnm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_3789_amd as m
    return m


@pytest.fixture(scope="module")
def mixture():
    with open(os.path.join(GOLDEN, "mixture64_oracle.json")) as f:
        want = json.load(f)
    X, _ = W.mixture64(0)
    assert W.sha256(X) == want["x_sha256"]
    return X, want


def _tree_digest(u, v, s, w):
    h = hashlib.sha256()
    for a, t in ((u, "<i4"), (v, "<i4"), (s, "<f8"), (w, "<f8")):
        h.update(np.ascontiguousarray(a, dtype=t).tobytes())
    return h.hexdigest()


def _same_tree(got, ref):
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_mixture64_full_size(nnm, mixture, prec):
    X, want = mixture
    _say("mixture64 full", prec)
    tree = nnm.mst_build(torch.from_numpy(X).to("cuda:0"), precision=prec)
    torch.cuda.synchronize()
    assert _tree_digest(*tree.to_numpy()) == want["tree_sha256"]
    c = want["cut"]
    labels, k = nnm.cluster_cut(tree, kl1=c["kl1"], kl4=c["kl4"], dmax=c["dmax"])
    assert k == c["clusters"]
    assert hashlib.sha256(np.ascontiguousarray(labels, "<i4").tobytes()).hexdigest() == c["labels_sha256"]
    _say("mixture64", prec, "tree and cut identical;", k, "clusters")


def _structure(n, u, v, s):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    assert len(u) == n - 1
    if n == 1:
        return
    assert np.all(u < v) and u.min() >= 0 and v.max() < n
    ds = np.diff(s)
    du = np.diff(u.astype(np.int64))
    dv = np.diff(v.astype(np.int64))
    assert np.all((ds > 0) | ((ds == 0) & ((du > 0) | ((du == 0) & (dv > 0)))))
    g = coo_matrix((np.ones(n - 1), (u, v)), shape=(n, n))
    assert connected_components(g, directed=False)[0] == 1


@pytest.fixture(scope="module")
def batch():
    with open(os.path.join(GOLDEN, "batch256_oracle.json")) as f:
        want = json.load(f)
    Xs, ks = W.batch256(0, with_components=True)
    assert len(Xs) == want["count"] == 256
    for x, k, wi in zip(Xs, ks, want["instances"]):
        assert W.sha256(x) == wi["x_sha256"] and k == wi["components"]
    return Xs, want["instances"]


def _labels_digest(labels):
    return hashlib.sha256(np.ascontiguousarray(labels, "<i4").tobytes()).hexdigest()


@pytest.mark.parametrize("prec", ["auto", "fp32", "bf16", "fp16-graph", "bf16-tuned"])
def test_batch256_full_size(nnm, batch, prec):
    """All 256 instances in one batched call: every tree, and every cut at
    KL1 = the instance's own component count, identical to the oracle's
    (digests written by tests/golden/make_fullsize_digests.py); also with the
    rounds replayed from the round graph, and with the autotuner's options."""
    Xs, want = batch
    sizes = np.array([x.shape[0] for x in Xs])
    _say("batch256", prec, len(Xs), "instances,", int(sizes.sum()), "points")
    p, _, how = prec.partition("-")
    trees = nnm.mst_build_batched([torch.from_numpy(x).to("cuda:0") for x in Xs], precision=p,
                                  graph=how == "graph", tuned=how == "tuned")
    torch.cuda.synchronize()
    host = [t.to_numpy() for t in trees]
    bad = [b for b, (h, wi) in enumerate(zip(host, want)) if _tree_digest(*h) != wi["tree_sha256"]]
    assert not bad, f"{prec}: {len(bad)} trees differ from the oracle, first {bad[:8]}"
    for b, (x, h, wi) in enumerate(zip(Xs, host, want)):
        c = wi["cut"]
        labels, k = nnm.cluster_cut(h, n=x.shape[0], kl1=c["kl1"])
        assert k == c["clusters"] and _labels_digest(labels) == c["labels_sha256"], \
            f"{prec}: instance {b} cut differs"
    _say("batch256", prec, "all 256 trees and cuts identical to the oracle")
    if prec != "auto":
        return
    for x, (u, v, s, w) in zip(Xs, host):
        _structure(x.shape[0], u, v, s)
        assert np.array_equal(w, np.sqrt(s))
    rng = np.random.default_rng(31)
    big = int(np.argmax(sizes))
    X = Xs[big]
    u, v, s, w = host[big]
    keys = set(zip(u.tolist(), v.tolist()))
    rows = rng.choice(X.shape[0], size=200, replace=False)
    j, _ = oracle.nn_outside(X, None, rows=rows)
    for i, jj in zip(rows.tolist(), j.tolist()):
        assert (min(i, jj), max(i, jj)) in keys
    _say("batch256 largest instance", X.shape, "nearest-neighbour edges ok")
