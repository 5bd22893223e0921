"""Full-size parity on the two other benchmark workloads.

* mixture64 (N = 262,144, D = 25: 64 isotropic Gaussians plus 5 % uniform
  noise): the whole tree is compared bit for bit with the oracle's, for every
  candidate precision, and so is the constrained cut (KL1 = 64, KL4 = 50,
  dmax = 0.2), through SHA-256 digests of the oracle's tree and labels that
  tests/golden/make_mixture64_digest.py wrote (oracle dense Prim and oracle
  cut; minutes of CPU time, so not repeated here).
* batch256 (256 independent instances, N log-uniform in [1024, 65536], D in
  4..25), built in one batched call: every instance's tree is checked for
  structure (n - 1 edges, u < v, sorted by key, spanning); sampled instances
  are compared bit for bit with the oracle's Prim, and their KL1 = 8 cuts with
  the oracle's; on the largest instance, the smallest pair of sampled points
  (the cut property for a single point) must be a tree edge.
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


def test_batch256_full_size(nnm):
    Xs = W.batch256(0)
    sizes = np.array([x.shape[0] for x in Xs])
    _say("batch256", len(Xs), "instances,", int(sizes.sum()), "points")
    trees = nnm.mst_build_batched([torch.from_numpy(x).to("cuda:0") for x in Xs])
    torch.cuda.synchronize()
    host = [t.to_numpy() for t in trees]
    for x, (u, v, s, w) in zip(Xs, host):
        _structure(x.shape[0], u, v, s)
        assert np.array_equal(w, np.sqrt(s))
    _say("batch256 structure ok")
    rng = np.random.default_rng(31)
    order = np.argsort(sizes, kind="stable")
    mid = [int(i) for i in order if sizes[i] <= 12_000]
    pick = sorted(set(mid[:6]) | set(rng.choice(mid, size=min(10, len(mid)), replace=False).tolist()))
    for b in pick:
        ref = oracle.prim_mst(Xs[b])
        _same_tree(host[b], ref)
        n = Xs[b].shape[0]
        labels, k = nnm.cluster_cut(host[b], n=n, kl1=8)
        want, wk = oracle.cut(*ref, n, kl1=8)
        assert k == wk and np.array_equal(labels, want)
    _say("batch256:", len(pick), "sampled instances identical to the oracle")
    big = int(order[-1])
    X = Xs[big]
    u, v, s, w = host[big]
    keys = set(zip(u.tolist(), v.tolist()))
    rows = rng.choice(X.shape[0], size=200, replace=False)
    j, _ = oracle.nn_outside(X, None, rows=rows)
    for i, jj in zip(rows.tolist(), j.tolist()):
        assert (min(i, jj), max(i, jj)) in keys
    _say("batch256 largest instance", X.shape, "nearest-neighbour edges ok")
