"""Other metrics (L1, L-infinity, cosine) against the oracle, bit for bit:
trees (u, v, s, w), neighbour lists, cuts, the batched call, forced paths
and graph-replayed rounds."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

METRICS = ["l1", "linf", "cosine"]


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def nnm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_3789_amd as m
    return m


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X, np.float32)).to("cuda:0")


def _same_tree(X, tree, metric):
    u, v, s, w = tree.to_numpy()
    ou, ov, os_, ow = oracle.prim_mst(X, metric=metric)
    bad = np.nonzero((u != ou) | (v != ov) | (s != os_))[0]
    assert bad.size == 0, f"{metric}: first mismatches at {bad[:5]}"
    assert np.array_equal(w, ow)
    return ou, ov, os_, ow


@pytest.mark.parametrize("metric", METRICS)
@pytest.mark.parametrize("data", ["mixture", "grid", "blobs"])
def test_tree_matches_oracle(nnm, metric, data):
    if data == "mixture":
        X, _ = W.mixture64(11, n=3000, d=12)
    elif data == "grid":
        X = W.int16grid(5, n=2500, d=6)                      # ties
    else:
        X, _ = W.blobs8(3, n=2048)
    precs = ["auto", "fp32"] if metric != "cosine" else ["auto", "fp16", "bf16", "fp32"]
    for prec in precs:
        _say("metric tree", metric, data, prec, X.shape)
        tree = nnm.mst_build(_dev(X), precision=prec, metric=metric)
        torch.cuda.synchronize()
        ou, ov, os_, ow = _same_tree(X, tree, metric)
    lab, k = nnm.cluster_cut(tree, kl1=8, kl4=5)
    olab, ok = oracle.cut(ou, ov, os_, ow, X.shape[0], kl1=8, kl4=5)
    assert k == ok and np.array_equal(lab, olab)


@pytest.mark.parametrize("metric", METRICS)
def test_knn_matches_oracle(nnm, metric):
    X, _ = W.mixture64(12, n=2500, d=16)
    _say("metric knn", metric, X.shape)
    idx, s, ln = nnm.knn_build(_dev(X), k=12, metric=metric)
    torch.cuda.synchronize()
    oi, os_, ol = oracle.knn(X, 12, metric=metric)
    assert np.array_equal(ln.cpu().numpy(), ol)
    assert np.array_equal(idx.cpu().numpy(), oi)
    assert np.array_equal(s.cpu().numpy(), os_)


@pytest.mark.parametrize("knob", ["fallback", "noprune", "k1", "cap64", "graph"])
def test_forced_paths(nnm, knob):
    X, _ = W.mixture64(13, n=3000, d=10)
    kw = {"fallback": dict(force_fallback=True), "noprune": dict(disable_prune=True),
          "k1": dict(knn_k=1), "cap64": dict(survivor_cap=64), "graph": dict(graph=True)}[knob]
    for metric in ("l1", "linf"):
        _say("metric forced", knob, metric, X.shape)
        tree = nnm.mst_build(_dev(X), precision="fp32", metric=metric, **kw)
        torch.cuda.synchronize()
        _same_tree(X, tree, metric)


def test_cosine_zero_rows_and_scale(nnm):
    rng = np.random.default_rng(14)
    X = rng.standard_normal((1500, 9)).astype(np.float32)
    X[[3, 700, 1499]] = 0.0
    X[10:20] *= 1e6                                            # scale never matters
    _say("cosine zero rows", X.shape)
    tree = nnm.mst_build(_dev(X), metric="cosine")
    torch.cuda.synchronize()
    _same_tree(X, tree, "cosine")


@pytest.mark.parametrize("metric", METRICS)
def test_batched_matches_oracle(nnm, metric):
    Xs = W.batch256(4, count=8, n_lo=300, n_hi=2000)
    _say("metric batched", metric, [x.shape for x in Xs])
    trees = nnm.mst_build_batched([_dev(x) for x in Xs], metric=metric)
    torch.cuda.synchronize()
    for X, t in zip(Xs, trees):
        _same_tree(X, t, metric)
