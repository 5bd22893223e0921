"""Merge rounds replayed from a captured hipGraph (options.graph = 1).

After the first round (host-sized, as without the option) every round is
one replay of a graph captured once: all launch sizes come from device
counts, the candidate passes are persistent grids that pop (tile, split)
items from a queue, and the host reads the counters once per round.  The
result must be the oracle's tree bit for bit, for single and batched calls,
in every precision and through the forced paths; a later call with the same
buffers and settings replays the kept graph.
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _same_as_oracle(X, tree):
    u, v, s, w = tree.to_numpy()
    ou, ov, os_, ow = oracle.prim_mst(X)
    bad = np.nonzero((u != ou) | (v != ov) | (s != os_))[0]
    assert bad.size == 0, f"first mismatches at {bad[:5]}"
    assert np.array_equal(w, ow)


@pytest.mark.parametrize("prec", ["fp16", "bf16", "fp32", "fp8"])
def test_graph_rounds_match_oracle(nnm, prec):
    if prec == "fp8":
        X = W.int16grid(4, n=3000, d=9)
    else:
        X, _ = W.mixture64(3, n=3000, d=12)
    _say("graph rounds", prec, X.shape)
    tree = nnm.mst_build(_dev(X), precision=prec, graph=True)
    torch.cuda.synchronize()
    rep = tree.report
    _say("rounds", rep["rounds"], "graph rounds", rep["graph_rounds"], "nodes", rep["graph_nodes"])
    assert rep["graph_rounds"] == rep["rounds"] - 1 and rep["graph_nodes"] > 0
    _same_as_oracle(X, tree)
    eager = nnm.mst_build(_dev(X), precision=prec)
    torch.cuda.synchronize()
    assert np.array_equal(tree.host_bytes(), eager.host_bytes())


@pytest.mark.parametrize("knob", ["fallback", "noprune", "overflow", "splits4", "k1"])
def test_graph_forced_paths(nnm, knob):
    if knob == "overflow":
        # binary features: hundreds of ties at every distance overflow the
        # survivor lists again and again, down to the exact scan
        X = np.random.default_rng(12).integers(0, 2, size=(3000, 6)).astype(np.float32)
        kw = dict(survivor_cap=64, knn_k=32)
    else:
        X, _ = W.mixture64(1, n=3000, d=12)
        kw = {"fallback": dict(force_fallback=True), "noprune": dict(disable_prune=True),
              "splits4": dict(col_splits=4), "k1": dict(knn_k=1)}[knob]
    for prec in ("fp16", "fp32"):
        _say("graph forced path", knob, prec, X.shape)
        tree = nnm.mst_build(_dev(X), precision=prec, graph=True, **kw)
        torch.cuda.synchronize()
        _same_as_oracle(X, tree)


def test_graph_kept_and_replayed_on_new_data(nnm):
    X, _ = W.mixture64(6, n=4000, d=16)
    Xd = _dev(X)
    _say("graph kept across calls", X.shape)
    t1 = nnm.mst_build(Xd, precision="fp16", graph=True)
    t2 = nnm.mst_build(Xd, precision="fp16", graph=True)
    torch.cuda.synchronize()
    assert t2.report["graph_captured"] == 0
    assert np.array_equal(t1.host_bytes(), t2.host_bytes())
    _same_as_oracle(X, t2)
    # the same buffers holding other points with the same feature ranges (a
    # row permutation: same frame, same settings) replay the kept graph
    X2 = X[np.random.default_rng(1).permutation(X.shape[0])]
    Xd.copy_(_dev(X2))
    t3 = nnm.mst_build(Xd, precision="fp16", graph=True)
    torch.cuda.synchronize()
    assert t3.report["graph_captured"] == 0
    _same_as_oracle(X2, t3)


@pytest.mark.parametrize("prec", ["fp16", "bf16", "fp32"])
def test_graph_batched_matches_oracle(nnm, prec):
    Xs = W.batch256(0, count=10, n_lo=300, n_hi=3000)
    rng = np.random.default_rng(3)
    Xs.insert(3, rng.standard_normal((1, 7)).astype(np.float32))     # single point
    Xs.insert(5, rng.standard_normal((2, 3)).astype(np.float32))     # one edge
    Xs.append(rng.integers(0, 3, size=(400, 4)).astype(np.float32))  # ties
    _say("graph batched", prec, [x.shape for x in Xs])
    trees = nnm.mst_build_batched([_dev(x) for x in Xs], precision=prec, graph=True)
    torch.cuda.synchronize()
    assert trees[0].report["graph_rounds"] >= 1
    for X, t in zip(Xs, trees):
        _same_as_oracle(X, t)


@pytest.mark.parametrize("knob", ["force_fallback", "tiny_cap"])
def test_graph_batched_exact_scan_stays_in_instance(nnm, knob):
    Xs = W.batch256(1, count=6, n_lo=200, n_hi=1500)
    _say("graph batched exact scan", knob, [x.shape for x in Xs])
    kw = {"force_fallback": True} if knob == "force_fallback" else {"survivor_cap": 16}
    trees = nnm.mst_build_batched([_dev(x) for x in Xs], precision="fp16", graph=True, **kw)
    torch.cuda.synchronize()
    for X, t in zip(Xs, trees):
        _same_as_oracle(X, t)
