"""GPU parity: the HIP path against the CPU oracle, element by element.

Bar: tree edges (u, v) and FP64 weights s, w bit-exact; cut labels
bit-exact; neighbour lists (idx, s) bit-exact.  Every case prints its name,
seed and shape before it touches the GPU.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRECS = ["fp32", "fp16", "bf16"]


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


def _tree_equal(nnm, X, **kw):
    tree = nnm.mst_build(_dev(X), **kw)
    torch.cuda.synchronize()
    u, v, s, w = tree.to_numpy()
    ou, ov, os_, ow = oracle.prim_mst(X)
    assert len(u) == len(ou)
    bad = np.nonzero((u != ou) | (v != ov) | (s != os_))[0]
    assert bad.size == 0, f"first mismatches at {bad[:5]}: gpu {list(zip(u[bad[:5]], v[bad[:5]], s[bad[:5]]))} oracle {list(zip(ou[bad[:5]], ov[bad[:5]], os_[bad[:5]]))}"
    assert np.array_equal(w, ow)
    return tree, (ou, ov, os_, ow)


@pytest.mark.parametrize("prec", PRECS)
def test_blobs8_tree_and_cut(nnm, prec):
    X, y = W.blobs8(0)
    _say("blobs8", prec, X.shape)
    tree, (ou, ov, os_, ow) = _tree_equal(nnm, X, precision=prec)
    lab, k = nnm.cluster_cut(tree, kl1=8)
    olab, ok = oracle.cut(ou, ov, os_, ow, X.shape[0], kl1=8)
    assert k == ok == 8 and np.array_equal(lab, olab)
    rep = tree.report
    assert rep["rounds"] >= 1


@pytest.mark.parametrize("prec", PRECS)
def test_mixture_reduced_with_constraints(nnm, prec):
    X, _ = W.mixture64(0, n=6000)
    _say("mixture64 reduced", prec, X.shape)
    tree, (ou, ov, os_, ow) = _tree_equal(nnm, X, precision=prec)
    lab, k = nnm.cluster_cut(tree, kl1=64, kl4=50, dmax=0.2)
    olab, ok = oracle.cut(ou, ov, os_, ow, X.shape[0], kl1=64, kl4=50, dmax=0.2)
    assert k == ok and np.array_equal(lab, olab)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_aniso_reduced(nnm, prec):
    X, _ = W.aniso500(0, n=12000, k=40)
    _say("aniso500 reduced", prec, X.shape)
    _tree_equal(nnm, X, precision=prec)


@pytest.mark.parametrize("prec", ["fp8", "bf16", "fp16", "fp32", "auto"])
def test_integer_grid_ties(nnm, prec):
    X = W.int16grid(0, n=5000)
    _say("int16grid reduced", prec, X.shape)
    tree, (ou, ov, os_, ow) = _tree_equal(nnm, X, precision=prec)
    if prec != "fp32":
        assert tree.report["integer_mode"] == 1
        assert tree.report["max_abs_err"] == 0.0
    lab, k = nnm.cluster_cut(tree, kl1=64)
    olab, ok = oracle.cut(ou, ov, os_, ow, X.shape[0], kl1=64)
    assert k == ok and np.array_equal(lab, olab)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16", "fp8"])
@pytest.mark.parametrize("data", ["aniso", "mixture", "grid"])
def test_error_report_within_applied_bound(nnm, prec, data):
    """Every rescored candidate's |t - s| is within the bound E(t) that the
    candidate pass applied to it (report: max ratio <= 1), and the largest
    error is within the largest bound; exact on integer data."""
    if data == "aniso":
        X, _ = W.aniso500(1, n=20000, k=40)
    elif data == "mixture":
        X, _ = W.mixture64(1, n=20000)
    else:
        X = W.int16grid(1, n=8000)
    if prec == "fp8" and data != "grid":
        pytest.skip("FP8 serves integer grids only")
    _say("error report", prec, data, X.shape)
    tree = nnm.mst_build(_dev(X), precision=prec)
    torch.cuda.synchronize()
    rep = tree.report
    assert rep["survivors"] > 0
    assert rep["max_err_ratio"] <= 1.0, rep
    assert rep["max_abs_err"] <= rep["max_bound"] or rep["max_abs_err"] == 0.0
    if data == "grid" and prec != "fp32":
        assert rep["integer_mode"] == 1
        assert rep["max_abs_err"] == 0.0 and rep["max_bound"] == 0.0
    else:
        assert rep["max_bound"] > 0.0


@pytest.mark.parametrize("n", [1, 2, 3, 17, 255, 256, 257, 1000, 4097])
def test_ragged_sizes(nnm, n):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 5)).astype(np.float32)
    _say("ragged", n)
    for prec in ("fp16", "fp32"):
        tree = nnm.mst_build(_dev(X), precision=prec)
        torch.cuda.synchronize()
        u, v, s, w = tree.to_numpy()
        ou, ov, os_, ow = oracle.prim_mst(X)
        assert np.array_equal(u, ou) and np.array_equal(v, ov) and np.array_equal(s, os_)


@pytest.mark.parametrize("kind", ["dups", "all_same", "collinear", "lattice", "d1", "d26"])
def test_degenerate_inputs(nnm, kind):
    rng = np.random.default_rng(7)
    if kind == "dups":
        base = rng.standard_normal((50, 6)).astype(np.float32)
        X = base[rng.integers(0, 50, size=700)]
    elif kind == "all_same":
        X = np.ones((300, 4), np.float32)
    elif kind == "collinear":
        X = (np.arange(600)[:, None] * np.array([[0.25, -1.0, 3.0]])).astype(np.float32)
        X = X[rng.permutation(600)]
    elif kind == "lattice":
        X = rng.integers(0, 3, size=(900, 3)).astype(np.float32) * 0.5 + 0.25
    elif kind == "d1":
        X = rng.standard_normal((800, 1)).astype(np.float32)
    else:
        X = rng.uniform(0, 1, size=(1500, 26)).astype(np.float32)
    _say("degenerate", kind, X.shape)
    for prec in ("fp16", "bf16", "fp32"):
        _tree_equal(nnm, X, precision=prec)


def test_near_ties_below_half_precision(nnm):
    # pairs whose squared distances differ far below FP16/BF16 resolution
    rng = np.random.default_rng(11)
    base = rng.uniform(0, 1, size=(40, 8)).astype(np.float32)
    jit = rng.integers(-3, 4, size=(40 * 25, 8)) * 2.0 ** -20
    X = (np.repeat(base, 25, axis=0) + jit).astype(np.float32)
    _say("near ties", X.shape)
    for prec in ("fp16", "bf16", "fp32"):
        _tree_equal(nnm, X, precision=prec)


@pytest.mark.parametrize("knob", ["k1", "k32", "cap64", "fallback", "noprune", "splits4",
                                  "fixed_chunks"])
def test_forced_paths_give_identical_trees(nnm, knob):
    X, _ = W.mixture64(1, n=3000, d=12)
    kw = {"k1": dict(knn_k=1), "k32": dict(knn_k=32), "cap64": dict(survivor_cap=64),
          "fallback": dict(force_fallback=True), "noprune": dict(disable_prune=True),
          "splits4": dict(col_splits=4), "fixed_chunks": dict(fixed_chunks=True)}[knob]
    _say("forced path", knob, X.shape)
    for prec in ("fp16", "fp32"):
        _tree_equal(nnm, X, precision=prec, **kw)


@pytest.mark.parametrize("prec", ["fp16", "bf16", "fp32"])
def test_component_aligned_chunks_ragged_segments(nnm, prec):
    """Few large components of sizes that are no multiple of the chunk (and
    some far below it): the merge rounds cut column chunks along the
    components; the tree must equal the oracle's and the fixed-chunk run's."""
    rng = np.random.default_rng(77)
    sizes = [37, 300, 1023, 4097, 2500, 9000, 13, 700, 256, 257, 3]
    d = 10
    centres = rng.uniform(0, 40, size=(len(sizes), d))
    X = np.concatenate([c + rng.standard_normal((m, d)) * rng.uniform(0.2, 1.5)
                        for c, m in zip(centres, sizes)])
    X = X[rng.permutation(X.shape[0])].astype(np.float32)
    _say("aligned chunks, ragged components", prec, X.shape)
    tree, _ = _tree_equal(nnm, X, precision=prec)
    fixed = nnm.mst_build(_dev(X), precision=prec, fixed_chunks=True)
    torch.cuda.synchronize()
    assert np.array_equal(tree.host_bytes(), fixed.host_bytes())


def test_overflow_twice_goes_to_exact_scan(nnm):
    # binary features: hundreds of columns tie at every distance, so even the
    # bounded re-scan overflows a 64-entry survivor list
    X = np.random.default_rng(12).integers(0, 2, size=(3000, 6)).astype(np.float32)
    _say("overflow twice", X.shape)
    for prec in ("fp16", "fp32", "fp8"):
        tree, _ = _tree_equal(nnm, X, precision=prec, survivor_cap=64, knn_k=32)
        assert tree.report["overflow_rows"] > 0 and tree.report["rescanned_bounded"] > 0


def test_nonfinite_and_fp8_rejected(nnm):
    X = np.zeros((10, 3), np.float32)
    X[4, 1] = np.nan
    _say("nonfinite")
    with pytest.raises(nnm.NNMError) as e:
        nnm.mst_build(_dev(X))
    assert e.value.code == -4
    X = np.random.default_rng(0).uniform(0, 1, (20, 3)).astype(np.float32)
    with pytest.raises(nnm.NNMError) as e:
        nnm.mst_build(_dev(X), precision="fp8")
    assert e.value.code == -5


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16", "fp8"])
def test_knn_matches_oracle(nnm, prec):
    if prec == "fp8":
        X = W.int16grid(3, n=2500, d=10)
    else:
        X, _ = W.mixture64(2, n=2500, d=16)
    k = 12
    _say("knn", prec, X.shape, k)
    idx, s, ln = nnm.knn_build(_dev(X), k=k, precision=prec)
    torch.cuda.synchronize()
    oi, os_, ol = oracle.knn(X, k)
    assert np.array_equal(ln.cpu().numpy(), ol)
    assert np.array_equal(idx.cpu().numpy(), oi)
    assert np.array_equal(s.cpu().numpy(), os_)


def test_knn_short_rows(nnm):
    X = np.random.default_rng(4).standard_normal((5, 3)).astype(np.float32)
    _say("knn short rows")
    idx, s, ln = nnm.knn_build(_dev(X), k=8, precision="fp16")
    oi, os_, ol = oracle.knn(X, 8)
    assert np.array_equal(ln.cpu().numpy(), ol)
    assert np.array_equal(idx.cpu().numpy(), oi)
    assert np.array_equal(s.cpu().numpy(), os_)


def test_determinism_across_runs_and_settings(nnm):
    X, _ = W.mixture64(5, n=4000, d=25)
    _say("determinism", X.shape)
    ref = None
    for kw in (dict(precision="fp16"), dict(precision="fp16"), dict(precision="bf16", knn_k=8),
               dict(precision="fp32", knn_k=4), dict(precision="fp16", col_splits=3)):
        t = nnm.mst_build(_dev(X), **kw)
        raw = t.host_bytes().copy()
        if ref is None:
            ref = raw
        assert np.array_equal(raw, ref)


def test_batched_matches_single(nnm):
    Xs = W.batch256(0, count=10, n_lo=300, n_hi=3000)
    rng = np.random.default_rng(3)
    Xs.insert(3, rng.standard_normal((1, 7)).astype(np.float32))     # single point
    Xs.insert(5, rng.standard_normal((2, 3)).astype(np.float32))     # one edge
    Xs.append(rng.integers(0, 3, size=(400, 4)).astype(np.float32))  # ties
    _say("batched", [x.shape for x in Xs])
    for prec in ("fp16", "fp32"):
        trees = nnm.mst_build_batched([_dev(x) for x in Xs], precision=prec)
        torch.cuda.synchronize()
        for X, t in zip(Xs, trees):
            u, v, s, w = t.to_numpy()
            ou, ov, os_, ow = oracle.prim_mst(X)
            assert np.array_equal(u, ou) and np.array_equal(v, ov) and np.array_equal(s, os_)
            assert np.array_equal(w, ow)


@pytest.mark.parametrize("knob", ["force_fallback", "tiny_cap"])
def test_batched_exact_scan_stays_in_instance(nnm, knob):
    # Rows that reach the exact full scan (forced, or after repeated survivor
    # overflows with the smallest cap) must only pair inside their instance.
    Xs = W.batch256(1, count=6, n_lo=200, n_hi=1500)
    _say("batched exact scan", knob, [x.shape for x in Xs])
    kw = {"force_fallback": True} if knob == "force_fallback" else {"survivor_cap": 16}
    trees = nnm.mst_build_batched([_dev(x) for x in Xs], precision="fp16", **kw)
    torch.cuda.synchronize()
    for X, t in zip(Xs, trees):
        got = t.to_numpy()
        for g, r in zip(got, oracle.prim_mst(X)):
            assert np.array_equal(g, r)
