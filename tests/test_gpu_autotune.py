"""The run-option autotuner on the GPU: it times the caller's own data over
its grid (every trial's trees checked against the first's inside the
library), stores the fastest options per size bucket, and a tuned call gives
the oracle's tree."""
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


def test_tune_single_then_tuned_call(nnm, tmp_path):
    from paper_1402_3789_amd import autotune as A
    X, _ = W.mixture64(8, n=3000, d=12)
    cache = str(tmp_path / "tune.json")
    _say("autotune single", X.shape)
    ent = A.tune(_dev(X), precision="fp16", reps=1, cache=cache)
    _say("entry", ent)
    assert ent["knn_k"] in (4, 6, 8, 12) and ent["graph"] in (0, 1)
    assert 2 <= len(ent["trials_ms"]) <= 13 and ent["ms"] <= ent["default_ms"]
    assert A.lookup(3000, 12, "fp16", cache=cache) == ent
    tree = nnm.mst_build(_dev(X), precision="fp16", tuned=cache)
    torch.cuda.synchronize()
    # 0: the tuner kept the default depth (6 on the FP16 path)
    assert tree.report["knn_k"] == (ent["knn_k"] or 6)
    u, v, s, w = tree.to_numpy()
    ou, ov, os_, ow = oracle.prim_mst(X)
    assert np.array_equal(u, ou) and np.array_equal(v, ov) and np.array_equal(s, os_)
    assert np.array_equal(w, ow)


def test_tune_batch_then_tuned_call(nnm, tmp_path):
    from paper_1402_3789_amd import autotune as A
    Xs = W.batch256(2, count=8, n_lo=300, n_hi=2000)
    cache = str(tmp_path / "tune.json")
    _say("autotune batch", [x.shape for x in Xs])
    ent = A.tune([_dev(x) for x in Xs], precision="fp16", reps=1, cache=cache)
    _say("entry", ent)
    ntot = sum(x.shape[0] for x in Xs)
    dmax = max(x.shape[1] for x in Xs)
    assert A.lookup(ntot, dmax, "fp16", count=len(Xs), cache=cache) == ent
    trees = nnm.mst_build_batched([_dev(x) for x in Xs], precision="fp16", tuned=cache)
    torch.cuda.synchronize()
    for X, t in zip(Xs, trees):
        for g, r in zip(t.to_numpy(), oracle.prim_mst(X)):
            assert np.array_equal(g, r)
