"""The constrained process over all pairs (cluster_cut_allpairs) against the
oracle's (oracle_cut_allpairs), label for label: random small cases with
every setting, neighbour prefixes short enough that most points need
several GPU rescans, ties, a hand example where the process bypasses a
blocked tree edge, a mixture with size caps, and equality with the tree cut
when the size caps are off."""
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


def test_hand_example_bypasses_blocked_tree_edge(nnm):
    X = np.array([[-0.75], [0.0], [0.125], [0.25], [1.125]], np.float32)
    _say("allpairs hand example")
    lab, k = nnm.cluster_cut_allpairs(_dev(X), kl3=3, k=1)
    assert k == 2 and lab.tolist() == [0, 1, 1, 1, 0]


@pytest.mark.parametrize("depth", [1, 2, 4, 16])
def test_random_settings_match_oracle(nnm, depth):
    rng = np.random.default_rng(100 + depth)
    for trial in range(40):
        n = int(rng.integers(2, 300))
        d = int(rng.integers(1, 6))
        X = rng.standard_normal((n, d)).astype(np.float32)
        if trial % 4 == 0:
            X = np.round(X * 2).astype(np.float32)          # ties
        kw = dict(kl1=int(rng.integers(0, 8)),
                  kl2=int(rng.choice([-1, 2, 5, 20, 60])),
                  kl3=int(rng.choice([-1, 3, 8, 30, 90])),
                  kl4=int(rng.choice([0, 2, 5, 12])),
                  dmax=float(rng.choice([np.inf, 0.5, 1.2, 3.0])))
        _say("allpairs random", depth, trial, X.shape, kw)
        want, wk = oracle.cut_allpairs(X, **kw)
        got, gk = nnm.cluster_cut_allpairs(_dev(X), k=depth, precision="fp32", **kw)
        assert gk == wk and np.array_equal(got, want), (trial, kw)


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
def test_mixture_with_size_caps_matches_oracle(nnm, prec):
    X, _ = W.mixture64(9, n=3000, d=8)
    for kw in (dict(kl1=10, kl2=200, kl3=300), dict(kl2=120, kl4=20, dmax=0.6),
               dict(kl1=30, kl3=150, kl4=8)):
        _say("allpairs mixture", prec, X.shape, kw)
        want, wk = oracle.cut_allpairs(X, **kw)
        got, gk, st = nnm.cluster_cut_allpairs(_dev(X), precision=prec, with_stats=True, **kw)
        _say("stats", st)
        assert gk == wk and np.array_equal(got, want), kw


def test_equals_tree_cut_without_size_caps(nnm):
    X, _ = W.mixture64(10, n=20000, d=12)
    Xd = _dev(X)
    tree = nnm.mst_build(Xd, precision="fp16")
    torch.cuda.synchronize()
    for kw in (dict(kl1=64), dict(kl1=64, kl4=50, dmax=0.2), dict(dmax=0.1)):
        _say("allpairs vs tree cut", X.shape, kw)
        want, wk = nnm.cluster_cut(tree, **kw)
        got, gk = nnm.cluster_cut_allpairs(Xd, tree, **kw)
        assert gk == wk and np.array_equal(got, want), kw
