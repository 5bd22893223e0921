"""GPU: the cut of a sorted tree on the device (cluster_cut_device).

Without KL2, KL3 and KL4 the cut takes the first min(prefix, n - KL1) tree
edges (the prefix with w <= dmax) and the clusters are the components of
that forest.  Labels and K must equal the oracle's cut of the oracle's tree
(small n) and the host cut of the same edges (any n), element by element.
Every case prints its name and shape before it touches the GPU.
"""
import math

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


def _tree_from_edges(nnm, u, v, s, w):
    """A Tree on the device holding the given edge records."""
    m = len(u)
    buf = np.zeros((max(m, 1), 3), np.float64)
    iv = buf.view(np.int32).reshape(-1, 6)
    iv[:m, 0] = u
    iv[:m, 1] = v
    buf[:m, 1] = s
    buf[:m, 2] = w
    return nnm.Tree(torch.from_numpy(buf[:m]).to("cuda:0"), m + 1)


def test_matches_oracle_cut_on_oracle_tree(nnm):
    X, _ = W.blobs8(0)
    n = X.shape[0]
    _say("blobs8 device cut vs oracle", X.shape)
    tree = nnm.mst_build(_dev(X), precision="fp32")
    u, v, s, w = oracle.prim_mst(X)
    qs = [float(np.quantile(w, q)) for q in (0.0, 0.5, 0.99)]
    for kl1, dmax in [(8, math.inf), (1, math.inf), (0, math.inf), (0, qs[1]), (8, qs[2]),
                      (0, qs[0]), (n, math.inf), (n + 3, math.inf), (0, -1.0), (3, 0.0)]:
        lab, k = nnm.cluster_cut_device(tree, kl1=kl1, dmax=dmax)
        olab, ok = oracle.cut(u, v, s, w, n, kl1=kl1, dmax=dmax)
        assert k == ok and np.array_equal(lab, olab), (kl1, dmax, k, ok)


def test_matches_host_cut_mixture(nnm):
    X = W.mixture64(0)[0][:65536]
    n = X.shape[0]
    _say("mixture64 first 65536 device cut vs host cut", X.shape)
    tree = nnm.mst_build(_dev(X), precision="fp16")
    w = tree.to_numpy()[3]
    for kl1, dmax in [(64, math.inf), (64, 0.2), (0, 0.05), (1, math.inf), (5000, float(np.median(w)))]:
        lab, k = nnm.cluster_cut_device(tree, kl1=kl1, dmax=dmax)
        hlab, hk = nnm.cluster_cut(tree, kl1=kl1, dmax=dmax)
        assert k == hk and np.array_equal(lab, hlab), (kl1, dmax)
    dl, dk = nnm.cluster_cut_device(tree, kl1=64, host=False)
    assert dl.is_cuda and dl.dtype == torch.int32 and dk == 64


@pytest.mark.parametrize("n", [2, 3, 1000, 300001])
def test_random_trees(nnm, n):
    """Random trees with ragged sizes: point i > 0 hangs off a random
    earlier point, keys random with ties in s broken by (u, v)."""
    rng = np.random.default_rng(n)
    i = np.arange(1, n)
    par = (rng.random(n - 1) * i).astype(np.int64)
    u = np.minimum(par, i).astype(np.int32)
    v = np.maximum(par, i).astype(np.int32)
    s = np.floor(rng.random(n - 1) * 64.0)          # many equal s
    o = np.lexsort((v, u, s))
    u, v, s = u[o], v[o], s[o]
    w = np.sqrt(s)
    _say("random tree", n)
    tree = _tree_from_edges(nnm, u, v, s, w)
    for kl1, dmax in [(1, math.inf), (max(n // 7, 1), math.inf), (0, 4.0), (2, 5.0), (n, math.inf)]:
        lab, k = nnm.cluster_cut_device(tree, kl1=kl1, dmax=dmax)
        hlab, hk = nnm.cluster_cut(tree, kl1=kl1, dmax=dmax)
        assert k == hk and np.array_equal(lab, hlab), (n, kl1, dmax)


def test_single_point(nnm):
    _say("n = 1")
    tree = nnm.Tree(torch.zeros((0, 3), dtype=torch.float64, device="cuda:0"), 1)
    lab, k = nnm.cluster_cut_device(tree, kl1=0)
    assert k == 1 and lab.tolist() == [0]


def test_rejections(nnm):
    n = 1000
    rng = np.random.default_rng(7)
    i = np.arange(1, n)
    par = (rng.random(n - 1) * i).astype(np.int64)
    u = np.minimum(par, i).astype(np.int32)
    v = np.maximum(par, i).astype(np.int32)
    s = np.sort(rng.random(n - 1))
    _say("rejections", n)
    good = (u, v, s, np.sqrt(s))
    tree = _tree_from_edges(nnm, *good)
    _caps_unsupported(nnm, tree)
    # keys out of order
    bad = (u, v, s[::-1].copy(), np.sqrt(s[::-1]))
    with pytest.raises(nnm.NNMError, match="-1"):
        nnm.cluster_cut_device(_tree_from_edges(nnm, *bad), kl1=3)
    # a cycle among the edges the cut takes: edge 10 repeats edge 3's ends
    u2, v2 = u.copy(), v.copy()
    u2[10], v2[10] = u[3], v[3]
    with pytest.raises(nnm.NNMError, match="-1"):
        nnm.cluster_cut_device(_tree_from_edges(nnm, u2, v2, s, np.sqrt(s)), kl1=1)
    # an end out of range
    v3 = v.copy()
    v3[5] = n
    with pytest.raises(nnm.NNMError, match="-1"):
        nnm.cluster_cut_device(_tree_from_edges(nnm, u, v3, s, np.sqrt(s)), kl1=1)
    # still fine afterwards
    lab, k = nnm.cluster_cut_device(tree, kl1=3)
    hlab, hk = nnm.cluster_cut(tree, kl1=3)
    assert k == hk == 3 and np.array_equal(lab, hlab)


def _caps_unsupported(nnm, tree):
    """The size caps and the priority are the host cut's: NNM_EUNSUPPORTED."""
    import ctypes
    from paper_1402_3789_amd import _native as N
    L = N.lib()
    n = tree.n
    nb = ctypes.c_size_t(0)
    N.check("ws", L.cluster_cut_device_workspace_size(n, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda:0")
    labels = torch.empty(n, dtype=torch.int32, device="cuda:0")
    k = ctypes.c_int64(0)
    for caps in [(3, 10, -1, 0), (3, -1, 50, 0), (3, -1, -1, 5)]:
        p = N.CutParams(*caps, math.inf)
        code = L.cluster_cut_device(ctypes.c_void_p(tree.raw.data_ptr()), n, ctypes.byref(p),
                                    ctypes.c_void_p(ws.data_ptr()), nb.value,
                                    ctypes.c_void_p(labels.data_ptr()), ctypes.byref(k),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert code == N.NNM_EUNSUPPORTED, caps
