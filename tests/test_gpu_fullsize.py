"""Full-size parity (N = 2,000,000, D = 25) on properties the oracle can
check one row at a time, in the launch configuration the benchmark times
(and the exact kNN of sampled rows for knn_build at full size).

A spanning tree is the key-ordered minimum spanning tree iff every tree
edge is the smallest pair across the cut it defines.  At full size the
oracle cannot build the whole tree, so these tests check:
  * structure: n-1 edges, u < v, strictly sorted by key, one component;
  * weights: s of sampled edges equals the oracle's FP64 key, w = sqrt(s);
  * for sampled points i, the smallest pair (i, j) over all j (oracle, one
    row) is a tree edge -- the cut property for the cut {i};
  * for sampled tree edges whose smaller side A has at most 48 points, the
    smallest pair between A and the rest (oracle, |A| rows) is that edge.
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_FULL = 2_000_000


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def nnm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_3789_amd as m
    return m


def _structure(n, u, v, s):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    assert len(u) == n - 1
    assert np.all(u < v) and u.min() >= 0 and v.max() < n
    ds = np.diff(s)
    tie = ds == 0
    du = np.diff(u.astype(np.int64))
    dv = np.diff(v.astype(np.int64))
    assert np.all((ds > 0) | (tie & ((du > 0) | ((du == 0) & (dv > 0)))))
    g = coo_matrix((np.ones(n - 1), (u, v)), shape=(n, n))
    nc, _ = connected_components(g, directed=False)
    assert nc == 1


def _tree_children(n, u, v):
    """BFS order from 0, parent of every node, subtree sizes."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import breadth_first_order
    g = coo_matrix((np.ones(n - 1), (u, v)), shape=(n, n)).tocsr()
    order, parent = breadth_first_order(g, 0, directed=False, return_predecessors=True)
    size = np.ones(n, np.int64)
    for x in order[::-1][:-1]:
        size[parent[x]] += size[x]
    return order, parent, size


def _check_full(nnm, X, precision, rng):
    n = X.shape[0]
    Xd = torch.from_numpy(X).to("cuda:0")
    tree = nnm.mst_build(Xd, precision=precision)
    torch.cuda.synchronize()
    u, v, s, w = tree.to_numpy()
    _say("tree built", precision, tree.report["rounds"], "rounds")
    _structure(n, u, v, s)
    # weights of sampled edges
    for e in rng.choice(n - 1, size=1500, replace=False):
        assert s[e] == oracle.sqdist(X[u[e]], X[v[e]])
    assert np.array_equal(w, np.sqrt(s))
    # nearest-neighbour edges of sampled points
    keys = set(zip(u.tolist(), v.tolist()))
    rows = rng.choice(n, size=160, replace=False)
    j, sj = oracle.nn_outside(X, None, rows=rows)
    for i, jj, ss in zip(rows.tolist(), j.tolist(), sj.tolist()):
        assert (min(i, jj), max(i, jj)) in keys, (i, jj, ss)
    _say("nearest-neighbour edges ok")
    # cut property for small-side edges
    order, parent, size = _tree_children(n, u, v)
    small = np.nonzero((size <= 48) & (size >= 2) & (parent >= 0))[0]
    pick = rng.choice(small, size=min(12, small.size), replace=False)
    children = {}
    for x in order[1:]:
        children.setdefault(int(parent[x]), []).append(int(x))
    for c in pick.tolist():
        side = [c]
        k = 0
        while k < len(side):
            side.extend(children.get(side[k], []))
            k += 1
        lab = np.zeros(n, np.int32)
        lab[np.array(side)] = 1
        jj, ss = oracle.nn_outside(X, lab, rows=np.array(side))
        best = min((float(ss[q]), min(side[q], int(jj[q])), max(side[q], int(jj[q])))
                   for q in range(len(side)))
        p = int(parent[c])
        e_lo, e_hi = min(c, p), max(c, p)
        assert (best[1], best[2]) == (e_lo, e_hi), (c, p, best)
        assert best[0] == oracle.sqdist(X[e_lo], X[e_hi])
    _say("cut property ok on", len(pick), "edges")
    return tree


@pytest.fixture(scope="module")
def aniso():
    X, _ = W.aniso500(0, n=N_FULL)
    return X


def test_aniso500_full_size_fp16(nnm, aniso):
    rng = np.random.default_rng(2024)
    X = aniso
    _say("aniso500 full", X.shape)
    tree = _check_full(nnm, X, "fp16", rng)
    labels, k = nnm.cluster_cut(tree, kl1=500)
    assert k == 500 and labels.shape[0] == N_FULL


def test_int16grid_full_size_fp8(nnm):
    rng = np.random.default_rng(2025)
    X = W.int16grid(0, n=N_FULL)
    _say("int16grid full", X.shape)
    tree = _check_full(nnm, X, "fp8", rng)
    assert tree.report["integer_mode"] == 1 and tree.report["max_abs_err"] == 0.0


@pytest.mark.parametrize("k", [16, 32])
def test_aniso500_full_size_knn(nnm, aniso, k):
    # exact k nearest neighbours of every point at full size: sampled rows
    # against the oracle's exact kNN of those rows
    X = aniso
    rng = np.random.default_rng(2026 + k)
    rows = rng.choice(X.shape[0], size=96, replace=False)
    _say("aniso500 full knn", k)
    idx, s, ln = nnm.knn_build(torch.from_numpy(X).to("cuda:0"), k=k, precision="fp16")
    torch.cuda.synchronize()
    oi, os_, ol = oracle.knn(X, k, rows=rows)
    assert np.array_equal(idx.cpu().numpy()[rows], oi)
    assert np.array_equal(s.cpu().numpy()[rows], os_)
    assert np.array_equal(ln.cpu().numpy()[rows], ol)
    _say("knn rows identical", k)
