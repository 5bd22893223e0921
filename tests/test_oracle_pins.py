"""Pins for the CPU oracle against facts other than the oracle itself.

Each test ties one part of the oracle to something the paper or mathematics
fixes: exact rational arithmetic for the key of eq. (1), brute-force Kruskal
for the tree (unique under the (s, min, max) key), the cycle property, closed
forms, SciPy's single-linkage merge heights, hand-derived fixtures, the
epsilon-graph for the distance threshold and the paper's all-pairs process
for the KL1 / KL4 / threshold cut.
"""
import zlib
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import checks
from golden_io import read_fixture

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ---- the key of eq. (1) ------------------------------------------------

def _exact_sq(a, b):
    return sum((Fraction(float(x)) - Fraction(float(y))) ** 2 for x, y in zip(a, b))


@pytest.mark.parametrize("scale", [1e-30, 1e-3, 1.0, 7.5, 1e6, 1e30])
def test_key_within_fp64_bound_of_exact(scale):
    rng = np.random.default_rng(11)
    for _ in range(200):
        d = int(rng.integers(1, 33))
        a = (rng.standard_normal(d) * scale).astype(np.float32)
        b = (a + rng.standard_normal(d) * scale * 10.0 ** rng.uniform(-6, 0)).astype(np.float32)
        s = oracle.sqdist(a, b)
        ex = _exact_sq(a, b)
        bound = (d + 2) * 2.0 ** -53 * float(ex)
        assert abs(Fraction(s) - ex) <= Fraction(bound) + Fraction(0)


def test_key_is_exact_on_small_integers():
    rng = np.random.default_rng(5)
    X = rng.integers(0, 16, size=(300, 25)).astype(np.float32)
    for _ in range(500):
        i, j = rng.integers(0, 300, size=2)
        s = oracle.sqdist(X[i], X[j])
        assert s == float(int(((X[i].astype(np.int64) - X[j].astype(np.int64)) ** 2).sum()))


def test_key_summation_order_is_fixed():
    # Squares of 2^-27 are 2^-54, below half an ulp of 1.0.  Added left to
    # right after 1.0 they vanish one by one; added before 1.0 they reach
    # 1.5 * 2^-53 and round 1.0 up.  The key must add features in order
    # 0..D-1, each widened exactly from FP32.
    t = 2.0 ** -27
    z = np.zeros(4, np.float32)
    assert oracle.sqdist(np.array([1.0, t, t, t], np.float32), z) == 1.0
    assert oracle.sqdist(np.array([t, t, t, 1.0], np.float32), z) == 1.0 + 2.0 ** -52


# ---- the tree --------------------------------------------------------------

def _inputs(kind, n, d, rng):
    if kind == "normal":
        return rng.standard_normal((n, d)).astype(np.float32)
    if kind == "lattice":
        return rng.integers(0, 3, size=(n, d)).astype(np.float32)
    if kind == "dups":
        base = rng.standard_normal((max(n // 4, 1), d)).astype(np.float32)
        return base[rng.integers(0, base.shape[0], size=n)]
    if kind == "collinear":
        t = rng.standard_normal(n)
        v = rng.standard_normal(d)
        return (t[:, None] * v[None, :]).astype(np.float32)
    if kind == "tiny":
        return (1.0 + rng.integers(0, 4, size=(n, d)) * 2.0 ** -20).astype(np.float32)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["normal", "lattice", "dups", "collinear", "tiny"])
def test_prim_equals_full_kruskal(kind):
    seed = zlib.crc32(kind.encode())      # fixed per kind, unlike str hash()
    rng = np.random.default_rng(seed)
    for trial in range(40):
        n = int(rng.integers(2, 160))
        d = int(rng.choice([1, 2, 3, 8, 25]))
        X = _inputs(kind, n, d, rng)
        u, v, s, w = oracle.prim_mst(X)
        ku, kv, ks = checks.kruskal_full(X)
        assert np.array_equal(u, ku) and np.array_equal(v, kv), (kind, seed, trial)
        assert np.array_equal(s, ks), (kind, seed, trial)
        assert np.array_equal(w, np.sqrt(s))


def test_prim_equals_kruskal_n512():
    rng = np.random.default_rng(3)
    X = rng.integers(0, 4, size=(512, 3)).astype(np.float32)
    u, v, s, _ = oracle.prim_mst(X)
    ku, kv, ks = checks.kruskal_full(X)
    assert np.array_equal(u, ku) and np.array_equal(v, kv) and np.array_equal(s, ks)


def _tree_invariants(n, u, v, s):
    assert len(u) == n - 1
    assert np.all(u < v) and np.all(u >= 0) and np.all(v < n)
    keys = list(zip(s.tolist(), u.tolist(), v.tolist()))
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    par = list(range(n))

    def find(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x
    for a, b in zip(u.tolist(), v.tolist()):
        ra, rb = find(a), find(b)
        assert ra != rb, "cycle"
        par[ra] = rb
    assert len({find(i) for i in range(n)}) == 1


def test_blobs8_tree_cycle_property_and_invariants():
    from workloads import blobs8
    X, _ = blobs8(0)
    u, v, s, w = oracle.prim_mst(X)
    _tree_invariants(X.shape[0], u, v, s)
    assert checks.cycle_property_violations(X, u, v, s) == 0


def test_cycle_check_detects_a_wrong_tree():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((60, 4)).astype(np.float32)
    u, v, s, _ = oracle.prim_mst(X)
    # swap the heaviest tree edge for another pair that reconnects the tree
    S = checks.key_matrix(X)
    u2, v2, s2 = u.copy(), v.copy(), s.copy()
    keep = np.ones(len(u), bool)
    keep[-1] = False
    par = list(range(60))

    def find(x):
        while par[x] != x:
            x = par[x]
        return x
    for a, b in zip(u[keep].tolist(), v[keep].tolist()):
        par[find(a)] = find(b)
    side = np.array([find(i) == find(int(u[-1])) for i in range(60)])
    cand = [(S[i, j], i, j) for i in range(60) for j in range(i + 1, 60)
            if side[i] != side[j] and (i, j) != (int(u[-1]), int(v[-1]))]
    sn, a, b = max(cand)
    u2[-1], v2[-1], s2[-1] = a, b, sn
    order = np.lexsort((v2, u2, s2))
    assert checks.cycle_property_violations(X, u2[order], v2[order], s2[order]) > 0


def test_weights_match_scipy_single_linkage():
    from scipy.cluster.hierarchy import linkage
    rng = np.random.default_rng(7)
    for _ in range(10):
        n = int(rng.integers(5, 400))
        d = int(rng.integers(1, 26))
        X = rng.uniform(0, 1, size=(n, d)).astype(np.float32)
        _, _, _, w = oracle.prim_mst(X)
        h = np.sort(linkage(X.astype(np.float64), method="single")[:, 2])
        assert np.allclose(w, h, rtol=1e-12, atol=0)


def test_closed_form_one_feature():
    rng = np.random.default_rng(9)
    for _ in range(20):
        n = int(rng.integers(2, 300))
        x = rng.integers(0, n // 2 + 2, size=n).astype(np.float32)
        u, v, s, _ = oracle.prim_mst(x[:, None])
        # sort by value then index; adjacent pairs in that order are the tree
        order = np.lexsort((np.arange(n), x))
        exp = []
        for a, b in zip(order[:-1], order[1:]):
            lo, hi = min(a, b), max(a, b)
            exp.append((float(x[a] - x[b]) ** 2, int(lo), int(hi)))
        # equal values: every pair among duplicates has s=0 and the tie-break
        # links each duplicate to the smallest index of its group, which the
        # adjacency chain gives only when groups are index-sorted: compare the
        # multiset of s and the number of zero edges instead of the pairs
        assert sorted(e[0] for e in exp) == s.tolist()
        if len(np.unique(x)) == n:
            assert sorted(exp) == list(zip(s.tolist(), u.tolist(), v.tolist()))


def test_closed_form_equally_spaced_in_index_order():
    n = 100
    X = (np.arange(n, dtype=np.float32)[:, None] * np.array([[0.5, -1.0, 2.0]], np.float32))
    u, v, s, _ = oracle.prim_mst(X)
    assert np.array_equal(u, np.arange(n - 1)) and np.array_equal(v, np.arange(1, n))
    assert np.all(s == 0.25 + 1.0 + 4.0)


def test_small_cases():
    u, v, s, w = oracle.prim_mst(np.array([[0.0, 0.0], [3.0, 4.0]], np.float32))
    assert (u.tolist(), v.tolist(), s.tolist(), w.tolist()) == ([0], [1], [25.0], [5.0])
    u, v, s, w = oracle.prim_mst(np.array([[1.0, 2.0]], np.float32))
    assert len(u) == 0


@pytest.mark.parametrize("name", ["line5.txt", "square_ties.txt", "duplicates.txt"])
def test_golden_trees(name):
    X, edges, _ = read_fixture(name)
    u, v, s, _ = oracle.prim_mst(X)
    assert list(zip(u.tolist(), v.tolist(), s.tolist())) == edges


# ---- the constrained cut ---------------------------------------------------

def test_golden_cut_line7():
    X, _, cuts = read_fixture("cut_line7.txt")
    u, v, s, w = oracle.prim_mst(X)
    for kl1, kl4, dmax, lab in cuts:
        got, k = oracle.cut(u, v, s, w, X.shape[0], kl1=kl1, kl4=kl4, dmax=dmax)
        assert got.tolist() == lab, (kl1, kl4, dmax)
        assert k == max(lab) + 1


def test_golden_cut_size_limits_line7():
    # KL2 / KL3 (with KL1, KL4 and dmax) against a hand-derived fixture
    X, _, cuts = read_fixture("cut_kl23_line7.txt")
    u, v, s, w = oracle.prim_mst(X)
    assert s.tolist() == [1.0, 4.0, 9.0, 16.0, 25.0, 36.0]
    for kw, lab in cuts:
        got, k = oracle.cut(u, v, s, w, X.shape[0], **kw)
        assert got.tolist() == lab, kw
        assert k == max(lab) + 1


def test_cut_kl1_equals_dropping_heaviest_edges():
    rng = np.random.default_rng(21)
    for _ in range(30):
        n = int(rng.integers(2, 200))
        X = rng.standard_normal((n, 3)).astype(np.float32)
        u, v, s, w = oracle.prim_mst(X)
        k = int(rng.integers(1, n + 1))
        got, kk = oracle.cut(u, v, s, w, n, kl1=k)
        assert kk == k
        assert np.array_equal(got, checks.drop_heaviest(n, u, v, k))


def test_cut_dmax_equals_epsilon_graph_components():
    rng = np.random.default_rng(22)
    for _ in range(30):
        n = int(rng.integers(2, 200))
        X = rng.integers(0, 6, size=(n, 2)).astype(np.float32)
        u, v, s, w = oracle.prim_mst(X)
        dmax = float(rng.choice([0.0, 1.0, 1.5, np.sqrt(2.0), 2.0, 3.3]))
        got, k = oracle.cut(u, v, s, w, n, dmax=dmax)
        exp, ke = checks.eps_components(X, dmax)
        assert k == ke and np.array_equal(got, exp)


def test_cut_kl1_kl4_dmax_equals_all_pairs_process():
    rng = np.random.default_rng(23)
    for trial in range(60):
        n = int(rng.integers(2, 28))
        X = rng.standard_normal((n, 2)).astype(np.float32)
        if trial % 3 == 0:
            X = np.round(X * 2).astype(np.float32)   # ties
        kl1 = int(rng.integers(0, 6))
        kl4 = int(rng.integers(0, 6))
        dmax = float(rng.choice([np.inf, 0.5, 1.0, 2.0]))
        u, v, s, w = oracle.prim_mst(X)
        got, k = oracle.cut(u, v, s, w, n, kl1=kl1, kl4=kl4, dmax=dmax)
        exp, ke = checks.agglo_allpairs(X, kl1=kl1, kl4=kl4, dmax=dmax)
        assert k == ke and np.array_equal(got, exp), (trial, kl1, kl4, dmax)


def test_cut_separated_blobs_give_generating_labels():
    rng = np.random.default_rng(24)
    for _ in range(10):
        k = int(rng.integers(2, 9))
        r = 1.0
        centres = rng.uniform(0, 100, size=(k, 4))
        # reject draws where two centres are closer than 5 r
        dd = np.sqrt(((centres[:, None] - centres[None]) ** 2).sum(-1)) + np.eye(k) * 1e9
        if dd.min() <= 5 * r:
            continue
        lab = rng.integers(0, k, size=300)
        lab[:k] = np.arange(k)
        dirs = rng.standard_normal((300, 4))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        X = (centres[lab] + dirs * rng.uniform(0, r, size=(300, 1))).astype(np.float32)
        u, v, s, w = oracle.prim_mst(X)
        got, kk = oracle.cut(u, v, s, w, 300, kl1=k)
        assert kk == k
        assert np.array_equal(got, checks.canonical(lab))


def test_blobs8_cut_recovers_blobs():
    from workloads import blobs8
    X, y = blobs8(0)
    u, v, s, w = oracle.prim_mst(X)
    got, k = oracle.cut(u, v, s, w, X.shape[0], kl1=8)
    assert k == 8
    assert np.array_equal(got, checks.canonical(y))


def test_cut_size_caps_are_monotone_blocks():
    # KL2 / KL3 (no printed example; see also the hand-derived fixture): a
    # blocked edge stays blocked and no cluster grows from two sides that
    # violate the caps.
    rng = np.random.default_rng(25)
    for _ in range(20):
        n = int(rng.integers(2, 120))
        X = rng.standard_normal((n, 3)).astype(np.float32)
        u, v, s, w = oracle.prim_mst(X)
        kl2 = int(rng.integers(1, 10))
        kl3 = int(rng.integers(2, 20))
        lab, k = oracle.cut(u, v, s, w, n, kl2=kl2, kl3=kl3)
        sizes = np.bincount(lab)
        assert sizes.max() <= max(kl3, 1)
        assert k >= 1


def test_cut_rejects_unsorted_edges():
    u = np.array([0, 1], np.int32)
    v = np.array([1, 2], np.int32)
    s = np.array([2.0, 1.0])
    with pytest.raises(ValueError):
        oracle.cut(u, v, s, np.sqrt(s), 3)


# ---- neighbour queries ------------------------------------------------------

def test_knn_matches_brute_force():
    rng = np.random.default_rng(31)
    X = rng.integers(0, 5, size=(300, 3)).astype(np.float32)
    S = checks.key_matrix(X)
    idx, s, ln = oracle.knn(X, 7)
    for i in range(300):
        js = np.array([j for j in range(300) if j != i])
        order = np.lexsort((js, S[i, js]))[:7]
        assert idx[i].tolist() == js[order].tolist()
        assert s[i].tolist() == S[i, js[order]].tolist()
        assert ln[i] == 7
    idx, s, ln = oracle.knn(X[:4], 7)
    assert ln.tolist() == [3, 3, 3, 3] and np.all(idx[:, 3:] == -1)


def test_nn_outside_matches_brute_force():
    rng = np.random.default_rng(32)
    X = rng.integers(0, 5, size=(200, 2)).astype(np.float32)
    lab = rng.integers(0, 6, size=200).astype(np.int32)
    S = checks.key_matrix(X)
    j, s = oracle.nn_outside(X, lab)
    for i in range(200):
        js = np.nonzero(lab != lab[i])[0]
        o = np.lexsort((js, S[i, js]))[0]
        assert j[i] == js[o] and s[i] == S[i, js[o]]
    j, s = oracle.nn_outside(X, np.zeros(200, np.int32))
    assert np.all(j == -1) and np.all(np.isinf(s))


# ---- the constrained process over all pairs ("Problem settings", KL1..KL4;
# "General description of the algorithm for constructing the set of minimum
# distances") -------------------------------------------------------------

def test_allpairs_process_equals_brute_force_with_size_caps():
    """oracle_cut_allpairs against the step-by-step brute force (every
    cluster pair's single-link key recomputed at every step), with KL2 and
    KL3 on as well as KL1, KL4 and dmax."""
    rng = np.random.default_rng(31)
    for trial in range(120):
        n = int(rng.integers(2, 26))
        X = rng.standard_normal((n, 2)).astype(np.float32)
        if trial % 3 == 0:
            X = np.round(X * 2).astype(np.float32)   # ties
        kl1 = int(rng.integers(0, 5))
        kl2 = int(rng.choice([-1, 1, 2, 3, 5, 8]))
        kl3 = int(rng.choice([-1, 2, 3, 4, 6, 10]))
        kl4 = int(rng.choice([0, 2, 3, 4]))
        dmax = float(rng.choice([np.inf, 0.7, 1.5, 3.0]))
        got, k = oracle.cut_allpairs(X, kl1=kl1, kl2=kl2, kl3=kl3, kl4=kl4, dmax=dmax)
        exp, ke = checks.agglo_allpairs(X, kl1=kl1, kl2=kl2, kl3=kl3, kl4=kl4, dmax=dmax)
        assert k == ke and np.array_equal(got, exp), (trial, kl1, kl2, kl3, kl4, dmax)


def test_allpairs_process_equals_tree_cut_without_size_caps():
    """With KL2 and KL3 off the process takes only tree edges (cut
    property), so it equals the cut of the tree."""
    rng = np.random.default_rng(32)
    for trial in range(12):
        n = int(rng.integers(50, 400))
        X = rng.standard_normal((n, 3)).astype(np.float32)
        kl1 = int(rng.integers(0, 12))
        kl4 = int(rng.choice([0, 2, 5, 20]))
        dmax = float(rng.choice([np.inf, 0.3, 0.8]))
        u, v, s, w = oracle.prim_mst(X)
        exp, ke = oracle.cut(u, v, s, w, n, kl1=kl1, kl4=kl4, dmax=dmax)
        got, k = oracle.cut_allpairs(X, kl1=kl1, kl4=kl4, dmax=dmax)
        assert k == ke and np.array_equal(got, exp), (trial, kl1, kl4, dmax)


def test_allpairs_process_bypasses_a_blocked_tree_edge():
    """Hand example on a line (KL3 = 3).  B = {0, 0.125, 0.25} unites first
    (keys 1/64); the tree edges A-B (A = -0.75, key 0.5625) and c-B
    (c = 1.125, key 0.765625) are then blocked (4 > 3 points); the pair A-c
    (key 1.875^2 = 3.515625) is not a tree edge, but the process over all
    pairs takes it: clusters {A, c} and B.  The cut of the tree keeps A and c
    apart."""
    X = np.array([[-0.75], [0.0], [0.125], [0.25], [1.125]], np.float32)
    got, k = oracle.cut_allpairs(X, kl3=3)
    assert k == 2 and got.tolist() == [0, 1, 1, 1, 0]
    u, v, s, w = oracle.prim_mst(X)
    assert (0, 4) not in set(zip(u.tolist(), v.tolist()))
    tl, tk = oracle.cut(u, v, s, w, 5, kl3=3)
    assert tk == 3 and tl.tolist() == [0, 1, 1, 1, 2]
    # KL1 = 2 stops there as well; KL1 = 3 stops before the bypass
    assert oracle.cut_allpairs(X, kl1=3, kl3=3)[1] == 3


# ---- other metrics ("Overall idea of the algorithm": another metric may be
# chosen in place of eq. (1)) ------------------------------------------------

@pytest.mark.parametrize("metric,name", [("l1", "cityblock"), ("linf", "chebyshev")])
def test_metric_keys_match_scipy(metric, name):
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(41)
    X = (rng.standard_normal((60, 7)) * rng.uniform(0.01, 100, size=7)).astype(np.float32)
    D = cdist(X.astype(np.float64), X.astype(np.float64), name)
    for i in range(0, 60, 7):
        for j in range(60):
            got = oracle.pair_key(X[i], X[j], metric)
            if metric == "linf":
                assert got == D[i, j]                       # a max of exact terms
            else:
                assert abs(got - D[i, j]) <= 8 * 2.0 ** -53 * D[i, j]
    # integer data: every key exact
    Xi = rng.integers(-50, 50, size=(30, 5)).astype(np.float32)
    Di = cdist(Xi.astype(np.float64), Xi.astype(np.float64), name)
    for i in range(30):
        for j in range(30):
            assert oracle.pair_key(Xi[i], Xi[j], metric) == Di[i, j]


@pytest.mark.parametrize("metric,name", [("l1", "cityblock"), ("linf", "chebyshev"),
                                         ("euclidean", "euclidean")])
def test_metric_tree_weights_match_scipy_single_linkage(metric, name):
    from scipy.cluster.hierarchy import linkage
    rng = np.random.default_rng(42)
    X = rng.standard_normal((300, 6)).astype(np.float32)
    u, v, s, w = oracle.prim_mst(X, metric=metric)
    Z = linkage(X.astype(np.float64), method="single", metric=name)
    assert np.allclose(np.sort(w), np.sort(Z[:, 2]), rtol=1e-12, atol=0)
    if metric != "euclidean":
        assert np.array_equal(s, w)


@pytest.mark.parametrize("metric", ["l1", "linf"])
def test_metric_tree_equals_kruskal(metric):
    """Prim under L1 / L-infinity against Kruskal over every pair's key
    (scipy's union-find-free minimum_spanning_tree on the dense matrix gives
    the same edge set when the keys are distinct)."""
    from scipy.sparse.csgraph import minimum_spanning_tree
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(43)
    X = rng.uniform(0, 1, size=(200, 5)).astype(np.float32)
    u, v, s, w = oracle.prim_mst(X, metric=metric)
    D = np.array([[oracle.pair_key(X[i], X[j], metric) for j in range(200)] for i in range(200)])
    T = minimum_spanning_tree(D).tocoo()
    # the tree's weights are unique whatever the ties; its edges are when
    # the keys are distinct
    assert np.array_equal(np.sort(T.data), s)
    if len(np.unique(D[np.triu_indices(200, 1)])) == 200 * 199 // 2:
        want = sorted((min(a, b), max(a, b)) for a, b in zip(T.row.tolist(), T.col.tolist()))
        assert sorted(zip(u.tolist(), v.tolist())) == want
    name = "cityblock" if metric == "l1" else "chebyshev"
    Dc = cdist(X.astype(np.float64), X.astype(np.float64), name)
    assert np.allclose(D, Dc, rtol=1e-14, atol=0)


def test_cosine_rows_and_tree():
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(44)
    X = rng.standard_normal((150, 8)).astype(np.float32)
    X[7] = 0.0                                   # a zero row stays zero
    Xn = oracle.normalize_rows(X)
    ref = X.astype(np.float64) / np.linalg.norm(X.astype(np.float64), axis=1, keepdims=True)
    ref[7] = 0.0
    assert np.array_equal(Xn, ref.astype(np.float32))
    norms = np.linalg.norm(Xn.astype(np.float64), axis=1)
    assert np.all(np.abs(norms[np.arange(150) != 7] - 1.0) < 1e-6) and norms[7] == 0.0
    u, v, s, w = oracle.prim_mst(X, metric="cosine")
    keep = np.arange(150) != 7
    C = cdist(X[keep].astype(np.float64), X[keep].astype(np.float64), "cosine")
    # tree edges between non-zero rows: s = |x^ - y^|^2 = 2 (1 - cos) up to rounding
    idx = np.cumsum(keep) - 1
    for a, b, sv in zip(u.tolist(), v.tolist(), s.tolist()):
        if a != 7 and b != 7:
            assert abs(sv - 2.0 * C[idx[a], idx[b]]) < 1e-6
    uu, vv, ss, ww = oracle.prim_mst(Xn)
    assert np.array_equal(uu, u) and np.array_equal(ss, s)
