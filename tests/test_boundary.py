"""The C-ABI boundary on the CPU: symbols, argument checks, host-side cut.

No test here launches GPU work: only calls that fail their argument checks
(before any device call) and the host-only cluster_cut are exercised.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from golden_io import read_fixture
from paper_1402_3789_amd import _native as N
import paper_1402_3789_amd as nnm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nnm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(?:nnm_status|void|const char \*)\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = N.lib()
    declared = _declared()
    assert set(declared) == set(N.exported_symbols())
    for name in declared:
        assert hasattr(L, name), name


def test_struct_layouts():
    assert ctypes.sizeof(N.Edge) == 24
    assert ctypes.sizeof(N.CutParams) == 40
    assert ctypes.sizeof(N.Options) == 64
    assert ctypes.sizeof(N.Instance) == 40


def test_strerror_and_defaults():
    assert N.strerror(0) == "ok"
    assert "non-finite" in N.strerror(N.NNM_ENONFINITE)
    assert N.strerror(-99) == "unknown status"
    o = N.Options()
    N.lib().nnm_default_options(ctypes.byref(o))
    assert o.precision == N.PREC["auto"] and o.knn_k == 0


def _ws(n, d, **kw):
    o = nnm.options(**kw)
    nb = ctypes.c_size_t(0)
    code = N.lib().mst_workspace_size(n, d, ctypes.byref(o), ctypes.byref(nb))
    return code, nb.value


def test_workspace_size_checks():
    assert _ws(0, 8)[0] == N.NNM_EINVAL
    assert _ws(10, 0)[0] == N.NNM_EINVAL
    assert _ws(10, 33)[0] == N.NNM_EINVAL
    assert _ws(10, 27, precision="bf16")[0] == N.NNM_EUNSUPPORTED
    assert _ws(10, 27, precision="fp8")[0] == N.NNM_EUNSUPPORTED
    code, b = _ws(10, 27, precision="auto")
    assert code == 0 and b > 0
    code, b1 = _ws(1000, 25)
    code2, b2 = _ws(100000, 25)
    assert code == 0 and code2 == 0 and b2 > b1
    nb = ctypes.c_size_t(0)
    assert N.lib().knn_workspace_size(100, 8, 0, None, ctypes.byref(nb)) == N.NNM_EINVAL
    assert N.lib().knn_workspace_size(100, 8, 33, None, ctypes.byref(nb)) == N.NNM_EINVAL
    assert N.lib().knn_workspace_size(100, 8, 8, None, ctypes.byref(nb)) == 0


def test_entry_points_reject_bad_arguments_before_device_work():
    L = N.lib()
    o = nnm.options()
    rep = N.Report()
    fake = ctypes.c_void_p(0x1000)    # never dereferenced: checks fail first
    # null X, n < 1, d out of range, ld < d, short workspace
    assert L.mst_build(None, 10, 4, 4, ctypes.byref(o), fake, 1 << 30, fake, None,
                       ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.mst_build(fake, 0, 4, 4, ctypes.byref(o), fake, 1 << 30, fake, None,
                       ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.mst_build(fake, 10, 0, 4, ctypes.byref(o), fake, 1 << 30, fake, None,
                       ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.mst_build(fake, 10, 40, 40, ctypes.byref(o), fake, 1 << 30, fake, None,
                       ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.mst_build(fake, 10, 4, 3, ctypes.byref(o), fake, 1 << 30, fake, None,
                       ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.mst_build(fake, 10, 4, 4, ctypes.byref(o), fake, 16, fake, None,
                       ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.mst_build(fake, 10, 4, 4, ctypes.byref(o), fake, 1 << 30, None, None,
                       ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.knn_build(fake, 10, 4, 4, 0, ctypes.byref(o), fake, 1 << 30, fake, fake, fake,
                       None, ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.knn_build(fake, 10, 4, 4, 4, ctypes.byref(o), fake, 1 << 30, None, fake, fake,
                       None, ctypes.byref(rep)) == N.NNM_EINVAL


def test_noalloc_rejects_bad_and_oversized_inputs_before_device_work():
    L = N.lib()
    o = nnm.options()
    rep = N.Report()
    fake = ctypes.c_void_p(0x1000)    # never dereferenced: checks fail first
    assert L.mst_build_noalloc(None, 10, 4, 4, ctypes.byref(o), fake, None,
                               ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.mst_build_noalloc(fake, 0, 4, 4, ctypes.byref(o), fake, None,
                               ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.mst_build_noalloc(fake, 10, 33, 33, ctypes.byref(o), fake, None,
                               ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.mst_build_noalloc(fake, 10, 4, 3, ctypes.byref(o), fake, None,
                               ctypes.byref(rep)) == N.NNM_EINVAL
    assert L.mst_build_noalloc(fake, 10, 4, 4, ctypes.byref(o), None, None,
                               ctypes.byref(rep)) == N.NNM_EINVAL
    # the largest n whose workspace fits the fixed scratch, and one far past it
    nb = ctypes.c_size_t(0)
    assert L.mst_workspace_size(65536, 25, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert nb.value <= N.NOALLOC_SCRATCH_BYTES
    assert L.mst_workspace_size(300_000, 25, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert nb.value > N.NOALLOC_SCRATCH_BYTES
    code = L.mst_build_noalloc(fake, 300_000, 25, 25, ctypes.byref(o), fake, None,
                               ctypes.byref(rep))
    assert code == N.NNM_ETOOLARGE and "scratch" in N.strerror(code)


def _random_tree(rng, n, d=3, ties=False):
    X = rng.standard_normal((n, d)).astype(np.float32)
    if ties:
        X = np.round(X * 2).astype(np.float32)
    return X, oracle.prim_mst(X)


def test_cut_matches_oracle_cut_on_random_settings():
    rng = np.random.default_rng(101)
    for trial in range(300):
        n = int(rng.integers(1, 120))
        X, (u, v, s, w) = _random_tree(rng, n, ties=trial % 2 == 0)
        kl1 = int(rng.choice([0, 1, 2, 3, 5, 10]))
        kl2 = int(rng.choice([-1, 1, 3, 8]))
        kl3 = int(rng.choice([-1, 2, 5, 12]))
        kl4 = int(rng.choice([0, 1, 2, 4, 9]))
        dmax = float(rng.choice([math.inf, 0.5, 1.0, 2.0]))
        got, k = nnm.cluster_cut((u, v, s, w), n, kl1, kl2, kl3, kl4, dmax)
        exp, ke = oracle.cut(u, v, s, w, n, kl1, kl2, kl3, kl4, dmax)
        assert k == ke and np.array_equal(got, exp), (trial, kl1, kl2, kl3, kl4, dmax)


def test_cut_golden_line7():
    X, _, cuts = read_fixture("cut_line7.txt")
    u, v, s, w = oracle.prim_mst(X)
    for kl1, kl4, dmax, lab in cuts:
        got, k = nnm.cluster_cut((u, v, s, w), X.shape[0], kl1=kl1, kl4=kl4, dmax=dmax)
        assert got.tolist() == lab


def test_cut_golden_size_limits_line7():
    X, _, cuts = read_fixture("cut_kl23_line7.txt")
    u, v, s, w = oracle.prim_mst(X)
    for kw, lab in cuts:
        got, k = nnm.cluster_cut((u, v, s, w), X.shape[0], **kw)
        assert got.tolist() == lab, kw
        assert k == max(lab) + 1


def test_cut_rejects_bad_edges():
    u = np.array([0, 1], np.int32)
    v = np.array([1, 2], np.int32)
    s = np.array([2.0, 1.0])
    with pytest.raises(N.NNMError):
        nnm.cluster_cut((u, v, s, np.sqrt(s)), 3)                       # unsorted
    with pytest.raises(N.NNMError):
        nnm.cluster_cut((np.array([1, 1], np.int32), np.array([0, 2], np.int32),
                         np.array([1.0, 2.0]), np.array([1.0, 1.5])), 3)   # u > v
    with pytest.raises(N.NNMError):
        nnm.cluster_cut((u, np.array([1, 5], np.int32), np.array([1.0, 2.0]),
                         np.array([1.0, 1.5])), 3)                      # v out of range
    lab, k = nnm.cluster_cut((u[:0], v[:0], s[:0], s[:0]), 1)
    assert k == 1 and lab.tolist() == [0]
    # w decreasing along the key order (w must be sqrt(s), nondecreasing)
    with pytest.raises(N.NNMError):
        nnm.cluster_cut((u, v, np.array([1.0, 2.0]), np.array([1.5, 1.0])), 3)
    # not a tree: the third edge closes a cycle (heap path, with and without KL4)
    cu = np.array([0, 0, 1], np.int32)
    cv = np.array([1, 2, 2], np.int32)
    cs = np.array([1.0, 2.0, 3.0])
    for kw in ({}, dict(kl4=3), dict(kl2=5)):
        with pytest.raises(N.NNMError):
            nnm.cluster_cut((cu, cv, cs, np.sqrt(cs)), 4, **kw)


def test_cut_rejects_cycle_on_forest_path():
    rng = np.random.default_rng(17)
    n = 70_001
    u, v, s, w = _big_sorted_tree(rng, n)
    # the last edge repeats an earlier one (with a larger key): a cycle
    u, v, s = u.copy(), v.copy(), s.copy()
    u[-1], v[-1], s[-1] = u[10], v[10], s[-2] + 1.0
    w = np.sqrt(s)
    with pytest.raises(N.NNMError):
        nnm.cluster_cut((u, v, s, w), n)
    with pytest.raises(N.NNMError):
        nnm.cluster_cut((u, v, s, w), n, dmax=1e9)


def _big_sorted_tree(rng, n):
    """A random spanning tree with key-sorted edges (ties included)."""
    i = np.arange(1, n, dtype=np.int64)
    par = (rng.random(n - 1) * i).astype(np.int64)
    u = np.minimum(par, i).astype(np.int32)
    v = np.maximum(par, i).astype(np.int32)
    s = np.round(rng.random(n - 1) * 1000.0) / 1000.0      # many equal keys
    o = np.lexsort((v, u, s))
    u, v, s = u[o], v[o], s[o]
    return u, v, s, np.sqrt(s)


def test_cut_large_forest_path_matches_oracle():
    """n >= 65536 without KL2/KL3/KL4 takes the threaded forest path."""
    rng = np.random.default_rng(7)
    n = 200_003
    u, v, s, w = _big_sorted_tree(rng, n)
    for kl1, dmax in [(0, math.inf), (500, math.inf), (1, math.inf), (n + 5, math.inf),
                      (0, float(np.median(w))), (64, 0.2), (500, 0.0), (0, math.nan)]:
        got, k = nnm.cluster_cut((u, v, s, w), n, kl1=kl1, dmax=dmax)
        exp, ke = oracle.cut(u, v, s, w, n, kl1, -1, -1, 0, dmax)
        assert k == ke and np.array_equal(got, exp), (kl1, dmax)
    # and the general path at the same size
    got, k = nnm.cluster_cut((u, v, s, w), n, kl1=100, kl4=3)
    exp, ke = oracle.cut(u, v, s, w, n, 100, -1, -1, 3, math.inf)
    assert k == ke and np.array_equal(got, exp)


def test_autotune_rejects_bad_arguments_before_device_work():
    L = N.lib()
    o = nnm.options("fp16")
    inst = (N.Instance * 1)()
    inst[0].X_dev = 1234
    inst[0].n = 100
    inst[0].d = 4
    inst[0].ld = 4
    inst[0].edges_dev = 5678
    best = N.Options()
    nb = ctypes.c_size_t(0)
    assert L.mst_autotune_workspace_size(inst, 1, ctypes.byref(o), ctypes.byref(nb)) == N.NNM_OK
    assert nb.value > 0
    # null workspace, reps out of range, short workspace, empty batch
    assert L.mst_autotune(inst, 1, ctypes.byref(o), None, nb.value, None, 1, ctypes.byref(best),
                          None, None) == N.NNM_EINVAL
    assert L.mst_autotune(inst, 1, ctypes.byref(o), ctypes.c_void_p(1), nb.value, None, 0,
                          ctypes.byref(best), None, None) == N.NNM_EINVAL
    assert L.mst_autotune(inst, 1, ctypes.byref(o), ctypes.c_void_p(1), nb.value - 1, None, 1,
                          ctypes.byref(best), None, None) == N.NNM_EINVAL
    assert L.mst_autotune(inst, 0, ctypes.byref(o), ctypes.c_void_p(1), nb.value, None, 1,
                          ctypes.byref(best), None, None) == N.NNM_EINVAL
    inst[0].d = 40
    assert L.mst_autotune_workspace_size(inst, 1, ctypes.byref(o), ctypes.byref(nb)) == N.NNM_EINVAL


def test_autotune_cache_keys_and_store(tmp_path):
    from paper_1402_3789_amd import autotune as A
    k1 = A.bucket_key(2_000_000, 25, "fp16", 1, "gfx950")
    assert k1 == "gfx950|fp16|n1048576|d26|single"
    assert A.bucket_key(3_000, 4, "bf16", 10, "gfx950") == "gfx950|bf16|n4096|d8|batch"
    assert A.bucket_key(1, 32, "fp32", 1, "gfx950") == "gfx950|fp32|n1|d32|single"
    path = str(tmp_path / "c.json")
    assert A.lookup(2_000_000, 25, "fp16", cache=path, arch_name="gfx950", shipped=False) is None
    ent = {"knn_k": 8, "split_target0": 2048, "split_target": 16384, "graph": 1, "ms": 1.0}
    A._store(path, k1, ent)
    A._store(path, A.bucket_key(5000, 9, "fp16", 1, "gfx950"), dict(ent, knn_k=4))
    assert A.lookup(1_900_000, 26, "fp16", cache=path, arch_name="gfx950") == ent
    assert A.lookup(1_900_000, 26, "fp16", cache=path, arch_name="gfx942") is None
    # the shipped table: every entry names a knob value of the tuner's grid
    import json
    for key, e in json.load(open(A.SHIPPED)).items():
        assert key.startswith("gfx950|") and e["knn_k"] in (0, 4, 6, 8, 12)
        assert e["split_target0"] in (0, 2048, 4096, 8192)
        assert e["split_target"] in (0, 4096, 8192, 16384) and e["graph"] in (0, 1)
    assert A.lookup(4096, 12, "fp16", cache=path, arch_name="gfx950")["knn_k"] == 4


def test_allpairs_cut_rejects_bad_arguments_before_device_work():
    L = N.lib()
    o = nnm.options("fp16")
    p = N.CutParams(0, 5, -1, 0, math.inf)
    nb = ctypes.c_size_t(0)
    assert L.allpairs_cut_workspace_size(1000, 8, 0, ctypes.byref(o), ctypes.byref(nb)) == N.NNM_OK
    assert nb.value > 0
    assert L.allpairs_cut_workspace_size(1000, 8, 33, ctypes.byref(o), ctypes.byref(nb)) == N.NNM_EINVAL
    labels = np.zeros(1000, np.int32)
    k = ctypes.c_int64(0)

    edges = np.zeros((999, 3), np.float64)
    ev = edges.view(np.int32).reshape(-1, 6)
    ev[:, 0] = 0
    ev[:, 1] = np.arange(1, 1000)

    def call(X=1234, n=1000, d=8, ld=8, prm=p, kk=0, ws=1, wsb=None, e=edges):
        return L.cluster_cut_allpairs(ctypes.c_void_p(X), n, d, ld,
                                      ctypes.c_void_p(e.ctypes.data if e is not None else None),
                                      ctypes.byref(prm), kk, ctypes.byref(o), ctypes.c_void_p(ws),
                                      nb.value if wsb is None else wsb, None,
                                      ctypes.c_void_p(labels.ctypes.data), ctypes.byref(k), None)
    assert call(X=0) == N.NNM_EINVAL
    assert call(e=None) == N.NNM_EINVAL
    bad = edges.copy()
    bad.view(np.int32).reshape(-1, 6)[5, 1] = 0          # u >= v
    assert call(e=bad) == N.NNM_EINVAL
    assert call(ws=0) == N.NNM_EINVAL
    assert call(kk=40) == N.NNM_EINVAL
    assert call(ld=4) == N.NNM_EINVAL
    assert call(wsb=nb.value - 1) == N.NNM_EINVAL
    assert call(prm=N.CutParams(0, 5, -1, 0, float("nan"))) == N.NNM_EINVAL
    assert call(prm=N.CutParams(0, 5, -1, 0, -1.0)) == N.NNM_EINVAL


def test_metric_option_checks():
    L = N.lib()
    nb = ctypes.c_size_t(0)
    for name, prec, want in (("l1", "bf16", N.NNM_EUNSUPPORTED), ("linf", "fp16", N.NNM_EUNSUPPORTED),
                             ("linf", "fp8", N.NNM_EUNSUPPORTED), ("l1", "auto", N.NNM_OK),
                             ("linf", "fp32", N.NNM_OK), ("cosine", "bf16", N.NNM_OK)):
        o = nnm.options(prec, metric=name)
        assert L.mst_workspace_size(1000, 8, ctypes.byref(o), ctypes.byref(nb)) == want, (name, prec)
    o = nnm.options("fp32")
    o.metric = 7
    assert L.mst_workspace_size(1000, 8, ctypes.byref(o), ctypes.byref(nb)) == N.NNM_EINVAL
    # the cosine metric keeps its scaled rows in the workspace
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    L.mst_workspace_size(1000, 8, ctypes.byref(nnm.options("fp16")), ctypes.byref(a))
    L.mst_workspace_size(1000, 8, ctypes.byref(nnm.options("fp16", metric="cosine")), ctypes.byref(b))
    assert b.value >= a.value + 1000 * 8 * 4


def test_pminimal_rejects_bad_arguments_before_device_work():
    L = N.lib()
    o = nnm.options("fp16")
    nb = ctypes.c_size_t(0)
    assert L.pminimal_workspace_size(5000, 10, ctypes.byref(o), ctypes.byref(nb)) == N.NNM_OK
    mb = ctypes.c_size_t(0)
    assert L.mst_workspace_size(5000, 10, ctypes.byref(o), ctypes.byref(mb)) == N.NNM_OK
    assert nb.value > mb.value
    rep = N.Report()
    bad = [dict(P=-1), dict(X=0), dict(ws=0), dict(wsb=nb.value - 1), dict(e=0), dict(d=40)]
    for b in bad:
        a = dict(X=1234, P=10, ws=1, wsb=nb.value, e=5678, d=10)
        a.update(b)
        code = L.mst_build_pminimal(ctypes.c_void_p(a["X"]), 5000, a["d"], max(a["d"], 10), a["P"],
                                    ctypes.byref(o), ctypes.c_void_p(a["ws"]), a["wsb"],
                                    ctypes.c_void_p(a["e"]), None, ctypes.byref(rep))
        assert code == N.NNM_EINVAL, b


def test_cut_device_argument_checks():
    """Refusals that happen before any device work (no GPU needed)."""
    L = N.lib()
    nb = ctypes.c_size_t(0)
    assert L.cluster_cut_device_workspace_size(0, ctypes.byref(nb)) == N.NNM_EINVAL
    assert L.cluster_cut_device_workspace_size(1 << 31, ctypes.byref(nb)) == N.NNM_EINVAL
    assert L.cluster_cut_device_workspace_size(1000, None) == N.NNM_EINVAL
    assert L.cluster_cut_device_workspace_size(1000, ctypes.byref(nb)) == 0 and nb.value >= 12 * 1000
    fake = ctypes.c_void_p(0x1000)                  # never dereferenced on these paths
    k = ctypes.c_int64(0)
    p = N.CutParams(3, -1, -1, 0, float("inf"))
    call = lambda n, e, prm, ws, wsb, lab, kk: L.cluster_cut_device(e, n, prm, ws, wsb, lab, kk, None)
    assert call(0, fake, ctypes.byref(p), fake, nb.value, fake, ctypes.byref(k)) == N.NNM_EINVAL
    assert call(1000, None, ctypes.byref(p), fake, nb.value, fake, ctypes.byref(k)) == N.NNM_EINVAL
    assert call(1000, fake, None, fake, nb.value, fake, ctypes.byref(k)) == N.NNM_EINVAL
    assert call(1000, fake, ctypes.byref(p), None, nb.value, fake, ctypes.byref(k)) == N.NNM_EINVAL
    assert call(1000, fake, ctypes.byref(p), fake, nb.value, None, ctypes.byref(k)) == N.NNM_EINVAL
    assert call(1000, fake, ctypes.byref(p), fake, nb.value, fake, None) == N.NNM_EINVAL
    assert call(1000, fake, ctypes.byref(p), fake, nb.value - 1, fake, ctypes.byref(k)) == N.NNM_EINVAL
    for caps in [(3, 10, -1, 0), (3, -1, 50, 0), (3, -1, -1, 5)]:
        q = N.CutParams(*caps, float("inf"))
        assert call(1000, fake, ctypes.byref(q), fake, nb.value, fake, ctypes.byref(k)) == N.NNM_EUNSUPPORTED
