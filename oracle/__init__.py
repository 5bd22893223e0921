"""CPU oracle for exact single-linkage clustering (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``liboracle.so`` (plain C, FP64, built from
``oracle.c`` by ``oracle/build.py``) and shares nothing with the GPU path.

Every function follows the paper's definitions as read in ``oracle.c``:
eq. (1) for the pair distance (as an FP64 squared distance with a fixed
summation order), the minimum-pair union process of the section on
constructing the set of minimum distances (as the key-ordered minimum
spanning tree) and the KL1..KL4 / distance-threshold settings of the
"Problem settings" and "Problem statement" sections (as a cut of that tree).

Parity status: every function here is pinned by the CPU tests in
``tests/test_oracle_pins.py``.  The KL2 / KL3 size caps have no printed
example in the paper: they are pinned, under the reading that applies them
to tree edges, by a fixture worked out by hand edge by edge
(``tests/golden/cut_kl23_line7.txt``); that reading itself differs from the
all-pairs process whenever a cap blocks a tree edge.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of oracle.c (a sanitizer build, say).
_LIBPATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    i64, i32, c_int, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.c_double
    vp = ctypes.c_void_p
    lib.oracle_prim_mst.argtypes = [_f32p, i64, i32, i64, _i32p, _i32p, _f64p, _f64p, c_int]
    lib.oracle_prim_mst.restype = c_int
    lib.oracle_cut.argtypes = [vp, vp, vp, vp, i64, i64, i64, i64, i64, dbl, _i32p,
                               ctypes.POINTER(i64)]
    lib.oracle_cut.restype = c_int
    lib.oracle_prim_mst_metric.argtypes = [_f32p, i64, i32, i64, i32, _i32p, _i32p, _f64p, _f64p,
                                            c_int]
    lib.oracle_prim_mst_metric.restype = c_int
    lib.oracle_knn_metric.argtypes = [_f32p, i64, i32, i64, i32, vp, i64, i32, _i32p, _f64p, _i32p,
                                       c_int]
    lib.oracle_knn_metric.restype = c_int
    lib.oracle_normalize_rows.argtypes = [_f32p, i64, i32, i64, _f32p]
    lib.oracle_normalize_rows.restype = c_int
    lib.oracle_pair_key.argtypes = [_f32p, _f32p, i32, i32]
    lib.oracle_pair_key.restype = dbl
    lib.oracle_cut_allpairs.argtypes = [_f32p, i64, i32, i64, i64, i64, i64, i64, dbl, _i32p,
                                         ctypes.POINTER(i64)]
    lib.oracle_cut_allpairs.restype = c_int
    lib.oracle_knn.argtypes = [_f32p, i64, i32, i64, vp, i64, i32, _i32p, _f64p, _i32p, c_int]
    lib.oracle_knn.restype = c_int
    lib.oracle_nn_outside.argtypes = [_f32p, i64, i32, i64, vp, vp, i64, _i32p, _f64p, c_int]
    lib.oracle_nn_outside.restype = c_int
    lib.oracle_sqdist.argtypes = [_f32p, _f32p, i32]
    lib.oracle_sqdist.restype = dbl
    _lib = lib
    return lib


def _as_x(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("X must be [N][D]")
    return X


def sqdist(a, b) -> float:
    """FP64 squared distance of eq. (1) between two FP32 feature vectors."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    return float(_load().oracle_sqdist(a, b, a.shape[0]))


# metric names -> the oracle's metric codes; "cosine" is the Euclidean
# metric on rows scaled to unit length
METRICS = {"euclidean": 0, "l1": 1, "linf": 2, "cosine": 0}


def normalize_rows(X):
    """Rows scaled to unit Euclidean length (FP64 norm, one rounding per
    feature; zero rows stay zero)."""
    X = _as_x(X)
    n, d = X.shape
    out = np.zeros((max(n, 1), d), np.float32)
    rc = _load().oracle_normalize_rows(X, n, d, d, out)
    if rc != 0:
        raise ValueError(f"oracle_normalize_rows failed ({rc})")
    return out[:n]


def pair_key(a, b, metric="euclidean") -> float:
    """The FP64 key of one pair under a metric (cosine: of the given rows)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    return float(_load().oracle_pair_key(a, b, a.shape[0], METRICS[metric]))


def prim_mst(X, threads: int = 0, metric: str = "euclidean"):
    """Key-ordered minimum spanning tree by dense Prim.

    Returns (u int32, v int32, s float64, w float64), n-1 edges sorted by
    (s, u, v), u < v, w the distance (sqrt(s) for the Euclidean and cosine
    metrics, s for L1 and L-infinity).
    """
    X = _as_x(X)
    if metric == "cosine":
        X = normalize_rows(X)
    n, d = X.shape
    m = max(n - 1, 0)
    u = np.zeros(max(m, 1), np.int32)
    v = np.zeros(max(m, 1), np.int32)
    s = np.zeros(max(m, 1), np.float64)
    w = np.zeros(max(m, 1), np.float64)
    rc = _load().oracle_prim_mst_metric(X, n, d, d, METRICS[metric], u, v, s, w, int(threads))
    if rc != 0:
        raise ValueError(f"oracle_prim_mst failed ({rc})")
    return u[:m], v[:m], s[:m], w[:m]


def cut(u, v, s, w, n, kl1=0, kl2=-1, kl3=-1, kl4=0, dmax=float("inf")):
    """Constrained cut of the sorted tree edges; returns (labels int32, K)."""
    u = np.ascontiguousarray(u, np.int32)
    v = np.ascontiguousarray(v, np.int32)
    s = np.ascontiguousarray(s, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    labels = np.zeros(max(int(n), 1), np.int32)
    k = ctypes.c_int64(0)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else None
    rc = _load().oracle_cut(ptr(u), ptr(v), ptr(s), ptr(w), int(n), int(kl1), int(kl2),
                            int(kl3), int(kl4), float(dmax), labels, ctypes.byref(k))
    if rc != 0:
        raise ValueError(f"oracle_cut failed ({rc})")
    return labels[: int(n)], int(k.value)


def cut_allpairs(X, kl1=0, kl2=-1, kl3=-1, kl4=0, dmax=float("inf")):
    """The constrained process over all pairs of points (not only tree
    edges); returns (labels int32, K).  O(n^2) memory: small n only."""
    X = _as_x(X)
    n, d = X.shape
    labels = np.zeros(max(int(n), 1), np.int32)
    k = ctypes.c_int64(0)
    rc = _load().oracle_cut_allpairs(X, int(n), int(d), int(d), int(kl1), int(kl2), int(kl3),
                                     int(kl4), float(dmax), labels, ctypes.byref(k))
    if rc != 0:
        raise ValueError(f"oracle_cut_allpairs failed ({rc})")
    return labels[: int(n)], int(k.value)


def knn(X, k: int, rows=None, threads: int = 0, metric: str = "euclidean"):
    """Exact k nearest neighbours by key (s, j), j != i, for the query rows."""
    X = _as_x(X)
    if metric == "cosine":
        X = normalize_rows(X)
    n, d = X.shape
    if rows is None:
        rows_a = np.arange(n, dtype=np.int64)
    else:
        rows_a = np.ascontiguousarray(rows, np.int64)
    q = rows_a.shape[0]
    idx = np.zeros((max(q, 1), k), np.int32)
    s = np.zeros((max(q, 1), k), np.float64)
    ln = np.zeros(max(q, 1), np.int32)
    rc = _load().oracle_knn_metric(X, n, d, d, METRICS[metric],
                                   rows_a.ctypes.data_as(ctypes.c_void_p), q, int(k), idx, s, ln,
                                   int(threads))
    if rc != 0:
        raise ValueError(f"oracle_knn failed ({rc})")
    return idx[:q], s[:q], ln[:q]


def nn_outside(X, label=None, rows=None, threads: int = 0):
    """Smallest key (s, j) over j outside the query row's label (or j != i)."""
    X = _as_x(X)
    n, d = X.shape
    rows_a = (np.arange(n, dtype=np.int64) if rows is None
              else np.ascontiguousarray(rows, np.int64))
    q = rows_a.shape[0]
    lab = None if label is None else np.ascontiguousarray(label, np.int32)
    oj = np.zeros(max(q, 1), np.int32)
    os_ = np.zeros(max(q, 1), np.float64)
    rc = _load().oracle_nn_outside(
        X, n, d, d, None if lab is None else lab.ctypes.data_as(ctypes.c_void_p),
        rows_a.ctypes.data_as(ctypes.c_void_p), q, oj, os_, int(threads))
    if rc != 0:
        raise ValueError(f"oracle_nn_outside failed ({rc})")
    return oj[:q], os_[:q]
