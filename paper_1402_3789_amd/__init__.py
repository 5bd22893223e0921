"""MI355X-native exact nearest-neighbour (single-linkage) clustering.

Python binding of the C ABI in ``include/nnm.h``: it only marshals
arguments.  Every step of the computation runs in the HIP kernels of
``libnnm.so``; PyTorch provides device memory and the current stream.  There
is no CPU fallback: if the library is missing, every call raises.

    tree = mst_build(X)                  # X: float32 CUDA tensor [n, d]
    labels, k = cluster_cut(tree, kl1=8)
    idx, s, ln = knn_build(X, k=16)
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _native as N
from ._native import NNMError, NativeMissing, PREC  # noqa: F401

__all__ = ["mst_build", "mst_build_noalloc", "mst_build_pminimal", "knn_build", "cluster_cut",
           "cluster_cut_device", "cluster_cut_allpairs",
           "mst_build_batched", "Tree",
           "options", "autotune", "NNMError", "NativeMissing"]


def _torch():
    import torch
    return torch


def options(precision="auto", knn_k=0, survivor_cap=0, disable_prune=False,
            force_fallback=False, col_splits=0, fixed_chunks=False, graph=False,
            split_target0=0, split_target=0, metric="euclidean") -> N.Options:
    o = N.Options()
    N.lib().nnm_default_options(ctypes.byref(o))
    o.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    o.knn_k = int(knn_k)
    o.survivor_cap = int(survivor_cap)
    o.disable_prune = int(bool(disable_prune))
    o.force_fallback = int(bool(force_fallback))
    o.col_splits = int(col_splits)
    o.fixed_chunks = int(bool(fixed_chunks))
    o.graph = int(bool(graph))
    o.split_target0 = int(split_target0)
    o.split_target = int(split_target)
    o.metric = N.METRIC[metric] if isinstance(metric, str) else int(metric)
    return o


def _tuned(tuned, n, d, precision, count, kw):
    """Fill the knobs the caller left at 0 from the autotuner's cache."""
    if not tuned:
        return kw
    from . import autotune
    ent = autotune.lookup(n, d, precision, count=count, cache=None if tuned is True else tuned)
    if ent is None:
        return kw
    out = dict(kw)
    for key in autotune.KNOBS:
        if not out.get(key):
            out[key] = ent[key]
    return out


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_x(X):
    torch = _torch()
    if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != torch.float32:
        raise TypeError("X must be a float32 CUDA tensor of shape [n, d]")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be 2-D with unit stride along features")
    n, d = X.shape
    ld = X.stride(0) if n > 1 else d
    return int(n), int(d), int(ld)


class _Workspace:
    """Reusable device workspace (grows on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
        return self.buf


_WS = _Workspace()


class Tree:
    """The key-sorted minimum spanning tree returned by mst_build.

    ``raw`` is the device buffer of n-1 nnm_edge records (24 bytes each) seen
    as float64 [n-1, 3]; u, v, s, w are views into it.
    """

    def __init__(self, raw, n, report=None):
        self.raw = raw
        self.n = int(n)
        self.report = report

    @property
    def u(self):
        return self.raw.view(_torch().int32)[:, 0]

    @property
    def v(self):
        return self.raw.view(_torch().int32)[:, 1]

    @property
    def s(self):
        return self.raw[:, 1]

    @property
    def w(self):
        return self.raw[:, 2]

    def host_bytes(self) -> np.ndarray:
        return self.raw.cpu().numpy().view(np.uint8).reshape(-1)

    def to_numpy(self):
        h = self.raw.cpu().numpy()
        iv = h.view(np.int32).reshape(-1, 6)
        return (iv[:, 0].copy(), iv[:, 1].copy(), h[:, 1].copy(), h[:, 2].copy())


def mst_build(X, precision="auto", knn_k=0, survivor_cap=0, disable_prune=False,
              force_fallback=False, col_splits=0, stream=None, workspace=None,
              fixed_chunks=False, graph=False, split_target0=0, split_target=0,
              tuned=False, metric="euclidean") -> Tree:
    """Exact key-ordered minimum spanning tree of the rows of X (device).
    graph=True replays the merge rounds after the first from a captured
    hipGraph (kept for later calls with the same buffers and settings).
    tuned=True (or a cache path) takes k, the split targets and graph replay
    from the autotuner's cache entry for this size, where the caller left
    them at 0."""
    torch = _torch()
    n, d, ld = _check_x(X)
    L = N.lib()
    kw = _tuned(tuned, n, d, precision, 1, dict(knn_k=knn_k, graph=graph,
                                                  split_target0=split_target0,
                                                  split_target=split_target))
    o = options(precision, kw["knn_k"], survivor_cap, disable_prune, force_fallback, col_splits,
                fixed_chunks, kw["graph"], kw["split_target0"], kw["split_target"], metric)
    nb = ctypes.c_size_t(0)
    N.check("mst_workspace_size", L.mst_workspace_size(n, d, ctypes.byref(o), ctypes.byref(nb)))
    ws = (workspace or _WS).get(nb.value, X.device)
    edges = torch.empty((max(n - 1, 1), 3), dtype=torch.float64, device=X.device)
    rep = N.Report()
    code = L.mst_build(ctypes.c_void_p(X.data_ptr()), n, d, ld, ctypes.byref(o),
                       ctypes.c_void_p(ws.data_ptr()), nb.value,
                       ctypes.c_void_p(edges.data_ptr()), _stream(stream), ctypes.byref(rep))
    N.check("mst_build", code)
    return Tree(edges[: n - 1], n, rep.as_dict())


def mst_build_pminimal(X, P=0, precision="auto", knn_k=0, metric="euclidean", stream=None,
                       workspace=None) -> Tree:
    """The same tree by the paper's pipeline of P minimal pairs per pass."""
    torch = _torch()
    n, d, ld = _check_x(X)
    L = N.lib()
    o = options(precision, knn_k, metric=metric)
    nb = ctypes.c_size_t(0)
    N.check("pminimal_workspace_size",
            L.pminimal_workspace_size(n, d, ctypes.byref(o), ctypes.byref(nb)))
    ws = (workspace or _WS).get(nb.value, X.device)
    edges = torch.empty((max(n - 1, 1), 3), dtype=torch.float64, device=X.device)
    rep = N.Report()
    code = L.mst_build_pminimal(ctypes.c_void_p(X.data_ptr()), n, d, ld, int(P), ctypes.byref(o),
                                ctypes.c_void_p(ws.data_ptr()), nb.value,
                                ctypes.c_void_p(edges.data_ptr()), _stream(stream),
                                ctypes.byref(rep))
    N.check("mst_build_pminimal", code)
    return Tree(edges[: n - 1], n, rep.as_dict())


def mst_build_noalloc(X, precision="auto", knn_k=0, survivor_cap=0, disable_prune=False,
                      force_fallback=False, col_splits=0, stream=None, edges=None) -> Tree:
    """mst_build with the library's fixed device scratch instead of a
    workspace (nothing is allocated by the library; ``edges``, if given, is a
    float64 CUDA tensor of at least [n-1, 3] that receives the tree)."""
    torch = _torch()
    n, d, ld = _check_x(X)
    o = options(precision, knn_k, survivor_cap, disable_prune, force_fallback, col_splits)
    if edges is None:
        edges = torch.empty((max(n - 1, 1), 3), dtype=torch.float64, device=X.device)
    rep = N.Report()
    code = N.lib().mst_build_noalloc(ctypes.c_void_p(X.data_ptr()), n, d, ld, ctypes.byref(o),
                                     ctypes.c_void_p(edges.data_ptr()), _stream(stream),
                                     ctypes.byref(rep))
    N.check("mst_build_noalloc", code)
    return Tree(edges[: n - 1], n, rep.as_dict())


def knn_build(X, k=16, precision="auto", survivor_cap=0, force_fallback=False,
              col_splits=0, stream=None, workspace=None, with_report=False, metric="euclidean"):
    """Exact k nearest neighbours of every row: (idx int32, s float64, len int32)."""
    torch = _torch()
    n, d, ld = _check_x(X)
    L = N.lib()
    o = options(precision, k, survivor_cap, False, force_fallback, col_splits, metric=metric)
    nb = ctypes.c_size_t(0)
    N.check("knn_workspace_size",
            L.knn_workspace_size(n, d, int(k), ctypes.byref(o), ctypes.byref(nb)))
    ws = (workspace or _WS).get(nb.value, X.device)
    idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
    s = torch.empty((n, k), dtype=torch.float64, device=X.device)
    ln = torch.empty((n,), dtype=torch.int32, device=X.device)
    rep = N.Report()
    code = L.knn_build(ctypes.c_void_p(X.data_ptr()), n, d, ld, int(k), ctypes.byref(o),
                       ctypes.c_void_p(ws.data_ptr()), nb.value, ctypes.c_void_p(idx.data_ptr()),
                       ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(ln.data_ptr()),
                       _stream(stream), ctypes.byref(rep))
    N.check("knn_build", code)
    if with_report:
        return idx, s, ln, rep.as_dict()
    return idx, s, ln


def _instances(Xs):
    """Instance descriptors and output buffers for a list of inputs."""
    torch = _torch()
    inst = (N.Instance * len(Xs))()
    outs = []
    for b, X in enumerate(Xs):
        n, d, ld = _check_x(X)
        e = torch.empty((max(n - 1, 1), 3), dtype=torch.float64, device=X.device)
        outs.append((e, n))
        inst[b].X_dev = X.data_ptr()
        inst[b].n = n
        inst[b].d = d
        inst[b].ld = ld
        inst[b].edges_dev = e.data_ptr()
    return inst, outs


def mst_build_batched(Xs, precision="auto", knn_k=0, survivor_cap=0, force_fallback=False,
                      stream=None, workspace=None, col_splits=0, graph=False, split_target0=0,
                      split_target=0, tuned=False, metric="euclidean"):
    """Independent trees of many instances in one call; list of Tree."""
    torch = _torch()
    L = N.lib()
    ntot = sum(int(X.shape[0]) for X in Xs)
    dmax = max((int(X.shape[1]) for X in Xs), default=1)
    kw = _tuned(tuned, ntot, dmax, precision, len(Xs), dict(knn_k=knn_k, graph=graph,
                                                            split_target0=split_target0,
                                                            split_target=split_target))
    o = options(precision, kw["knn_k"], survivor_cap, False, force_fallback, col_splits, False,
                kw["graph"], kw["split_target0"], kw["split_target"], metric)
    inst, outs = _instances(Xs)
    nb = ctypes.c_size_t(0)
    N.check("mst_batched_workspace_size",
            L.mst_batched_workspace_size(inst, len(Xs), ctypes.byref(o), ctypes.byref(nb)))
    dev = Xs[0].device if Xs else torch.device("cuda")
    ws = (workspace or _WS).get(nb.value, dev)
    reps = (N.Report * max(len(Xs), 1))()
    code = L.mst_build_batched(inst, len(Xs), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                               nb.value, _stream(stream), reps)
    N.check("mst_build_batched", code)
    return [Tree(e[: n - 1], n, reps[b].as_dict()) for b, (e, n) in enumerate(outs)]


_PINNED = {}


def _pinned(nbytes):
    """A reusable page-locked host buffer of at least nbytes (uint8 tensor)."""
    torch = _torch()
    b = _PINNED.get("edges")
    if b is None or b.numel() < nbytes:
        b = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, pin_memory=True)
        _PINNED["edges"] = b
    return b


def _edges_host(tree_or_edges, n):
    if isinstance(tree_or_edges, Tree):
        raw = tree_or_edges.raw
        if raw.is_cuda:
            # device -> page-locked host copy on the current stream
            torch = _torch()
            nb = raw.numel() * raw.element_size()
            h = _pinned(nb)[:nb].view(torch.float64).view(raw.shape)
            h.copy_(raw, non_blocking=True)
            torch.cuda.current_stream(raw.device).synchronize()
            return h.numpy(), tree_or_edges.n
        return np.ascontiguousarray(raw.numpy()), tree_or_edges.n
    u, v, s, w = tree_or_edges
    m = len(u)
    buf = np.zeros((max(m, 1), 3), np.float64)
    iv = buf.view(np.int32).reshape(-1, 6)
    iv[:m, 0] = np.asarray(u, np.int32)
    iv[:m, 1] = np.asarray(v, np.int32)
    buf[:m, 1] = np.asarray(s, np.float64)
    buf[:m, 2] = np.asarray(w, np.float64)
    if n is None:
        n = m + 1
    return buf, int(n)


def cluster_cut(tree, n=None, kl1=0, kl2=-1, kl3=-1, kl4=0, dmax=math.inf):
    """Constrained cut of a sorted tree (host): (labels int32 [n], K)."""
    buf, n = _edges_host(tree, n)
    p = N.CutParams(int(kl1), int(kl2), int(kl3), int(kl4), float(dmax))
    labels = np.empty(max(n, 1), np.int32)     # every entry is written
    k = ctypes.c_int64(0)
    code = N.lib().cluster_cut(ctypes.c_void_p(buf.ctypes.data), int(n), ctypes.byref(p),
                               ctypes.c_void_p(labels.ctypes.data), ctypes.byref(k))
    N.check("cluster_cut", code)
    return labels[:n], int(k.value)


def cluster_cut_device(tree, kl1=0, dmax=math.inf, stream=None, workspace=None, host=True):
    """The cut of mst_build's tree on the device, for settings without size
    caps or priority (only kl1 and dmax): (labels int32 [n], K), the same as
    cluster_cut.  The edges stay on the device; with host=True the labels
    come back as a numpy array, else as a CUDA tensor."""
    torch = _torch()
    if not isinstance(tree, Tree) or not tree.raw.is_cuda:
        raise TypeError("cluster_cut_device takes a Tree in device memory")
    n = tree.n
    L = N.lib()
    nb = ctypes.c_size_t(0)
    N.check("cluster_cut_device_workspace_size", L.cluster_cut_device_workspace_size(n, ctypes.byref(nb)))
    dev = tree.raw.device
    ws = (workspace or _WS).get(nb.value, dev)
    labels = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    p = N.CutParams(int(kl1), -1, -1, 0, float(dmax))
    k = ctypes.c_int64(0)
    code = L.cluster_cut_device(ctypes.c_void_p(tree.raw.data_ptr() if n > 1 else None), n,
                                ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()), nb.value,
                                ctypes.c_void_p(labels.data_ptr()), ctypes.byref(k), _stream(stream))
    N.check("cluster_cut_device", code)
    labels = labels[:n]
    return (labels.cpu().numpy() if host else labels), int(k.value)


def cluster_cut_allpairs(X, tree=None, kl1=0, kl2=-1, kl3=-1, kl4=0, dmax=math.inf, k=0,
                         precision="auto", stream=None, workspace=None, with_stats=False):
    """The clustering process under the settings over all pairs of points of
    X (a float32 CUDA tensor), given mst_build's tree of X (built here when
    None): (labels int32 [n], K), and with with_stats=True also {unions,
    scans, rows_rescanned, k, scan_ms}.  Equal to cluster_cut of the tree when kl2 and
    kl3 are off."""
    n, d, ld = _check_x(X)
    if tree is None:
        tree = mst_build(X, precision=precision, stream=stream)
    buf, _ = _edges_host(tree, n)
    L = N.lib()
    o = options(precision)
    nb = ctypes.c_size_t(0)
    N.check("allpairs_cut_workspace_size",
            L.allpairs_cut_workspace_size(n, d, int(k), ctypes.byref(o), ctypes.byref(nb)))
    ws = (workspace or _WS).get(nb.value, X.device)
    p = N.CutParams(int(kl1), int(kl2), int(kl3), int(kl4), float(dmax))
    labels = np.empty(max(n, 1), np.int32)
    kk = ctypes.c_int64(0)
    st = (ctypes.c_int64 * 5)()
    code = L.cluster_cut_allpairs(ctypes.c_void_p(X.data_ptr()), n, d, ld,
                                  ctypes.c_void_p(buf.ctypes.data if n > 1 else None),
                                  ctypes.byref(p), int(k),
                                  ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), nb.value,
                                  _stream(stream), ctypes.c_void_p(labels.ctypes.data),
                                  ctypes.byref(kk), st)
    N.check("cluster_cut_allpairs", code)
    if with_stats:
        return labels[:n], int(kk.value), {"unions": st[0], "scans": st[1],
                                          "rows_rescanned": st[2], "k": st[3],
                                          "scan_ms": st[4] / 1000.0}
    return labels[:n], int(kk.value)
