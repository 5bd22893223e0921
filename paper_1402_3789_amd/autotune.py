"""Autotuner cache: the run options the library's tuner (``mst_autotune`` in
``include/nnm.h``) found fastest, per GPU architecture, precision, size
bucket and shape (one instance or a batch).

    ent = autotune.tune(X, precision="fp16")      # measures, stores, returns
    tree = mst_build(X, precision="fp16", tuned=True)

The cache is a JSON file (``$NNM_AUTOTUNE_CACHE``, else
``~/.cache/paper_1402_3789_amd/autotune.json``; ``tuned.json`` beside this
module holds entries measured on an MI355X for buckets the cache lacks) keyed by
``arch|precision|n-bucket|d-bucket|single-or-batch``: n rounded to a power
of four, d to 8, 16, 26 or 32.  Every result is exact whatever the options,
so a stale or foreign entry can only cost time.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import tempfile

from . import _native as N

KNOBS = ("knn_k", "split_target0", "split_target", "graph")


def default_cache() -> str:
    p = os.environ.get("NNM_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1402_3789_amd", "autotune.json")


def arch(device=None) -> str:
    import torch
    props = torch.cuda.get_device_properties(device if device is not None else torch.cuda.current_device())
    return str(getattr(props, "gcnArchName", props.name)).split(":")[0]


def bucket_key(n: int, d: int, precision: str, count: int = 1, arch_name: str | None = None) -> str:
    nb = 4 ** max(0, round(math.log(max(int(n), 1), 4)))
    db = next(b for b in (8, 16, 26, 32) if int(d) <= b) if int(d) <= 32 else int(d)
    shape = "batch" if count > 1 else "single"
    return f"{arch_name or arch()}|{precision}|n{nb}|d{db}|{shape}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, entry: dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    data = _load(path)
    data[key] = entry
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


# entries measured with this package's tuner on an MI355X (gfx950), used
# where the cache has no entry of its own for a bucket
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def lookup(n: int, d: int, precision: str = "auto", count: int = 1, cache: str | None = None,
           arch_name: str | None = None, shipped: bool = True):
    """The cached entry for this size and shape (the cache file first, then
    the shipped table), or None."""
    key = bucket_key(n, d, precision, count, arch_name)
    ent = _load(cache or default_cache()).get(key)
    if ent is None and shipped:
        ent = _load(SHIPPED).get(key)
    return ent


def tune(X, precision: str = "auto", reps: int = 3, cache: str | None = None, save: bool = True,
         stream=None, **base) -> dict:
    """Measure the run options on X (a float32 CUDA tensor, or a list of them
    for a batched call) with the library's tuner; store and return the entry
    ``{knn_k, split_target0, split_target, graph, ms, default_ms, trials_ms}``."""
    from . import _instances, _stream, options, _WS, PREC  # noqa: F401
    Xs = list(X) if isinstance(X, (list, tuple)) else [X]
    inst, outs = _instances(Xs)
    o = options(precision, **base)
    L = N.lib()
    nb = ctypes.c_size_t(0)
    N.check("mst_autotune_workspace_size",
            L.mst_autotune_workspace_size(inst, len(Xs), ctypes.byref(o), ctypes.byref(nb)))
    ws = _WS.get(nb.value, Xs[0].device)
    best = N.Options()
    trials = (ctypes.c_double * N.TUNE_MAX_TRIALS)()
    nt = ctypes.c_int32(0)
    N.check("mst_autotune", L.mst_autotune(inst, len(Xs), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                                           nb.value, _stream(stream), int(reps), ctypes.byref(best),
                                           trials, ctypes.byref(nt)))
    tms = [round(trials[i], 3) for i in range(nt.value)]
    entry = {k: int(getattr(best, k)) for k in KNOBS}
    entry.update(ms=min(tms), default_ms=tms[0], trials_ms=tms)
    ntot = sum(int(x.shape[0]) for x in Xs)
    dmax = max(int(x.shape[1]) for x in Xs)
    if save:
        _store(cache or default_cache(), bucket_key(ntot, dmax, precision, len(Xs)), entry)
    return entry
