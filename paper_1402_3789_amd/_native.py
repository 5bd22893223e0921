"""ctypes view of the C ABI declared in include/nnm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# NNM_LIB names another build of the same library (for instance one whose
# host code is instrumented by a sanitizer).
LIBPATH = os.environ.get("NNM_LIB") or os.path.join(HERE, "libnnm.so")

NNM_OK = 0
NNM_EINVAL = -1
NNM_ENOMEM = -2
NNM_EDEVICE = -3
NNM_ENONFINITE = -4
NNM_EUNSUPPORTED = -5
NNM_ETOOLARGE = -6
NOALLOC_SCRATCH_BYTES = 128 << 20
TUNE_MAX_TRIALS = 32

PREC = {"fp32": 0, "bf16": 1, "fp8": 2, "auto": 3, "fp16": 4}
PREC_NAME = {v: k for k, v in PREC.items()}
METRIC = {"euclidean": 0, "l1": 1, "linf": 2, "cosine": 3}


class Edge(ctypes.Structure):
    _fields_ = [("u", ctypes.c_int32), ("v", ctypes.c_int32),
                ("s", ctypes.c_double), ("w", ctypes.c_double)]


class CutParams(ctypes.Structure):
    _fields_ = [("kl1_max_clusters", ctypes.c_int64), ("kl2_max_size", ctypes.c_int64),
                ("kl3_max_merged", ctypes.c_int64), ("kl4_min_size", ctypes.c_int64),
                ("dmax", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("knn_k", ctypes.c_int32),
                ("survivor_cap", ctypes.c_int32), ("disable_prune", ctypes.c_int32),
                ("force_fallback", ctypes.c_int32), ("col_splits", ctypes.c_int32),
                ("fixed_chunks", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("split_target0", ctypes.c_int32), ("split_target", ctypes.c_int32),
                ("metric", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class Report(ctypes.Structure):
    _fields_ = [("precision_used", ctypes.c_int32), ("integer_mode", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("knn_k", ctypes.c_int32),
                ("rows_scanned", ctypes.c_int64), ("pairs_evaluated", ctypes.c_int64),
                ("survivors", ctypes.c_int64), ("overflow_rows", ctypes.c_int64),
                ("max_abs_err", ctypes.c_double), ("max_rel_err", ctypes.c_double),
                ("max_bound", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_candidates", ctypes.c_double), ("ms_rescore", ctypes.c_double),
                ("ms_merge", ctypes.c_double), ("ms_sort", ctypes.c_double),
                ("rows_per_round", ctypes.c_int64 * 32),
                ("comps_per_round", ctypes.c_int64 * 32),
                ("cand_launches", ctypes.c_int64),
                ("rescanned_bounded", ctypes.c_int64),
                ("pairs_per_round", ctypes.c_int64 * 32),
                ("over_per_round", ctypes.c_int64 * 32),
                ("exact_per_round", ctypes.c_int64 * 32),
                ("cand_ms_per_round", ctypes.c_double * 32),
                ("surv_per_round", ctypes.c_int64 * 32),
                ("max_err_ratio", ctypes.c_double), ("ms_graph", ctypes.c_double),
                ("graph_rounds", ctypes.c_int32), ("graph_nodes", ctypes.c_int32),
                ("graph_captured", ctypes.c_int32), ("pad_", ctypes.c_int32)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if name.endswith("_per_round"):
                v = [round(float(x), 3) if name.startswith("cand_ms") else int(x)
                     for x in v[: max(self.rounds, 0)]]
            out[name] = v
        out["precision_used"] = PREC_NAME.get(self.precision_used, str(self.precision_used))
        return out


class Instance(ctypes.Structure):
    _fields_ = [("X_dev", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("ld", ctypes.c_int64), ("edges_dev", ctypes.c_void_p)]


# Every symbol include/nnm.h declares, with its ctypes signature.
_SIG = {
    "nnm_default_options": (None, [ctypes.POINTER(Options)]),
    "nnm_strerror": (ctypes.c_char_p, [ctypes.c_int32]),
    "mst_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32,
                                          ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]),
    "knn_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]),
    "knn_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_int32, ctypes.POINTER(Options), ctypes.c_void_p,
                                 ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Report)]),
    "mst_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_size_t,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Report)]),
    "mst_build_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.POINTER(Options), ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.POINTER(Report)]),
    "pminimal_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32,
                                               ctypes.POINTER(Options),
                                               ctypes.POINTER(ctypes.c_size_t)]),
    "mst_build_pminimal": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(Options),
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.POINTER(Report)]),
    "mst_batched_workspace_size": (ctypes.c_int, [ctypes.POINTER(Instance), ctypes.c_int32,
                                                  ctypes.POINTER(Options),
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "mst_build_batched": (ctypes.c_int, [ctypes.POINTER(Instance), ctypes.c_int32,
                                         ctypes.POINTER(Options), ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_void_p,
                                         ctypes.POINTER(Report)]),
    "mst_autotune_workspace_size": (ctypes.c_int, [ctypes.POINTER(Instance), ctypes.c_int32,
                                                   ctypes.POINTER(Options),
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "mst_autotune": (ctypes.c_int, [ctypes.POINTER(Instance), ctypes.c_int32,
                                    ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Options),
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int32)]),
    "allpairs_cut_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.POINTER(Options),
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "cluster_cut_allpairs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                            ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.POINTER(CutParams),
                                            ctypes.c_int32, ctypes.POINTER(Options),
                                            ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.c_void_p]),
    "cluster_cut": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(CutParams),
                                   ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "cluster_cut_device_workspace_size": (ctypes.c_int, [ctypes.c_int64,
                                                         ctypes.POINTER(ctypes.c_size_t)]),
    "cluster_cut_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(CutParams),
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
}

_lib = None


class NativeMissing(RuntimeError):
    pass


def lib():
    """The loaded libnnm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise NativeMissing(
            f"{LIBPATH} is missing: build it with paper_1402_3789_amd/build.py "
            "(or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIBPATH)
    for name, (res, args) in _SIG.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols():
    return sorted(_SIG)


def strerror(code: int) -> str:
    return lib().nnm_strerror(int(code)).decode()


class NNMError(RuntimeError):
    def __init__(self, where, code):
        self.code = int(code)
        super().__init__(f"{where}: {strerror(code)} ({code})")


def check(where, code):
    if code != NNM_OK:
        raise NNMError(where, code)
