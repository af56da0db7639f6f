"""ctypes binding of libpc.so (the C ABI declared in include/pc.h).

Argument marshalling only: every step of the skeleton runs in the library's HIP kernels. PyTorch
provides device memory and the stream. There is no CPU fallback: if libpc.so is missing the import
of the binding fails.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpc.so")

PC_MAX_LEVEL = 30

PC_OK = 0
PC_WARN_SAMPLE_LIMIT = 1
PC_WARN_LEVEL_CAP = 2
PC_ERR_INVALID_ARG = -1
PC_ERR_SHAPE = -2
PC_ERR_CONSTANT_COLUMN = -3
PC_ERR_NONFINITE = -4
PC_ERR_WORKSPACE = -5
PC_ERR_HIP = -6
PC_ERR_UNSUPPORTED = -7
PC_ERR_SEPSET_CAPACITY = -8

PC_PREC_FP64 = 0
PC_PREC_FP32 = 1
PC_PREC_BF16X3 = 2
PRECISIONS = {"fp64": PC_PREC_FP64, "fp32": PC_PREC_FP32, "bf16x3": PC_PREC_BF16X3}


class pc_options(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("max_level", ct.c_int32), ("margin_scale", ct.c_float),
                ("force_recheck_all", ct.c_int32), ("lds_budget", ct.c_int32),
                ("ranks_per_lane", ct.c_int32), ("grid", ct.c_int32), ("timing", ct.c_int32),
                ("recheck_cap", ct.c_int64), ("graph_levels", ct.c_int32), ("tests_per_lane", ct.c_int32),
                ("tail_tests", ct.c_int32)]


class pc_sep_rec(ct.Structure):
    _fields_ = [("i", ct.c_int32), ("j", ct.c_int32), ("level", ct.c_int32),
                ("S", ct.c_int32 * PC_MAX_LEVEL)]


class pc_sepset(ct.Structure):
    _fields_ = [("recs", ct.c_void_p), ("cap", ct.c_int64), ("count", ct.c_void_p)]


PC_MLP_IN = 8
PC_MLP_HID = 64
PC_MLP_PARAMS = 4801


class pc_order(ct.Structure):
    _fields_ = [("params", ct.c_void_p), ("row_params", ct.c_void_p), ("min_level", ct.c_int32),
                ("max_level", ct.c_int32), ("top", ct.c_int32), ("row_top", ct.c_int32),
                ("row_rank", ct.c_int32), ("row_short", ct.c_int32), ("row_sort", ct.c_int32),
                ("row_split", ct.c_int32)]


class pc_problem(ct.Structure):
    _fields_ = [("X", ct.c_void_p), ("m", ct.c_int64), ("n", ct.c_int64), ("alpha", ct.c_double),
                ("max_level", ct.c_int32), ("pad", ct.c_int32), ("adj_out", ct.c_void_p),
                ("sep", pc_sepset)]


_NL = PC_MAX_LEVEL + 1


class pc_run_stats(ct.Structure):
    _fields_ = [("tests", ct.c_int64 * _NL), ("removed", ct.c_int64 * _NL),
                ("rechecks", ct.c_int64 * _NL), ("items", ct.c_int64 * _NL),
                ("audit_violations", ct.c_int64 * _NL), ("probe_tests", ct.c_int64 * _NL),
                ("probe_removed", ct.c_int64 * _NL), ("max_degree", ct.c_int32 * _NL),
                ("levels_run", ct.c_int32), ("fp64_from", ct.c_int32), ("prep_ms", ct.c_float),
                ("corr_ms", ct.c_float), ("compact_ms", ct.c_float * _NL),
                ("level_ms", ct.c_float * _NL), ("recheck_ms", ct.c_float * _NL),
                ("wall_ms", ct.c_double)]

    def as_dict(self) -> dict:
        k = max(1, self.levels_run)
        return {
            "levels_run": self.levels_run,
            "fp64_from": self.fp64_from,
            "tests": list(self.tests[:k]),
            "removed": list(self.removed[:k]),
            "rechecks": list(self.rechecks[:k]),
            "items": list(self.items[:k]),
            "audit_violations": list(self.audit_violations[:k]),
            "probe_tests": list(self.probe_tests[:k]),
            "probe_removed": list(self.probe_removed[:k]),
            "max_degree": list(self.max_degree[:k]),
            "prep_ms": self.prep_ms,
            "corr_ms": self.corr_ms,
            "compact_ms": list(self.compact_ms[:k]),
            "level_ms": list(self.level_ms[:k]),
            "recheck_ms": list(self.recheck_ms[:k]),
            "wall_ms": self.wall_ms,
        }


class pc_tuning(ct.Structure):
    _fields_ = [("tests_per_lane", ct.c_int32 * _NL), ("ranks_per_lane", ct.c_int32 * _NL),
                ("lds_budget", ct.c_int32 * _NL), ("grid", ct.c_int32 * _NL),
                ("recheck_grid", ct.c_int32 * _NL), ("set_lanes", ct.c_int32 * _NL), ("level_ms", ct.c_float * _NL),
                ("default_ms", ct.c_float * _NL), ("levels", ct.c_int32), ("runs", ct.c_int32)]

    _SHAPES = ("tests_per_lane", "ranks_per_lane", "lds_budget", "grid", "recheck_grid", "set_lanes")

    def as_dict(self) -> dict:
        # the timed levels, and any level further on whose shape differs from the default
        k = max(1, self.levels)
        for key in self._SHAPES:
            arr, dflt = getattr(self, key), (-1 if key == "lds_budget" else 0)
            for l in range(k, _NL):
                if arr[l] != dflt:
                    k = l + 1
        return {"levels": self.levels, "runs": self.runs,
                "tests_per_lane": list(self.tests_per_lane[:k]), "ranks_per_lane": list(self.ranks_per_lane[:k]),
                "lds_budget": list(self.lds_budget[:k]), "grid": list(self.grid[:k]),
                "recheck_grid": list(self.recheck_grid[:k]), "set_lanes": list(self.set_lanes[:k]),
                "level_ms": list(self.level_ms[:k]),
                "default_ms": list(self.default_ms[:k])}

    @classmethod
    def from_dict(cls, d: dict) -> "pc_tuning":
        t = cls()
        for l in range(_NL):
            t.lds_budget[l] = -1
        for key in cls._SHAPES:
            for l, v in enumerate(d.get(key, [])):
                getattr(t, key)[l] = int(v)
        for key in ("level_ms", "default_ms"):
            for l, v in enumerate(d.get(key, [])):
                getattr(t, key)[l] = float(v)
        t.levels = int(d.get("levels", 0))
        t.runs = int(d.get("runs", 0))
        return t


_LIB_DIGEST = None


def _lib_digest() -> str:
    """Digest of the built library (a stored tuning belongs to the build that measured it)."""
    global _LIB_DIGEST
    if _LIB_DIGEST is None:
        import hashlib
        with open(LIB_PATH, "rb") as f:
            _LIB_DIGEST = hashlib.sha1(f.read()).hexdigest()[:16]
    return _LIB_DIGEST


TUNING_CACHE_ENV = "PC_TUNING_CACHE"


def default_tuning_cache() -> "str | None":
    """The tuning cache file that pc_tune reads and extends when a call names none: the path in the
    environment variable PC_TUNING_CACHE, if it is set and not empty; else None (no file)."""
    path = os.environ.get(TUNING_CACHE_ENV, "").strip()
    return path or None


def _read_tuning_cache(path: str) -> dict:
    import json
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return data if isinstance(data, dict) else {}


def _write_tuning_cache(path: str, entries: dict) -> None:
    import json
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1)
    os.replace(tmp, path)


class PCError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


_lib = None


def lib() -> ct.CDLL:
    """Loads libpc.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1812_08491_amd.build`")
        L = ct.CDLL(LIB_PATH)
        vp, i64 = ct.c_void_p, ct.c_int64
        L.pc_create.argtypes = [ct.POINTER(vp), vp, ct.POINTER(pc_options)]
        L.pc_create.restype = ct.c_int
        L.pc_destroy.argtypes = [vp]
        L.pc_destroy.restype = None
        L.pc_default_options.argtypes = [ct.POINTER(pc_options)]
        L.pc_default_options.restype = ct.c_int
        L.pc_workspace_bytes.argtypes = [i64, i64, ct.POINTER(pc_options)]
        L.pc_workspace_bytes.restype = ct.c_size_t
        L.pc_corr.argtypes = [vp, vp, i64, i64, ct.c_double, vp, ct.c_size_t, vp, vp]
        L.pc_corr.restype = ct.c_int
        L.pc_level.argtypes = [vp, ct.c_int, i64, i64, ct.c_double, vp, ct.POINTER(pc_sepset),
                               ct.POINTER(pc_run_stats), vp, ct.c_size_t]
        L.pc_level.restype = ct.c_int
        L.pc_skeleton.argtypes = [vp, vp, i64, i64, ct.c_double, ct.c_int, vp, ct.POINTER(pc_sepset),
                                  ct.POINTER(pc_run_stats), vp, ct.c_size_t]
        L.pc_skeleton.restype = ct.c_int
        L.pc_corr_workspace_bytes.argtypes = [i64, ct.POINTER(pc_options)]
        L.pc_corr_workspace_bytes.restype = ct.c_size_t
        L.pc_level_corr.argtypes = [vp, ct.c_int, vp, i64, ct.c_double, ct.c_double, vp, ct.POINTER(pc_sepset),
                                    ct.POINTER(pc_run_stats), vp, ct.c_size_t]
        L.pc_level_corr.restype = ct.c_int
        L.pc_skeleton_corr.argtypes = [vp, vp, i64, ct.c_double, ct.c_double, ct.c_int, vp, ct.POINTER(pc_sepset),
                                       ct.POINTER(pc_run_stats), vp, ct.c_size_t]
        L.pc_skeleton_corr.restype = ct.c_int
        L.pc_skeleton_noalloc.argtypes = [vp, vp, i64, i64, ct.c_double, ct.c_int, vp, ct.POINTER(pc_sepset),
                                          ct.POINTER(pc_run_stats)]
        L.pc_skeleton_noalloc.restype = ct.c_int
        L.pc_sync_status.argtypes = [vp, vp, ct.c_size_t]
        L.pc_sync_status.restype = ct.c_int
        L.pc_comb_unrank.argtypes = [ct.c_int32, ct.c_int32, ct.c_uint64, ct.c_int32,
                                     ct.POINTER(ct.c_int32)]
        L.pc_comb_unrank.restype = ct.c_int
        L.pc_threshold.argtypes = [ct.c_double, ct.c_double, ct.c_int]
        L.pc_threshold.restype = ct.c_double
        L.pc_batch_workspace_bytes.argtypes = [ct.POINTER(pc_problem), ct.c_int, ct.POINTER(pc_options)]
        L.pc_batch_workspace_bytes.restype = ct.c_size_t
        L.pc_batch_skeleton.argtypes = [vp, ct.POINTER(pc_problem), ct.c_int, ct.POINTER(pc_run_stats),
                                        ct.POINTER(ct.c_int), vp, ct.c_size_t]
        L.pc_batch_skeleton.restype = ct.c_int
        L.pc_batch_capture.argtypes = [vp, ct.POINTER(pc_problem), ct.c_int, vp, ct.c_size_t,
                                       ct.POINTER(vp)]
        L.pc_batch_capture.restype = ct.c_int
        L.pc_batch_capture_ordered.argtypes = [vp, ct.POINTER(pc_problem), ct.c_int, ct.POINTER(pc_order), vp,
                                               ct.c_size_t, ct.POINTER(vp)]
        L.pc_batch_capture_ordered.restype = ct.c_int
        L.pc_tune.argtypes = [vp, ct.POINTER(pc_problem), ct.c_int, ct.POINTER(pc_order), vp, ct.c_size_t,
                              ct.POINTER(pc_tuning)]
        L.pc_tune.restype = ct.c_int
        L.pc_set_tuning.argtypes = [vp, ct.POINTER(pc_tuning)]
        L.pc_set_tuning.restype = ct.c_int
        L.pc_graph_launch.argtypes = [vp]
        L.pc_graph_launch.restype = ct.c_int
        L.pc_graph_results.argtypes = [vp, ct.POINTER(pc_run_stats), ct.POINTER(ct.c_int)]
        L.pc_graph_results.restype = ct.c_int
        L.pc_graph_destroy.argtypes = [vp]
        L.pc_graph_destroy.restype = None
        fp, dp_ = ct.c_void_p, ct.c_void_p
        L.pc_ordered_workspace_bytes.argtypes = [i64, i64, ct.POINTER(pc_options), ct.POINTER(pc_order)]
        L.pc_ordered_workspace_bytes.restype = ct.c_size_t
        L.pc_skeleton_ordered.argtypes = [vp, vp, i64, i64, ct.c_double, ct.c_int, ct.POINTER(pc_order), vp,
                                          ct.POINTER(pc_sepset), ct.POINTER(pc_run_stats), vp, ct.c_size_t]
        L.pc_skeleton_ordered.restype = ct.c_int
        L.pc_features.argtypes = [vp, ct.c_int, i64, i64, ct.c_double, vp, fp, vp, i64, ct.POINTER(i64), vp,
                                  ct.c_size_t]
        L.pc_features.restype = ct.c_int
        L.pc_row_features.argtypes = [vp, ct.c_int, i64, i64, ct.c_double, vp, fp, fp, vp, i64, ct.POINTER(i64), vp,
                                      ct.c_size_t]
        L.pc_row_features.restype = ct.c_int
        L.pc_row_scores.argtypes = [vp, i64, i64, ct.c_double, vp, ct.POINTER(pc_order), fp, vp, vp, ct.c_size_t]
        L.pc_row_scores.restype = ct.c_int
        L.pc_orient_workspace_bytes.argtypes = [i64]
        L.pc_orient_workspace_bytes.restype = ct.c_size_t
        L.pc_orient.argtypes = [vp, i64, vp, vp, i64, vp, vp, ct.c_size_t, ct.POINTER(ct.c_int32)]
        L.pc_orient.restype = ct.c_int
        L.pc_mlp_forward.argtypes = [vp, fp, fp, i64, fp, fp]
        L.pc_mlp_forward.restype = ct.c_int
        L.pc_mlp_backward.argtypes = [vp, fp, fp, i64, fp, fp, fp, fp]
        L.pc_mlp_backward.restype = ct.c_int
        L.pc_mlp_bce.argtypes = [vp, fp, fp, i64, ct.c_float, fp, dp_]
        L.pc_mlp_bce.restype = ct.c_int
        L.pc_mlp_adam.argtypes = [vp, fp, fp, fp, fp, ct.c_int, ct.c_float, ct.c_float, ct.c_float, ct.c_float]
        L.pc_mlp_adam.restype = ct.c_int
        L.pc_abi_size.argtypes = [ct.c_int]
        L.pc_abi_size.restype = ct.c_size_t
        L.pc_status_str.argtypes = [ct.c_int]
        L.pc_status_str.restype = ct.c_char_p
        _check_abi(L)
        _lib = L
    return _lib


EXPORTED = ["pc_create", "pc_destroy", "pc_default_options", "pc_workspace_bytes", "pc_corr",
            "pc_level", "pc_skeleton", "pc_sync_status", "pc_comb_unrank", "pc_threshold",
            "pc_abi_size", "pc_status_str", "pc_batch_workspace_bytes", "pc_batch_skeleton",
            "pc_batch_capture", "pc_graph_launch", "pc_graph_results", "pc_graph_destroy",
            "pc_ordered_workspace_bytes", "pc_skeleton_ordered", "pc_features", "pc_row_features", "pc_mlp_forward",
            "pc_mlp_backward", "pc_mlp_bce", "pc_mlp_adam", "pc_orient_workspace_bytes", "pc_orient",
            "pc_corr_workspace_bytes", "pc_level_corr", "pc_skeleton_corr", "pc_row_scores",
            "pc_batch_capture_ordered", "pc_tune", "pc_set_tuning",
            "pc_skeleton_noalloc"]


def _check_abi(L: ct.CDLL) -> None:
    # A library built from a different include/pc.h than these structs would write past the
    # caller's buffers (statistics arrays are filled with the library's stride), so refuse it.
    for k, cls in enumerate([pc_options, pc_sep_rec, pc_sepset, pc_run_stats, pc_problem, pc_order, pc_tuning]):
        want = int(L.pc_abi_size(k))
        if ct.sizeof(cls) != want:
            raise ImportError(f"{LIB_PATH}: {cls.__name__} is {want} bytes in the library but "
                              f"{ct.sizeof(cls)} in the binding; rebuild the library")


def check_abi() -> None:
    """Raises if a ctypes struct disagrees in size with the library's."""
    _check_abi(lib())


def status_str(status: int) -> str:
    return lib().pc_status_str(status).decode()


def _check(status: int, what: str, allow_warn: bool = True) -> int:
    if status < 0 or (status > 0 and not allow_warn):
        raise PCError(status, what)
    return status


# ------------------------------------------------------------------------------------------------
# Host-only helpers (no GPU)
# ------------------------------------------------------------------------------------------------
def pc_comb_unrank(d: int, l: int, t: int, skip: int = -1) -> list:
    out = (ct.c_int32 * max(1, l))()
    _check(lib().pc_comb_unrank(d, l, t, skip, out), "pc_comb_unrank")
    return [int(out[k]) for k in range(l)]


def pc_threshold(alpha: float, m: float, level: int) -> float:
    return lib().pc_threshold(alpha, m, level)


def default_options(**kw) -> pc_options:
    o = pc_options()
    _check(lib().pc_default_options(ct.byref(o)), "pc_default_options")
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def pc_workspace_bytes(n: int, m: int, opt: pc_options | None = None) -> int:
    return int(lib().pc_workspace_bytes(n, m, ct.byref(opt) if opt is not None else None))


# ------------------------------------------------------------------------------------------------
# Device calls (torch tensors on the current HIP device)
# ------------------------------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def words_per_row(n: int) -> int:
    return (n + 63) // 64


class Context:
    """A pc_ctx bound to a torch stream (default: the current stream)."""

    def __init__(self, stream=None, **options):
        torch = _torch()
        self.opt = default_options(**options)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ct.c_void_p()
        _check(lib().pc_create(ct.byref(h), ct.c_void_p(stream.cuda_stream), ct.byref(self.opt)),
               "pc_create", allow_warn=False)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().pc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers ---------------------------------------------------------------------------
    def workspace(self, n: int, m: int):
        torch = _torch()
        nbytes = pc_workspace_bytes(n, m, self.opt)
        return torch.empty(nbytes, dtype=torch.uint8, device="cuda")

    @staticmethod
    def adjacency(n: int):
        torch = _torch()
        return torch.zeros((n, words_per_row(n)), dtype=torch.int64, device="cuda")

    @staticmethod
    def sepsets(cap: int):
        torch = _torch()
        recs = torch.empty((max(1, cap), 3 + PC_MAX_LEVEL), dtype=torch.int32, device="cuda")
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
        return recs, count

    # -- entry points --------------------------------------------------------------------------
    def pc_corr(self, X, alpha: float, ws, C_out=None, adj_out=None) -> int:
        m, n = X.shape
        assert X.is_cuda and X.dtype == _torch().float64 and X.is_contiguous()
        return _check(lib().pc_corr(self.h, ct.c_void_p(X.data_ptr()), m, n, alpha,
                                    ct.c_void_p(ws.data_ptr()), ws.numel(),
                                    ct.c_void_p(C_out.data_ptr()) if C_out is not None else None,
                                    ct.c_void_p(adj_out.data_ptr()) if adj_out is not None else None),
                      "pc_corr")

    def pc_level(self, level: int, n: int, m: int, alpha: float, adj, recs, count, ws,
                 stats: pc_run_stats | None = None) -> int:
        sep = pc_sepset(recs.data_ptr(), recs.shape[0], count.data_ptr())
        return _check(lib().pc_level(self.h, level, n, m, alpha, ct.c_void_p(adj.data_ptr()),
                                     ct.byref(sep), ct.byref(stats) if stats is not None else None,
                                     ct.c_void_p(ws.data_ptr()), ws.numel()), "pc_level")

    def pc_skeleton(self, X, alpha: float, adj, recs, count, ws, max_level: int = -1,
                    stats: pc_run_stats | None = None) -> int:
        m, n = X.shape
        assert X.is_cuda and X.dtype == _torch().float64 and X.is_contiguous()
        sep = pc_sepset(recs.data_ptr(), recs.shape[0], count.data_ptr())
        return _check(lib().pc_skeleton(self.h, ct.c_void_p(X.data_ptr()), m, n, alpha, max_level,
                                        ct.c_void_p(adj.data_ptr()), ct.byref(sep),
                                        ct.byref(stats) if stats is not None else None,
                                        ct.c_void_p(ws.data_ptr()), ws.numel()), "pc_skeleton")

    # -- a caller's correlation matrix (FP64 contexts) ----------------------------------------
    def corr_workspace(self, n: int):
        torch = _torch()
        nbytes = int(lib().pc_corr_workspace_bytes(n, ct.byref(self.opt)))
        return torch.empty(nbytes, dtype=torch.uint8, device="cuda")

    def pc_level_corr(self, level: int, C, m: float, alpha: float, adj, recs, count, ws,
                      stats: pc_run_stats | None = None) -> int:
        n = C.shape[0]
        assert C.is_cuda and C.dtype == _torch().float64 and C.is_contiguous() and C.shape == (n, n)
        sep = pc_sepset(recs.data_ptr(), recs.shape[0], count.data_ptr())
        return _check(lib().pc_level_corr(self.h, level, ct.c_void_p(C.data_ptr()), n, float(m), alpha,
                                          ct.c_void_p(adj.data_ptr()), ct.byref(sep),
                                          ct.byref(stats) if stats is not None else None,
                                          ct.c_void_p(ws.data_ptr()), ws.numel()), "pc_level_corr")

    def pc_skeleton_corr(self, C, m: float, alpha: float, adj, recs, count, ws, max_level: int = -1,
                         stats: pc_run_stats | None = None) -> int:
        n = C.shape[0]
        assert C.is_cuda and C.dtype == _torch().float64 and C.is_contiguous() and C.shape == (n, n)
        sep = pc_sepset(recs.data_ptr(), recs.shape[0], count.data_ptr())
        return _check(lib().pc_skeleton_corr(self.h, ct.c_void_p(C.data_ptr()), n, float(m), alpha, max_level,
                                             ct.c_void_p(adj.data_ptr()), ct.byref(sep),
                                             ct.byref(stats) if stats is not None else None,
                                             ct.c_void_p(ws.data_ptr()), ws.numel()), "pc_skeleton_corr")

    def pc_skeleton_noalloc(self, X, alpha: float, adj, recs, count, max_level: int = -1,
                            stats: pc_run_stats | None = None) -> int:
        m, n = X.shape
        assert X.is_cuda and X.dtype == _torch().float64 and X.is_contiguous()
        sep = pc_sepset(recs.data_ptr(), recs.shape[0], count.data_ptr())
        return _check(lib().pc_skeleton_noalloc(self.h, ct.c_void_p(X.data_ptr()), m, n, alpha, max_level,
                                                ct.c_void_p(adj.data_ptr()), ct.byref(sep),
                                                ct.byref(stats) if stats is not None else None),
                      "pc_skeleton_noalloc")

    # -- batches ---------------------------------------------------------------------------------
    @staticmethod
    def problems(items) -> "ct.Array":
        """items: iterable of (X, alpha, max_level, adj, recs, count) torch tensors on the device."""
        items = list(items)
        arr = (pc_problem * len(items))()
        for k, (X, alpha, max_level, adj, recs, count) in enumerate(items):
            assert X.is_cuda and X.dtype == _torch().float64 and X.is_contiguous()
            m, n = X.shape
            arr[k] = pc_problem(X.data_ptr(), m, n, alpha, max_level, 0, adj.data_ptr(),
                                pc_sepset(recs.data_ptr(), recs.shape[0], count.data_ptr()))
        # The descriptors hold raw device pointers (and a captured graph keeps using them): the
        # array keeps the tensors alive for as long as it lives.
        arr._keep = items
        return arr

    def batch_workspace(self, probs):
        torch = _torch()
        nbytes = int(lib().pc_batch_workspace_bytes(probs, len(probs), ct.byref(self.opt)))
        if nbytes == 0:
            raise PCError(PC_ERR_INVALID_ARG, "pc_batch_workspace_bytes")
        return torch.empty(nbytes, dtype=torch.uint8, device="cuda")

    def pc_batch_skeleton(self, probs, ws, stats=None):
        count = len(probs)
        status = (ct.c_int * count)()
        r = lib().pc_batch_skeleton(self.h, probs, count, stats, status, ct.c_void_p(ws.data_ptr()),
                                    ws.numel())
        return r, [int(x) for x in status]

    def tuning_key(self, probs, order: "pc_order | None" = None) -> str:
        """Key of a tuning in a cache file: the problems' shapes, alphas and level caps, the
        context's options, the order's form and the library build."""
        import hashlib
        import json
        shapes = [(int(p.n), int(p.m), float(p.alpha), int(p.max_level)) for p in probs]
        opt = ct.string_at(ct.addressof(self.opt), ct.sizeof(self.opt)).hex()
        form = None
        if order is not None:
            form = [int(order.min_level), int(order.max_level), int(order.top), int(order.row_top),
                    int(order.row_rank), int(order.row_short), int(order.row_sort), int(order.row_split),
                    bool(order.params), bool(order.row_params)]
        blob = json.dumps({"shapes": shapes, "opt": opt, "order": form, "lib": _lib_digest()})
        return hashlib.sha1(blob.encode()).hexdigest()[:20]

    def pc_tune(self, probs, ws, order: "pc_order | None" = None, cache: "str | bool | None" = None) -> pc_tuning:
        """Times the level kernels of the problems under candidate shapes and applies the fastest per
        level (pc_tune); returns the tuning. With a cache (a JSON file: `cache`, or when it is None
        the file that PC_TUNING_CACHE names; False for none): a tuning stored there under this
        workload's key (tuning_key) is applied without a search (no skeleton runs, the outputs are
        left as they are); otherwise the search runs and its result is added to the file."""
        if cache is None:
            cache = default_tuning_cache()
        elif cache is False:
            cache = None
        key = None
        if cache is not None:
            key = self.tuning_key(probs, order)
            stored = _read_tuning_cache(cache).get(key)
            if stored is not None:
                t = pc_tuning.from_dict(stored)
                self.pc_set_tuning(t)
                return t
        t = pc_tuning()
        _check(lib().pc_tune(self.h, probs, len(probs), ct.byref(order) if order is not None else None,
                             ct.c_void_p(ws.data_ptr()), ws.numel(), ct.byref(t)), "pc_tune", allow_warn=False)
        if cache is not None:
            entries = _read_tuning_cache(cache)
            entries[key] = t.as_dict()
            _write_tuning_cache(cache, entries)
        return t

    def pc_set_tuning(self, tuning: "pc_tuning | None") -> None:
        _check(lib().pc_set_tuning(self.h, ct.byref(tuning) if tuning is not None else None), "pc_set_tuning",
               allow_warn=False)

    def pc_batch_capture(self, probs, ws, order: "pc_order | None" = None) -> "Graph":
        g = ct.c_void_p()
        if order is None:
            _check(lib().pc_batch_capture(self.h, probs, len(probs), ct.c_void_p(ws.data_ptr()), ws.numel(),
                                          ct.byref(g)), "pc_batch_capture", allow_warn=False)
        else:
            _check(lib().pc_batch_capture_ordered(self.h, probs, len(probs), ct.byref(order),
                                                  ct.c_void_p(ws.data_ptr()), ws.numel(), ct.byref(g)),
                   "pc_batch_capture_ordered", allow_warn=False)
        return Graph(g, len(probs), keep=(probs, ws, self, order))

    # -- learned ordering ----------------------------------------------------------------------
    @staticmethod
    def order(params=None, min_level: int = 2, top: int = 4, max_level: int = 0, row_params=None,
              row_top: int = 0, row_rank: str = "model", row_short: int = 0, row_sort: bool = False,
              row_split: int = 0) -> pc_order:
        """Learned order: the probe pass of the edge model `params` at levels min_level .. max_level
        (0 = 8) that are <= top, and/or the shared-set order at level 1 (the row_top best candidates
        per node first), ranked by the row model `row_params` (row_rank "model"; with row_short > 0
        it scores only the row_short candidates of largest |C_ik|) or by |C_ik| alone
        (row_rank "abs"); row_sort enumerates the remaining candidates by descending |C_ik|, and
        row_split > row_top runs the remaining ranks in two passes split there."""
        torch = _torch()
        for p in (params, row_params):
            assert p is None or (p.is_cuda and p.dtype == torch.float32 and p.numel() == PC_MLP_PARAMS)
        rank = {"model": 0, "abs": 1}[row_rank]
        o = pc_order(params.data_ptr() if params is not None else None,
                     row_params.data_ptr() if row_params is not None else None,
                     min_level, max_level, top, row_top, rank, row_short, int(row_sort), row_split)
        o._keep = (params, row_params)    # the struct holds raw pointers: keep the tensors alive
        return o

    def ordered_workspace(self, n: int, m: int, order: pc_order):
        torch = _torch()
        nbytes = int(lib().pc_ordered_workspace_bytes(n, m, ct.byref(self.opt), ct.byref(order)))
        if nbytes == 0:
            raise PCError(PC_ERR_INVALID_ARG, "pc_ordered_workspace_bytes")
        return torch.empty(nbytes, dtype=torch.uint8, device="cuda")

    def pc_skeleton_ordered(self, X, alpha: float, adj, recs, count, ws, order: pc_order,
                            max_level: int = -1, stats: pc_run_stats | None = None) -> int:
        m, n = X.shape
        assert X.is_cuda and X.dtype == _torch().float64 and X.is_contiguous()
        sep = pc_sepset(recs.data_ptr(), recs.shape[0], count.data_ptr())
        return _check(lib().pc_skeleton_ordered(self.h, ct.c_void_p(X.data_ptr()), m, n, alpha, max_level,
                                                ct.byref(order), ct.c_void_p(adj.data_ptr()), ct.byref(sep),
                                                ct.byref(stats) if stats is not None else None,
                                                ct.c_void_p(ws.data_ptr()), ws.numel()), "pc_skeleton_ordered")

    def pc_features(self, level: int, n: int, m: int, alpha: float, adj, feats, meta, ws) -> int:
        assert feats.is_cuda and feats.dtype == _torch().float32 and feats.shape[1:] == (PC_MLP_IN,)
        assert meta is None or (meta.is_cuda and meta.dtype == _torch().int32 and meta.numel() >= 3 * feats.shape[0])
        rows = ct.c_int64()
        r = lib().pc_features(self.h, level, n, m, alpha, ct.c_void_p(adj.data_ptr()),
                              ct.c_void_p(feats.data_ptr()),
                              ct.c_void_p(meta.data_ptr()) if meta is not None else None,
                              feats.shape[0], ct.byref(rows), ct.c_void_p(ws.data_ptr()), ws.numel())
        if r == PC_ERR_WORKSPACE:
            return -int(rows.value)          # negative: the capacity needed
        _check(r, "pc_features")
        return int(rows.value)

    def pc_row_features(self, level: int, n: int, m: int, alpha: float, adj, feats, labels, meta, ws) -> int:
        """Training rows of the shared-set order (see include/pc.h); returns the row count, or minus
        the capacity needed when feats holds too few rows."""
        torch = _torch()
        assert feats.is_cuda and feats.dtype == torch.float32 and feats.shape[1:] == (PC_MLP_IN,)
        assert labels.is_cuda and labels.dtype == torch.float32 and labels.numel() >= feats.shape[0]
        assert meta is None or (meta.is_cuda and meta.dtype == torch.int32 and meta.numel() >= 2 * feats.shape[0])
        rows = ct.c_int64()
        r = lib().pc_row_features(self.h, level, n, m, alpha, ct.c_void_p(adj.data_ptr()),
                                  ct.c_void_p(feats.data_ptr()), ct.c_void_p(labels.data_ptr()),
                                  ct.c_void_p(meta.data_ptr()) if meta is not None else None,
                                  feats.shape[0], ct.byref(rows), ct.c_void_p(ws.data_ptr()), ws.numel())
        if r == PC_ERR_WORKSPACE:
            return -int(rows.value)
        _check(r, "pc_row_features")
        return int(rows.value)

    def pc_row_scores(self, n: int, m: int, alpha: float, adj, order: pc_order, scores, top, ws) -> int:
        torch = _torch()
        assert scores.is_cuda and scores.dtype == torch.float32 and scores.shape == (n, n)
        assert top.is_cuda and top.dtype == torch.int32 and top.shape == (n, order.row_top)
        return _check(lib().pc_row_scores(self.h, n, m, alpha, ct.c_void_p(adj.data_ptr()), ct.byref(order),
                                          ct.c_void_p(scores.data_ptr()), ct.c_void_p(top.data_ptr()),
                                          ct.c_void_p(ws.data_ptr()), ws.numel()), "pc_row_scores")

    def orient_workspace(self, n: int):
        torch = _torch()
        nbytes = int(lib().pc_orient_workspace_bytes(n))
        if nbytes == 0:
            raise PCError(PC_ERR_SHAPE, "pc_orient_workspace_bytes")
        return torch.empty(nbytes, dtype=torch.uint8, device="cuda")

    def pc_orient(self, n: int, adj, recs, nrec: int, arrows, ws) -> int:
        """CPDAG arrowheads of a skeleton and its SepSet records (see include/pc.h); returns the
        number of propagation rounds that oriented something."""
        torch = _torch()
        W = (n + 63) // 64
        assert adj.is_cuda and adj.dtype == torch.int64 and adj.numel() == n * W
        assert arrows.is_cuda and arrows.dtype == torch.int64 and arrows.numel() == n * W
        assert nrec == 0 or (recs.is_cuda and recs.numel() * recs.element_size() >= nrec * ct.sizeof(pc_sep_rec))
        rounds = ct.c_int32()
        _check(lib().pc_orient(self.h, n, ct.c_void_p(adj.data_ptr()),
                               ct.c_void_p(recs.data_ptr()) if nrec > 0 else None, nrec,
                               ct.c_void_p(arrows.data_ptr()), ct.c_void_p(ws.data_ptr()), ws.numel(),
                               ct.byref(rounds)), "pc_orient")
        return int(rounds.value)

    @staticmethod
    def _mlp_shapes(params, X, **bufs):
        # Device buffers carry no size across the C ABI: check them here, before any launch.
        torch = _torch()
        rows = X.shape[0]
        assert params.is_cuda and params.dtype == torch.float32 and params.numel() == PC_MLP_PARAMS
        assert X.is_cuda and X.dtype == torch.float32 and X.is_contiguous() and X.shape[1:] == (PC_MLP_IN,)
        need = {"scores": rows, "dscore": rows, "labels": rows, "act": rows * 2 * PC_MLP_HID,
                "grads": PC_MLP_PARAMS, "partial": (rows + 63) // 64 * PC_MLP_PARAMS}
        for name, t in bufs.items():
            if t is None:
                continue
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous(), name
            assert t.numel() >= need[name], f"{name}: {t.numel()} < {need[name]} floats"
        return rows

    def pc_mlp_forward(self, params, X, scores, act=None) -> int:
        self._mlp_shapes(params, X, scores=scores, act=act)
        return _check(lib().pc_mlp_forward(self.h, params.data_ptr(), X.data_ptr(), X.shape[0], scores.data_ptr(),
                                           act.data_ptr() if act is not None else None), "pc_mlp_forward")

    def pc_mlp_backward(self, params, X, act, dscore, grads, partial) -> int:
        self._mlp_shapes(params, X, act=act, dscore=dscore, grads=grads, partial=partial)
        return _check(lib().pc_mlp_backward(self.h, params.data_ptr(), X.data_ptr(), X.shape[0], act.data_ptr(),
                                            dscore.data_ptr(), grads.data_ptr(), partial.data_ptr()),
                      "pc_mlp_backward")

    def pc_mlp_bce(self, scores, labels, pos_weight, dscore, loss) -> int:
        torch = _torch()
        rows = scores.shape[0]
        for name, t in (("labels", labels), ("dscore", dscore)):
            assert t.is_cuda and t.dtype == torch.float32 and t.numel() >= rows, name
        assert loss.is_cuda and loss.dtype == torch.float64 and loss.numel() >= 1
        return _check(lib().pc_mlp_bce(self.h, scores.data_ptr(), labels.data_ptr(), scores.shape[0], pos_weight,
                                       dscore.data_ptr(), loss.data_ptr()), "pc_mlp_bce")

    def pc_mlp_adam(self, params, grads, m1, m2, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> int:
        for t in (params, grads, m1, m2):
            assert t.is_cuda and t.dtype == _torch().float32 and t.numel() == PC_MLP_PARAMS
        return _check(lib().pc_mlp_adam(self.h, params.data_ptr(), grads.data_ptr(), m1.data_ptr(), m2.data_ptr(),
                                        step, lr, beta1, beta2, eps), "pc_mlp_adam")

    def pc_sync_status(self, ws=None) -> int:
        return _check(lib().pc_sync_status(self.h, ct.c_void_p(ws.data_ptr()) if ws is not None else None,
                                           ws.numel() if ws is not None else 0), "pc_sync_status")


class Graph:
    """A captured batch (pc_graph)."""

    def __init__(self, h, count, keep):
        self.h, self.count, self._keep = h, count, keep

    def pc_graph_launch(self) -> int:
        return _check(lib().pc_graph_launch(self.h), "pc_graph_launch")

    def pc_graph_results(self, stats=None):
        status = (ct.c_int * self.count)()
        r = lib().pc_graph_results(self.h, stats, status)
        return r, [int(x) for x in status]

    def close(self):
        if getattr(self, "h", None):
            lib().pc_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------------
# Result decoding (host)
# ------------------------------------------------------------------------------------------------
def bits_to_dense(adj_words: np.ndarray, n: int) -> np.ndarray:
    """n x W little-endian uint64 bit matrix -> n x n uint8 adjacency."""
    w = np.ascontiguousarray(adj_words).view(np.uint64).reshape(n, -1)
    b = np.unpackbits(w.view(np.uint8), axis=1, bitorder="little")
    return b[:, :n].astype(np.uint8)


def dense_to_bits(G: np.ndarray) -> np.ndarray:
    """n x n 0/1 adjacency -> n x W uint64 bit matrix (as int64 for torch)."""
    n = G.shape[0]
    W = words_per_row(n)
    padded = np.zeros((n, W * 64), np.uint8)
    padded[:, :n] = G != 0
    packed = np.packbits(padded, axis=1, bitorder="little")
    return packed.view(np.uint64).reshape(n, W).view(np.int64)


def decode_sepsets(recs: np.ndarray, count: int) -> dict:
    """(i, j) -> (level, S tuple) from the record table (first `count` rows)."""
    out = {}
    for r in recs[:count]:
        i, j, l = int(r[0]), int(r[1]), int(r[2])
        out[(i, j)] = (l, tuple(int(x) for x in r[3:3 + l]))
    return out
