"""Python access to the plain FP64 CPU oracle (``oracle/pc_oracle.c``).

TEST INFRASTRUCTURE ONLY. The product path never imports this package: only the test suite, the
smoke check and the benchmark's CPU-baseline leg do. It shares no code with the HIP library.

Functions follow the cuPC paper (Zarebavani et al., TPDS 2019): Algorithm 1 (PC-stable skeleton,
Sec. 2.4), Eq. 3-6 (CI test from the correlation matrix, Sec. 4.3), Sec. 4.4 (pseudo-inverse).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OC_OK, OC_PINV, OC_WARN_SAMPLE_LIMIT = 0, 1, 2
OC_ERR_SHAPE, OC_ERR_CONSTANT, OC_ERR_NONFINITE, OC_ERR_ALLOC = -1, -2, -3, -4


class OracleError(RuntimeError):
    pass


# Built with -O3 -march=native, so the library is tied to the CPU it was built on; a stamp file
# records that CPU and the flags, and a library built elsewhere is rebuilt before it is loaded.
_FLAGS = ["-O3", "-march=native", "-fopenmp", "-std=c11", "-fPIC", "-shared", "-Wall"]
_STAMP = _LIB + ".host"


def _host_stamp() -> str:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model + " | " + " ".join(_FLAGS)


def _stale() -> bool:
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        return True
    try:
        with open(_STAMP) as f:
            return f.read() != _host_stamp()
    except OSError:
        return True


def build(force: bool = True) -> str:
    """Compiles the oracle with gcc (-O3 -march=native, OpenMP; single-threaded unless
    set_threads says otherwise). -std=c11 keeps floating-point contraction off, so the arithmetic
    is the plain sequence of the source."""
    if force or _stale():
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc"] + _FLAGS + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
        with open(_STAMP, "w") as f:
            f.write(_host_stamp())
    return _LIB


_lib = None


class _Sep(ct.Structure):
    _fields_ = [("i", ct.POINTER(ct.c_int32)), ("j", ct.POINTER(ct.c_int32)),
                ("level", ct.POINTER(ct.c_int32)), ("S", ct.POINTER(ct.c_int32)),
                ("cap", ct.c_int64), ("count", ct.c_int64), ("max_level", ct.c_int32)]


class _Stats(ct.Structure):
    _fields_ = [("tests", ct.c_int64), ("removed", ct.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build(force=True)
        L = ct.CDLL(_LIB)
        dp, ip = ct.POINTER(ct.c_double), ct.POINTER(ct.c_int)
        up = ct.POINTER(ct.c_ubyte)
        L.oc_corr.argtypes = [dp, ct.c_int64, ct.c_int64, dp]
        L.oc_corr_pair.argtypes = [dp, ct.c_int64, ct.c_int64, ct.c_int64, ct.c_int64, dp]
        L.oc_ppnd.argtypes = [ct.c_double]
        L.oc_ppnd.restype = ct.c_double
        L.oc_tau.argtypes = [ct.c_double, ct.c_double, ct.c_int]
        L.oc_tau.restype = ct.c_double
        L.oc_fisher_z.argtypes = [ct.c_double]
        L.oc_fisher_z.restype = ct.c_double
        L.oc_pinv_sym.argtypes = [dp, ct.c_int, dp]
        L.oc_pcor.argtypes = [dp, ct.c_int64, ct.c_int, ct.c_int, ip, ct.c_int, dp]
        L.oc_ci_test.argtypes = [dp, ct.c_int64, ct.c_int, ct.c_int, ip, ct.c_int, ct.c_double, dp]
        L.oc_level0.argtypes = [dp, ct.c_int64, ct.c_double, ct.c_double, up, ct.POINTER(_Stats)]
        L.oc_level.argtypes = [dp, ct.c_int64, ct.c_double, ct.c_double, ct.c_int, up,
                               ct.POINTER(_Sep), ct.POINTER(_Stats)]
        L.oc_max_degree.argtypes = [up, ct.c_int64]
        L.oc_set_threads.argtypes = [ct.c_int]
        L.oc_set_threads.restype = None
        L.oc_skeleton_corr.argtypes = [dp, ct.c_int64, ct.c_double, ct.c_double, ct.c_int, up,
                                       ct.POINTER(_Sep), ct.POINTER(_Stats), ct.c_int, up,
                                       ct.POINTER(ct.c_int)]
        L.oc_skeleton.argtypes = [dp, ct.c_int64, ct.c_int64, ct.c_double, ct.c_int, up,
                                  ct.POINTER(_Sep), ct.POINTER(_Stats), ct.c_int, up,
                                  ct.POINTER(ct.c_int)]
        _lib = L
    return _lib


def set_threads(k: int) -> None:
    """Threads the level loop uses (edges of a level are decided in parallel from the snapshot G'
    and applied in canonical order, so every result is the same for any k)."""
    lib().oc_set_threads(int(k))


def _dp(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _up(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_ubyte))


def _check(st, what):
    if st < 0:
        raise OracleError(f"{what}: oracle status {st}")
    return st


def corr(X: np.ndarray) -> np.ndarray:
    """Pearson correlation of the columns of X (m x n, FP64), C_aa = 1."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    C = np.empty((n, n))
    _check(lib().oc_corr(_dp(X), m, n, _dp(C)), "corr")
    return C


def corr_pair(X: np.ndarray, a: int, b: int) -> float:
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    out = ct.c_double()
    _check(lib().oc_corr_pair(_dp(X), m, n, a, b, ct.byref(out)), "corr_pair")
    return out.value


def ppnd(p: float) -> float:
    return lib().oc_ppnd(p)


def tau(alpha: float, m: float, level: int) -> float:
    return lib().oc_tau(alpha, m, level)


def fisher_z(rho: float) -> float:
    return lib().oc_fisher_z(rho)


def pinv_sym(A: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    k = A.shape[0]
    P = np.empty((k, k))
    _check(lib().oc_pinv_sym(_dp(A), k, _dp(P)), "pinv_sym")
    return P


def pcor(C: np.ndarray, i: int, j: int, S) -> tuple[float, bool]:
    """Partial correlation rho(V_i, V_j | S) (Eq. 3-4); second value: the pseudo-inverse was used."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    Sa = np.ascontiguousarray(np.asarray(S, dtype=np.int32).reshape(-1))
    out = ct.c_double()
    st = _check(lib().oc_pcor(_dp(C), C.shape[0], i, j,
                              Sa.ctypes.data_as(ct.POINTER(ct.c_int)), Sa.size, ct.byref(out)),
                "pcor")
    return out.value, st == OC_PINV


def ci_test(C: np.ndarray, i: int, j: int, S, m: float, alpha: float) -> tuple[bool, float, float]:
    """Returns (independent, z, tau) for I(V_i, V_j | S) at sample size m and level alpha."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    Sa = np.ascontiguousarray(np.asarray(S, dtype=np.int32).reshape(-1))
    t = tau(alpha, m, Sa.size)
    z = ct.c_double()
    r = _check(lib().oc_ci_test(_dp(C), C.shape[0], i, j, Sa.ctypes.data_as(ct.POINTER(ct.c_int)),
                                Sa.size, t, ct.byref(z)), "ci_test")
    return bool(r == 1), z.value, t


def ci_test_tau(C: np.ndarray, i: int, j: int, S, tau_value: float) -> tuple[bool, float]:
    """I(V_i, V_j | S) against an explicit threshold: returns (independent, z)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    Sa = np.ascontiguousarray(np.asarray(S, dtype=np.int32).reshape(-1))
    z = ct.c_double()
    r = _check(lib().oc_ci_test(_dp(C), C.shape[0], i, j, Sa.ctypes.data_as(ct.POINTER(ct.c_int)),
                                Sa.size, tau_value, ct.byref(z)), "ci_test")
    return bool(r == 1), z.value


@dataclass
class SepSets:
    """Level >= 1 SepSet records: (i < j, level, S ids ascending). Level-0 SepSets are empty."""
    i: np.ndarray
    j: np.ndarray
    level: np.ndarray
    S: np.ndarray          # count x max_level, -1 padded

    def as_dict(self):
        return {(int(a), int(b)): (int(l), tuple(int(x) for x in s[:l]))
                for a, b, l, s in zip(self.i, self.j, self.level, self.S)}


class _SepBuf:
    def __init__(self, cap: int, max_level: int):
        cap = max(int(cap), 1)
        self.i = np.zeros(cap, np.int32)
        self.j = np.zeros(cap, np.int32)
        self.level = np.zeros(cap, np.int32)
        self.S = np.full((cap, max_level), -1, np.int32)
        ip = lambda a: a.ctypes.data_as(ct.POINTER(ct.c_int32))
        self.c = _Sep(ip(self.i), ip(self.j), ip(self.level), ip(self.S), cap, 0, max_level)

    def result(self) -> SepSets:
        k = int(self.c.count)
        if k > self.c.cap:
            raise OracleError("SepSet buffer overflow")
        return SepSets(self.i[:k].copy(), self.j[:k].copy(), self.level[:k].copy(),
                       self.S[:k].copy())


def level0(C: np.ndarray, m: float, alpha: float):
    """Level 0 on the complete graph: returns (G as n x n uint8, tests, removed)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    n = C.shape[0]
    G = np.ones((n, n), np.uint8)
    st = _Stats()
    _check(lib().oc_level0(_dp(C), n, m, alpha, _up(G), ct.byref(st)), "level0")
    return G, st.tests, st.removed


def level(C: np.ndarray, m: float, alpha: float, l: int, G: np.ndarray, max_level: int = 64):
    """One level l >= 1 given G (the snapshot G' is taken inside). Returns (G_new, SepSets, tests)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    n = C.shape[0]
    Gn = np.ascontiguousarray(G, dtype=np.uint8).copy()
    cap = int(Gn.sum()) // 2 + 1
    buf = _SepBuf(cap, max(max_level, l))
    st = _Stats()
    r = _check(lib().oc_level(_dp(C), n, m, alpha, l, _up(Gn), ct.byref(buf.c), ct.byref(st)),
               "level")
    return Gn, buf.result(), st.tests, r


@dataclass
class Skeleton:
    G: np.ndarray                  # final adjacency, n x n uint8
    sepsets: SepSets
    tests: list                    # canonical executed tests per level (level 0 first)
    removed: list
    G_after: list = field(default_factory=list)   # adjacency after each level
    status: int = 0

    @property
    def levels_run(self):
        return len(self.tests)


def _skeleton_common(fn, args, n, max_level, keep_levels):
    ML = 32
    cap = 8 * n + 1024
    while True:
        G = np.zeros((n, n), np.uint8)
        buf = _SepBuf(cap, ML)
        stats = (_Stats * ML)()
        Gafter = np.zeros((ML, n, n), np.uint8) if keep_levels else None
        run = ct.c_int(0)
        st = _check(fn(*args, max_level, _up(G), ct.byref(buf.c), stats, ML,
                       _up(Gafter) if keep_levels else None, ct.byref(run)), "skeleton")
        if buf.c.count <= buf.c.cap:
            break
        cap = int(buf.c.count)          # SepSet buffer was too small: run again with room
    k = run.value
    if k > ML:
        raise OracleError("more levels than the oracle wrapper records")
    return Skeleton(G=G, sepsets=buf.result(), tests=[stats[l].tests for l in range(k)],
                    removed=[stats[l].removed for l in range(k)],
                    G_after=[Gafter[l].copy() for l in range(k)] if keep_levels else [],
                    status=st)


def skeleton(X: np.ndarray, alpha: float, max_level: int = -1, keep_levels: bool = False) -> Skeleton:
    """PC-stable skeleton from data X (m x n)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    return _skeleton_common(lib().oc_skeleton, (_dp(X), m, n, alpha), n, max_level, keep_levels)


def skeleton_corr(C: np.ndarray, m: float, alpha: float, max_level: int = -1,
                  keep_levels: bool = False) -> Skeleton:
    """PC-stable skeleton from a correlation matrix at nominal sample size m."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    n = C.shape[0]
    return _skeleton_common(lib().oc_skeleton_corr, (_dp(C), n, float(m), alpha), n, max_level,
                            keep_levels)
