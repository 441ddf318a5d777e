"""CPU oracle for the L_d norms -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps the plain C enumeration in ld_oracle.c (ctypes) and shares
no code with the GPU library.  Every function returns a Python int.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ld_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

INT64_MIN = -(1 << 63)


def build(force: bool = False) -> str:
    """Compile ld_oracle.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        for name, args in [("oracle_l1", [P, i32, i32, i32]),
                           ("oracle_l1_all", [P, i32, i32, i32]),
                           ("oracle_lmarg", [P, i32, i32, i32]),
                           ("oracle_ld", [P, i32, i32, i32, i32]),
                           ("oracle_ld_all", [P, i32, i32, i32, i32]),
                           ("oracle_range", [P, i32, i32, i32, i32, i32, u64, u64, i32]),
                           ("oracle_l1_split", [P, i32, i32, i32, i32]),
                           ("oracle_ld_split", [P, i32, i32, i32, i32]),
                           ("oracle_ld_classes", [P, i32, i32, i32, i32]),
                           ("oracle_value_of", [P, i32, i32, i32, i32, P])]:
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = i64
        lib.oracle_rgs_count.argtypes = [i32, i32]
        lib.oracle_rgs_count.restype = u64
        _lib = lib
    return _lib


def _mat(M):
    a = np.ascontiguousarray(np.asarray(M, dtype=np.int32))
    if a.ndim != 2:
        raise ValueError("matrix must be 2-D")
    return a


def _threads(t):
    """t, or the CPUs this process may run on (capped by OMP_NUM_THREADS when set): more
    threads than that only time-slice."""
    if t:
        return t
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(omp))) if omp.isdigit() and int(omp) > 0 else max(1, n)


def l1(M, threads: int = 0) -> int:
    a = _mat(M)
    return int(_load().oracle_l1(a.ctypes.data, a.shape[0], a.shape[1], _threads(threads)))


def l1_all(M, threads: int = 0) -> int:
    a = _mat(M)
    return int(_load().oracle_l1_all(a.ctypes.data, a.shape[0], a.shape[1], _threads(threads)))


def lmarg(M, threads: int = 0) -> int:
    a = _mat(M)
    return int(_load().oracle_lmarg(a.ctypes.data, a.shape[0], a.shape[1], _threads(threads)))


def ld(M, d: int, threads: int = 0) -> int:
    a = _mat(M)
    return int(_load().oracle_ld(a.ctypes.data, a.shape[0], a.shape[1], d, _threads(threads)))


def ld_all(M, d: int, threads: int = 0) -> int:
    a = _mat(M)
    return int(_load().oracle_ld_all(a.ctypes.data, a.shape[0], a.shape[1], d, _threads(threads)))


def norm(M, d: int, marginals: int = 0, threads: int = 0) -> int:
    """The value the library's ld_norm must return: d = 1 is Eq. (LM2) (or Eq. (LMarg)
    with marginals), d >= 2 is Eq. (L_o_norm)."""
    if d == 1:
        return lmarg(M, threads) if marginals else l1(M, threads)
    return ld(M, d, threads)


def range_max(M, d: int, marginals: int, q: int, pfx_begin: int, pfx_end: int,
              threads: int = 0) -> int:
    a = _mat(M)
    return int(_load().oracle_range(a.ctypes.data, a.shape[0], a.shape[1], d, marginals, q,
                                    pfx_begin, pfx_end, _threads(threads)))


def l1_split(M, marginals: int = 0, threads: int = 0) -> int:
    a = _mat(M)
    return int(_load().oracle_l1_split(a.ctypes.data, a.shape[0], a.shape[1], marginals,
                                       _threads(threads)))


def ld_split(M, d: int, threads: int = 0) -> int:
    a = _mat(M)
    return int(_load().oracle_ld_split(a.ctypes.data, a.shape[0], a.shape[1], d, _threads(threads)))


def ld_classes(M, d: int, threads: int = 0) -> int:
    """L_d by one assignment per relabelling class (restricted-growth strings)."""
    a = _mat(M)
    return int(_load().oracle_ld_classes(a.ctypes.data, a.shape[0], a.shape[1], d, _threads(threads)))


def rgs_count(n: int, d: int) -> int:
    return int(_load().oracle_rgs_count(n, d))


def norm_split(M, d: int, marginals: int = 0, threads: int = 0) -> int:
    """The same value as norm(), by the split-table forms (for the larger inputs)."""
    if d == 1:
        return l1_split(M, marginals, threads)
    return ld_split(M, d, threads)


def value_of(M, d: int, marginals: int, assignment) -> int:
    a = _mat(M)
    s = np.ascontiguousarray(np.asarray(assignment, dtype=np.int8))
    return int(_load().oracle_value_of(a.ctypes.data, a.shape[0], a.shape[1], d, marginals,
                                       s.ctypes.data))
