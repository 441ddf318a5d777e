"""Python binding of the MI355X L_d-norm library (libld.so, C ABI in include/ld.h).

Argument marshalling only: every step of the computation runs in the HIP library.
The library must have been built (``paper_2503_21596_amd._build.build()``); if it
is missing, importing the binding's functions raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libld.so")
TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_mi355x.json")
INT64_MIN = -(1 << 63)

LD_OK, LD_EINVAL, LD_EMARG_D, LD_ETOOBIG, LD_EHIP, LD_EBUSY, LD_PENDING, LD_ENOTFOUND, LD_ECANCELED, \
    LD_ESCRATCH = range(10)

PLAN_KINDS = {0: "L1", 1: "L_marg", 2: "L2", 3: "L_d", 4: "sum|M|", 5: "zero"}


class LdError(RuntimeError):
    def __init__(self, code: int, text: str):
        super().__init__(f"ld error {code}: {text}")
        self.code = code


class ld_problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_void_p), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("d", ctypes.c_int32), ("marginals", ctypes.c_int32)]


class ld_plan_info(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("d", ctypes.c_int32), ("transposed", ctypes.c_int32), ("i64", ctypes.c_int32),
                ("mp", ctypes.c_int32), ("R", ctypes.c_int32), ("C", ctypes.c_int32),
                ("P", ctypes.c_int32), ("P_tab", ctypes.c_int32), ("n_prefix", ctypes.c_uint64),
                ("words", ctypes.c_double), ("kernel", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ld_server_config(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("max_inflight_problems", ctypes.c_int32),
                ("max_items_per_launch", ctypes.c_int32), ("words_per_item", ctypes.c_double),
                ("step_ms", ctypes.c_double), ("max_queued", ctypes.c_int32), ("device", ctypes.c_int32),
                ("express_ms", ctypes.c_double), ("idle_spin_ms", ctypes.c_double),
                ("min_items", ctypes.c_int32)]


class ld_request_timing(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("lane", ctypes.c_int32), ("items", ctypes.c_int32),
                ("words", ctypes.c_double), ("plan_ms", ctypes.c_double), ("wait_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double)]


class ld_valu_probe_result(ctypes.Structure):
    _fields_ = [("sclk_hz", ctypes.c_double), ("sclk_max_hz", ctypes.c_double),
                ("valu_lane_ops_per_s", ctypes.c_double), ("seconds", ctypes.c_double),
                ("compute_units", ctypes.c_int32), ("waves", ctypes.c_int32)]


class ld_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("items", ctypes.c_uint64), ("inflight", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("mean_wait_ms", ctypes.c_double),
                ("mean_plan_ms", ctypes.c_double), ("mean_run_ms", ctypes.c_double)]


# exported symbols and their signatures: name -> (restype, argtypes)
_P, _I32, _U32, _I64, _U64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64,
                              ctypes.c_uint64)
SIGNATURES = {
    "ld_norm": (_I64, [_P, _I32, _I32, _I32, _I32]),
    "ld_norm_batch": (ctypes.c_int, [_P, _I32, _P, _P, _P]),
    "ld_norm_range": (_I64, [_P, _I32, _I32, _I32, _I32, _I32, _U64, _U64]),
    "ld_norm_noalloc": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P, _P]),
    "ld_argmax": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P, _P, _P]),
    "ld_norm_resumable": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, ctypes.c_char_p, ctypes.c_double,
                                         ctypes.c_double, _P]),
    "ld_last_error": (ctypes.c_int, []),
    "ld_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ld_plan": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P]),
    "ld_plan_batch": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P]),
    "ld_gray_digit": (_U32, [_U32, _U32, _U64]),
    "ld_gray_change": (_I32, [_U32, _U64, _P, _P]),
    "ld_set_sweep_shape": (None, [_I32, _I32, _I32, _I32, _I32, _I32]),
    "ld_set_lane_fill": (None, [_I32]),
    "ld_set_launch_waves": (None, [_I32]),
    "ld_prepare": (_P, [_P, _I32, _I32, _I32, _I32]),
    "ld_run": (ctypes.c_int, [_P, _P, _P]),
    "ld_last_kernel_ms": (ctypes.c_float, [_P]),
    "ld_prepared_plan": (ctypes.c_int, [_P, _P]),
    "ld_release": (None, [_P]),
    "ld_batch_prepare": (_P, [_P, _I32, _P]),
    "ld_batch_run": (ctypes.c_int, [_P, _P, _P]),
    "ld_batch_last_ms": (ctypes.c_float, [_P]),
    "ld_batch_release": (None, [_P]),
    "ld_server_create": (_P, [_P]),
    "ld_server_submit": (ctypes.c_int, [_P, _P, _P]),
    "ld_server_poll": (ctypes.c_int, [_P, _U64, _P]),
    "ld_server_wait": (ctypes.c_int, [_P, _U64, _P]),
    "ld_server_cancel": (ctypes.c_int, [_P, _U64]),
    "ld_server_stats": (None, [_P, _P]),
    "ld_server_timings": (_I32, [_P, _P, _I32]),
    "ld_server_destroy": (None, [_P]),
    "ld_autotune": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_double]),
    "ld_load_tuning": (ctypes.c_int, [ctypes.c_char_p]),
    "ld_valu_probe": (ctypes.c_int, [ctypes.c_double, _P]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libld.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2503_21596_amd._build.build()")
        # torch ships its own libamdhip64.so.7; loading it first makes libld.so bind to
        # that same HIP runtime, so streams and events pass between the two and torch
        # still sees the GPU (two runtimes in one process do not share devices)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)   # a missing export is a broken build: raise
            f.restype = res
            f.argtypes = args
        # the shapes the autotuner measured on MI355X (its JSON, kept with the
        # package; the library's built-in defaults are the same values)
        if os.path.exists(TUNING_PATH) and os.environ.get("LD_TUNING", "1") != "0":
            L.ld_load_tuning(TUNING_PATH.encode())
        _lib = L
    return _lib


def _err(code: Optional[int] = None) -> LdError:
    L = lib()
    c = L.ld_last_error() if code is None else code
    return LdError(c, L.ld_error_string(c).decode())


def _mat(M) -> np.ndarray:
    if hasattr(M, "detach"):          # a CPU torch tensor
        M = M.detach().cpu().numpy()
    a = np.ascontiguousarray(np.asarray(M), dtype=np.int32)
    if a.ndim != 2:
        raise ValueError("M must be a 2-D integer matrix")
    if not np.array_equal(a, np.asarray(M)):
        raise ValueError("M must hold integers representable in int32 (convert real entries first)")
    return a


def ld_norm(M, d: int = 1, marginals: int = 0) -> int:
    a = _mat(M)
    v = lib().ld_norm(a.ctypes.data, a.shape[0], a.shape[1], int(d), int(marginals))
    if v == INT64_MIN:
        raise _err()
    return int(v)


def ld_norm_range(M, d: int, marginals: int, q: int, prefix_begin: int, prefix_end: int) -> int:
    a = _mat(M)
    v = lib().ld_norm_range(a.ctypes.data, a.shape[0], a.shape[1], int(d), int(marginals), int(q),
                            int(prefix_begin), int(prefix_end))
    if v == INT64_MIN:
        raise _err()
    return int(v)


def ld_norm_noalloc(M, d: int = 1, marginals: int = 0, stream=None) -> int:
    """ld_norm on the library's static device scratch array (no device allocation)."""
    a = _mat(M)
    v = ctypes.c_int64(0)
    s = stream.cuda_stream if stream is not None else None
    rc = lib().ld_norm_noalloc(a.ctypes.data, a.shape[0], a.shape[1], int(d), int(marginals), ctypes.byref(v), s)
    if rc != LD_OK:
        raise _err(rc)
    return int(v.value)


def ld_argmax(M, d: int = 1, marginals: int = 0):
    """(value, a, b): the value and one assignment reaching it.  a holds one entry
    per row (signs for d = 1, messages for d >= 2); b the column signs for d = 1
    (None for d >= 2)."""
    a = _mat(M)
    n, m = a.shape
    v = np.zeros(1, dtype=np.int64)
    rows = np.zeros(n, dtype=np.int32)
    cols = np.zeros(m, dtype=np.int32)
    rc = lib().ld_argmax(a.ctypes.data, n, m, int(d), int(marginals), v.ctypes.data, rows.ctypes.data,
                         cols.ctypes.data if d == 1 else None)
    if rc != LD_OK:
        raise _err(rc)
    return int(v[0]), rows, (cols if d == 1 else None)


def ld_norm_resumable(M, d: int, marginals: int, state_path: str, chunk_seconds: float = 10.0,
                      max_seconds: float = float("inf")):
    """The value once the whole search space has been swept (possibly over several
    calls), or None when max_seconds ran out first; progress is kept in state_path."""
    a = _mat(M)
    v = np.zeros(1, dtype=np.int64)
    ms = float(max_seconds) if max_seconds != float("inf") else 1e300
    rc = lib().ld_norm_resumable(a.ctypes.data, a.shape[0], a.shape[1], int(d), int(marginals),
                                 os.fsencode(state_path), float(chunk_seconds), ms, v.ctypes.data)
    if rc == LD_PENDING:
        return None
    if rc != LD_OK:
        raise _err(rc)
    return int(v[0])


def ld_norm_batch(problems: Sequence[Tuple], stream=None, return_status: bool = False):
    """problems: sequence of (M, d, marginals).  Returns the values (INT64_MIN where a
    problem failed) and, with return_status, the per-problem error codes."""
    mats = [_mat(p[0]) for p in problems]
    arr = (ld_problem * max(1, len(problems)))()
    for i, (a, p) in enumerate(zip(mats, problems)):
        arr[i] = ld_problem(a.ctypes.data, a.shape[0], a.shape[1], int(p[1]), int(p[2]))
    out = np.zeros(len(problems), dtype=np.int64)
    st = np.zeros(len(problems), dtype=np.int32)
    s = _stream_handle(stream)
    rc = lib().ld_norm_batch(ctypes.addressof(arr), len(problems), out.ctypes.data, st.ctypes.data, s)
    if rc != LD_OK and not return_status:
        raise _err(rc)
    return (out, st) if return_status else out


def _stream_handle(stream):
    if stream is None:
        return None
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class Prepared:
    """A planned problem whose tables stay resident on the GPU (ld_prepare)."""

    def __init__(self, M, d: int = 1, marginals: int = 0):
        a = _mat(M)
        self._h = lib().ld_prepare(a.ctypes.data, a.shape[0], a.shape[1], int(d), int(marginals))
        if not self._h:
            raise _err()

    def run(self, stream=None) -> int:
        v = ctypes.c_int64()
        rc = lib().ld_run(self._h, _stream_handle(stream), ctypes.byref(v))
        if rc != LD_OK:
            raise _err(rc)
        return int(v.value)

    def kernel_ms(self) -> float:
        return float(lib().ld_last_kernel_ms(self._h))

    def plan(self) -> dict:
        info = ld_plan_info()
        lib().ld_prepared_plan(self._h, ctypes.byref(info))
        out = {f[0]: getattr(info, f[0]) for f in ld_plan_info._fields_}
        out["kind_name"] = PLAN_KINDS.get(info.kind, "?")
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().ld_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A reusable batch (ld_batch_prepare): tables resident, launches in a HIP graph."""

    def __init__(self, problems: Sequence[Tuple]):
        mats = [_mat(p[0]) for p in problems]
        arr = (ld_problem * max(1, len(problems)))()
        for i, (a, p) in enumerate(zip(mats, problems)):
            arr[i] = ld_problem(a.ctypes.data, a.shape[0], a.shape[1], int(p[1]), int(p[2]))
        self.count = len(problems)
        self.status = np.zeros(self.count, dtype=np.int32)
        self._h = lib().ld_batch_prepare(ctypes.addressof(arr), self.count, self.status.ctypes.data)
        if not self._h:
            raise _err()

    def run(self, stream=None, check: bool = True) -> np.ndarray:
        out = np.zeros(self.count, dtype=np.int64)
        rc = lib().ld_batch_run(self._h, _stream_handle(stream), out.ctypes.data)
        if rc != LD_OK and check:
            raise _err(rc)
        return out

    def last_ms(self) -> float:
        return float(lib().ld_batch_last_ms(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().ld_batch_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan(M, d: int = 1, marginals: int = 0, batch: bool = False) -> dict:
    """The plan ld_norm makes for M (batch=True: the plan of a batch member)."""
    a = _mat(M)
    info = ld_plan_info()
    f = lib().ld_plan_batch if batch else lib().ld_plan
    rc = f(a.ctypes.data, a.shape[0], a.shape[1], int(d), int(marginals), ctypes.byref(info))
    out = {f[0]: getattr(info, f[0]) for f in ld_plan_info._fields_}
    out["status"] = rc
    out["kind_name"] = PLAN_KINDS.get(info.kind, "?")
    return out


def gray_digit(d: int, i: int, j: int) -> int:
    return int(lib().ld_gray_digit(d, i, j))


def gray_change(d: int, j: int):
    f, t = ctypes.c_uint32(), ctypes.c_uint32()
    i = lib().ld_gray_change(d, j, ctypes.byref(f), ctypes.byref(t))
    return int(i), int(f.value), int(t.value)


def set_sweep_shape(p_target: int = 0, c_min: int = 0, r_drop: int = -1, dary_ptab: int = 0,
                    sgpr_r: int = -1, dary_sgpr: int = -1) -> None:
    lib().ld_set_sweep_shape(p_target, c_min, r_drop, dary_ptab, sgpr_r, dary_sgpr)


def set_lane_fill(p_fill: int = 16) -> None:
    lib().ld_set_lane_fill(p_fill)


def set_launch_waves(waves_per_simd: int = 0) -> None:
    lib().ld_set_launch_waves(waves_per_simd)


def autotune(path: Optional[str] = None, budget_seconds: float = 20.0) -> None:
    rc = lib().ld_autotune(path.encode() if path else None, float(budget_seconds))
    if rc != LD_OK:
        raise _err(rc)


def load_tuning(path: str) -> None:
    rc = lib().ld_load_tuning(path.encode())
    if rc != LD_OK:
        raise _err(rc)


def valu_probe(target_ms: float = 200.0) -> dict:
    """Engine clock under a VALU-bound load and the VALU issue rate the device
    sustains (ld_valu_probe)."""
    r = ld_valu_probe_result()
    rc = lib().ld_valu_probe(float(target_ms), ctypes.byref(r))
    if rc != LD_OK:
        raise _err(rc)
    return {f[0]: getattr(r, f[0]) for f in ld_valu_probe_result._fields_}


class Server:
    """Continuous-batching request server (ld_server_* in include/ld.h)."""

    def __init__(self, arena_bytes: int = 256 << 20, max_inflight_problems: int = 1024,
                 max_items_per_launch: int = 65536, words_per_item: float = 0.0, step_ms: float = 0.0,
                 max_queued: int = 0, device: int = 0, express_ms: float = 0.0, idle_spin_ms: float = 0.0,
                 min_items: int = 0):
        cfg = ld_server_config(arena_bytes, max_inflight_problems, max_items_per_launch, words_per_item,
                               step_ms, max_queued, device, express_ms, idle_spin_ms, min_items)
        self._h = lib().ld_server_create(ctypes.byref(cfg))
        if not self._h:
            raise _err()

    def submit(self, M, d: int = 1, marginals: int = 0, check: bool = True):
        """Returns the ticket; with check=False returns (rc, ticket) and never raises."""
        a = _mat(M)
        p = ld_problem(a.ctypes.data, a.shape[0], a.shape[1], int(d), int(marginals))
        t = ctypes.c_uint64()
        rc = lib().ld_server_submit(self._h, ctypes.byref(p), ctypes.byref(t))
        if not check:
            return rc, int(t.value)
        if rc != LD_OK:
            raise _err(rc)
        return int(t.value)

    def poll(self, ticket: int):
        v = ctypes.c_int64()
        rc = lib().ld_server_poll(self._h, ticket, ctypes.byref(v))
        if rc == LD_PENDING:
            return None
        if rc != LD_OK:
            raise _err(rc)
        return int(v.value)

    def wait(self, ticket: int, check: bool = True):
        """The value; with check=False returns (rc, value) and never raises."""
        v = ctypes.c_int64()
        rc = lib().ld_server_wait(self._h, ticket, ctypes.byref(v))
        if not check:
            return rc, int(v.value)
        if rc != LD_OK:
            raise _err(rc)
        return int(v.value)

    def cancel(self, ticket: int) -> int:
        return int(lib().ld_server_cancel(self._h, ticket))

    def stats(self) -> dict:
        s = ld_stats()
        lib().ld_server_stats(self._h, ctypes.byref(s))
        return {f[0]: getattr(s, f[0]) for f in ld_stats._fields_}

    def timings(self, max_records: int = 1 << 20) -> list:
        """Per completed request: ticket, lane, items, words, plan_ms, wait_ms, run_ms."""
        cap = max(1, min(int(max_records), int(self.stats()["completed"])))
        buf = (ld_request_timing * cap)()
        n = lib().ld_server_timings(self._h, buf, cap)
        if n < 0:
            raise _err(LD_EINVAL)
        return [{f[0]: getattr(buf[i], f[0]) for f in ld_request_timing._fields_} for i in range(n)]

    def close(self):
        if self._h:
            lib().ld_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
