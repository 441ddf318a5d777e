"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle scripts.

This module holds no arithmetic of the method: it only draws integer matrices and
problem parameters.  The generator is SplitMix64 (Steele, Lea, Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw number i of stream `key` is mix64(key + (i + 1) * GAMMA).  A uniform
integer in [lo, hi] is lo + (draw mod (hi - lo + 1)); the modulo bias is below
2^-50 for every span used here.

Matrices are int32, row-major (M[x, y], x = row, y = column), drawn row by row.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def stream_key(seed: int, tag: str = "") -> int:
    """64-bit key of the stream named `tag` under `seed`."""
    h = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    for ch in tag.encode():
        with np.errstate(over="ignore"):
            h = _mix64(np.array([h ^ np.uint64(ch)], dtype=np.uint64))[0]
    return int(h)


def draws(key: int, count: int, start: int = 0) -> np.ndarray:
    """Raw 64-bit draws start .. start+count-1 of stream `key`."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + idx * GAMMA
    return _mix64(z)


def uniform_ints(key: int, count: int, lo: int, hi: int, start: int = 0) -> np.ndarray:
    span = np.uint64(hi - lo + 1)
    d = draws(key, count, start)
    return (d % span).astype(np.int64) + lo


def matrix(seed: int, n: int, m: int, lo: int, hi: int, tag: str = "M") -> np.ndarray:
    """n x m int32 matrix with i.i.d. uniform entries in [lo, hi]."""
    v = uniform_ints(stream_key(seed, tag), n * m, lo, hi)
    return np.ascontiguousarray(v.reshape(n, m).astype(np.int32))


# ---------------------------------------------------------------------------
# the workloads (shapes and value laws of the benchmark configurations)

def config_small_l1(seed: int = 0) -> np.ndarray:
    """One 20x20 matrix, entries uniform in [-10, 10] (plain L1)."""
    return matrix(seed, 20, 20, -10, 10, "small_l1")


def config_42_l1(seed: int = 0) -> np.ndarray:
    """One 42x42 matrix, entries uniform in [-100, 100] (plain L1)."""
    return matrix(seed, 42, 42, -100, 100, "l1_42")


def config_42_marg(seed: int = 0) -> np.ndarray:
    """41x41 correlation block plus a marginal row and column: a 42x42 matrix whose
    row 0 / column 0 hold the marginals and M[0,0] the constant term, all entries
    uniform in [-100, 100]."""
    return matrix(seed, 42, 42, -100, 100, "marg_42")


def config_pm(seed: int = 0) -> np.ndarray:
    """16x32 prepare-and-measure matrix, entries uniform in [-50, 50] (used at d=2,3,4)."""
    return matrix(seed, 16, 32, -50, 50, "pm_16x32")


def config_pm24(seed: int = 0) -> np.ndarray:
    """24x24 matrix, entries uniform in [-50, 50] (used at d=2)."""
    return matrix(seed, 24, 24, -50, 50, "pm_24x24")


def batch_problems(seed: int = 0, count: int = 4096, d3_max_n: int = 20):
    """The mixed batch: n ~ U[12,28], m ~ U[8,40], d ~ U{1,2,3} (at most n),
    20% with marginals (those use d = 1), entries uniform in [-1000, 1000].
    Problems drawn with d = 3 redraw n ~ U[12, d3_max_n] (see the design notes:
    the literal law puts hours of work into a few d = 3 draws).
    Returns a list of (M, d, marginals)."""
    key = stream_key(seed, "batch")
    raw = uniform_ints(key, 5 * count, 0, 1 << 30)
    out = []
    for i in range(count):
        r = raw[5 * i: 5 * i + 5]
        n = 12 + int(r[0] % 17)
        m = 8 + int(r[1] % 33)
        d = 1 + int(r[2] % 3)
        marg = int(r[3] % 5) == 0
        if marg:
            d = 1
        if d == 3:
            n = 12 + int(r[4] % (d3_max_n - 12 + 1))
        d = min(d, n)
        M = matrix(seed * 1000003 + i, n, m, -1000, 1000, "batch_M")
        out.append((M, d, int(marg)))
    return out


def served_requests(seed: int = 0, count: int = 1000, rate: float = 200.0, d3_max_n: int = 20):
    """Poisson request stream: exponential inter-arrival times with mean 1/rate,
    n ~ U[16,34], m ~ U[16,48], d ~ U{1,2,3}, entries uniform in [-100, 100].
    Requests drawn with d = 3 redraw n ~ U[16, d3_max_n].
    Returns a list of (arrival_seconds, M, d)."""
    key = stream_key(seed, "serve")
    raw = uniform_ints(key, 5 * count, 0, (1 << 53) - 1)
    t = 0.0
    out = []
    for i in range(count):
        r = raw[5 * i: 5 * i + 5]
        u = (int(r[0]) + 0.5) / float(1 << 53)
        t += -np.log(u) / rate
        n = 16 + int(r[1] % 19)
        m = 16 + int(r[2] % 33)
        d = 1 + int(r[3] % 3)
        if d == 3:
            n = 16 + int(r[4] % (d3_max_n - 16 + 1))
        M = matrix(seed * 1000003 + i, n, m, -100, 100, "serve_M")
        out.append((t, M, d))
    return out
