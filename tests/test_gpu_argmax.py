"""GPU: ld_argmax returns the value and an assignment that attains it.

The optimum is never unique (sign symmetry, relabelled messages, ties), so the
returned assignment is checked by attainment: the oracle evaluates the definition
at it (Eqs. LM2, LMarg, L_o_norm) and must get the value, which itself must equal
the oracle's maximum.  For d = 1 the column signs b must also give a^T M b = value."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2503_21596_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "configs_seed0.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(M, d, marg, want=None):
    M = np.asarray(M, dtype=np.int32)
    v, a, b = L.ld_argmax(M, d, marg)
    if want is None:
        want = oracle.norm(M, d, marg)
    assert v == want, (M.shape, d, marg, v, want)
    assert a.shape == (M.shape[0],)
    if d == 1:
        assert set(np.unique(a)) <= {-1, 1}
        assert set(np.unique(b)) <= {-1, 1}
        if marg:
            assert a[0] == 1 and b[0] == 1
        assert int(a.astype(np.int64) @ M.astype(np.int64) @ b.astype(np.int64)) == v
    else:
        assert b is None
        assert a.min() >= 0 and a.max() < d
    assert oracle.value_of(M, d, marg, a) == v, (M.shape, d, marg, a)
    return v, a, b


def test_worked_example():
    """The 3 x 3 example of Sec. 2.1.2: L1 = 29 at a = +-(+,-,+)."""
    say("argmax worked example")
    M = np.array([[4, -7, -2], [-5, 2, 3], [9, -1, 4]], dtype=np.int32)
    v, a, _ = check(M, 1, 0, 29)
    assert list(a) in ([1, -1, 1], [-1, 1, -1])
    check(M, 1, 1, 29)
    check(M, 2, 0, 33)
    check(M, 3, 0, 37)


@pytest.mark.parametrize("d,marg", [(1, 0), (1, 1), (2, 0), (3, 0), (4, 0)])
def test_random_shapes(d, marg):
    """Tall (transposed for d = 1), wide, square, with zero rows and columns."""
    say("argmax random", d, marg)
    shapes = [(2, 3), (5, 4), (9, 13), (14, 6), (12, 20), (16, 16), (7, 30)]
    if d >= 3:
        shapes = [(n, m) for n, m in shapes if n <= 12]
    for i, (n, m) in enumerate(shapes):
        M = synth.matrix(300 + 17 * i + d, n, m, -60, 60, "argmax")
        if i % 3 == 1:
            M[n // 2, :] = 0
            M[:, m // 2] = 0
        check(M, d, marg)


def test_edges():
    say("argmax edges")
    check(np.zeros((3, 4), np.int32), 1, 0, 0)
    check(np.zeros((3, 4), np.int32), 2, 0, 0)
    check(np.array([[-5]], np.int32), 1, 1, -5)
    check(np.array([[3, -4, 5]], np.int32), 1, 0, 12)
    check(np.array([[3], [-4], [5]], np.int32), 1, 0, 12)
    M = synth.matrix(5, 4, 7, -9, 9, "argmax_sum")
    check(M, 5, 0, int(np.abs(M).sum()))             # d >= rows: every row its own message
    # marginals, none set: L1 of the block
    M = synth.matrix(6, 6, 6, -9, 9, "argmax_nomarg")
    M[0, :] = 0
    M[:, 0] = 0
    check(M, 1, 1)


@pytest.mark.parametrize("d,marg", [(1, 0), (1, 1), (2, 0), (3, 0)])
def test_merged_rows_map_back(d, marg):
    """Rows merged by the planner (proportional, either sign for d = 1) get the
    sign or message that attains the value in the caller's matrix."""
    say("argmax merged rows", d, marg)
    for i, (n, m) in enumerate([(9, 8), (12, 10), (7, 14)]):
        M = synth.matrix(700 + i, n, m, -30, 30, "argmax_merge").astype(np.int64)
        M[n - 1] = -2 * M[1]
        M[n - 2] = 3 * M[2]
        M[:, m - 1] = -M[:, 1]
        M[:, 0] = np.abs(M[:, 0])
        M[:, 3] = np.abs(M[:, 3])
        if d >= 3:
            M = M[:9]
        check(M.astype(np.int32), d, marg)


def test_int64_and_wide():
    say("argmax int64 and wide")
    big = synth.matrix(7, 9, 11, -(2**30), 2**30, "argmax_big")
    check(big, 1, 0)
    check(big, 2, 0)
    wide = synth.matrix(8, 9, 70, -100, 100, "argmax_wide")   # m > 64: the LDS-state kernel
    check(wide, 2, 0)
    check(wide, 3, 0)


def test_full_size_l1():
    """42 x 42 L1 (2^41 words): the value is the oracle's stored one, the
    assignment attains it."""
    g = json.load(open(GOLDEN))["values"] if os.path.exists(GOLDEN) else {}
    if "l1_42" not in g:
        pytest.skip("l1_42 not yet written by tests/golden/make_golden.py")
    say("argmax 42x42")
    check(synth.config_42_l1(0), 1, 0, g["l1_42"])
