"""GPU: the binary sweep whose Gray-code state update runs on the matrix cores
(int8 MFMA) against the oracle, bit-exactly.

The kernel is selected with sweep variant 8.  It takes the place of the
SGPR-operand kernel with R = 5 low rows, whose tables it shares, for int32 binary
problems (L1, L_marg, L2) whose mid-row deltas fit int8 (after preprocessing:
|entry| <= 127 for L1 and L_marg, entry in [-128, 127] for L2) and that have
1 <= C <= 16 mid rows; other problems keep the SGPR-operand kernel.  Each case
checks which kernel the plan used, so the tests cover both sides of that rule."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2503_21596_amd")

VARIANT_MFMA = 8
KERNEL_MFMA = 2
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "configs_seed0.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture
def mfma():
    # small problems here keep mid rows (the kernel needs 1 <= C <= 16) instead of
    # trading them for lanes
    L.set_sweep_shape(0, 0, -1, 0, VARIANT_MFMA, -1)
    L.set_lane_fill(0)
    try:
        yield
    finally:
        L.set_lane_fill(16)
        L.set_sweep_shape(20, 4, -1, 0, 5, -1)
        if os.path.exists(L.TUNING_PATH):
            L.load_tuning(L.TUNING_PATH)


def eligible(p):
    return p["i64"] == 0 and p["kind"] in (0, 1, 2) and p["R"] == 5 and 1 <= p["C"] <= 16 and p["kernel"] >= 0


def check(M, d, marg):
    p = L.plan(M, d, marg)
    got = L.ld_norm(M, d, marg)
    want = oracle.norm(M, d, marg)
    assert got == want, (M.shape, d, marg, got, want, p)
    return p


def test_widths_and_kinds(mfma):
    """Every accumulator-tile count (1 to 4 tiles of 16 columns) and column
    remainder, rows from 7 (C = 1, two words per prefix) up, L1, L_marg and L2."""
    widths = [1, 2, 3, 5, 8, 13, 16, 17, 24, 31, 32, 33, 42, 47, 48, 49, 57, 63, 64]
    used = 0
    for i, m in enumerate(widths):
        for n in (7, 9, 12, 14):
            M = synth.matrix(1300 + 7 * i + n, n, m, -127, 127, "mfma")
            for d, marg in [(1, 0), (1, 1), (2, 0)]:
                p = check(M, d, marg)
                if p["kernel"] == KERNEL_MFMA:
                    used += 1
                    assert eligible(p), p
    say("mfma widths: kernel used in", used, "cases")
    assert used >= 100


def test_operand_limits(mfma):
    """Entries of magnitude 127 and 128 (the last that fit the int8 operands and
    the first that do not), and merged rows whose sum leaves the range: every
    case gives the oracle's value, on whichever kernel the planner picks."""
    n, m = 12, 20
    for lo, hi, want_mfma in [(-127, 127, True), (-1, 1, True), (-128, 128, None), (-300, 300, False)]:
        M = synth.matrix(1400 + hi, n, m, lo, hi, "mfma_lim")
        if hi == 1:
            M = np.where(M >= 0, 127, -127).astype(np.int32)   # every entry at the limit
        if lo == -128:
            M[3, 5] = 128   # L1 / L_marg: a delta of 256 does not fit
        for d, marg in [(1, 0), (1, 1), (2, 0)]:
            p = check(M, d, marg)
            if want_mfma is True:
                assert p["kernel"] == KERNEL_MFMA, (lo, hi, d, marg, p)
            elif want_mfma is False:
                assert p["kernel"] != KERNEL_MFMA, (lo, hi, d, marg, p)
    # two proportional rows merge into one of twice the entries (> 127)
    M = synth.matrix(1410, n, m, -100, 100, "mfma_merge")
    M[7] = M[2]
    for d, marg in [(1, 0), (2, 0)]:
        check(M, d, marg)


def test_mid_row_count_limits(mfma):
    """C = 16 (the most reduction slots of the operands) and C = 17 (falls back),
    forced with a small lane count."""
    try:
        L.set_sweep_shape(2, 0, -1, 0, -1, -1)
        for n, want in [(24, True), (25, False)]:
            M = synth.matrix(1500 + n, n, 30, -90, 90, "mfma_c")
            for d, marg in [(1, 0), (2, 0)]:
                p = check(M, d, marg)
                assert p["C"] == n - 8, p
                assert (p["kernel"] == KERNEL_MFMA) == want, p
    finally:
        L.set_sweep_shape(20, 0, -1, 0, -1, -1)


def test_argmax_and_ranges(mfma):
    """The per-prefix maxima the argmax search records, and prefix sub-ranges."""
    for i, (n, m) in enumerate([(12, 20), (14, 33), (11, 47)]):
        M = synth.matrix(1600 + i, n, m, -90, 90, "mfma_arg")
        for d, marg in [(1, 0), (1, 1), (2, 0)]:
            assert L.plan(M, d, marg)["kernel"] == KERNEL_MFMA
            v, a, b = L.ld_argmax(M, d, marg)
            assert v == oracle.norm(M, d, marg)
            assert oracle.value_of(M, d, marg, a) == v
    M = synth.config_42_l1(0)
    q = 25
    key = synth.stream_key(11, "mfma_spots")
    for p in [int(x) for x in synth.uniform_ints(key, 3, 0, (1 << q) - 1)]:
        assert L.ld_norm_range(M, 1, 0, q, p, p + 1) == oracle.range_max(M, 1, 0, q, p, p + 1)


def test_batch(mfma):
    """A batch mixing problems that take the MFMA kernel with ones that do not."""
    probs = []
    for i in range(24):
        n = 7 + (i % 9)
        m = 3 + (5 * i) % 60
        hi = 127 if i % 4 else 1000
        M = synth.matrix(1700 + i, n, m, -hi, hi, "mfma_batch")
        d, marg = [(1, 0), (1, 1), (2, 0)][i % 3]
        probs.append((M, d, marg))
    got = L.ld_norm_batch(probs)
    want = [oracle.norm(M, d, marg) for M, d, marg in probs]
    assert list(got) == want


def test_full_size_golden(mfma):
    """The 42 x 42 L1 and L_marg solves (C = 16, 2^41 words each) against the
    oracle's stored values."""
    g = json.load(open(GOLDEN))["values"] if os.path.exists(GOLDEN) else {}
    if "l1_42" not in g or "marg_42" not in g:
        pytest.skip("42x42 values not yet written by tests/golden/make_golden.py")
    M = synth.config_42_l1(0)
    assert L.plan(M, 1, 0)["kernel"] == KERNEL_MFMA
    say("mfma 42x42 L1")
    assert L.ld_norm(M, 1, 0) == g["l1_42"]
    say("mfma 42x42 L_marg")
    assert L.ld_norm(synth.config_42_marg(0), 1, 1) == g["marg_42"]
