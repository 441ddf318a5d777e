"""GPU parity: the HIP library against the CPU oracle, bit-exact (integer work).

Every case is seeded and synthetic.  Sizes are chosen so the oracle finishes in
well under a second per case while the GPU plans still span several lanes, mid
Gray steps, low-row patterns and padded columns.
"""
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


def check(M, d, marg, expect=None):
    got = L.ld_norm(M, d, marg)
    want = oracle.norm(M, d, marg) if expect is None else expect
    assert got == want, (M.shape, d, marg, got, want, L.plan(M, d, marg))
    return got


# ---------------------------------------------------------------------------
# edge cases


def test_edges():
    say("edges")
    check(np.array([[3, -4, 5]], dtype=np.int32), 1, 0, 12)
    check(np.array([[3, -4, 5]], dtype=np.int32), 1, 1, 12)
    check(np.array([[3], [-4], [5]], dtype=np.int32), 1, 0, 12)
    check(np.array([[3], [-4], [5]], dtype=np.int32), 1, 1)
    check(np.zeros((4, 3), dtype=np.int32), 1, 0, 0)
    check(np.zeros((4, 3), dtype=np.int32), 1, 1, 0)
    check(np.zeros((4, 3), dtype=np.int32), 3, 0, 0)
    check(np.array([[-5]], dtype=np.int32), 1, 1, -5)
    check(np.array([[-5]], dtype=np.int32), 1, 0, 5)
    check(np.array([[-5]], dtype=np.int32), 2, 0, 5)
    check(np.array([[1, 1], [1, -1]], dtype=np.int32), 1, 0, 2)           # CHSH
    for n in (1, 2, 5, 9, 17):
        check(np.eye(n, dtype=np.int32), 1, 0, n)
    W = np.array([[4, -7, -2], [-5, 2, 3], [9, -1, 4]], dtype=np.int32)   # Sec. 2.1.2 example
    check(W, 1, 0, 29)
    check(W, 1, 1, 29)
    check(W, 2, 0, 33)
    check(W, 3, 0, 37)
    check(W, 9, 0, 37)                                                     # d >= n


def test_zero_rows_cols_and_marginal_structure():
    say("zero rows / marginal structure")
    M = synth.matrix(3, 6, 7, -9, 9, "gpu")
    Z = np.zeros((9, 10), dtype=np.int32)
    Z[2:8, 1:8] = M
    for d in (1, 2, 3):
        check(Z, d, 0)
    X = M.copy()
    X[0, :] = 0
    X[:, 0] = 0
    check(X, 1, 1)
    Y = M.copy()
    Y[0, :] = 0
    check(Y, 1, 1)


# ---------------------------------------------------------------------------
# random shapes


def _shapes():
    key = synth.stream_key(7, "shapes")
    raw = synth.uniform_ints(key, 4 * 400, 0, 1 << 30)
    out = []
    for i in range(400):
        r = raw[4 * i: 4 * i + 4]
        d = [1, 1, 1, 2, 2, 3, 3, 4, 5][int(r[0] % 9)]
        marg = int(d == 1 and r[1] % 2 == 1)
        nmax = {1: 18, 2: 16, 3: 11, 4: 9, 5: 8}[d]
        n = 1 + int(r[2] % nmax)
        m = 1 + int(r[3] % (48 if d <= 2 else 40))
        out.append((i, n, m, d, marg))
    return out


@pytest.mark.parametrize("block", range(8))
def test_random_shapes(block):
    cases = [c for c in _shapes() if c[0] % 8 == block]
    say("random shapes block", block, len(cases))
    for i, n, m, d, marg in cases:
        M = synth.matrix(1000 + i, n, m, -60, 60, "rand")
        check(M, d, marg)


def test_small_value_ranges():
    say("value ranges")
    for i in range(40):
        n, m = 3 + i % 12, 2 + (i * 5) % 40
        M = synth.matrix(2000 + i, n, m, -1, 1, "tiny")        # many ties
        check(M, 1, i % 2)
        check(M, 2, 0)


def test_int64_path():
    say("int64 path")
    for i in range(6):
        n, m = 4 + i, 5 + 2 * i
        M = synth.matrix(3000 + i, n, m, -(1 << 28), 1 << 28, "big")
        assert L.plan(M, 1, 0)["i64"] == 1
        check(M, 1, 0)
        check(M, 1, 1)
        check(M, 2, 0)
        if n >= 4:
            check(M, 3, 0)


def test_int32_boundary():
    say("int32 boundary")
    # sum |M| = 2^31 - 1 (int32 path) and 2^31 (int64 path); extremes fit int32
    a = np.array([[2**30, -(2**30 - 1)]], dtype=np.int32)
    b = np.array([[2**30, -(2**30)]], dtype=np.int32)
    assert L.plan(a, 1, 0)["i64"] == 0 and L.plan(b, 1, 0)["i64"] == 1
    check(a, 1, 0, 2**31 - 1)
    check(b, 1, 0, 2**31)
    c = np.array([[2**29, -(2**29)], [2**29, 2**29 - 1], [0, 1]], dtype=np.int32)
    check(c, 1, 0)
    check(c, 1, 1)
    check(c, 2, 0)


def test_sweep_shapes_agree():
    """Different lane / chunk splits of the same problem give the same value."""
    say("sweep shapes")
    M = synth.matrix(11, 22, 30, -100, 100, "shape")
    want = oracle.l1(M)
    try:
        for p_target, c_min, r_drop, sgpr_r in [(20, 4, 0, 4), (6, 10, 0, 5), (12, 1, 1, 0), (3, 4, 1, 0),
                                                (3, 4, 0, 4)]:
            L.set_sweep_shape(p_target, c_min, r_drop, 8, sgpr_r, -1)
            assert L.ld_norm(M, 1, 0) == want
            assert L.ld_norm(M, 1, 1) == oracle.lmarg(M)
    finally:
        L.set_sweep_shape(20, 4, 0, 8, 5, -1)


def planted(seed, n, m):
    """A random matrix with proportional rows and columns of both signs and some
    single-signed columns: every reduction of the planner applies somewhere."""
    M = synth.matrix(seed, n, m, -30, 30, "planted").astype(np.int64)
    M[n - 1] = -2 * M[1]
    M[n - 2] = 3 * M[2]
    M[:, m - 1] = -M[:, 1]
    M[:, m - 2] = 2 * M[:, 3]
    M[:, 0] = np.abs(M[:, 0])
    M[:, 4] = -np.abs(M[:, 4])
    return M.astype(np.int32)


@pytest.mark.parametrize("d,marg", [(1, 0), (1, 1), (2, 0), (3, 0), (4, 0)])
def test_reductions_planted(d, marg):
    """Proportional rows / columns (rules A1-A3) and single-signed columns
    (Appendix A) are merged before the sweep; the values stay the oracle's."""
    say("planted reductions", d, marg)
    for i, (n, m) in enumerate([(8, 9), (11, 7), (13, 12), (6, 16)]):
        M = planted(40 + i, n, m)
        p = L.plan(M, d, marg)
        assert p["n"] * p["m"] < n * m or p["kind_name"] in ("sum|M|", "zero")
        check(M, d, marg)


@pytest.mark.parametrize("dary_sgpr", [0, 1, 16])
def test_dary_kernel_variants(dary_sgpr):
    """The int32 d-ary kernels (subset operands in VGPRs with up to two low rows,
    streamed through SGPRs with three, or two columns per register as 16-bit
    halves with five low rows for d = 3 and four for d = 4, or one fewer where a
    single problem would have too few lanes) against the oracle, d = 3, 4, every
    column count up to the SGPR kernels' limits, row counts around R + 1 and plans
    with several mid rows, plain (the smaller R at these sizes) and batched (the
    larger R)."""
    say("dary variants", dary_sgpr)
    try:
        L.set_sweep_shape(0, 0, -1, 0, -1, dary_sgpr)
        for i, (n, m, d) in enumerate([(4, 5, 3), (5, 8, 3), (7, 13, 3), (9, 32, 3), (10, 52, 3), (8, 3, 3),
                                       (5, 6, 4), (7, 17, 4), (8, 40, 4), (9, 24, 4), (6, 1, 4),
                                       (12, 20, 3), (13, 47, 3), (12, 64, 3), (11, 9, 4), (10, 48, 4),
                                       (11, 52, 4), (6, 2, 3), (6, 10, 3)]):
            M = synth.matrix(950 + i, n, m, -500, 500, "dvariants")
            p = L.plan(M, d, 0)
            if p["kind_name"] == "L_d" and p["i64"] == 0:
                if dary_sgpr == 1 and p["mp"] * d <= 160:
                    assert p["R"] == 3 and p["kernel"] == 1, p
                packed_r = 5 if d == 3 else 4
                if dary_sgpr == 16 and n >= packed_r and p["mp"] // 2 * d <= 96:
                    assert p["R"] in (packed_r, packed_r - 1) and p["kernel"] == 5, p
                    if n >= 1 + packed_r:
                        assert L.plan(M, d, 0, batch=True)["R"] == packed_r
            want = check(M, d, 0)
            if dary_sgpr == 16:
                assert L.ld_norm_batch([(M, d, 0)])[0] == want   # the batch plan's kernel
        # plans that walk mid rows with the Gray code (and batch plans with more),
        # against the oracle's split-table form
        for i, (n, m, d) in enumerate([(14, 20, 3), (15, 24, 3), (13, 20, 4), (14, 16, 4)]):
            M = synth.matrix(1950 + i, n, m, -500, 500, "dvariants2")
            assert L.plan(M, d, 0)["C"] >= 1
            if dary_sgpr == 16:
                # plain: the smaller R (too few lanes at the larger); batched: the larger
                assert L.plan(M, d, 0)["R"] == (4 if d == 3 else 3)
                assert L.plan(M, d, 0, batch=True)["R"] == (5 if d == 3 else 4)
            want = oracle.ld_split(M, d)
            check(M, d, 0, want)
            assert L.ld_norm_batch([(M, d, 0)])[0] == want
    finally:
        L.set_sweep_shape(0, 0, -1, 0, -1, 1)


def test_dary_paired_widths():
    """The packed d = 3 kernel with five low rows at two waves per SIMD (more than 28
    columns) re-scores both messages a mid step changes from one stream of operand
    loads, by the pair {0, 1} or {1, 2}: batch plans that walk a mid row (both pairs
    occur) at every such width, odd column counts padded, against the oracle."""
    say("dary paired widths")
    try:
        L.set_sweep_shape(0, 0, -1, 0, -1, 16)
        for i, m in enumerate([29, 30, 33, 36, 39, 42, 45, 48, 52, 57, 61, 64]):
            M = synth.matrix(2950 + i, 14, m, -500, 500, "paired")
            p = L.plan(M, 3, 0, batch=True)
            assert p["R"] == 5 and p["kernel"] == 5 and p["C"] >= 1 and p["mp"] > 28, p
            want = oracle.ld_split(M, 3)
            assert L.ld_norm_batch([(M, 3, 0)])[0] == want, (m, p)
    finally:
        L.set_sweep_shape(0, 0, -1, 0, -1, 1)


def test_dary_packed_bounds():
    """The packed 16-bit d-ary kernel at the edge of its range: a column with
    sum |M_xy| = 2^15 - 1 is taken, 2^15 falls back to the SGPR-operand kernel;
    all rows of the extreme column sent to one message reach a sum of 2^15 - 1."""
    say("dary packed bounds")
    try:
        L.set_sweep_shape(0, 0, -1, 0, -1, 16)
        for n, m, d in [(9, 10, 3), (11, 21, 4), (13, 30, 3)]:
            key = synth.stream_key(n + 100 * d, "dedge")
            sg = np.where(synth.uniform_ints(key, n * m, 0, 1) == 0, -1, 1).reshape(n, m)
            mag = synth.uniform_ints(synth.stream_key(n, "dmag"), n * m, 1, 50).reshape(n, m)
            for target, packed in [(32767, True), (32768, False)]:
                A = (sg * mag).astype(np.int64)
                col = np.abs(A[:, 3])
                A[:, 3] = sg[:, 3] * (col * (target // col.sum()))
                A[0, 3] += sg[0, 3] * (target - np.abs(A[:, 3]).sum())
                assert np.abs(A[:, 3]).sum() == target
                A = A.astype(np.int32)
                p = L.plan(A, d, 0)
                assert p["kernel"] == (5 if packed else 1), (target, d, p)
                check(A, d, 0)
    finally:
        L.set_sweep_shape(0, 0, -1, 0, -1, 1)
        L.load_tuning(L.TUNING_PATH)


@pytest.mark.parametrize("sgpr_r", [0, 4, 5, 16])
def test_binary_kernel_variants(sgpr_r):
    """The int32 binary kernels (low-row operands in VGPRs, or streamed through
    SGPRs with 4 or 5 low rows, or two columns per register as 16-bit halves)
    against the oracle for L1, L_marg and L2, over every column-chunk shape
    (m = 1 .. 64 in steps that hit each remainder mod 8) and row counts below, at
    and above the low-row count."""
    say("binary variants", sgpr_r)
    try:
        L.set_sweep_shape(0, 0, -1, 0, sgpr_r, -1)
        cases = [(n, m) for n, m in [(1, 5), (2, 3), (3, 8), (4, 1), (5, 17), (6, 64), (7, 63), (9, 42),
                                     (12, 9), (13, 33), (14, 50), (15, 2), (16, 24), (11, 57)]]
        for i, (n, m) in enumerate(cases):
            M = synth.matrix(900 + i, n, m, -1000, 1000, "variants")
            for d, marg in [(1, 0), (1, 1), (2, 0)]:
                p = L.plan(M, d, marg)
                if p["i64"] == 0 and sgpr_r and p["kind"] != 4 and p["mp"] <= 64 and p["n"] > 1:
                    assert p["R"] == (5 if sgpr_r == 16 else sgpr_r), p
                if sgpr_r == 16 and p["kind_name"] in ("L1", "L2") and p["n"] > 1:
                    assert p["kernel"] == 5, p           # every column sum fits 16 bits here
                check(M, d, marg)
    finally:
        L.set_sweep_shape(0, 0, -1, 0, 5, -1)


def test_packed_kernel_bounds():
    """The packed 16-bit kernel at the edge of its range: a column with sum |M_xy|
    = 2^15 - 1 (every reachable column sum fits 16 bits offset by 2^15) is taken,
    2^15 is not; for L_marg the linear column 0 carries an offset of half its bound
    (ceil(B_0 / 2)), so it is taken up to B_0 = 21844.  Values stay the oracle's
    at the extremes, where some sign vectors reach column sums of +-(2^15 - 1)."""
    say("packed bounds")
    try:
        L.set_sweep_shape(0, 0, -1, 0, 16, -1)
        key = synth.stream_key(31, "edge")
        for n, m in [(9, 10), (14, 21), (18, 34)]:      # n <= m: L1 is not transposed
            sg = np.where(synth.uniform_ints(key, n * m, 0, 1) == 0, -1, 1).reshape(n, m)
            mag = synth.uniform_ints(synth.stream_key(n, "mag"), n * m, 1, 50).reshape(n, m)
            for target, packed in [(32767, True), (32768, False)]:
                A = (sg * mag).astype(np.int64)
                # scale column 3 so that sum |A_x3| is exactly `target`
                col = np.abs(A[:, 3])
                A[:, 3] = sg[:, 3] * (col * (target // col.sum()))
                A[0, 3] += sg[0, 3] * (target - np.abs(A[:, 3]).sum())
                assert np.abs(A[:, 3]).sum() == target
                A = A.astype(np.int32)
                for d in (1, 2):
                    p = L.plan(A, d, 0)
                    assert p["kernel"] == (5 if packed else 1), (target, d, p)
                    check(A, d, 0)
        # L_marg: column 0 is linear; its bound with the offset
        for b0, packed in [(21844, True), (21845, False)]:
            A = synth.matrix(77, 12, 16, -60, 60, "medge").astype(np.int64)
            A[:, 0] = np.abs(A[:, 0])
            A[:, 0] = A[:, 0] * (b0 // A[:, 0].sum())
            A[1, 0] += b0 - A[:, 0].sum()
            A[2, 0] = -A[2, 0]
            assert np.abs(A[:, 0]).sum() == b0
            A = A.astype(np.int32)
            p = L.plan(A, 1, 1)
            assert p["kernel"] == (5 if packed else 1), (b0, p)
            check(A, 1, 1)
            check(-A, 1, 1)
        # a linear column whose values are all negative: the score is negative
        N = -np.abs(synth.matrix(78, 9, 12, 1, 40, "neg"))
        assert L.plan(N, 1, 1)["kernel"] == 5
        check(N, 1, 1)
    finally:
        L.set_sweep_shape(0, 0, -1, 0, 5, -1)
        L.load_tuning(L.TUNING_PATH)


def test_packed_six_low_rows(tmp_path):
    """The packed kernel with six low rows (plain L1 / L_marg calls with many mid
    rows; by default only 40-odd-row problems) against the oracle for 24 and 25 rows
    at widths from 24 to 63 columns (12 to 32 dwords, odd column counts padded),
    under a tuning table whose mid-row threshold is lowered to 1.  Fewer columns
    than rows cannot reach it: L1 and L_marg put the smaller side in the rows."""
    say("six low rows")
    t = json.load(open(L.TUNING_PATH))
    t.pop("measured", None)
    t["plain_big_r_c"] = 1
    path = tmp_path / "big_r.json"
    path.write_text(json.dumps(t))
    try:
        L.load_tuning(str(path))
        for i, (n, m) in enumerate([(24, 24), (25, 33), (24, 42), (24, 57), (24, 63)]):
            M = synth.matrix(950 + i, n, m, -1000, 1000, "six")
            for marg in (0, 1):
                p = L.plan(M, 1, marg)
                assert p["R"] == 6 and p["kernel"] == 5 and p["C"] >= 1, p
                check(M, 1, marg)
    finally:
        L.load_tuning(L.TUNING_PATH)


# ---------------------------------------------------------------------------
# the benchmark configurations


@pytest.mark.parametrize("seed", range(3))
def test_config_small_l1(seed):
    say("20x20 L1 seed", seed)
    check(synth.config_small_l1(seed), 1, 0)


def test_config_pm_oracle_direct():
    say("16x32 d=2,3 and 24x24 d=2")
    M = synth.config_pm(0)
    v2 = check(M, 2, 0)
    v3 = check(M, 3, 0)
    assert L.ld_norm(M, 1, 0) <= v2 <= v3
    check(synth.config_pm24(0), 2, 0)


def _golden():
    if not os.path.exists(GOLDEN):
        return {}
    return json.load(open(GOLDEN)).get("values", {})


def test_config_pm_golden():
    g = _golden()
    say("16x32 golden", sorted(g))
    M = synth.config_pm(0)
    for d in (2, 3, 4):
        key = f"pm16x32_d{d}"
        if key not in g:
            pytest.skip(f"{key} not yet written by tests/golden/make_golden.py")
        assert L.ld_norm(M, d, 0) == g[key]
    if "pm24x24_d2" in g:
        assert L.ld_norm(synth.config_pm24(0), 2, 0) == g["pm24x24_d2"]


def test_full_size_planted_block_diagonal():
    """42x42 with a known value: L1 of a block-diagonal matrix is the sum of the
    blocks' L1 (each 21x21 block is oracle-cheap); rows and columns are then
    shuffled and sign-flipped, which keeps L1."""
    say("42x42 planted")
    A = synth.matrix(21, 21, 21, -100, 100, "blockA")
    B = synth.matrix(22, 21, 21, -100, 100, "blockB")
    want = oracle.l1(A) + oracle.l1(B)
    D = np.zeros((42, 42), dtype=np.int64)
    D[:21, :21] = A
    D[21:, 21:] = B
    key = synth.stream_key(5, "scramble")
    r = np.argsort(synth.draws(key, 42, 0))
    c = np.argsort(synth.draws(key, 42, 100))
    rs = np.where(synth.draws(key, 42, 200) % 2 == 0, 1, -1)
    cs = np.where(synth.draws(key, 42, 300) % 2 == 0, 1, -1)
    S = (D[r][:, c] * rs[:, None] * cs[None, :]).astype(np.int32)
    assert L.plan(S, 1, 0)["words"] == 2.0 ** 41
    assert L.ld_norm(S, 1, 0) == want


@pytest.mark.parametrize("key", ["l1_42", "marg_42"])
def test_full_size_configs_golden(key):
    """The full 42x42 solves (2^41 words each) against values the oracle wrote."""
    g = _golden()
    if key not in g:
        pytest.skip(f"{key} not yet written by tests/golden/make_golden.py")
    say("42x42 golden", key)
    if key == "l1_42":
        assert L.ld_norm(synth.config_42_l1(0), 1, 0) == g[key]
    else:
        assert L.ld_norm(synth.config_42_marg(0), 1, 1) == g[key]


@pytest.mark.parametrize("d,marg", [(1, 0), (1, 1)])
def test_full_size_range_spot_checks(d, marg):
    """Prefix sub-ranges of the 42x42 search space, each small enough for the oracle."""
    say("42x42 range", d, marg)
    M = synth.config_42_l1(0) if marg == 0 else synth.config_42_marg(0)
    q = 25
    key = synth.stream_key(9, "spots")
    pfx = [int(x) for x in synth.uniform_ints(key, 6, 0, (1 << q) - 1)]
    for p in pfx:
        got = L.ld_norm_range(M, d, marg, q, p, p + 1)
        want = oracle.range_max(M, d, marg, q, p, p + 1)
        assert got == want, (p, got, want)
    got = L.ld_norm_range(M, d, marg, q, pfx[0], pfx[0] + 3)
    want = max(oracle.range_max(M, d, marg, q, p, p + 1) for p in range(pfx[0], pfx[0] + 3))
    assert got == want


@pytest.mark.parametrize("d", [2, 3, 4])
def test_range_dary(d):
    say("range d", d)
    M = synth.matrix(40 + d, 9, 20, -50, 50, "rng")
    q = 3
    for p in (0, 1, d ** q - 1, d ** 2 + 1):
        assert L.ld_norm_range(M, d, 0, q, p, p + 1) == oracle.range_max(M, d, 0, q, p, p + 1)
    parts = [L.ld_norm_range(M, d, 0, q, p, p + 1) for p in range(d ** q)]
    assert max(parts) == oracle.ld(M, d)


def _dary_high_cases(d):
    """Matrices for alphabet d with more rows than messages (else the value is
    sum |M| without a search), sized for the oracle's class walk (about Bell(n)
    assignments).  With two restricted-growth prefix rows the plans walk at least
    two mid rows with the d-ary Gray code."""
    n = d + 1 if d >= 9 else d + 2
    ms = [5, 3] if d <= 10 else [3]
    cases = [synth.matrix(7000 + 37 * d + i, n, m, -300, 300, "dhi") for i, m in enumerate(ms)]
    if d == 9:
        cases.append(synth.matrix(7200, n, 70, -300, 300, "dhi"))   # more than 64 columns too
    return cases


def _plan_two_mid_rows(M, d):
    """Set the fewest restricted-growth prefix rows (from 2 up) whose plan walks at
    least two mid rows with at most 10^8 words, and return that plan; the words
    bound keeps the wide kernel's share (one wave per prefix) to a fraction of a
    second.  Raises on the host if no such shape exists."""
    for ptab in (2, 4, 6, 8, 10, 12):
        L.set_sweep_shape(0, 0, -1, ptab, -1, -1)
        p = L.plan(M, d, 0)
        if p["C"] >= 2 and p["words"] <= 1e8:
            return p
    raise AssertionError(("no plan with two mid rows and at most 1e8 words", M.shape, d))


@pytest.mark.parametrize("d", [5, 6, 7, 8, 9, 10, 12])
def test_dary_high_alphabets(d):
    """d >= 5: the d-ary reflected Gray code (Eqs. N_ary_G1-G3, d_aryGrayChange_1)
    over at least two mid rows, in the register kernels (d <= 8) and the wide LDS
    kernel (d >= 9, or more than 64 columns), plain and batched, against the
    oracle's walk over one assignment per relabelling class."""
    say("dary high alphabets", d)
    probs, want, ptabs = [], [], []
    try:
        for M in _dary_high_cases(d):
            p = _plan_two_mid_rows(M, d)
            assert p["kind_name"] == "L_d" and p["C"] >= 2, p
            assert p["kernel"] == (4 if (d > 8 or M.shape[1] > 64) else 0), p
            say("  ", M.shape, "C", p["C"], "P_tab", p["P_tab"], "words", p["words"])
            ptabs.append(p["P_tab"])
            w = oracle.ld_classes(M, d)
            check(M, d, 0, w)
            probs.append((M, d, 0))
            want.append(w)
        # the batch under the largest of those prefix shapes, its size checked first
        L.set_sweep_shape(0, 0, -1, max(ptabs), -1, -1)
        assert all(L.plan(M, d, 0, batch=True)["words"] <= 1e8 for M, d, _ in probs)
        assert list(L.ld_norm_batch(probs)) == want
    finally:
        L.set_sweep_shape(0, 0, -1, 8, -1, -1)


@pytest.mark.parametrize("d", [13, 17, 20])
def test_dary_range_large_alphabets(d):
    """Alphabets beyond the restricted-growth table (d > 16 fixes row 0 only) are
    checked on prefix sub-ranges: two free rows walk the d-ary Gray code in the
    wide kernel, the other rows are fixed by the prefix."""
    say("dary range d", d)
    n, m, q = 8, 4, 5
    M = synth.matrix(7300 + d, n, m, -300, 300, "dhr")
    key = synth.stream_key(d, "dhr_pfx")
    for p in [0, d ** q - 1] + [int(x) for x in synth.uniform_ints(key, 3, 0, d ** q - 1)]:
        assert L.ld_norm_range(M, d, 0, q, p, p + 1) == oracle.range_max(M, d, 0, q, p, p + 1), p
    assert L.ld_norm_range(M, d, 0, q, 7, 7 + 3 * d) == oracle.range_max(M, d, 0, q, 7, 7 + 3 * d)
    # a whole problem with more rows than messages has at least d^(d-1) classes
    # (d > 16: above 2^62, refused); with at most d rows it is sum |M|
    p = L.plan(synth.matrix(7400 + d, d + 2, m, -300, 300, "dhr"), d, 0)
    assert p["status"] == (L.LD_ETOOBIG if d > 16 else L.LD_OK), p
    S = synth.matrix(7500 + d, d, m, -300, 300, "dhr")
    assert L.ld_norm(S, d, 0) == int(np.abs(S).sum())       # the closed form for d >= rows


def test_batch_matches_plain():
    say("batch vs plain")
    probs = []
    for i in range(60):
        n, m = 2 + i % 13, 3 + (i * 7) % 30
        d = [1, 1, 2, 3][i % 4]
        marg = int(d == 1 and i % 8 == 1)
        probs.append((synth.matrix(500 + i, n, m, -1000, 1000, "batch"), d, marg))
    out = L.ld_norm_batch(probs)
    for (M, d, marg), v in zip(probs, out):
        assert v == oracle.norm(M, d, marg)


def test_autotune_writes_table_and_keeps_values(tmp_path):
    """A short autotuner run writes its table; whatever it picks, values stay the
    oracle's."""
    say("autotune")
    probs = [(synth.matrix(990 + i, 10 + i % 7, 12 + i % 9, -99, 99, "tune"), 1 + i % 3, 0) for i in range(12)]
    before = [oracle.norm(M, d, marg) for M, d, marg in probs]
    assert [L.ld_norm(M, d, marg) for M, d, marg in probs] == before
    path = str(tmp_path / "tuning.json")
    try:
        L.autotune(path, 2.0)
        table = json.load(open(path))
        for key in ("bin_c_target", "dary_cwords", "item_words", "plain_p_target", "plain_c_goal", "sgpr_r",
                    "dary_variant", "plain_dary_lanes", "variant_l1_2", "measured"):
            assert key in table, key
        assert len(table["measured"]) >= 1
        assert table["plain_dary_lanes"] in (0, 1 << 18, 1 << 19, 1 << 20, 1 << 21)
        assert table["dary_variant"] in (0, 1, 16) and table["sgpr_r"] in (0, 4, 5, 8, 16)
        assert [L.ld_norm(M, d, marg) for M, d, marg in probs] == before
        # the written table loads back and still gives the same values
        L.load_tuning(path)
        assert [L.ld_norm(M, d, marg) for M, d, marg in probs] == before
    finally:
        L.load_tuning(L.TUNING_PATH)
