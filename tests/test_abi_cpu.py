"""Host-side checks of the C-ABI library: it loads without a GPU, exports every
symbol include/ld.h declares, validates arguments before touching the device, and
its planner and Gray-code helpers match what the paper fixes."""
import json
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

L = pytest.importorskip("paper_2503_21596_amd")


@pytest.fixture(scope="module")
def lib():
    return L.lib()


def header_functions():
    src = open(os.path.join(ROOT, "include", "ld.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(ld_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert "ld_norm" in names and "ld_norm_batch" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, name


@pytest.mark.parametrize("args,code", [
    ((None, 2, 2, 1, 0), 1),
    (("M", 0, 2, 1, 0), 1),
    (("M", 2, 0, 1, 0), 1),
    (("M", 2, 2, 0, 0), 1),
    (("M", 2, 2, 1, 2), 1),
    (("M", 2, 2, 2, 1), 2),     # marginals are defined only for the local bound
])
def test_validation_before_device(lib, args, code):
    M = np.ones((2, 2), dtype=np.int32)
    ptr = None if args[0] is None else M.ctypes.data
    v = lib.ld_norm(ptr, *args[1:])
    assert v == L.INT64_MIN
    assert lib.ld_last_error() == code
    assert lib.ld_error_string(code)


def test_range_validation(lib):
    M = np.ones((4, 3), dtype=np.int32)
    assert lib.ld_norm_range(M.ctypes.data, 4, 3, 1, 0, 2, 3, 3) == L.INT64_MIN   # empty range
    assert lib.ld_last_error() == L.LD_EINVAL
    assert lib.ld_norm_range(M.ctypes.data, 4, 3, 1, 0, 2, 0, 5) == L.INT64_MIN   # past 2^q
    assert lib.ld_norm_range(M.ctypes.data, 4, 3, 1, 0, 4, 0, 1) == L.INT64_MIN   # q > n - 1


def test_plan_transpose_and_zero_removal():
    M = np.zeros((9, 5), dtype=np.int32)
    M[1:8, 0:4] = synth.matrix(0, 7, 4, -5, 5, "abi")
    M[1:8, 0:4][M[1:8, 0:4] == 0] = 1
    p = L.plan(M, 1, 0)
    assert p["status"] == 0 and p["kind_name"] == "L1"
    assert (p["n"], p["m"], p["transposed"]) == (4, 7, 1)     # 7x4 after dropping zeros, transposed
    p2 = L.plan(M, 2, 0)
    assert (p2["n"], p2["m"], p2["transposed"]) == (7, 4, 0)  # no transposition for d >= 2


def test_plan_marginal_rules():
    M = synth.matrix(1, 5, 5, -5, 5, "abi")
    Z = M.copy()
    Z[0, :] = 0
    Z[:, 0] = 0
    p = L.plan(Z, 1, 1)
    assert p["kind_name"] == "L1" and (p["n"], p["m"]) == (4, 4)   # Sec. 2.2: no marginals left
    p = L.plan(M, 1, 1)
    assert p["kind_name"] == "L_marg"


def test_plan_reductions_worked_example(golden_dir):
    """Sec. 2.1.1: the zero row goes and row 2 = 2 x row 1 merges into row 1,
    leaving the printed 2 x 4 matrix.  For d >= 2 the row merge is allowed too
    (c = 2 > 0, rule A3) and the three single-signed columns then unite into one
    (Appendix A), so 2 rows and 2 columns remain and d = 2 needs no search."""
    g = json.load(open(os.path.join(golden_dir, "preprocessing_example.json")))
    M = np.array(g["matrix"], dtype=np.int32)
    p = L.plan(M, 1, 0)
    assert (p["n"], p["m"], p["transposed"]) == (2, 4, 0)
    p2 = L.plan(M, 2, 0)
    assert (p2["n"], p2["m"]) == (2, 2) and p2["kind_name"] == "sum|M|"


def test_plan_reduction_rules():
    base = np.array([[3, -1, 4, 1], [5, 9, -2, 6], [5, 3, 5, -8], [9, 7, 9, 3]], dtype=np.int32)
    # a negative multiple of a row: merged for d = 1 (rule A1), kept for d >= 2 (A3)
    M = np.vstack([base, -2 * base[1:2]]).astype(np.int32)
    assert L.plan(M, 1, 0)["n"] == 4
    assert L.plan(M, 3, 0)["n"] == 5
    # a positive multiple: merged for every d
    M = np.vstack([base, 3 * base[2:3]]).astype(np.int32)
    assert L.plan(M, 1, 0)["n"] == 4 and L.plan(M, 3, 0)["n"] == 4
    # a negative multiple of a column: merged for every d (rules A1, A2)
    M = np.hstack([base, -base[:, 1:2]]).astype(np.int32)
    assert L.plan(M, 1, 0)["m"] == 4 and L.plan(M, 3, 0)["m"] == 4
    # single-signed columns (base column 0 and the two added) unite for d >= 2 only
    # (Appendix A)
    U = np.hstack([base, np.array([[1], [0], [2], [5]]), -np.array([[4], [1], [1], [0]])]).astype(np.int32)
    assert L.plan(U, 1, 0)["m"] == 6
    assert L.plan(U, 2, 0)["m"] == 4
    # marginals: the first row and column take part in no merge (Sec. 2.2)
    M = base.copy()
    M[2] = 2 * M[0]
    assert L.plan(M, 1, 1)["n"] == 4
    M[3] = -M[1]
    assert L.plan(M, 1, 1)["n"] == 3


def test_plan_int64_boundary():
    # int32 path iff sum |M_xy| <= 2^31 - 1
    M = np.array([[2**30, 2**30 - 1], [0, 0]], dtype=np.int64)
    M = M[:1].astype(np.int32)
    assert L.plan(M, 1, 0)["i64"] == 0
    M2 = np.array([[2**30, 2**30]], dtype=np.int32)
    assert L.plan(M2, 1, 0)["i64"] == 1


def stirling2_upto(n, d):
    """sum_{k <= d} S(n, k): the number of restricted-growth strings of length n
    with at most d distinct digits (assignments of n rows to d messages up to
    relabelling the messages)."""
    S = [1] + [0] * d
    for _ in range(n):
        S = [0] + [k * S[k] + S[k - 1] for k in range(1, d + 1)]
    return sum(S)


def test_plan_dary_counts():
    # restricted-growth prefixes of length P_tab, then free digits: every class of
    # assignments up to message relabelling is covered at least once
    for d in (3, 4):
        p = L.plan(synth.config_pm(0), d, 0)
        assert p["kind_name"] == "L_d" and p["P_tab"] >= 1
        assert p["words"] == stirling2_upto(p["P_tab"], d) * d ** (16 - p["P_tab"])
        assert stirling2_upto(16, d) <= p["words"] <= d ** 15
    assert stirling2_upto(8, 3) == 1094 and stirling2_upto(8, 4) == 2795
    # d >= rows: the value is sum |M|, no search
    assert L.plan(synth.matrix(0, 3, 4, -3, 3, "abi"), 3, 0)["kind_name"] in ("sum|M|",)


def test_plan_headline_shape():
    p = L.plan(synth.config_42_l1(0), 1, 0)
    assert p["words"] == 2.0 ** 41
    assert p["R"] + p["C"] + p["P"] == 41


def test_plan_wide_and_too_big():
    # more than 64 columns: the wide (LDS-state) kernel takes it
    M = synth.matrix(2, 3, 70, 1, 9, "abi")
    p = L.plan(M, 1, 0)
    assert p["status"] == 0 and p["words"] == 4
    # 64 rows and 64 columns: 2^63 sign vectors even after the sign symmetry (Sec. 2.1.3)
    B = synth.matrix(3, 64, 64, 1, 9, "abi")
    assert L.plan(B, 1, 0)["status"] == L.LD_ETOOBIG


def test_brgc_table1(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "brgc_table1.json")))
    for i, row in g["rows_by_digit"].items():
        assert [L.gray_digit(2, int(i), j) for j in range(16)] == row
    for j, tag in enumerate(g["change_row"]):
        if j == 0:
            continue  # word 0 differs from word 15 (cyclic); the helper starts at j >= 1
        i, f, t = L.gray_change(2, j)
        assert tag == f"{i}{'+' if t == 1 else '-'}" and f == 1 - t


def test_trgc_table3(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "trgc_table3.json")))
    for i, row in g["rows_by_digit"].items():
        assert [L.gray_digit(3, int(i), j) for j in range(27)] == row
    for j, dig in enumerate(g["change_row"]):
        if dig is None:
            continue
        i, f, t = L.gray_change(3, j)
        assert i == dig
        assert f == L.gray_digit(3, i, j - 1) and t == L.gray_digit(3, i, j)


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_gray_hamming_one(d):
    # consecutive words differ in exactly the reported digit
    for j in range(1, d ** 4):
        i, f, t = L.gray_change(d, j)
        prev = [L.gray_digit(d, k, j - 1) for k in range(5)]
        cur = [L.gray_digit(d, k, j) for k in range(5)]
        diff = [k for k in range(5) if prev[k] != cur[k]]
        assert diff == [i] and prev[i] == f and cur[i] == t


def test_tuning_file_round_trip(tmp_path):
    """ld_load_tuning reads the autotuner's JSON (host only) and new plans follow
    it; a missing file is an error.  The shipped table is restored afterwards."""
    path = tmp_path / "t.json"
    path.write_text('{"bin_c_target": 10, "plain_p_target": 18, "plain_p_min": 12, "plain_c_goal": 14, '
                    '"sgpr_r": 4, "variant_l1_2": -1, "measured": []}')
    M = synth.config_42_l1(0)
    p0 = L.plan(M, 1, 0)
    try:
        L.load_tuning(str(path))
        p = L.plan(M, 1, 0)
        assert p["P"] == 18 and p["R"] == 4 and p["words"] == 2.0 ** 41
        with pytest.raises(L.LdError):
            L.load_tuning(str(tmp_path / "missing.json"))
    finally:
        L.load_tuning(L.TUNING_PATH)
    p = L.plan(M, 1, 0)
    assert (p["R"], p["P"], p["C"], p["kernel"]) == (p0["R"], p0["P"], p0["C"], p0["kernel"])


def test_plan_dary_lane_trading():
    """Plain d-ary calls trade mid rows for lanes (prefixes) in two stages: down to
    two mid rows until 2^17 lanes exist, then up to 2^19 lanes only while a lane
    keeps at least 2^12 words (d^(C+R) >= 4096).  Values never depend on this."""
    def lane_words(p, d):
        return d ** (p["C"] + p["R"])

    # small: fills 2^17 lanes as far as two mid rows allow
    p = L.plan(synth.config_pm(0), 3, 0)
    assert p["C"] == 2 or p["n_prefix"] >= 2 ** 17, p
    # mid-size d = 3: more lanes than 2^17, each still long
    M = synth.matrix(95, 22, 40, -100, 100, "ab")
    p = L.plan(M, 3, 0)
    assert p["n_prefix"] > 2 ** 17 and lane_words(p, 3) >= 4096, p
    # large d = 3: already beyond 2^19 lanes with long lanes, so nothing moves
    M = synth.matrix(155, 24, 40, -100, 100, "ab")
    p = L.plan(M, 3, 0)
    assert p["n_prefix"] >= 2 ** 19 and lane_words(p, 3) >= 4096, p
    # d = 4 near the floor: the second stage stops at 4^(C + 3) = 4096
    M = synth.matrix(102, 17, 30, -100, 100, "ab")
    p = L.plan(M, 4, 0)
    assert lane_words(p, 4) >= 4096 or p["n_prefix"] < 2 ** 17, p
    for d, n, m in [(3, 22, 40), (3, 20, 40), (4, 18, 16), (4, 19, 30)]:
        p = L.plan(synth.matrix(55 + n + m, n, m, -100, 100, "ab"), d, 0)
        assert p["C"] >= 2
        # beyond 2^17 lanes a lane keeps 2^12 words, unless the first stage had to
        # go down to two mid rows to reach 2^17 (one trade multiplies the lanes by
        # d or more, so it can land past 2^17)
        if p["n_prefix"] > 2 ** 17:
            assert lane_words(p, d) >= 4096 or p["C"] == 2, (d, n, m, p)


def test_plan_kernel_family_and_mfma_selection():
    """ld_plan_info.kernel names the sweep kernel: the headline takes the packed 16-bit
    kernel (5, six low rows); with variant 8 the int8-MFMA kernel (2, five low rows)
    where the mid-row deltas fit int8 and 1 <= C <= 16, else the SGPR-operand kernel
    with 5 low rows (1)."""
    M = synth.config_42_l1(0)
    p = L.plan(M, 1, 0)
    assert p["kernel"] == 5 and p["R"] == 6
    rc0 = p["R"] + p["C"]
    try:
        L.set_sweep_shape(0, 0, -1, 0, 8, -1)
        p = L.plan(M, 1, 0)
        # the same prefix rows, one low row fewer and one mid row more
        assert p["kernel"] == 2 and p["R"] == 5 and p["R"] + p["C"] == rc0 and 1 <= p["C"] <= 16
        big = synth.matrix(4, 20, 20, -1000, 1000, "abi")      # deltas 2 * 1000 do not fit int8
        p = L.plan(big, 1, 0)
        assert p["kernel"] == 1 and p["R"] == 5
        assert L.plan(synth.matrix(5, 26, 26, -120, 120, "abi"), 2, 0)["kernel"] == 2
        assert L.plan(synth.matrix(6, 12, 20, -9, 9, "abi"), 3, 0)["kernel"] in (0, 1, 5)   # d >= 3: d-ary
        assert L.plan(synth.matrix(7, 3, 70, 1, 9, "abi"), 1, 0)["kernel"] == 4          # > 64 columns: wide
    finally:
        L.load_tuning(L.TUNING_PATH)
    assert L.plan(M, 1, 0)["kernel"] == 5


def test_packed_binary_low_rows_by_size():
    """The packed binary kernel scores five low rows, six for a plain L1 / L_marg call
    with at least 11 mid rows at five (one row update per 64 words; the same
    prefixes, one mid row fewer); L2 and batch plans keep five."""
    for n in (30, 36, 40, 41, 42):
        M = synth.matrix(7 + n, n, 40, -100, 100, "bigr")
        for d, marg in ((1, 0), (1, 1), (2, 0)):
            p = L.plan(M, d, marg)
            if p["kernel"] != 5:
                continue
            rows = p["n"]                             # after preprocessing (L1 may transpose)
            c5 = rows - 1 - 5 - p["P"]                # mid rows at five low rows
            want = 6 if d == 1 and c5 >= 11 else 5
            assert p["R"] == want and p["R"] + p["C"] + p["P"] == rows - 1, (n, d, marg, p)
            assert L.plan(M, d, marg, batch=True)["R"] == 5
    assert L.plan(synth.config_42_l1(0), 1, 0)["R"] == 6
    assert L.plan(synth.config_42_marg(0), 1, 1)["R"] == 6


def test_big_r_threshold_from_the_tuning_table(tmp_path):
    """`plain_big_r_c` of a loaded table moves the switch to six low rows: 0 turns it
    off (the 42 x 42 solve plans five), 1 lets a 24 x 24 L1 problem with one mid row
    take it; the row split stays whole either way."""
    t = json.load(open(L.TUNING_PATH))
    t.pop("measured", None)
    M42, M24 = synth.config_42_l1(0), synth.matrix(5, 24, 24, -100, 100, "bigr")
    try:
        for c, want42, want24 in ((0, 5, 5), (1, 6, 6), (13, 6, 5)):
            t["plain_big_r_c"] = c
            path = tmp_path / ("t%d.json" % c)
            path.write_text(json.dumps(t))
            L.load_tuning(str(path))
            p42, p24 = L.plan(M42, 1, 0), L.plan(M24, 1, 0)
            assert (p42["R"], p24["R"]) == (want42, want24), (c, p42, p24)
            for p in (p42, p24):
                assert p["R"] + p["C"] + p["P"] == p["n"] - 1, p
    finally:
        L.load_tuning(L.TUNING_PATH)


def test_batch_plan_dary_step_count_fits_32_bits(tmp_path):
    """The d-ary register kernels count a lane's d^C Gray words in 32 bits.  A batch
    prefix cap moves prefix rows into the Gray walk; the planner must still keep
    d^C < 2^32 (moving rows back into the prefix), whatever the tuned cap."""
    path = tmp_path / "cap.json"
    path.write_text('{"batch_pfx_cap": 16, "dary_cwords": 729, "measured": []}')
    try:
        L.load_tuning(str(path))
        for d, n, m in [(3, 36, 12), (4, 30, 12), (5, 28, 12), (3, 24, 20), (6, 20, 8)]:
            M = synth.matrix(d * 100 + n, n, m, -100, 100, "cap")
            p = L.plan(M, d, 0, batch=True)
            assert p["status"] == L.LD_OK, (d, n, p)
            assert d ** p["C"] < 2 ** 32, (d, n, p)
            # the prefix rows and the walk still cover every restricted-growth class
            assert p["words"] == L.plan(M, d, 0)["words"], (d, n)
    finally:
        L.load_tuning(L.TUNING_PATH)


def test_error_strings_cover_every_code(lib):
    texts = {code: lib.ld_error_string(code).decode() for code in range(10)}
    fallback = lib.ld_error_string(99).decode()
    assert fallback == "unknown error code"
    assert fallback not in texts.values(), texts
    assert len(set(texts.values())) == 10


def test_small_problems_take_lanes_before_mid_rows(tmp_path):
    """A small binary problem keeps 2^16 prefixes (one wave per SIMD) before any row
    becomes a mid row; mid rows beyond those go up to the usual minimum of four,
    and large problems keep their shape (lane bounds 2^19 .. 2^20, 2^12 words per
    prefix between them)."""
    path = tmp_path / "shape.json"
    path.write_text('{"plain_p_target": 20, "plain_p_min": 19, "plain_c_goal": 12, "measured": []}')
    L.load_tuning(str(path))
    try:
        _check_small_problem_shapes()
    finally:
        L.load_tuning(L.TUNING_PATH)


def _check_small_problem_shapes():
    p = L.plan(synth.config_pm(0), 2, 0)              # 16 x 32 L2: every free row is a lane row
    assert p["R"] == 5 and p["C"] == 0 and p["P"] == 10, p
    p = L.plan(synth.config_pm24(0), 2, 0)            # 24 x 24 L2: 2^16 lanes, two mid rows
    assert p["R"] == 5 and p["C"] == 2 and p["P"] == 16, p
    p = L.plan(synth.config_small_l1(0), 1, 0)        # 20 x 20 L1
    assert p["C"] == 0 and p["P"] == 14, p
    p = L.plan(synth.matrix(3, 27, 27, -100, 100, "fill"), 1, 0)
    assert p["C"] == 4 and p["P"] == 17, p
    # 42 x 42 L1: 16 mid rows at five low rows, so six low rows and 15 mid rows
    p = L.plan(synth.config_42_l1(0), 1, 0)
    assert p["R"] == 6 and p["C"] == 15 and p["P"] == 20, p


def test_noalloc_refuses_images_beyond_its_array():
    """ld_norm_noalloc checks the problem's device image against its static array
    before any device call: a plan whose int64 tables exceed it gets LD_ESCRATCH
    (no GPU needed), invalid arguments their usual codes."""
    import ctypes
    big = synth.matrix(8111, 20, 8000, -3, 3, "noalloc_big")
    assert L.plan(big, 1, 0)["status"] == L.LD_OK
    v = ctypes.c_int64(7)
    rc = L.lib().ld_norm_noalloc(big.ctypes.data, 20, 8000, 1, 0, ctypes.byref(v), None)
    assert rc == L.LD_ESCRATCH and v.value == np.iinfo(np.int64).min
    assert L.lib().ld_last_error() == L.LD_ESCRATCH
    M = synth.matrix(8110, 4, 4, -5, 5, "noalloc")
    assert L.lib().ld_norm_noalloc(M.ctypes.data, 4, 4, 2, 1, ctypes.byref(v), None) == L.LD_EMARG_D
    assert L.lib().ld_norm_noalloc(None, 4, 4, 1, 0, ctypes.byref(v), None) == L.LD_EINVAL
    assert L.lib().ld_norm_noalloc(M.ctypes.data, 4, 4, 1, 0, None, None) == L.LD_EINVAL
