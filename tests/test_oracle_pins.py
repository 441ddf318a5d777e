"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage of arXiv:2503.21596 (or the mathematical fact) it
relies on.  The brute-force helpers here are independent of the oracle: they
enumerate both parties of the bilinear form (Eq. (LM2) written as max over a and b
of a^T M b) or the b_y^a variables of Eq. (L2Mv2), with numpy matrix products.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import synth

# ---------------------------------------------------------------------------
# independent brute force


def _signs(k):
    return np.array(list(itertools.product([-1, 1], repeat=k)), dtype=np.int64)


def bf_l1_bilinear(M):
    """max over a in {+-1}^n, b in {+-1}^m of a^T M b (equals Eq. (LM2) because the
    best b for a given a is b_y = sign((aM)_y))."""
    M = np.asarray(M, dtype=np.int64)
    A = _signs(M.shape[0])
    B = _signs(M.shape[1])
    return int((A @ M @ B.T).max())


def bf_lmarg_bilinear(M):
    """max over a_0 = b_0 = +1 of a^T M b (Eq. (LMarg): b_0 = +1 makes column 0 linear)."""
    M = np.asarray(M, dtype=np.int64)
    A = _signs(M.shape[0])
    A = A[A[:, 0] == 1]
    B = _signs(M.shape[1])
    B = B[B[:, 0] == 1]
    return int((A @ M @ B.T).max())


def bf_ld_with_b(M, d):
    """Eq. (L2Mv2): max over messages a_x in 0..d-1 and Bob's outputs b_y^k = +-1 of
    sum_x sum_y M_xy b_y^{a_x}, with nothing eliminated."""
    M = np.asarray(M, dtype=np.int64)
    n, m = M.shape
    B = _signs(m)                                   # every output column b^k
    best = None
    for a in itertools.product(range(d), repeat=n):
        a = np.array(a)
        # R[k, j] = sum_{x: a_x = k} (M_x . B_j): the part of message k under choice B_j
        R = np.stack([(M[a == k].sum(axis=0) @ B.T) for k in range(d)])
        v = int(R.max(axis=1).sum())                # choose b^k independently per message
        best = v if best is None else max(best, v)
    return best


def bf_l2_identity(M):
    """max over a in {+-1}^n of sum_y max(|c_y|, |(aM)_y|), c = column totals: for two
    groups with sums u, v one has |u| + |v| = max(|u + v|, |u - v|)."""
    M = np.asarray(M, dtype=np.int64)
    A = _signs(M.shape[0])
    c = np.abs(M.sum(axis=0))
    S = np.abs(A @ M)
    return int(np.maximum(S, c[None, :]).sum(axis=1).max())


def rnd(seed, n, m, lo=-9, hi=9):
    return synth.matrix(seed, n, m, lo, hi, "pins")


# ---------------------------------------------------------------------------
# P1: the worked example of Sec. 2.1.2


def test_worked_example_printed_values(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "worked_example.json")))
    M = np.array(g["matrix"], dtype=np.int32)
    for step in g["steps"]:
        a = np.array(step["a"], dtype=np.int8)
        assert list(a.astype(np.int64) @ M.astype(np.int64)) == step["m"]
        assert oracle.value_of(M, 1, 0, a) == step["bell_value"]
        # the same strategy with every sign flipped has the same value (Sec. 2.1.2)
        assert oracle.value_of(M, 1, 0, -a) == step["bell_value"]


def test_worked_example_norms():
    M = np.array([[4, -7, -2], [-5, 2, 3], [9, -1, 4]], dtype=np.int32)
    assert oracle.l1(M) == bf_l1_bilinear(M) == 29
    assert oracle.l1(M.T.copy()) == 29
    assert oracle.lmarg(M) == bf_lmarg_bilinear(M) == 29
    assert oracle.ld(M, 2) == bf_ld_with_b(M, 2) == 33
    assert oracle.ld(M, 3) == np.abs(M).sum() == 37


# ---------------------------------------------------------------------------
# P2: the preprocessing example of Sec. 2.1.1 (rules A1, A3 of Appendix A)


def test_preprocessing_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "preprocessing_example.json")))
    M = np.array(g["matrix"], dtype=np.int32)
    R = np.array(g["reduced"], dtype=np.int32)
    assert oracle.l1(M) == oracle.l1(R) == bf_l1_bilinear(M) == 48
    for d in (2, 3):
        assert oracle.ld(M, d) == oracle.ld(R, d)
    assert oracle.ld(M, 2) == 54


# ---------------------------------------------------------------------------
# P5 / P6: closed forms


def test_chsh():
    assert oracle.l1(np.array([[1, 1], [1, -1]])) == 2


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_identity(n):
    assert oracle.l1(np.eye(n, dtype=np.int32)) == n


@pytest.mark.parametrize("seed", range(6))
def test_rank_one(seed):
    u = synth.uniform_ints(synth.stream_key(seed, "u"), 6, -7, 7)
    v = synth.uniform_ints(synth.stream_key(seed, "v"), 5, -7, 7)
    M = np.outer(u, v).astype(np.int32)
    assert oracle.l1(M) == int(np.abs(u).sum() * np.abs(v).sum())


@pytest.mark.parametrize("seed", range(4))
def test_nonnegative(seed):
    M = rnd(seed, 5, 6, 0, 9)
    total = int(M.sum())
    assert oracle.l1(M) == total
    for d in (2, 3):
        assert oracle.ld(M, d) == total


@pytest.mark.parametrize("seed", range(4))
def test_single_column(seed):
    M = rnd(seed, 7, 1)
    s = int(np.abs(M).sum())
    assert oracle.l1(M) == s
    for d in (2, 3):
        assert oracle.ld(M, d) == s


@pytest.mark.parametrize("seed", range(5))
def test_ld_full_and_monotone(seed):
    M = rnd(seed, 5, 4)
    vals = [oracle.l1(M)] + [oracle.ld(M, d) for d in range(2, 6)]
    assert all(vals[i] <= vals[i + 1] for i in range(len(vals) - 1))
    assert vals[-1] == int(np.abs(M).sum())          # d >= n: every row alone
    assert oracle.ld(M, 7) == int(np.abs(M).sum())


# ---------------------------------------------------------------------------
# P7 / P8: independent brute force


@pytest.mark.parametrize("seed", range(25))
def test_bilinear_bruteforce(seed):
    n = 1 + seed % 6
    m = 1 + (seed * 7) % 6
    M = rnd(seed, n, m)
    assert oracle.l1(M) == bf_l1_bilinear(M)
    assert oracle.l1_all(M) == oracle.l1(M)
    assert oracle.lmarg(M) == bf_lmarg_bilinear(M)


@pytest.mark.parametrize("seed", range(12))
def test_ld_bob_outputs_bruteforce(seed):
    n = 1 + seed % 4
    m = 1 + (seed * 5) % 4
    d = 2 + seed % 3
    M = rnd(seed, n, m)
    assert oracle.ld(M, d) == bf_ld_with_b(M, d)
    assert oracle.ld_all(M, d) == oracle.ld(M, d)


@pytest.mark.parametrize("seed", range(15))
def test_l2_identity(seed):
    M = rnd(seed, 2 + seed % 7, 1 + seed % 9, -20, 20)
    assert oracle.ld(M, 2) == bf_l2_identity(M)


# ---------------------------------------------------------------------------
# P9: invariances


def _signed_perm(seed, M, rows=True, cols=True, keep_first=False):
    key = synth.stream_key(seed, "perm")
    n, m = M.shape
    r = np.argsort(synth.draws(key, n, 0)) if rows else np.arange(n)
    c = np.argsort(synth.draws(key, m, 100)) if cols else np.arange(m)
    rs = np.where(synth.draws(key, n, 200) % 2 == 0, 1, -1) if rows else np.ones(n, int)
    cs = np.where(synth.draws(key, m, 300) % 2 == 0, 1, -1) if cols else np.ones(m, int)
    if keep_first:
        r = np.concatenate([[0], 1 + np.argsort(synth.draws(key, n - 1, 400))])
        c = np.concatenate([[0], 1 + np.argsort(synth.draws(key, m - 1, 500))])
        rs[0] = 1
        cs[0] = 1
    P = (M[r][:, c] * rs[:, None] * cs[None, :]).astype(np.int32)
    return P


@pytest.mark.parametrize("seed", range(8))
def test_l1_invariances(seed):
    M = rnd(seed, 6, 5)
    v = oracle.l1(M)
    assert oracle.l1(M.T.copy()) == v                   # Sec. 2.1.1: transposition
    assert oracle.l1(_signed_perm(seed, M)) == v          # sign flips, permutations
    assert oracle.l1((3 * M).astype(np.int32)) == 3 * v   # L(cM) = |c| L(M)
    assert oracle.l1((-2 * M).astype(np.int32)) == 2 * v


@pytest.mark.parametrize("seed", range(8))
def test_ld_invariances(seed):
    M = rnd(seed, 6, 5)
    for d in (2, 3):
        v = oracle.ld(M, d)
        # column sign flips and row / column permutations keep L_d (Sec. 2.3.1)
        assert oracle.ld(_signed_perm(seed, M, rows=False), d) == v
        key = synth.stream_key(seed, "rowperm")
        r = np.argsort(synth.draws(key, M.shape[0]))
        assert oracle.ld(np.ascontiguousarray(M[r]), d) == v


def test_ld_not_transposition_invariant():
    # Sec. 2.3.1: transposition does not keep L_d for d > 1; a witness matrix
    # (two rows, d = 2: each row alone gives sum |M| = 6; the 3 x 2 transpose has
    # three rows to split over two messages, and every split scores at most 4)
    M = np.array([[1, -1, 1], [1, 1, -1]], dtype=np.int32)
    assert oracle.ld(M, 2) == 6 and oracle.ld(M.T.copy(), 2) == 4


@pytest.mark.parametrize("seed", range(8))
def test_lmarg_invariances(seed):
    M = rnd(seed, 5, 6)
    v = oracle.lmarg(M)
    assert oracle.lmarg(M.T.copy()) == v
    assert oracle.lmarg(_signed_perm(seed, M, keep_first=True)) == v


# ---------------------------------------------------------------------------
# P10: the reductions of Appendices A and B as metamorphic relations


@pytest.mark.parametrize("seed", range(6))
def test_proportional_rows_and_cols(seed):
    M = rnd(seed, 5, 5)
    # a row that is c times row 1, c > 0: rows merge by addition (A1, A3)
    P = np.vstack([M, 2 * M[1:2]]).astype(np.int32)
    R = M.copy(); R[1] *= 3
    assert oracle.l1(P) == oracle.l1(R)
    for d in (2, 3):
        assert oracle.ld(P, d) == oracle.ld(R, d)
    # c < 0: L1 merges by subtraction (A1) ...
    N = np.vstack([M, -2 * M[1:2]]).astype(np.int32)
    assert oracle.l1(N) == oracle.l1(R)
    # a column that is c times column 2, c < 0: columns merge for every d (A1, A2)
    C = np.hstack([M, -3 * M[:, 2:3]]).astype(np.int32)
    Q = M.copy(); Q[:, 2] *= 4
    assert oracle.l1(C) == oracle.l1(Q)
    for d in (2, 3):
        assert oracle.ld(C, d) == oracle.ld(Q, d)


def test_negative_row_multiple_changes_ld():
    # rule A3 allows only c > 0 for rows when d >= 2; with c < 0 the merge is wrong
    M = np.array([[1, 2], [-1, -2], [3, -1]], dtype=np.int32)
    merged = np.array([[2, 4], [3, -1]], dtype=np.int32)
    assert oracle.ld(M, 2) != oracle.ld(merged, 2)


@pytest.mark.parametrize("seed", range(6))
def test_uniform_sign_columns(seed):
    M = rnd(seed, 5, 4)
    pos = synth.uniform_ints(synth.stream_key(seed, "pos"), 5, 0, 9)
    neg = -synth.uniform_ints(synth.stream_key(seed, "neg"), 5, 0, 9)
    W = np.hstack([M, pos[:, None], neg[:, None]]).astype(np.int32)
    U = np.hstack([M, (np.abs(pos) + np.abs(neg))[:, None]]).astype(np.int32)
    for d in (2, 3):                                   # Appendix B
        assert oracle.ld(W, d) == oracle.ld(U, d)


@pytest.mark.parametrize("seed", range(4))
def test_zero_rows_cols(seed):
    M = rnd(seed, 4, 4)
    Z = np.zeros((6, 6), dtype=np.int32)
    Z[1:5, 0:4] = M
    assert oracle.l1(Z) == oracle.l1(M)
    for d in (2, 3):
        assert oracle.ld(Z, d) == oracle.ld(M, d)


# ---------------------------------------------------------------------------
# P11: block-diagonal additivity


@pytest.mark.parametrize("seed", range(4))
def test_block_diagonal(seed):
    A = rnd(seed, 4, 3)
    B = rnd(seed + 100, 3, 4)
    D = np.zeros((7, 7), dtype=np.int32)
    D[:4, :3] = A
    D[4:, 3:] = B
    assert oracle.l1(D) == oracle.l1(A) + oracle.l1(B)
    for d in (2, 3):
        assert oracle.ld(D, d) == oracle.ld(A, d) + oracle.ld(B, d)


# ---------------------------------------------------------------------------
# P12 / P15: marginal closed forms and edge values


def test_marginal_only():
    M = np.array([[3, -2, 5], [-4, 0, 0], [7, 0, 0]], dtype=np.int32)
    assert oracle.lmarg(M) == 3 + 11 + 7 == 21


@pytest.mark.parametrize("seed", range(4))
def test_marginal_structure(seed):
    M = rnd(seed, 5, 5)
    Z = M.copy(); Z[0, :] = 0; Z[:, 0] = 0
    assert oracle.lmarg(Z) == oracle.l1(np.ascontiguousarray(M[1:, 1:]))   # Sec. 2.2
    C = M.copy(); C[:, 0] = 0
    assert oracle.lmarg(C) == oracle.l1(np.ascontiguousarray(M[:, 1:]))
    S = M.copy(); S[0, 0] += 17
    assert oracle.lmarg(S) == oracle.lmarg(M) + 17


def test_edges():
    r = np.array([[3, -4, 5]], dtype=np.int32)
    assert oracle.l1(r) == 12
    assert oracle.lmarg(r) == 3 + 9
    c = np.array([[3], [-4], [5]], dtype=np.int32)
    assert oracle.l1(c) == 12
    assert oracle.l1(np.zeros((4, 3), dtype=np.int32)) == 0
    assert oracle.lmarg(np.array([[-5]], dtype=np.int32)) == -5
    assert oracle.ld(np.array([[-5]], dtype=np.int32), 2) == 5


# ---------------------------------------------------------------------------
# the split-table form and the prefix-range form against the plain enumeration


# The split-table forms visit the pairs (p, q) of half-assignments in tiles of
# 512 p-values by 64 q-values, and split the q-values into one contiguous range per
# thread.  The sizes below reach several tiles of both tables (n = 22..26: 2^10 ..
# 2^12 p-values), a single partial p-tile (n <= 19) and ragged thread ranges
# (3 and 7 threads).
SPLIT_TILE_P, SPLIT_TILE_Q = 512, 64


@pytest.mark.parametrize("seed", range(6))
def test_split_table_agrees(seed):
    n = 3 + 3 * seed
    M = rnd(seed, n, 7, -30, 30)
    assert oracle.l1_split(M, 0) == oracle.l1(M)
    assert oracle.l1_split(M, 1) == oracle.lmarg(M)


@pytest.mark.parametrize("n,m,threads", [(22, 9, 8), (24, 7, 3), (24, 6, 7), (26, 5, 8)])
def test_split_table_agrees_multi_tile(n, m, threads):
    M = rnd(n * 10 + m, n, m, -30, 30)
    assert (1 << ((n - 1) // 2)) > SPLIT_TILE_P
    assert oracle.l1_split(M, 0, threads) == oracle.l1(M)
    assert oracle.l1_split(M, 1, threads) == oracle.lmarg(M)


@pytest.mark.parametrize("d,n,m,threads", [(2, 22, 6, 8), (2, 23, 5, 3), (3, 14, 5, 7), (3, 15, 4, 8),
                                           (4, 11, 4, 3), (5, 8, 3, 8), (2, 3, 4, 8), (4, 3, 3, 2),
                                           (2, 1, 3, 1), (3, 2, 2, 4), (6, 7, 3, 5)])
def test_ld_split_agrees(d, n, m, threads):
    M = rnd(d * 100 + n, n, m, -30, 30)
    assert oracle.ld_split(M, d, threads) == oracle.ld(M, d)


@pytest.mark.parametrize("seed", range(4))
def test_ld_split_bob_outputs_bruteforce(seed):
    n, m, d = 3 + seed % 2, 2 + seed % 3, 2 + seed % 3
    M = rnd(seed + 40, n, m)
    assert oracle.ld_split(M, d) == bf_ld_with_b(M, d)


def _split_position(n, radix, p, q):
    """Assignment digits whose half-assignments are p (rows 1..ka) and q (rows
    ka+1..n-1), digit i of p / q (base radix) belonging to the i-th row of its half;
    row 0 takes digit 1 (a_0 = +1) for radix 2 and message 0 otherwise."""
    f = n - 1
    ka = f // 2
    digits = [1 if radix == 2 else 0]
    for i in range(ka):
        digits.append(p // radix ** i % radix)
    for i in range(f - ka):
        digits.append(q // radix ** i % radix)
    return np.array(digits)


def _ragged_q(nb, threads):
    """A q-value inside the last (partial) q-tile of thread 0's range."""
    per, rem = divmod(nb, threads)
    length = per + (1 if rem else 0)
    return length - 1 if length % SPLIT_TILE_Q else length - SPLIT_TILE_Q // 2


@pytest.mark.parametrize("where", ["last_p_ragged_q", "first_p_last_q", "mid"])
@pytest.mark.parametrize("marg", [0, 1])
def test_split_planted_maximum(where, marg):
    """A matrix K a* v^T + E with small noise E has its maximum at a = a* only (up to
    the global sign, removed by a_0 = +1): for a != a*, |a . a*| <= n - 2, which
    costs 2K sum|v| > 2 n sum_y max|E_.y|.  Placing a* in a chosen tile of the split
    form makes a skipped or misplaced tile visible."""
    n, m, threads = 24, 6, 7
    ka, kb = (n - 1) // 2, (n - 1) - (n - 1) // 2
    na, nb = 1 << ka, 1 << kb
    if where == "last_p_ragged_q":
        p, q = na - 1, _ragged_q(nb, threads)
    elif where == "first_p_last_q":
        p, q = 0, nb - 1
    else:
        p, q = 1234 % na, 2345 % nb
    a = np.where(_split_position(n, 2, p, q) == 1, 1, -1).astype(np.int64)
    v = synth.uniform_ints(synth.stream_key(p + q, "planted_v"), m, 1, 3) * \
        np.where(synth.uniform_ints(synth.stream_key(p, "planted_s"), m, 0, 1) == 0, -1, 1)
    v[0] = abs(v[0])
    E = rnd(q + 7, n, m, -2, 2).astype(np.int64)
    K = 100
    assert 2 * K * np.abs(v).sum() > 2 * n * m * 2
    M = (K * np.outer(a, v) + E).astype(np.int32)
    s = a @ M.astype(np.int64)
    want = int(s[0] + np.abs(s[1:]).sum()) if marg else int(np.abs(s).sum())
    assert oracle.l1_split(M, marg, threads) == want
    assert (oracle.lmarg(M) if marg else oracle.l1(M)) == want


@pytest.mark.parametrize("d,n,threads", [(2, 22, 7), (3, 14, 3), (4, 11, 5)])
@pytest.mark.parametrize("where", ["last_p_ragged_q", "first_p_last_q"])
def test_ld_split_planted_maximum(d, n, threads, where):
    """Rows K h_{t(x)} + E_x built from d rows h_k of an 8 x 8 Hadamard matrix.  Two
    Hadamard rows differ in half of the columns, so a message holding c >= 1 rows
    of type k and one row of another type has norm 8Kc, the same as without that
    row: every row away from its own type's group costs 8K.  The maximum is
    therefore at the planted grouping t (up to relabelling the messages), as long
    as the noise moves each value by less than 4K."""
    m = 8
    H = np.array([[1]], dtype=np.int64)
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    ka, kb = (n - 1) // 2, (n - 1) - (n - 1) // 2
    na, nb = d ** ka, d ** kb
    p, q = (na - 1, _ragged_q(nb, threads)) if where == "last_p_ragged_q" else (0, nb - 1)
    t = _split_position(n, d, p, q)
    K = 200
    E = rnd(p + 3 * q, n, m, -2, 2).astype(np.int64)
    assert 2 * n * m * 2 < 4 * K
    M = (K * H[t] + E).astype(np.int32)
    want = int(sum(np.abs(M[t == k].astype(np.int64).sum(axis=0)).sum() for k in range(d)))
    assert oracle.ld_split(M, d, threads) == want
    assert oracle.ld(M, d) == want


@pytest.mark.parametrize("d,marg", [(1, 0), (1, 1), (2, 0), (3, 0)])
def test_range_partition(d, marg):
    M = rnd(d * 10 + marg, 6, 4)
    q = 2
    radix = 2 if d == 1 else d
    parts = [oracle.range_max(M, d, marg, q, p, p + 1) for p in range(radix ** q)]
    assert max(parts) == oracle.norm(M, d, marg)
    # one prefix by brute force: rows 4, 5 carry the digits of p
    p = 1
    best = None
    for rest in itertools.product(range(radix), repeat=3):
        digits = [1 if d == 1 else 0] + list(rest) + [p % radix, p // radix]
        a = [(1 if g else -1) for g in digits] if d == 1 else digits
        v = oracle.value_of(M, d, marg, a)
        best = v if best is None else max(best, v)
    assert parts[p] == best


# ---------------------------------------------------------------------------
# one assignment per relabelling class (Sec. 2.3.2: the value does not depend on
# how the messages are named)


def _stirling2_row(n):
    """S(n, k) for k = 0..n by the textbook recurrence S(n, k) = k S(n-1, k) + S(n-1, k-1)."""
    row = [1]
    for i in range(1, n + 1):
        new = [0] * (i + 1)
        for k in range(1, i + 1):
            new[k] = k * (row[k] if k < len(row) else 0) + row[k - 1]
        row = new
    return row


@pytest.mark.parametrize("n,d", [(1, 2), (4, 2), (5, 3), (7, 3), (8, 4), (9, 9), (10, 4), (11, 12), (6, 20)])
def test_class_count_is_stirling(n, d):
    assert oracle.rgs_count(n, d) == sum(_stirling2_row(n)[1:d + 1])


@pytest.mark.parametrize("seed", range(10))
def test_ld_classes_agrees(seed):
    d = 2 + seed % 5
    n = 2 + seed % 7
    m = 1 + (seed * 3) % 6
    M = rnd(seed + 500, n, m, -40, 40)
    v = oracle.ld(M, d)
    assert oracle.ld_classes(M, d) == v
    assert oracle.ld_classes(M, d, 3) == v
    if d ** n <= 2e6:
        assert oracle.ld_all(M, d) == v


@pytest.mark.parametrize("d", [3, 4])
def test_ld_classes_planted(d):
    """The planted-grouping matrix of test_ld_split_planted_maximum: its maximum is
    the planted grouping (up to relabelling), which the class walk must reach."""
    n, m, K = 9, 8, 200
    H = np.array([[1]], dtype=np.int64)
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    t = np.array([(x * 5 + 3) % d for x in range(n)])
    M = (K * H[t] + rnd(d + 90, n, m, -2, 2)).astype(np.int32)
    want = int(sum(np.abs(M[t == k].astype(np.int64).sum(axis=0)).sum() for k in range(d)))
    assert oracle.ld_classes(M, d) == want


def test_batch_golden_matches_the_generator():
    """tests/golden/batch_seed0.json holds the oracle's value of every batch problem:
    a sample of the cheap members, recomputed here by the naive enumeration, agrees
    (so the file belongs to the current generator and split-table forms)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_seed0.json")
    g = json.load(open(path))
    assert g["count"] == 4096 and len(g["values"]) == 4096
    probs = synth.batch_problems(0, 4096)
    cheap = [i for i, (M, d, marg) in enumerate(probs) if (d <= 2 and M.shape[0] <= 15) or (d == 3 and M.shape[0] <= 11)]
    assert len(cheap) >= 100
    for i in cheap[::len(cheap) // 40]:
        M, d, marg = probs[i]
        assert g["values"][i] == oracle.norm(M, d, marg), i
