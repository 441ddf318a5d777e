"""GPU: ld_norm_noalloc, the plain solve on the library's static device scratch
array (no device allocation), against ld_norm on the same inputs, called through
the C ABI; two calls in a row, the second with a smaller input."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2503_21596_amd")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def noalloc(M, d, marg):
    a = np.ascontiguousarray(M, dtype=np.int32)
    v = ctypes.c_int64(0)
    rc = L.lib().ld_norm_noalloc(a.ctypes.data, a.shape[0], a.shape[1], d, marg, ctypes.byref(v), None)
    return rc, v.value


def test_noalloc_matches_plain_calls():
    """Larger problems first, then smaller ones on the same array: every value equals
    ld_norm's (and the oracle's where it is cheap), so nothing left in the array by
    one call leaks into the next."""
    cases = [
        (synth.matrix(8100, 30, 40, -100, 100, "noalloc"), 1, 0),   # binary, many prefixes
        (synth.matrix(8101, 12, 9, -100, 100, "noalloc"), 1, 0),    # smaller right after
        (synth.matrix(8102, 20, 24, -100, 100, "noalloc"), 3, 0),   # d-ary, restricted-growth table
        (synth.matrix(8103, 9, 7, -100, 100, "noalloc"), 3, 0),
        (synth.matrix(8104, 18, 33, -100, 100, "noalloc"), 1, 1),   # marginals
        (synth.matrix(8105, 6, 5, -100, 100, "noalloc"), 2, 0),
        (synth.matrix(8106, 10, 80, -50, 50, "noalloc"), 2, 0),     # wide kernel (m > 64)
        (synth.matrix(8107, 5, 4, -50, 50, "noalloc"), 9, 0),       # d >= rows: sum |M|
        (np.zeros((4, 3), np.int32), 1, 0),                         # all zero
    ]
    for i, (M, d, marg) in enumerate(cases):
        say("noalloc case", i, M.shape, d, marg)
        rc, v = noalloc(M, d, marg)
        assert rc == L.LD_OK, (i, rc)
        assert v == L.ld_norm(M, d, marg), (i, v)
        if M.shape[0] <= 12:
            assert v == oracle.norm(M, d, marg), (i, v)
    # the same two calls again, larger then smaller
    for M, d, marg in [cases[0], cases[1]]:
        rc, v = noalloc(M, d, marg)
        assert rc == L.LD_OK and v == L.ld_norm(M, d, marg)


def test_noalloc_errors():
    """Validation as ld_norm; a problem whose device image exceeds the array is
    refused with LD_ESCRATCH and launches nothing."""
    M = synth.matrix(8110, 4, 4, -5, 5, "noalloc")
    assert noalloc(M, 2, 1)[0] == L.LD_EMARG_D
    assert noalloc(M, 0, 0)[0] == L.LD_EINVAL
    big = synth.matrix(8111, 20, 8000, -3, 3, "noalloc_big")   # wide kernel, int64 tables > 1 MiB
    assert L.plan(big, 1, 0)["status"] == L.LD_OK
    rc, v = noalloc(big, 1, 0)
    assert rc == L.LD_ESCRATCH and v == np.iinfo(np.int64).min
    assert "scratch" in L.lib().ld_error_string(L.LD_ESCRATCH).decode()
    # the array is still usable after a refusal
    small = synth.matrix(8112, 8, 6, -50, 50, "noalloc")
    rc, v = noalloc(small, 1, 0)
    assert rc == L.LD_OK and v == oracle.norm(small, 1, 0)
