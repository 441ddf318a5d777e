"""GPU: a chunked, resumable solve gives the oracle's value however often it is
interrupted, and ignores state saved for another problem."""
import os
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


@pytest.mark.parametrize("d,marg", [(1, 0), (1, 1), (2, 0), (3, 0)])
def test_resume_after_interruptions(d, marg, tmp_path):
    say("resume", d, marg)
    n, m = (26, 30) if d < 3 else (15, 20)
    M = synth.matrix(60 + d + marg, n, m, -100, 100, "resume")
    want = oracle.norm_split(M, d, marg)
    assert L.ld_norm(M, d, marg) == want
    path = str(tmp_path / "state.txt")
    calls = 0
    v = None
    while v is None:
        v = L.ld_norm_resumable(M, d, marg, path, chunk_seconds=1e-4, max_seconds=1e-4)
        calls += 1
        assert calls < 100000
    assert v == want
    assert calls > 3                         # it really was interrupted
    text = open(path).read()
    assert text.startswith("ld_norm_resumable 1")
    # complete state: a further call returns at once with the value
    assert L.ld_norm_resumable(M, d, marg, path) == want


def test_resume_other_problem_starts_over(tmp_path):
    say("resume other problem")
    A = synth.matrix(70, 24, 28, -100, 100, "resume")
    B = synth.matrix(71, 24, 28, -100, 100, "resume")
    path = str(tmp_path / "state.txt")
    assert L.ld_norm_resumable(A, 1, 0, path, chunk_seconds=1e-4, max_seconds=1e-4) is None
    assert L.ld_norm_resumable(B, 1, 0, path) == oracle.l1_split(B)
    small = synth.matrix(72, 12, 9, -9, 9, "resume")
    assert L.ld_norm_resumable(small, 1, 0, path) == oracle.l1(small)
    assert L.ld_norm_resumable(np.zeros((3, 3), np.int32), 1, 0, path) == 0
