"""GPU batches: every problem of a mixed batch equals its plain ld_norm value and the
oracle's (bit-exact); a prepared batch replays its captured HIP graph correctly
many times, with other GPU work in between."""
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


def mixed(seed, count, nmax=14):
    key = synth.stream_key(seed, "mixed")
    raw = synth.uniform_ints(key, 4 * count, 0, 1 << 30)
    probs = []
    for i in range(count):
        r = raw[4 * i: 4 * i + 4]
        d = 1 + int(r[0] % 4)
        marg = int(d == 1 and r[1] % 3 == 0)
        n = 2 + int(r[2] % (nmax - 1 if d <= 2 else 9))
        m = 1 + int(r[3] % 70)          # some columns beyond 64: the wide kernel
        probs.append((synth.matrix(seed * 7919 + i, n, m, -1000, 1000, "mix"), d, marg))
    return probs


def test_batch_mixed_vs_oracle():
    say("mixed batch vs oracle")
    probs = mixed(1, 120)
    out = L.ld_norm_batch(probs)
    for (M, d, marg), v in zip(probs, out):
        assert v == oracle.norm(M, d, marg), (M.shape, d, marg)


def test_batch_errors_are_per_problem():
    say("batch errors")
    good = synth.matrix(3, 5, 6, -9, 9, "err")
    probs = [(good, 1, 0), (good, 2, 1), (good, 3, 0), (np.zeros((3, 3), np.int32), 1, 0)]
    out, st = L.ld_norm_batch(probs, return_status=True)
    assert list(st) == [0, L.LD_EMARG_D, 0, 0]
    assert out[1] == L.INT64_MIN
    assert out[0] == oracle.l1(good) and out[2] == oracle.ld(good, 3) and out[3] == 0


def test_batch_workload_sample_vs_plain():
    """A slice of the 4096-problem workload: batch == plain == oracle (oracle on the
    cheaper members)."""
    say("workload slice")
    probs = synth.batch_problems(0, count=4096)[:96]
    out = L.ld_norm_batch(probs)
    for (M, d, marg), v in zip(probs, out):
        assert v == L.ld_norm(M, d, marg)
        words = 2 ** (M.shape[0] - 1) if d == 1 else d ** (M.shape[0] - 1)
        if words * M.shape[0] * M.shape[1] * d < 3e8:
            assert v == oracle.norm(M, d, marg)


def test_prepared_batch_graph_replays():
    say("graph replays")
    import torch
    probs = mixed(2, 64, nmax=16)
    want = np.array([oracle.norm(M, d, marg) for M, d, marg in probs])
    B = L.Batch(probs)
    x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
    for rep in range(5):
        got = B.run()
        assert np.array_equal(got, want), rep
        # unrelated eager work and a sync between replays
        x = (x * 1.0001 + 1).contiguous()
        torch.cuda.synchronize()
        assert B.last_ms() > 0
    stream = torch.cuda.Stream()
    got = B.run(stream)
    assert np.array_equal(got, want)
    B.close()


def test_prepared_single_runs_repeat():
    say("prepared repeat")
    M = synth.matrix(9, 18, 30, -50, 50, "prep")
    h = L.Prepared(M, 1, 1)
    want = oracle.lmarg(M)
    for _ in range(4):
        assert h.run() == want
    h.close()


def test_full_batch_sampled_against_oracle():
    """The 4096-problem batch workload exactly as the benchmark runs it (one device
    program, graph replay): every value equals the plain call's, and a seeded sample
    of the problems small enough for the oracle equals the oracle's value."""
    say("full batch sampled")
    probs = synth.batch_problems(0, 4096)
    B = L.Batch(probs)
    got = B.run()
    again = B.run()
    B.close()
    assert list(got) == list(again)
    cheap = [i for i, (M, d, marg) in enumerate(probs)
             if (d <= 2 and M.shape[0] <= 17) or (d == 3 and M.shape[0] <= 12)]
    key = synth.stream_key(11, "batch_sample")
    pick = sorted({cheap[int(r) % len(cheap)] for r in synth.uniform_ints(key, 80, 0, 1 << 30)})
    for i in pick:
        M, d, marg = probs[i]
        assert got[i] == oracle.norm(M, d, marg), (i, M.shape, d, marg)
    plain = [L.ld_norm(M, d, marg) for M, d, marg in probs[:512]]
    assert list(got[:512]) == plain
