"""GPU: the largest members of the batch and serving workloads against values the
oracle wrote (tests/golden/configs_seed0.json, from oracle/ only): each through a
plain call, the batch members inside the full 4096-problem batch, and the served
members through the request server mixed with other requests."""
import json
import os
import sys
import time

import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2503_21596_amd")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "configs_seed0.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def members(prefix):
    g = json.load(open(GOLDEN))
    out = []
    for key, info in sorted(g.get("members", {}).items()):
        if key.startswith(prefix):
            out.append((key, info, g["values"][key]))
    return out


def batch_member_inputs():
    probs = synth.batch_problems(0, 4096)
    return probs, [(key, info["index"], value) for key, info, value in members("batch_")]


def serve_member_inputs():
    reqs = synth.served_requests(0, 2000, 200.0)
    return [(key, reqs[info["index"]][1], info["d"], value) for key, info, value in members("serve_")]


def test_golden_members_present():
    b, s = members("batch_"), members("serve_")
    assert len(b) == 16 and len(s) == 3
    assert {(i["d"], i["n"]) for _, i, _ in b} >= {(1, 28), (2, 28), (3, 20)}
    assert {(i["d"], i["n"], i["m"]) for _, i, _ in s} >= {(2, 34, 48), (3, 20, 48)}


def test_batch_members_plain():
    probs, mem = batch_member_inputs()
    for key, i, want in mem:
        M, d, marg = probs[i]
        say("plain", key, M.shape, d, marg)
        assert L.ld_norm(M, d, marg) == want, (key, L.plan(M, d, marg))


def test_batch_members_in_full_batch():
    say("full batch, golden members")
    probs, mem = batch_member_inputs()
    out = L.ld_norm_batch(probs)
    B = L.Batch(probs)
    rep = B.run()
    B.close()
    for key, i, want in mem:
        assert out[i] == want and rep[i] == want, (key, out[i], rep[i], want)


def test_serve_members_plain():
    for key, M, d, want in serve_member_inputs():
        say("plain", key, M.shape, d)
        assert L.ld_norm(M, d, 0) == want, (key, L.plan(M, d, 0))


def test_serve_members_in_the_mix():
    """The served members submitted while other requests arrive and run (continuous
    batching); every result equals the oracle's."""
    say("served members in the mix")
    big = serve_member_inputs()
    key = synth.stream_key(5, "golden_mix")
    raw = synth.uniform_ints(key, 3 * 40, 0, 1 << 30)
    small = []
    for i in range(40):
        r = raw[3 * i: 3 * i + 3]
        d = 1 + int(r[0] % 3)
        n = 6 + int(r[1] % (12 if d < 3 else 6))
        m = 4 + int(r[2] % 40)
        M = synth.matrix(880 + i, n, m, -100, 100, "gmix")
        small.append((M, d, oracle.norm(M, d, 0)))
    with L.Server(step_ms=1.0) as S:
        tickets = []
        for i, (M, d, want) in enumerate(small):
            tickets.append((S.submit(M, d, 0), want, f"small{i}"))
            if i % 13 == 0 and i // 13 < len(big):
                k, B, db, wb = big[i // 13]
                tickets.append((S.submit(B, db, 0), wb, k))
            time.sleep(0.0005)
        for t, want, tag in tickets:
            assert S.wait(t) == want, tag


BATCH_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_seed0.json")


def test_full_batch_every_problem_against_oracle():
    """Every one of the 4096 problems of the batch workload, through a plain batch
    call and through a prepared batch replayed from its HIP graph, against the
    oracle's values (tests/golden/batch_seed0.json, written by
    tests/golden/make_batch_golden.py from oracle/ only)."""
    g = json.load(open(BATCH_GOLDEN))
    assert g["count"] == 4096 and len(g["values"]) == 4096
    probs = synth.batch_problems(0, 4096)
    say("full batch vs oracle")
    assert [int(v) for v in L.ld_norm_batch(probs)] == g["values"]
    B = L.Batch(probs)
    try:
        for _ in range(2):
            assert [int(v) for v in B.run()] == g["values"]
    finally:
        B.close()
