"""GPU serving: requests submitted while others run give the same values as plain
calls and the oracle (continuous batching does not change results); invalid
requests fail alone; cancellation and backpressure behave."""
import sys
import threading
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2503_21596_amd")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_mix(seed, count):
    key = synth.stream_key(seed, "serve_mix")
    raw = synth.uniform_ints(key, 4 * count, 0, 1 << 30)
    out = []
    for i in range(count):
        r = raw[4 * i: 4 * i + 4]
        d = 1 + int(r[0] % 3)
        marg = int(d == 1 and r[1] % 4 == 0)
        n = 2 + int(r[2] % (15 if d < 3 else 9))
        m = 1 + int(r[3] % 48)
        out.append((synth.matrix(seed * 131 + i, n, m, -100, 100, "serve"), d, marg))
    return out


def test_serve_matches_oracle_and_plain():
    say("serve mix")
    probs = small_mix(1, 150)
    want = [oracle.norm(M, d, marg) for M, d, marg in probs]
    with L.Server(step_ms=1.0) as S:
        tickets = []
        for i, (M, d, marg) in enumerate(probs):
            tickets.append(S.submit(M, d, marg))
            if i % 25 == 0:
                time.sleep(0.002)          # let steps start between arrivals
        got = [S.wait(t) for t in tickets]
        st = S.stats()
    assert got == want
    assert st["completed"] == len(probs) and st["p50_ms"] > 0
    for (M, d, marg), v in list(zip(probs, got))[:30]:
        assert v == L.ld_norm(M, d, marg)      # alone == in the mix


def test_serve_threads_and_big_requests():
    """Several submitting threads; a few large requests span many steps while small
    ones keep arriving."""
    say("serve threads")
    big = [(synth.matrix(70 + i, 26, 30, -100, 100, "big"), 1 + i % 2, 0) for i in range(3)]
    small = small_mix(2, 90)
    results = {}
    with L.Server(step_ms=0.5) as S:
        def run(chunk, tag):
            for j, (M, d, marg) in enumerate(chunk):
                results[(tag, j)] = (S.submit(M, d, marg), M, d, marg)
                time.sleep(0.0005)
        th = [threading.Thread(target=run, args=(big, "big"))] + \
             [threading.Thread(target=run, args=(small[k::3], f"s{k}")) for k in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for key, (tk, M, d, marg) in results.items():
            v = S.wait(tk)
            if key[0] == "big":
                assert v == L.ld_norm(M, d, marg), key
            else:
                assert v == oracle.norm(M, d, marg), key
        st = S.stats()
        assert st["launches"] > 3


def test_serve_errors_do_not_disturb():
    say("serve errors")
    good = small_mix(3, 20)
    with L.Server() as S:
        tk = [S.submit(M, d, marg) for M, d, marg in good[:10]]
        rc, bad = S.submit(good[0][0], 2, 1, check=False)       # marginals with d = 2
        assert rc == L.LD_EMARG_D
        rc2, _ = S.wait(bad, check=False)
        assert rc2 == L.LD_EMARG_D
        z = S.submit(np.zeros((3, 4), np.int32), 1, 0)          # value 0 without a search
        s3 = S.submit(synth.matrix(5, 3, 7, -9, 9, "sum"), 5, 0)  # d >= rows: sum |M|
        tk += [S.submit(M, d, marg) for M, d, marg in good[10:]]
        assert [S.wait(t) for t in tk] == [oracle.norm(M, d, marg) for M, d, marg in good]
        assert S.wait(z) == 0
        assert S.wait(s3) == int(np.abs(synth.matrix(5, 3, 7, -9, 9, "sum")).sum())
        with pytest.raises(L.LdError):            # unknown ticket
            S.poll(99999999)


def test_serve_cancel():
    say("serve cancel")
    M = synth.matrix(9, 38, 40, -100, 100, "cancel")   # 2^37 words: many steps
    small = small_mix(4, 12)
    with L.Server(step_ms=1.0) as S:
        t_big = S.submit(M, 1, 0)
        time.sleep(0.01)
        assert S.cancel(t_big) == L.LD_OK
        rc, _ = S.wait(t_big, check=False)
        assert rc == L.LD_ECANCELED
        tk = [S.submit(A, d, marg) for A, d, marg in small]
        assert [S.wait(t) for t in tk] == [oracle.norm(A, d, marg) for A, d, marg in small]


def test_serve_backpressure():
    say("serve backpressure")
    M = synth.matrix(10, 30, 30, -100, 100, "bp")
    with L.Server(max_inflight_problems=2, max_queued=3, step_ms=1.0) as S:
        codes = [S.submit(M, 1, 0, check=False) for _ in range(12)]
        rcs = [c for c, _ in codes]
        assert L.LD_EBUSY in rcs and L.LD_OK in rcs
        want = L.ld_norm(M, 1, 0)
        for rc, t in codes:
            if rc == L.LD_OK:
                assert S.wait(t) == want
        assert S.stats()["rejected"] == rcs.count(L.LD_EBUSY)


def test_serve_cancel_after_admission():
    """Requests admitted by a bulk step that runs none of their items, cancelled at
    once, while express requests arrive: the cancelled requests keep their slots
    until the admitting step retires (that step still writes their descriptors and
    counters), so no express request is handed such a slot meanwhile.  Every
    express value is the oracle's, and a cancelled request ends either cancelled
    or with the oracle's value."""
    say("serve cancel after admission")
    big = synth.matrix(11, 34, 36, -100, 100, "adm_big")          # items of 2^26 words: ~35 ms each
    mids = [synth.matrix(300 + i, 23, 30, -100, 100, "adm_mid") for i in range(24)]
    smalls = small_mix(6, 60)
    want_small = [oracle.norm(A, d, marg) for A, d, marg in smalls]
    # tiny steps (a few mid requests each), express below 1 us of estimated work (the
    # mid requests, 2^22 words, estimate about 1.9 us and stay bulk; the small ones are
    # express), and items of 2^26 words whatever the request size (no floor on the
    # item count)
    with L.Server(step_ms=0.01, express_ms=0.001, words_per_item=float(1 << 26), min_items=-1) as S:
        t_big = S.submit(big, 1, 0)
        time.sleep(0.005)                       # the first bulk step (one long item) runs
        # more than 16 live bulk requests: a second step is issued behind the first and
        # admits the mid requests queued at that moment (at least 16); it cannot run
        # before the first step's long item ends
        tm = [S.submit(A, 1, 0) for A in mids]
        t0 = time.perf_counter()
        while S.stats()["inflight"] < 17 and time.perf_counter() - t0 < 2.0:
            time.sleep(0.0002)
        time.sleep(0.001)
        admitted = S.stats()["inflight"]
        for t in tm:
            S.cancel(t)
        held = S.stats()["inflight"]
        ts = []
        for i, (A, d, marg) in enumerate(smalls):
            ts.append(S.submit(A, d, marg))
            if i % 10 == 9:
                time.sleep(0.001)
        got = [S.wait(t) for t in ts]
        assert got == want_small
        for A, t in zip(mids, tm):
            rc, v = S.wait(t, check=False)
            assert rc in (L.LD_OK, L.LD_ECANCELED), rc
            if rc == L.LD_OK:
                assert v == oracle.norm(A, 1, 0)
        S.cancel(t_big)
        rc, _ = S.wait(t_big, check=False)
        assert rc in (L.LD_OK, L.LD_ECANCELED)
    # the queued step admitted mid requests, and none was released before it retired
    assert admitted >= 17, admitted
    assert held == admitted, (held, admitted)


def test_serve_timings_split_each_latency():
    """ld_server_timings: one record per completed request, whose plan, wait and run
    parts are non-negative and add up to the latency the statistics report; the
    idle scheduler's polling window (idle_spin_ms) can be switched off."""
    say("serve timings")
    probs = small_mix(5, 40)
    for spin in (0.0, -1.0):
        with L.Server(idle_spin_ms=spin) as S:
            tickets = []
            for i, (M, d, marg) in enumerate(probs):
                tickets.append(S.submit(M, d, marg))
                if i % 7 == 0:
                    time.sleep(0.002)       # some arrive at an idle scheduler
            vals = [S.wait(t) for t in tickets]
            st = S.stats()
            tm = S.timings()
        assert vals == [oracle.norm(M, d, marg) for M, d, marg in probs]
        assert len(tm) == st["completed"] == len(probs)
        assert sorted(t["ticket"] for t in tm) == sorted(tickets)
        for t in tm:
            assert t["plan_ms"] >= 0 and t["wait_ms"] >= 0 and t["run_ms"] >= 0, t
            assert t["lane"] in (0, 1) and t["words"] >= 0, t
        total = np.array([t["plan_ms"] + t["wait_ms"] + t["run_ms"] for t in tm])
        assert abs(float(total.mean()) - st["mean_ms"]) < 1e-6 * max(1.0, st["mean_ms"]) + 1e-9
