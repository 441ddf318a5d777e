"""Benchmark: exhaustive Gray-code search for the L1 norm of one 42x42 int32 matrix
(entries uniform in [-100, 100], seed 0; 2^41 sign vectors after the sign symmetry).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]

One step = one complete L1 solve of the 42x42 matrix on the GPU (result reset,
sweep kernel, 8-byte result copy), with the matrix tables already resident in HBM.
Prints one JSON line.  Only one GPU is used; --gpus above 1 is refused.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes x 2.4 GHz, one 32-bit VALU op per lane per clock
INT32_VALU_PEAK = 256 * 64 * 2.4e9
METRIC = "Gray-code steps/s (% INT32 VALU peak); 42×42 L1 secs; batched vs plain solves/s"


def alg_ops_per_word(kind: str, m: int) -> int:
    """Algorithmic int32 VALU work per Gray step of the paper's method (one row update
    and one fused |.|-accumulate per column, plus the running max): 2m + 1 for L1 and
    L_marg, 3m + 1 for L2 (Eq. update, Eq. LM2)."""
    if kind in ("L1", "L_marg"):
        return 2 * m + 1
    if kind == "L2":
        return 3 * m + 1
    raise ValueError(kind)


def scoring_ops_per_word(kind: str, m: int) -> int:
    """The scoring part alone: one |.|-accumulate per column (two for L2) and the max.
    The kernels share one row update among 2^R low-row patterns, so with one column
    per instruction this is the count they cannot go below."""
    if kind in ("L1", "L_marg"):
        return m + 1
    if kind == "L2":
        return 2 * m + 1
    raise ValueError(kind)


KERNEL_SOURCES = ["paper_2503_21596_amd/csrc/ld_sweep.h", "paper_2503_21596_amd/csrc/ld_kernels_bin.hip"]
# the registry lines that shape the headline kernel (its low-row count)
KERNEL_REGISTRY = ("paper_2503_21596_amd/csrc/ld_registry.h", "PACK16_R")
HEADLINE_PROFILE = "profiles/k_bin16s_l1_42x42.md"


def kernel_source_bytes() -> bytes:
    """The headline kernel's sources, and the registry lines that set its shape."""
    reg, key = KERNEL_REGISTRY
    lines = [l for l in open(os.path.join(ROOT, reg), "rb").read().split(b"\n") if key.encode() in l]
    return b"".join(open(os.path.join(ROOT, p), "rb").read() for p in KERNEL_SOURCES) + b"\n".join(lines)


def profile_fields(path: str = HEADLINE_PROFILE, plan: dict | None = None) -> dict:
    """The `key: value` lines of a committed rocprofv3 summary, or {} when the kernel
    sources changed after the profile was taken, or the live plan's sweep shape
    (R, C, P) differs from the profiled one: its counters then describe another
    kernel or another launch."""
    import hashlib
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return {}
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", " ", "#", "-")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256(kernel_source_bytes()).hexdigest()
    if fields.get("kernel_source_sha256_16") != h[:16]:
        return {}
    if plan is not None and fields.get("plan_r_c_p") != "%d %d %d" % (plan["R"], plan["C"], plan["P"]):
        return {}
    return fields


def cpu_baseline(M, target_s: float = 15.0):
    """The oracle (as it stands) on a bounded sample of the same problem: the
    sign vectors whose last q = 20 rows take a few fixed prefix values."""
    import oracle
    threads = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
    n = M.shape[0]
    q = 20
    words_per_prefix = 2 ** (n - 1 - q)
    t0 = time.perf_counter()
    oracle.range_max(M, 1, 0, q, 0, 1, threads)
    t1 = time.perf_counter() - t0
    k = max(1, min(512, int(target_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    oracle.range_max(M, 1, 0, q, 1, 1 + k, threads)
    dt = time.perf_counter() - t0
    return {"value": words_per_prefix * k / dt, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} prefixes x 2^{n - 1 - q} sign vectors of the 42x42 L1 problem "
                      f"(last {q} rows fixed per prefix), {dt:.1f} s, {threads} threads"}


def bench_batch(L, synth, seed: int = 0):
    """The 4096-problem batch: one ld_norm_batch call, a prepared batch replayed from its
    HIP graph, and 4096 separate ld_norm calls; solves/s for each (wall clock)."""
    probs = synth.batch_problems(seed, count=4096)
    t0 = time.perf_counter()
    out = L.ld_norm_batch(probs)
    t_batch = time.perf_counter() - t0
    B = L.Batch(probs)
    B.run()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        rep = B.run()
    t_replay = (time.perf_counter() - t0) / reps
    dev_ms = B.last_ms()
    B.close()
    t0 = time.perf_counter()
    plain = [L.ld_norm(M, d, marg) for M, d, marg in probs]
    t_plain = time.perf_counter() - t0
    n = len(probs)
    return {"problems": n, "batch_solves_per_s": n / t_batch, "replay_solves_per_s": n / t_replay,
            "plain_solves_per_s": n / t_plain, "batch_s": t_batch, "replay_s": t_replay,
            "replay_device_ms": dev_ms, "plain_s": t_plain,
            "speedup_vs_plain": t_plain / t_batch,
            "identical": bool(list(out) == plain and list(rep) == plain)}


def bench_serve(L, synth, seed: int = 0, rate: float = 200.0, seconds: float = 30.0, warm_s: float = 5.0):
    """Poisson request stream into the server (continuous batching) against the same
    trace replayed in real time through sequential plain calls (first come, first
    served, so queueing is included).  The trace lasts warm_s + seconds; latencies
    count the requests that arrive after the first warm_s seconds."""
    import numpy as np
    count = int(round(rate * (seconds + warm_s)))
    reqs = synth.served_requests(seed, count=count, rate=rate)
    warm = sum(1 for t, _, _ in reqs if t < warm_s)
    S = L.Server()
    tickets = []
    t_start = time.perf_counter()
    for t_arr, M, d in reqs:
        delay = t_start + t_arr - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets.append(S.submit(M, d, 0))
    vals = [S.wait(t) for t in tickets]
    t_end = time.perf_counter()
    st = S.stats()
    tm = {t["ticket"]: t for t in S.timings()}
    S.close()
    tm = [tm[t] for t in tickets[warm:]]
    lat = np.array([t["plan_ms"] + t["wait_ms"] + t["run_ms"] for t in tm])
    served = {"requests": count, "warmup_requests": warm, "rate_per_s": rate,
              "solves_per_s": count / (t_end - t_start),
              "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
              "mean_ms": float(lat.mean()), "launches": st["launches"],
              # medians of the latency split (plan: submitting thread; wait: until the first
              # step with the request's items is issued; run: from there to completion)
              "p50_split_ms": {k: float(np.median([t[k] for t in tm])) for k in ("plan_ms", "wait_ms", "run_ms")},
              "express_share": float(np.mean([t["lane"] for t in tm]))}
    # the same trace in real time through sequential plain calls: one thread waits
    # for each arrival (when idle) and serves the requests first come, first served
    durs = []
    seq_vals = []
    lat = []
    t_start = time.perf_counter()
    for t_arr, M, d in reqs:
        delay = t_start + t_arr - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        t0 = time.perf_counter()
        seq_vals.append(L.ld_norm(M, d, 0))
        t1 = time.perf_counter()
        durs.append(t1 - t0)
        lat.append(t1 - (t_start + t_arr))
    t_end = time.perf_counter()
    lat = np.array(lat[warm:]) * 1e3
    seq = {"solves_per_s": count / (t_end - t_start), "p50_ms": float(np.percentile(lat, 50)),
           "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()), "busy_s": float(sum(durs))}
    return {"served": served, "sequential_plain": seq, "identical": vals == seq_vals,
            "offered_load_of_sequential": float(sum(durs)) / reqs[-1][0]}


def bench_serve_burst(L, synth, seed: int = 2, count: int = 1000):
    """Saturation throughput: every request of a trace submitted at once to the
    server (continuous batching) against the same requests as sequential plain
    calls."""
    reqs = synth.served_requests(seed, count=count, rate=200.0)
    L.ld_norm(reqs[0][1], reqs[0][2], 0)
    t0 = time.perf_counter()
    seq_vals = [L.ld_norm(M, d, 0) for _, M, d in reqs]
    t_seq = time.perf_counter() - t0
    with L.Server() as S:
        S.wait(S.submit(reqs[0][1], reqs[0][2], 0))
        t0 = time.perf_counter()
        tickets = [S.submit(M, d, 0) for _, M, d in reqs]
        vals = [S.wait(t) for t in tickets]
        t_srv = time.perf_counter() - t0
        launches = S.stats()["launches"]
    return {"requests": count, "server_solves_per_s": count / t_srv, "sequential_solves_per_s": count / t_seq,
            "speedup": t_seq / t_srv, "launches": launches, "identical": vals == seq_vals}


def bench_small_configs(L, synth, stream):
    """The other workloads: 20x20 L1 (a plain call including host planning and copies,
    median of 20, plus the kernel alone), 16x32 at d = 2, 3, 4 and 24x24 at d = 2
    (kernel time of a prepared solve, words/s)."""
    import numpy as np
    out = {}
    M = synth.config_small_l1(0)
    L.ld_norm(M, 1, 0)
    walls = []
    for _ in range(20):
        t0 = time.perf_counter()
        L.ld_norm(M, 1, 0)
        walls.append(time.perf_counter() - t0)
    h = L.Prepared(M, 1, 0)
    h.run(stream)
    ks = []
    for _ in range(5):
        h.run(stream)
        ks.append(h.kernel_ms())
    out["l1_20x20"] = {"plain_call_ms_median": 1e3 * float(np.median(walls)), "kernel_ms": min(ks),
                       "words": h.plan()["words"]}
    h.close()
    for name, A, d in [("pm16x32_d2", synth.config_pm(0), 2), ("pm16x32_d3", synth.config_pm(0), 3),
                       ("pm16x32_d4", synth.config_pm(0), 4), ("pm24x24_d2", synth.config_pm24(0), 2)]:
        h = L.Prepared(A, d, 0)
        v = h.run(stream)
        ks = []
        for _ in range(3):
            h.run(stream)
            ks.append(h.kernel_ms())
        w = h.plan()["words"]
        out[name] = {"value": v, "kernel_ms": min(ks), "words": w, "words_per_s": w / (min(ks) / 1e3)}
        h.close()
    return out


def bench_mfma_variant(L, synth, stream, default_ms, golden, tuning=""):
    """The headline solve with the int8-MFMA state-update kernel in place of the
    default one (same tables, same value)."""
    L.set_sweep_shape(0, 0, -1, 0, 8, -1)
    try:
        h = L.Prepared(synth.config_42_l1(0), 1, 0)
        kernel = h.plan()["kernel"]
        v = h.run(stream)
        ms = h.kernel_ms()
        h.close()
    finally:
        L.set_sweep_shape(0, 0, -1, 0, 5, -1)
        if tuning:
            L.load_tuning(tuning)
        elif os.path.exists(L.TUNING_PATH) and os.environ.get("LD_TUNING", "1") != "0":
            L.load_tuning(L.TUNING_PATH)
    return {"kernel": kernel, "kernel_ms": ms, "vs_default_kernel": default_ms / ms,
            "value": v, "matches_oracle": (v == golden) if golden is not None else None}


def bench_low_rows(L, synth, stream, reps: int = 3):
    """Kernel time of plain L1 solves of 36 .. 42 rows with five and with six low
    rows scored per state (a tuning table whose plain_big_r_c is 0: never six, or 1:
    six wherever a mid row is left), the measurement behind the mid-row count at
    which plain calls switch to six."""
    import tempfile
    tuned = os.path.exists(L.TUNING_PATH) and os.environ.get("LD_TUNING", "1") != "0"
    base = json.load(open(L.TUNING_PATH)) if tuned else {}
    base.pop("measured", None)
    out = {}
    try:
        for n in (36, 38, 39, 40, 41, 42):
            M = synth.config_42_l1(0) if n == 42 else synth.matrix(91 + 2 * n, n, n, -100, 100, "prof")
            row, vals = {}, set()
            for c in (0, 1):
                with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as f:
                    json.dump(dict(base, plain_big_r_c=c), f)
                L.load_tuning(f.name)
                os.unlink(f.name)
                h = L.Prepared(M, 1, 0)
                vals.add(h.run(stream))
                ks = []
                for _ in range(reps):
                    vals.add(h.run(stream))
                    ks.append(h.kernel_ms())
                p = h.plan()
                h.close()
                row["R%d" % p["R"]] = {"C": p["C"], "P": p["P"], "ms": min(ks)}
            if len(vals) != 1:
                raise RuntimeError("values differ between low-row counts: %s" % sorted(vals))
            row["mid_rows_at_five"] = row["R5"]["C"]
            row["six_over_five"] = row["R6"]["ms"] / row["R5"]["ms"]
            out["L1_%dx%d" % (n, n)] = row
            print("low rows", n, json.dumps(row), file=sys.stderr, flush=True)
    finally:
        if tuned:
            L.load_tuning(L.TUNING_PATH)
    return out


def bench_sweep(L, synth, stream, reps: int = 3):
    """Kernel time of one solve against the number of lanes (prefixes, one per lane)
    and the resident waves per SIMD, for L1, L2, L_3 and L_4: the launch-shape
    question of the paper's Sec. 4 (Fig. 3), where the best total thread count
    followed no general rule.  Lanes: binary 2^P for P = 12 .. 22 (ld_set_sweep_shape
    p_target); d-ary the plan's lane count for lane targets 2^12 .. 2^20 (a tuning
    table carrying plain_dary_lanes).  Waves per SIMD 1 .. 8 at the tuned lane count
    (ld_set_launch_waves; the kernel's occupancy caps the count)."""
    import tempfile
    workloads = [("L1_36x36", 1, 36, 36), ("L2_31x31", 2, 31, 31), ("L3_22x32", 3, 22, 32), ("L4_18x24", 4, 18, 24)]
    tuned = os.path.exists(L.TUNING_PATH) and os.environ.get("LD_TUNING", "1") != "0"

    def dary_lanes(n):
        with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as f:
            f.write('{"plain_dary_lanes": %d}' % n)
        L.load_tuning(f.name)
        os.unlink(f.name)

    def restore():
        L.set_launch_waves(0)
        L.set_sweep_shape(20, 0, -1, 0, -1, -1)
        if tuned:
            L.load_tuning(L.TUNING_PATH)
        else:
            dary_lanes(1 << 19)   # the compiled default

    def timed(M, d):
        h = L.Prepared(M, d, 0)
        v = h.run(stream)
        ks = []
        for _ in range(reps):
            h.run(stream)
            ks.append(h.kernel_ms())
        p = h.plan()
        h.close()
        return {"lanes": p["n_prefix"], "C": p["C"], "R": p["R"], "kernel": p["kernel"], "ms": min(ks),
                "words_per_s": p["words"] / (min(ks) / 1e3), "value": v}

    out = {}
    for name, d, n, m in workloads:
        M = synth.matrix(500 + n + m + d, n, m, -100, 100, "sweep")
        rows = []
        try:
            for k in range(12, 23 if d <= 2 else 21):
                if d <= 2:
                    L.set_sweep_shape(k, 0, -1, 0, -1, -1)
                else:
                    dary_lanes(1 << k)
                r = timed(M, d)
                r["target"] = k
                rows.append(r)
        finally:
            restore()
        waves = []
        try:
            for w in range(1, 9):
                L.set_launch_waves(w)
                r = timed(M, d)
                r["waves_per_simd"] = w
                waves.append(r)
        finally:
            restore()
        ref = timed(M, d)
        assert all(r["value"] == ref["value"] for r in rows + waves), name
        best = min(rows, key=lambda r: r["ms"])
        out[name] = {"lanes": rows, "waves": waves, "tuned": ref, "best_lanes": best["lanes"],
                     "best_is_power_of_d": best["lanes"] & (best["lanes"] - 1) == 0 if d <= 2
                     else _is_power(best["lanes"], d)}
        print(f"sweep {name}: best {best['lanes']} lanes {best['ms']:.3f} ms, tuned {ref['lanes']} lanes "
              f"{ref['ms']:.3f} ms", file=sys.stderr, flush=True)
    return out


def _is_power(x: int, b: int) -> bool:
    while x > 1 and x % b == 0:
        x //= b
    return x == 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tuning", default="", help="load this autotuner table before measuring")
    ap.add_argument("--kernel-variant", type=int, default=-1,
                    help="sweep kernel variant: 16 (packed 16-bit, binary and d-ary), 5 or 4 (binary, SGPR "
                         "operands, that many low rows), 1 (d-ary, SGPR operands), 0 (VGPR operands), "
                         "8 (binary, int8-MFMA state update); default: tuned")
    ap.add_argument("--solve", default="",
                    help="D,N,M: instead of the benchmark, time one solve of L_D on a seeded N x M matrix "
                         "(entries U[-100,100]) and print its plan and kernel time (for profiling)")
    ap.add_argument("--small", action="store_true",
                    help="instead of the benchmark, run only the smaller workloads (20x20 L1, 16x32 at d = 2, "
                         "3, 4, 24x24 L2) and print their timings as one JSON line (for profiling)")
    ap.add_argument("--serve", type=float, default=0.0,
                    help="only the served trace at this rate (requests/s): server against sequential calls "
                         "(for profiling)")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark, time one solve each of L1, L2, L_3 and L_4 across lane "
                         "counts and waves per SIMD and print the table as one JSON line")
    ap.add_argument("--low-rows", action="store_true",
                    help="instead of the benchmark, time plain L1 solves of 36 .. 42 rows with five and "
                         "with six low rows per state and print the table as one JSON line")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB on the GPU (a kernel of "
                         "known traffic, to scale the HBM counters of a profiler run)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the prefix space would shard across GPUs with one int64 max per problem)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2503_21596_amd as L
    import synth

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if a.tuning:
        L.load_tuning(a.tuning)
    if a.kernel_variant >= 0:
        kv = a.kernel_variant
        L.set_sweep_shape(0, 0, -1, 0, kv if kv in (0, 4, 5, 8, 16) else -1, kv if kv in (0, 1, 16) else -1)
    if a.sweep:
        print(json.dumps({"sweep": bench_sweep(L, synth, stream)}), flush=True)
        return
    if a.low_rows:
        print(json.dumps({"low_rows": bench_low_rows(L, synth, stream)}), flush=True)
        return
    if a.small:
        print(json.dumps({"other_configs": bench_small_configs(L, synth, stream)}), flush=True)
        return
    if a.serve > 0:
        warm = min(5.0, a.serve_seconds / 6)
        print(json.dumps({"served": bench_serve(L, synth, seed=0 if a.serve == 200.0 else 1, rate=a.serve,
                                                seconds=a.serve_seconds, warm_s=warm)}), flush=True)
        return
    if a.solve:
        d, n, m = (int(x) for x in a.solve.split(","))
        Ms = synth.matrix(91 + n + m, n, m, -100, 100, "prof")
        hs = L.Prepared(Ms, d, 0)
        value = [hs.run(stream) for _ in range(2)][-1]
        plan = hs.plan()
        print(json.dumps({"solve": {"d": d, "n": n, "m": m, "value": value, "kernel_ms": hs.kernel_ms(),
                                    "plan": {k: plan[k] for k in ("kernel", "mp", "R", "C", "P", "P_tab",
                                                                  "n_prefix", "words")}}}), flush=True)
        hs.close()
        return
    M = synth.config_42_l1(0)
    h = L.Prepared(M, 1, 0)
    plan = h.plan()
    words = plan["words"]

    for _ in range(a.warmup):
        h.run(stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    kernel_ms = []
    value = None
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(a.steps):
        value = h.run(stream)
        kernel_ms.append(h.kernel_ms())
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / a.steps
    steps_per_s = words * a.steps / (total_ms / 1e3)
    kavg = sum(kernel_ms) / len(kernel_ms)
    ops = alg_ops_per_word("L1", plan["m"])
    sops = scoring_ops_per_word("L1", plan["m"])
    achieved = words * ops / (kavg / 1e3)
    # engine clock under a VALU-bound load, and the issue rate the chip sustains
    probe = L.valu_probe(200.0)
    prof = profile_fields(plan=plan)
    valu_issue = None
    # the kernel's own clock from the profile (busy cycles per shader engine over its
    # time), else the probe's clock under its VALU load
    sclk = float(prof.get("sclk_from_busy_cycles_hz", 0) or probe["sclk_hz"])
    if prof.get("valu_insts_per_launch") and sclk > 0:
        # wave-level VALU instructions of the profiled launch against the issue
        # capacity of this launch (one wave64 instruction per SIMD per 4 clocks,
        # 4 SIMDs per CU) at that clock
        valu_issue = float(prof["valu_insts_per_launch"]) / (kavg / 1e3 * probe["compute_units"] * sclk)
    packed = plan["kernel"] == 5
    note = ("frac counts the paper's per-step work, 2m + 1 int32 ops (row update, one |.|-accumulate per "
            "column, max); it exceeds 1 because the kernel shares one row update among 2^R = %d low-row "
            "patterns%s. valu_issue_frac (profiled instruction count over issue capacity at the measured "
            "clock) is the hardware utilisation." %
            (1 << plan["R"], " and scores two columns per v_sad_u16 (16-bit halves)" if packed else ""))

    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "configs_seed0.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath)).get("values", {}).get("l1_42")

    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "L1 (local bound) of one 42x42 int32 matrix, entries U[-100,100], seed 0; "
                               "2^41 Gray-code steps per solve",
                   "n": 42, "m": 42, "d": 1, "marginals": 0,
                   "plan": {k: plan[k] for k in ("mp", "R", "C", "P", "n_prefix", "i64", "kernel")}},
        "l1_42_seconds": ms_per_step / 1e3,
        "pct_int32_valu_peak": 100.0 * achieved / INT32_VALU_PEAK,
        "pct_int32_valu_issue": 100.0 * valu_issue if valu_issue else None,
        "result": value,
        "matches_oracle": (value == golden) if golden is not None else None,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_VALU_PEAK / 1e12,
                     "unit": "Tops/s (int32 VALU)", "frac": achieved / INT32_VALU_PEAK,
                     "traffic": float(prof["traffic_bytes"]) if "traffic_bytes" in prof else None,
                     "ops_per_step": ops, "note": note,
                     "scoring_ops_per_step": sops,
                     "frac_scoring_only": words * sops / (kavg / 1e3) / INT32_VALU_PEAK,
                     # lane-level: each wave64 instruction serves 64 lanes, one word each
                     "valu_insts_per_step": (64.0 * float(prof["valu_insts_per_launch"]) / words
                                             if prof.get("valu_insts_per_launch") else None),
                     "valu_issue_frac": valu_issue,
                     "sclk_kernel_hz": sclk, "sclk_probe_hz": probe["sclk_hz"],
                     "sclk_rated_hz": probe["sclk_max_hz"],
                     "peak_at_measured_clock": probe["compute_units"] * 64 * sclk / 1e12,
                     "probe_valu_frac": probe["valu_lane_ops_per_s"] / INT32_VALU_PEAK,
                     "kernel_ms": kavg, "profile": HEADLINE_PROFILE if prof else None},
        "wall_s": wall,
    }

    if not a.no_extras:
        print("bench: matrix-core variant", file=sys.stderr, flush=True)
        out["mfma_variant_42"] = bench_mfma_variant(L, synth, stream, kavg, golden, a.tuning)
        print("bench: batch", file=sys.stderr, flush=True)
        out["batched_vs_plain"] = bench_batch(L, synth)
        print("bench: serve", file=sys.stderr, flush=True)
        out["served"] = bench_serve(L, synth)
        out["served_600"] = bench_serve(L, synth, seed=1, rate=600.0, seconds=10.0, warm_s=2.0)
        out["served_burst"] = bench_serve_burst(L, synth)
        Mm = synth.config_42_marg(0)
        hm = L.Prepared(Mm, 1, 1)
        vm = hm.run(stream)
        gm = json.load(open(gpath)).get("values", {}).get("marg_42") if os.path.exists(gpath) else None
        out["marg_42"] = {"value": vm, "seconds": hm.kernel_ms() / 1e3,
                          "steps_per_s": hm.plan()["words"] / (hm.kernel_ms() / 1e3),
                          "matches_oracle": (vm == gm) if gm is not None else None}
        hm.close()
        print("bench: small configs", file=sys.stderr, flush=True)
        out["other_configs"] = bench_small_configs(L, synth, stream)
        print("bench: argmax", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        va, av, bv = L.ld_argmax(M, 1, 0)
        ta = time.perf_counter() - t0
        attained = int(av.astype(np.int64) @ M.astype(np.int64) @ bv.astype(np.int64))
        out["argmax_42"] = {"seconds": ta, "value": va, "attained": attained == va,
                            "vs_value_pass": ta / (ms_per_step / 1e3)}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(M)
    h.close()
    if a.calib_copy_mib:
        nbytes = a.calib_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = nbytes
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
