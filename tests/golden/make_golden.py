"""Write the oracle's values for the benchmark configurations (seed 0) to
tests/golden/configs_seed0.json.  Calls only oracle/ and synth/.

    python tests/golden/make_golden.py [--threads N] [--only KEY ...]

Keys:
  pm16x32_d2, pm16x32_d3, pm16x32_d4   16x32, entries U[-50,50], Eq. (L_o_norm)
  pm24x24_d2                           24x24, entries U[-50,50], Eq. (L_o_norm), d = 2
  l1_42                                42x42, entries U[-100,100], Eq. (LM2) (split-table form)
  marg_42                              42x42 with marginal row/column, Eq. (LMarg) (split-table form)
  batch_<i>                            member i of synth.batch_problems(0), 4096 problems:
                                       one per (d, marginals, n) stratum among the largest
                                       (d <= 2 with n = 25..28, d = 3 with n = 17..20), the
                                       widest member of each (split-table forms)
  serve_<i>                            request i of synth.served_requests(0, 2000, 200):
                                       the largest L1, L2 (34x48) and L_3 (20x48) requests
The 42x42 values take about an hour each on 8 cores, the others about two minutes
together; the file is rewritten after every value so a run can be resumed with --only.
The "members" map names where each batch_ / serve_ input comes from.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "configs_seed0.json")

JOBS = {
    "pm16x32_d2": lambda t: oracle.ld(synth.config_pm(0), 2, t),
    "pm16x32_d3": lambda t: oracle.ld(synth.config_pm(0), 3, t),
    "pm16x32_d4": lambda t: oracle.ld(synth.config_pm(0), 4, t),
    "pm24x24_d2": lambda t: oracle.ld(synth.config_pm24(0), 2, t),
    "l1_42": lambda t: oracle.l1_split(synth.config_42_l1(0), 0, t),
    "marg_42": lambda t: oracle.l1_split(synth.config_42_marg(0), 1, t),
}


BATCH_STRATA = [(1, 0, n) for n in range(25, 29)] + [(1, 1, n) for n in range(25, 29)] + \
               [(2, 0, n) for n in range(25, 29)] + [(3, 0, n) for n in range(17, 21)]
SERVE_COUNT, SERVE_RATE = 2000, 200.0


def batch_members():
    """{key: (index, M, d, marginals)}: the widest batch member of every stratum."""
    probs = synth.batch_problems(0, 4096)
    best = {}
    for i, (M, d, marg) in enumerate(probs):
        k = (d, marg, M.shape[0])
        if k in BATCH_STRATA and (k not in best or M.shape[1] > probs[best[k]][0].shape[1]):
            best[k] = i
    return {f"batch_{i}": (i,) + tuple(probs[i]) for i in sorted(best.values())}


def serve_members():
    """{key: (index, M, d, 0)}: the largest served L1 and L2 request (rows x columns)
    and the widest L_3 request with the most rows."""
    reqs = synth.served_requests(0, SERVE_COUNT, SERVE_RATE)
    out = {}
    for d in (1, 2, 3):
        cand = [(M.shape[0] * 100 + M.shape[1], i) for i, (_, M, dd) in enumerate(reqs) if dd == d]
        i = max(cand)[1]
        out[f"serve_{i}"] = (i, reqs[i][1], d, 0)
    return out


def member_jobs():
    jobs, info = {}, {}
    for src, members in (("synth.batch_problems(0, 4096)", batch_members()),
                         (f"synth.served_requests(0, {SERVE_COUNT}, {SERVE_RATE})", serve_members())):
        for key, (i, M, d, marg) in members.items():
            jobs[key] = (lambda M, d, marg: lambda t: oracle.norm_split(M, d, marg, t))(M, d, marg)
            info[key] = {"source": src, "index": i, "n": int(M.shape[0]), "m": int(M.shape[1]),
                         "d": int(d), "marginals": int(marg)}
    return jobs, info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*", default=None)
    a = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {
        "note": "values of the CPU oracle (oracle/) on the seeded inputs of synth/ (seed 0); "
                "written by tests/golden/make_golden.py",
        "values": {}, "seconds": {}}
    jobs, info = member_jobs()
    jobs.update(JOBS)
    data.setdefault("members", {}).update(info)
    for key in (a.only or list(jobs)):
        t0 = time.time()
        v = jobs[key](a.threads)
        data["values"][key] = v
        data["seconds"][key] = round(time.time() - t0, 1)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        print(key, v, data["seconds"][key], flush=True)


if __name__ == "__main__":
    main()
