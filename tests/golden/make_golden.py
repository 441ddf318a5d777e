"""Write the oracle's values for the benchmark configurations (seed 0) to
tests/golden/configs_seed0.json.  Calls only oracle/ and synth/.

    python tests/golden/make_golden.py [--threads N] [--only KEY ...]

Keys:
  pm16x32_d2, pm16x32_d3, pm16x32_d4   16x32, entries U[-50,50], Eq. (L_o_norm)
  pm24x24_d2                           24x24, entries U[-50,50], Eq. (L_o_norm), d = 2
  l1_42                                42x42, entries U[-100,100], Eq. (LM2) (split-table form)
  marg_42                              42x42 with marginal row/column, Eq. (LMarg) (split-table form)
The 42x42 values take about an hour each on 8 cores; the file is rewritten after
every value so a run can be resumed with --only.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*", default=None)
    a = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {
        "note": "values of the CPU oracle (oracle/) on the seeded inputs of synth/ (seed 0); "
                "written by tests/golden/make_golden.py",
        "values": {}, "seconds": {}}
    for key in (a.only or list(JOBS)):
        t0 = time.time()
        v = JOBS[key](a.threads)
        data["values"][key] = v
        data["seconds"][key] = round(time.time() - t0, 1)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        print(key, v, data["seconds"][key], flush=True)


if __name__ == "__main__":
    main()
