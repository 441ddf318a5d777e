"""Write tests/golden/batch_seed0.json: the oracle's value of every problem of the
4096-problem batch workload (synth.batch_problems(0, 4096)), computed by oracle/
only (the split-table forms of Eqs. (LM2), (LMarg), (L_o_norm)).

    python tests/golden/make_batch_golden.py [--threads T]

About 15 minutes on 8 cores.  The file is rewritten every 256 problems, and a run
resumes from the values already there.
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

OUT = os.path.join(HERE, "batch_seed0.json")
COUNT = 4096


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    probs = synth.batch_problems(0, COUNT)
    data = json.load(open(OUT)) if os.path.exists(OUT) else {
        "note": "oracle values of every problem of synth.batch_problems(0, 4096), in order; "
                "written by tests/golden/make_batch_golden.py (oracle/ only)",
        "count": COUNT, "values": [], "seconds": 0.0}
    values = data["values"]
    t0 = time.time()
    for i in range(len(values), COUNT):
        M, d, marg = probs[i]
        values.append(int(oracle.norm_split(M, d, marg, a.threads)))
        if (i + 1) % 256 == 0 or i + 1 == COUNT:
            data["seconds"] = round(data["seconds"] + time.time() - t0, 1)
            t0 = time.time()
            json.dump(data, open(OUT, "w"), indent=0)
            print(i + 1, "problems", data["seconds"], "s", flush=True)


if __name__ == "__main__":
    main()
