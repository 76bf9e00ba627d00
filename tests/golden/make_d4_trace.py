"""Writes tests/golden/d4_trace.json: the oracle's per-step list length and
least lower bound for the 4-D workload (100 inequalities, 2 equalities,
M = 2^16) over its first 33 steps.  Calls only the oracle."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ref  # noqa: E402
from paper_2003_01758_amd.instances import make_instance, truncate  # noqa: E402

STEPS = 33


def main():
    inst = truncate(make_instance(2, 0), 100).with_options(max_boxes=1 << 16)
    s = ref.RefSolver(inst)
    rows = []
    for _ in range(STEPS):
        out = s.step()
        r = s.result()
        rows.append({"k": int(r["list_len"]), "p_lo": r["p_lo"], "p_up": r["p_up"],
                     "outcome": int(out)})
        if out != ref.RUNNING:
            break
    with open(os.path.join(HERE, "d4_trace.json"), "w") as f:
        json.dump({"instance": "make_instance(2, 0) truncated to 100 inequalities, max_boxes 2^16",
                   "writer": "tests/golden/make_d4_trace.py (oracle only)", "steps": rows}, f, indent=1)


if __name__ == "__main__":
    main()
