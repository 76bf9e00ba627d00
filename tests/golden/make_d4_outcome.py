"""Writes tests/golden/d4_outcome.json: the oracle's run of the full 4-D
workload (4 variables, 100 inequalities and 2 equalities of multi-degree
(4,4,4,4) and (2,2,2,2)) to an outcome at a memory bound M that the oracle
reaches in about a minute: per step the list length, p_up and p_lo, then the
outcome, step count and peak list length.  Calls only the oracle."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ref  # noqa: E402
from paper_2003_01758_amd.instances import make_instance  # noqa: E402

M = 1 << 13
INDICES = (0, 1)


def run(k):
    inst = make_instance(2, k).with_options(max_boxes=M)
    s = ref.RefSolver(inst)
    rows = []
    while True:
        out = s.step()
        r = s.result()
        # a pass that ends at the memory test subdivides nothing: no record
        if r["steps"] > len(rows):
            rows.append({"k": int(r["list_len"]), "p_lo": r["p_lo"], "p_up": r["p_up"]})
        if out != ref.RUNNING:
            break
    r = s.result()
    return {"outcome": int(r["outcome"]), "steps": int(r["steps"]), "peak_len": int(r["peak_len"]),
            "p_up": r["p_up"], "p_lo": r["p_lo"], "has_x": bool(r["has_x"]),
            "x_index": [int(v) for v in r["x_index"]], "trace": rows}


def main():
    out = {"instance": "make_instance(2, k) at full size, max_boxes 2^13", "max_boxes": M,
           "writer": "tests/golden/make_d4_outcome.py (oracle only)",
           "runs": {str(k): run(k) for k in INDICES}}
    with open(os.path.join(HERE, "d4_outcome.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
