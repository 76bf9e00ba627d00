"""Writes tests/golden/c3_oracle.json: the oracle's results for the instances of
the 256-instance mixed batch (l in {2,3}, constraint degree 4..10, 50..1000
constraints) that it solves in seconds: every 2-variable instance and the
3-variable instances of at most 15,099 words per item.  Calls only the oracle."""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ref  # noqa: E402
from paper_2003_01758_amd.instances import make_instance  # noqa: E402

BATCH = 256
MAX_W_L3 = 15099


def selected():
    out = []
    for k in range(BATCH):
        inst = make_instance(3, k)
        if inst.l == 2 or inst.words_per_item() <= MAX_W_L3:
            out.append((k, inst))
    return out


def main():
    rows = {}
    t0 = time.time()
    for k, inst in selected():
        s = ref.RefSolver(inst)
        out = s.solve()
        r = s.result()
        rows[str(k)] = {"outcome": int(out), "p_up": r["p_up"], "p_lo": r["p_lo"],
                        "steps": int(r["steps"]), "peak_len": int(r["peak_len"]),
                        "x_index": [int(v) for v in r["x_index"][:inst.l]],
                        "x_depth": [int(v) for v in r["x_depth"][:inst.l]]}
        print(k, rows[str(k)]["outcome"], f"{time.time() - t0:.1f}s", flush=True)
    with open(os.path.join(HERE, "c3_oracle.json"), "w") as f:
        json.dump({"instances": "make_instance(3, k), k < 256: every l = 2 instance and l = 3 with "
                                f"at most {MAX_W_L3} words per item",
                   "writer": "tests/golden/make_c3_oracle.py (oracle only)", "results": rows}, f, indent=0)


if __name__ == "__main__":
    main()
