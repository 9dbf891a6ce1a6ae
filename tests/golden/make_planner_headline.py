"""Write planner_headline.json: the oracle planner (Sect. 3.4: eq. 5 search range, K(P)
on the planning subset, GPU form of eq. 9, eq. 10, Fig. 2 decision tree) on the
benchmark's inputs -- 4096^2 over 3 degrees, 50M rows of the 64-antenna array over 16 h
at 1.28 GHz, 288 GB, budget fraction 0.65, FP16 storage.  Calls only oracle/ and the
seeded input generators; run from the repository root:
    python tests/golden/make_planner_headline.py
"""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import wfsynth as ws  # noqa: E402
from oracle import planner  # noqa: E402
from oracle.operator import C_LIGHT  # noqa: E402


def main():
    obs = ws.precision_form(sky=False)
    w = obs.uvw_m[:, 2] * (obs.freqs_hz[0] / C_LIGHT)
    out = planner.plan(w, obs.nx, obs.ny, obs.cell_rad, 288e9, store="f16")
    rec = {
        "inputs": "precision form: 4096^2, 3 deg, 50M rows, 1.28 GHz, 288 GB, f16",
        "P": out["P"], "P_star": out["P_star"],
        "P_wsclean": out["P_wsclean"], "P_wsclean_ceil": int(math.ceil(out["P_wsclean"])),
        "strategy": out["strategy"],
        "K_at_P": [r[1] for r in out["table"] if r[0] == out["P"]][0],
        "mem_at_P": [r[3] for r in out["table"] if r[0] == out["P"]][0],
        "cost_at_P": [r[4] for r in out["table"] if r[0] == out["P"]][0],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "planner_headline.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(rec)


if __name__ == "__main__":
    main()
