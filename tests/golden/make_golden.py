"""Writes oracle_single_8kev.json: a regression record of the FP64 oracle on
the single 8 keV photon workload (2222 holes, seed 0).

It calls only the oracle and the seeded input generators; rerun it only
when a change of the oracle's arithmetic is justified by the paper, and
name that passage in the commit.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads import single_8kev  # noqa: E402


def main():
    oracle.build(force=False)
    s, b = single_8kev(seed=0)
    r = oracle.run(s, b)
    xyz = r["xyz"]
    rec = {
        "_source": "FP64 oracle (Sec. 2.1, Algorithm 1) on one 8 keV photon: 2222 holes, "
                   "sigma 1 um at z = 50 um, 320 um sensor, 150 V, V_dep 60 V, 293 K, dt 0.05 ns, "
                   "softening 0.01 um, Philox seed 0, event id 0",
        "status": r["status"],
        "steps": int(r["steps"][0]),
        "pairs": r["pairs"],
        "pix": r["pix"][0].tolist(),
        "cstep_hist": np.bincount(r["cstep"]).tolist(),
        "end_mean": xyz.mean(axis=0).tolist(),
        "end_std": xyz.std(axis=0).tolist(),
        "end_first": xyz[:8].tolist(),
    }
    with open(os.path.join(HERE, "oracle_single_8kev.json"), "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
