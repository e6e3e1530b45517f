"""Writes tests/golden/brute_force.json from the oracle's brute-force
enumeration on seeded instances (calls only oracle/ and the input generators).

    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1807_00699_amd import inputs as I  # noqa: E402


def main():
    out = {"_source": "oracle brute force (Gray-code / odometer enumeration), tests/golden/make_golden.py"}
    J = I.dense_pm1(64, 1)[:20, :20].astype(np.float64)
    e, s = O.brute_ising(J)
    out["ising_pm1_64_seed1_lead20"] = {
        "_note": "leading 20x20 block of the dense +-1 N=64 instance (inputs.dense_pm1(64, 1))",
        "E_min": int(e), "argmin": [int(v) for v in s]}
    for seed in (2, 3, 4):
        J = I.dense_pm1(18, seed).astype(np.float64)
        e, s = O.brute_ising(J)
        out[f"ising_pm1_18_seed{seed}"] = {"E_min": int(e), "argmin": [int(v) for v in s]}
    J = I.dense_uniform(8, 7).astype(np.float64)
    e, k = O.brute_potts(J, 3)
    out["potts3_uniform_8_seed7"] = {"E_min": e, "argmin": [int(v) for v in k]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "brute_force.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
