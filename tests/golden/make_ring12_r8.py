"""Writes tests/golden/ring12_r8.json: the FP64 oracle's FTLM of the
antiferromagnetic Heisenberg ring N = 12 (J = 1, 12 bonds), S^z = 0 sector
(D = 924), R = 8 +-1 start vectors with seed 1, M = 40 Lanczos steps:
E(T), C(T) on the 200-point grid T in [0.05, 10] (the sector alone, g = 1).

Calls only oracle/ (and the input definitions in ftlm_inputs/); seconds:
    python tests/golden/make_ring12_r8.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from ftlm_inputs import graphs  # noqa: E402

N, N_UP, SEED, R, M = 12, 6, 1, 8, 40


def main():
    temps = oracle.log_temperatures()
    th, recs = oracle.ftlm(N, graphs.ring(N), [N_UP], R, M, SEED, oracle.PM1, temps)
    out = {"about": "FP64 oracle FTLM, Heisenberg ring N=12 S^z=0, +-1 seed 1, R=8, M=40",
           "n_sites": N, "n_up": N_UP, "seed": SEED, "R": R, "M": M, "dist": "pm1",
           "temps": temps.tolist(), "E": th["E"].tolist(), "C": th["C"].tolist()}
    with open(os.path.join(HERE, "ring12_r8.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
