"""Writes tests/golden/ring18_r8.json: the FP64 oracle's FTLM over every
S^z >= 0 sector of the J1-J2 ring N = 18 (J1 = 1, J2 = 0.3, 36 bonds), +-1
start vectors, seed 21, R = 8 samples per sector, M = 60 steps: E(T), C(T),
chi(T) (g = 1, multiplicity-weighted) on the 200-point grid T in [0.05, 10],
and the lowest Ritz value per sector.

Calls only oracle/ (and the input definitions in ftlm_inputs/); a few
minutes on 8 cores:
    python tests/golden/make_ring18_r8.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from ftlm_inputs import graphs  # noqa: E402

N, SEED, M, R, J2 = 18, 21, 60, 8, 0.3


def main():
    bonds = graphs.j1j2_ring(N, 1.0, J2)
    t0 = time.time()
    temps = oracle.log_temperatures()
    th, recs = oracle.ftlm(N, bonds, list(range(N // 2, N + 1)), R, M, SEED, oracle.PM1, temps)
    out = {"about": "FP64 oracle FTLM, J1-J2 ring N=18 (J2=0.3), all S^z >= 0 sectors, +-1 seed 21, R=8, M=60",
           "n_sites": N, "seed": SEED, "R": R, "M": M, "dist": "pm1", "j2": J2,
           "n_ups": list(range(N // 2, N + 1)), "temps": temps.tolist(),
           "E": th["E"].tolist(), "C": th["C"].tolist(), "chi": th["chi"].tolist(),
           "e_min": [float(min(np.min(t) for t, _ in r["samples"])) for r in recs]}
    with open(os.path.join(HERE, "ring18_r8.json"), "w") as f:
        json.dump(out, f)
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
