"""Writes tests/golden/square4x6_r2.json: the FP64 oracle's Lanczos
coefficients for the first two samples (r = 0, 1) of every S^z >= 0 sector
of the periodic 6x4 J1-J2 square lattice (N = 24, J1 = 1, J2 = 0.5, 96 bonds),
+-1 start vectors, seed 3, M = 80 steps, and the resulting E(T), C(T),
chi(T) (g = 1, multiplicity-weighted).

Calls only oracle/ (and the input definitions in ftlm_inputs/); ~30 minutes
on 8 cores:
    python tests/golden/make_square4x6_r2.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from ftlm_inputs import graphs  # noqa: E402

N, SEED, M, R = 24, 3, 80, 2


def main():
    bonds = graphs.square_j1j2(6, 4, 1.0, 0.5)
    t0 = time.time()
    recs, sectors = [], []
    for n_up in range(N // 2, N + 1):
        rec, raw = oracle.ftlm_sector(N, n_up, bonds, R, M, SEED, oracle.PM1)
        recs.append(rec)
        sectors.append({"n_up": n_up, "dim": rec["dim"],
                        "samples": [{"r": r, "alpha": a.tolist(), "beta": b.tolist(), "steps": int(k)}
                                    for r, (a, b, k) in enumerate(raw)]})
        print(f"n_up {n_up}: D = {rec['dim']}, {time.time() - t0:.0f} s", flush=True)
    temps = oracle.log_temperatures()
    th = oracle.thermo(recs, temps, N, 1.0)
    out = {"about": "FP64 oracle reference, 6x4 J1-J2 lattice, all S^z >= 0 sectors, +-1 seed 3, r=0,1, M=80",
           "n_sites": N, "seed": SEED, "M": M, "dist": "pm1", "bonds": [[i, j, J] for i, j, J in bonds],
           "sectors": sectors, "temps": temps.tolist(),
           "E": th["E"].tolist(), "C": th["C"].tolist(), "chi": th["chi"].tolist()}
    with open(os.path.join(HERE, "square4x6_r2.json"), "w") as f:
        json.dump(out, f)
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
