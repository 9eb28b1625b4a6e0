"""Writes tests/golden/icosahedron_s1.json: the FP64 oracle's FTLM of the
spin-1 Heisenberg icosahedron (N = 12, 30 bonds, J = 1; the s = 1 system of
Table 1 and Table 3) over every sector with M >= 0 (digit sums A = 12 .. 24),
R = 4 +-1 start vectors with seed 7 per sector, M = 40 Lanczos steps:
per sector the Lanczos coefficients of every sample, and E(T), C(T), chi(T)
(g = 1, multiplicity-weighted) on the 200-point grid T in [0.05, 10];
and sigma_emp (Eq. 22) of each observable over 10 further seeds
(1000 .. 1009) at the same R and M, the scale of the stochastic error.

Calls only oracle/ (and the input definitions in ftlm_inputs/); a few
minutes on 8 cores:
    python tests/golden/make_icosahedron_s1.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import spin as sp  # noqa: E402
from ftlm_inputs import graphs  # noqa: E402

N, TWO_S, SEED, R, M = 12, 2, 7, 4, 40
SPREAD_SEEDS = list(range(1000, 1010))


def main():
    bonds = graphs.icosahedron()
    t0 = time.time()
    recs, sectors = [], []
    for a in range(N * TWO_S // 2, N * TWO_S + 1):
        rec, raw = sp.ftlm_sector(N, TWO_S, a, bonds, R, M, SEED, oracle.PM1)
        recs.append(rec)
        sectors.append({"a": a, "dim": rec["dim"],
                        "samples": [{"r": r, "alpha": al.tolist(), "beta": be.tolist(), "steps": int(k)}
                                    for r, (al, be, k) in enumerate(raw)]})
        print(f"A {a}: D = {rec['dim']}, {time.time() - t0:.0f} s", flush=True)
    temps = oracle.log_temperatures()
    th = sp.thermo(recs, temps, N, TWO_S)
    bases = {s["a"]: sp.basis(N, TWO_S, s["a"]) for s in sectors}
    runs = {k: [] for k in ("E", "C", "chi")}
    for seed in SPREAD_SEEDS:
        rs = [sp.ftlm_sector(N, TWO_S, s["a"], bonds, R, M, seed, oracle.PM1, bases[s["a"]])[0] for s in sectors]
        ts = sp.thermo(rs, temps, N, TWO_S)
        for k in runs:
            runs[k].append(ts[k])
    sigma = {k: oracle.seed_spread(runs[k])[1].tolist() for k in runs}
    out = {"about": "FP64 oracle FTLM, spin-1 icosahedron, all M >= 0 sectors, +-1 seed 7, R=4, M=40",
           "n_sites": N, "two_s": TWO_S, "seed": SEED, "R": R, "M": M, "dist": "pm1",
           "bonds": [[i, j, J] for i, j, J in bonds], "sectors": sectors, "temps": temps.tolist(),
           "E": th["E"].tolist(), "C": th["C"].tolist(), "chi": th["chi"].tolist(),
           "spread_seeds": SPREAD_SEEDS, "sigma": sigma}
    with open(os.path.join(HERE, "icosahedron_s1.json"), "w") as f:
        json.dump(out, f)
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
