"""Writes tests/golden/icosidodecahedron_r2.json: the FP64 oracle's Lanczos
coefficients for the first two samples (r = 0, 1) of the icosidodecahedron
workload (N = 30, 60 bonds, J = 1, S^z = 0, Gaussian start vectors, seed 2,
M = 100 steps) and the resulting single-sector E(T), C(T).

Calls only oracle/ (and the input definitions in ftlm_inputs/). Needs about
6 GB of memory and ~30-60 minutes on 8 cores:
    python tests/golden/make_icosidodecahedron_r2.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from ftlm_inputs import graphs  # noqa: E402

N, N_UP, SEED, M, R = 30, 15, 2, 100, 2


def main():
    bonds = graphs.icosidodecahedron()
    t0 = time.time()
    basis = oracle.basis(N, N_UP)
    table = oracle.full_table(N, basis)
    dim = len(basis)
    apply_h = lambda v: oracle.hv_table(N, N_UP, bonds, v, basis, table)  # noqa: E731
    samples, recs = [], []
    for r in range(R):
        q = oracle.start_vector(SEED, N_UP, r, oracle.GAUSS, dim)
        a, b, k = oracle.lanczos(apply_h, q, M)
        samples.append({"r": r, "alpha": a.tolist(), "beta": b.tolist(), "steps": int(k)})
        recs.append(oracle.ritz(a, b, k))
        print(f"sample {r}: {k} steps, {time.time() - t0:.0f} s", flush=True)
    temps = oracle.log_temperatures()
    th = oracle.thermo([{"n_up": N_UP, "dim": dim, "mult": 1, "samples": recs}], temps, N)
    out = {
        "about": "FP64 oracle reference, icosidodecahedron S^z=0, Gaussian seed 2, samples r=0,1, M=100",
        "n_sites": N, "n_up": N_UP, "seed": SEED, "M": M, "dist": "gauss",
        "bonds": [[i, j, J] for i, j, J in bonds],
        "samples": samples,
        "temps": temps.tolist(), "E": th["E"].tolist(), "C": th["C"].tolist(),
    }
    with open(os.path.join(HERE, "icosidodecahedron_r2.json"), "w") as f:
        json.dump(out, f)
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
