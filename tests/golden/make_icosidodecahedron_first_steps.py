"""Writes tests/golden/icosidodecahedron_first_steps.json: the FP64 oracle's
first two Lanczos steps (alpha_1, beta_1, alpha_2, beta_2) for every one of
the 20 samples r = 0..19 of the icosidodecahedron workload (N = 30, 60 bonds,
J = 1, S^z = 0, Gaussian start vectors, seed 2).

alpha_1 = <r|H|r> and alpha_1^2 + beta_1^2 = |H r|^2 for the normalized start
vector r (Sec. 2, the Lanczos recursion after Eq. 3); the second step is
still far from any loss of orthogonality, so an FP32 chain must reproduce
both steps at FP32 roundoff (Sec. 3.1, same seeds in both precisions).

Calls only oracle/ (and the input definitions in ftlm_inputs/). Needs about
9 GB of memory and ~10-20 minutes on 8 cores:
    python tests/golden/make_icosidodecahedron_first_steps.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from ftlm_inputs import graphs  # noqa: E402

N, N_UP, SEED, R, STEPS = 30, 15, 2, 20, 2


def main():
    bonds = graphs.icosidodecahedron()
    t0 = time.time()
    basis = oracle.basis(N, N_UP)
    table = oracle.full_table(N, basis)
    dim = len(basis)
    apply_h = lambda v: oracle.hv_table(N, N_UP, bonds, v, basis, table)  # noqa: E731
    samples = []
    for r in range(R):
        q = oracle.start_vector(SEED, N_UP, r, oracle.GAUSS, dim)
        a, b, k = oracle.lanczos(apply_h, q, STEPS)
        assert k == STEPS
        samples.append({"r": r, "alpha": a.tolist(), "beta": b.tolist()})
        print(f"sample {r}: alpha {a.tolist()} beta {b.tolist()}, {time.time() - t0:.0f} s", flush=True)
    out = {
        "about": "FP64 oracle, icosidodecahedron S^z=0, Gaussian seed 2, samples r=0..19, first two Lanczos steps",
        "n_sites": N, "n_up": N_UP, "seed": SEED, "dist": "gauss", "steps": STEPS,
        "bonds": [[i, j, J] for i, j, J in bonds],
        "samples": samples,
    }
    with open(os.path.join(HERE, "icosidodecahedron_first_steps.json"), "w") as f:
        json.dump(out, f)
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
