"""Writes tests/golden/ring34_first_step.json: the FP64 oracle's first
Lanczos step (alpha_1, beta_1) for samples r = 0..3 of the J1-J2 ring N = 34
(J1 = 1, J2 = 0.3, 68 bonds), S^z = 0 (D = 2,333,606,220), +-1 start vectors
with seed 5: alpha_1 = <x|H|x> / <x|x> and alpha_1^2 + beta_1^2 =
<Hx|Hx> / <x|x> (Sec. 2, the Lanczos recursion after Eq. 3), summed over
every row of the sector with the vector entries generated on demand.

Calls only oracle/ (and the input definitions in ftlm_inputs/). Needs little
memory and ~15-30 minutes on 8 cores:
    python tests/golden/make_ring34_first_step.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from ftlm_inputs import graphs  # noqa: E402

N, N_UP, SEED, R = 34, 17, 5, 4


def main():
    bonds = graphs.j1j2_ring(N, 1.0, 0.3)
    t0 = time.time()
    m = oracle.first_step_moments(N, N_UP, bonds, SEED, 0, R, oracle.PM1)
    a, b = oracle.first_step(m)
    out = {
        "about": "FP64 oracle, J1-J2 ring N=34 (J2=0.3) S^z=0, +-1 seed 5, samples r=0..3, first Lanczos step",
        "n_sites": N, "n_up": N_UP, "seed": SEED, "dist": "pm1", "j2": 0.3,
        "samples": [{"r": r, "xx": m[r, 0], "xHx": m[r, 1], "HxHx": m[r, 2], "alpha": [a[r]], "beta": [b[r]]}
                    for r in range(R)],
    }
    with open(os.path.join(HERE, "ring34_first_step.json"), "w") as f:
        json.dump(out, f)
    print(f"alpha {a.tolist()} beta {b.tolist()}; done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
