"""The served exchange-fit request stream: Poisson arrivals of FTLM jobs on
random spin-1/2 clusters.

Each request: N uniform in {16, ..., 28}; a random connected graph of mean
degree d ~ U[3, 4] (graphs.random_cluster); couplings J ~ U[0.2, 1.5]; one
S^z sector with M ~ U{0, ..., floor(N/2)}; R = 16 +-1 start vectors; 80
Lanczos steps. Inter-arrival gaps are exponential with mean 1/rate.
"""
import numpy as np

from .graphs import random_cluster


def exchange_fit_stream(count, seed=4, rate=50.0, n_range=(16, 28), R=16, M=80):
    """List of dicts: t (arrival, s), n_sites, n_up, bonds, R, M, seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        bonds = random_cluster(n, rng)
        m = int(rng.integers(0, n // 2 + 1))
        n_up = (n + 1) // 2 + m if n % 2 else n // 2 + m
        n_up = min(n_up, n)
        out.append({"t": t, "n_sites": n, "n_up": n_up, "bonds": bonds, "R": R, "M": M, "seed": 1000 + k})
    return out
