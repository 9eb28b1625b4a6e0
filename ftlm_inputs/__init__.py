"""Seeded synthetic inputs shared by the tests, the oracle checks and the
benchmark: cluster graphs, coupling sets and request streams.

This package holds none of the method's arithmetic (no ranks, no Hamiltonian
action, no Lanczos): only the definitions of the graphs and workloads.
"""
from .graphs import (  # noqa: F401
    dimer,
    dodecahedron,
    icosahedron,
    icosidodecahedron,
    j1j2_ring,
    random_cluster,
    relabel,
    ring,
    square_j1j2,
    triangle,
)
