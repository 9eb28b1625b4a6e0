"""Cluster graphs as bond lists [(i, j, J_ij)] with 0 <= i < j < N.

The paper's spin-1/2 systems (Sec. 3: rings, the dodecahedron, the
icosidodecahedron; Table 1's icosahedron) and the synthetic workloads built
around them. All are mathematical objects; nothing is read from disk.
"""
import itertools
import math

import numpy as np


def _norm(bonds):
    out = []
    for i, j, J in bonds:
        i, j = (i, j) if i < j else (j, i)
        out.append((int(i), int(j), float(J)))
    return out


def dimer(J=1.0):
    return [(0, 1, float(J))]


def triangle(J=1.0):
    return _norm([(0, 1, J), (1, 2, J), (0, 2, J)])


def ring(n, J=1.0):
    """Periodic chain of n sites with nearest-neighbour coupling J."""
    if n == 2:
        return dimer(J)
    return _norm([(i, (i + 1) % n, J) for i in range(n)])


def j1j2_ring(n, J1=1.0, J2=0.3):
    """Periodic chain with J1 on (i, i+1) and J2 on (i, i+2): 2n bonds."""
    return _norm([(i, (i + 1) % n, J1) for i in range(n)] +
                 [(i, (i + 2) % n, J2) for i in range(n)])


def square_j1j2(lx=6, ly=4, J1=1.0, J2=0.5):
    """Periodic lx x ly square lattice, site x + lx*y, J1 on the 2*lx*ly
    nearest-neighbour bonds and J2 on both diagonals of every plaquette."""
    def s(x, y):
        return (x % lx) + lx * (y % ly)
    bonds = []
    for y in range(ly):
        for x in range(lx):
            bonds.append((s(x, y), s(x + 1, y), J1))
            bonds.append((s(x, y), s(x, y + 1), J1))
    for y in range(ly):
        for x in range(lx):
            bonds.append((s(x, y), s(x + 1, y + 1), J2))
            bonds.append((s(x, y), s(x + 1, y - 1), J2))
    bonds = _norm(bonds)
    assert len({(i, j) for i, j, _ in bonds}) == len(bonds), "duplicate bond"
    return bonds


def dodecahedron(J=1.0):
    """The dodecahedron as the generalized Petersen graph GP(10, 2):
    outer 10-cycle u_i, spokes u_i - v_i, inner star v_i - v_{i+2}."""
    bonds = []
    for i in range(10):
        bonds.append((i, (i + 1) % 10, J))
        bonds.append((i, 10 + i, J))
        bonds.append((10 + i, 10 + (i + 2) % 10, J))
    return _norm(bonds)


def line_graph(bonds, J=1.0):
    """Vertices = edges of the input graph; adjacent when they share an end."""
    edges = [(i, j) for i, j, _ in bonds]
    out = []
    for a, b in itertools.combinations(range(len(edges)), 2):
        if set(edges[a]) & set(edges[b]):
            out.append((a, b, J))
    return _norm(out)


def icosidodecahedron(J=1.0, order="rcm"):
    """30 sites, 60 bonds, degree 4: the line graph of the dodecahedron.

    order="raw" keeps the line-graph numbering (edge order of GP(10, 2));
    order="rcm" relabels sites by reverse Cuthill-McKee, a low-bandwidth
    numbering. Observables do not depend on the numbering."""
    bonds = line_graph(dodecahedron(), J)
    if order == "rcm":
        bonds = relabel(bonds, rcm_order(30, bonds))
    return bonds


def icosahedron(J=1.0):
    """12 vertices (0, +-1, +-phi) and cyclic permutations; 30 edges of length 2."""
    phi = (1 + math.sqrt(5)) / 2
    pts = []
    for a in (-1, 1):
        for b in (-phi, phi):
            pts += [(0, a, b), (a, b, 0), (b, 0, a)]
    pts = np.array(pts)
    bonds = []
    for i, j in itertools.combinations(range(12), 2):
        if abs(np.linalg.norm(pts[i] - pts[j]) - 2.0) < 1e-9:
            bonds.append((i, j, J))
    assert len(bonds) == 30
    return _norm(bonds)


def relabel(bonds, new_of_old):
    """Rename site k to new_of_old[k]."""
    return sorted(_norm([(new_of_old[i], new_of_old[j], J) for i, j, J in bonds]))


def rcm_order(n, bonds):
    """new_of_old from scipy's reverse Cuthill-McKee on the bond graph."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    rows = [i for i, j, _ in bonds] + [j for i, j, _ in bonds]
    cols = [j for i, j, _ in bonds] + [i for i, j, _ in bonds]
    a = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    perm = reverse_cuthill_mckee(a, symmetric_mode=True)  # perm[new] = old
    new_of_old = np.empty(n, dtype=int)
    new_of_old[perm] = np.arange(n)
    return [int(v) for v in new_of_old]


def random_cluster(n, rng, degree_range=(3.0, 4.0), j_range=(0.2, 1.5)):
    """Random connected graph for the served exchange-fit stream: a uniform
    random spanning tree (decoded from a random Pruefer sequence) plus
    uniformly drawn extra edges until |E| = round(d * n / 2) with
    d ~ U[degree_range]; couplings J ~ U[j_range]."""
    prufer = rng.integers(0, n, size=n - 2) if n > 2 else np.array([], dtype=int)
    degree = np.ones(n, dtype=int)
    for v in prufer:
        degree[v] += 1
    edges = set()
    for v in prufer:
        leaf = int(np.flatnonzero(degree == 1)[0])
        edges.add((min(leaf, int(v)), max(leaf, int(v))))
        degree[leaf] -= 1
        degree[v] -= 1
    rest = np.flatnonzero(degree == 1)
    if n >= 2:
        edges.add((int(rest[0]), int(rest[-1])) if len(rest) > 1 else (0, 1))
    d = rng.uniform(*degree_range)
    target = min(int(round(d * n / 2)), n * (n - 1) // 2)
    while len(edges) < target:
        i, j = rng.integers(0, n, size=2)
        if i != j:
            edges.add((min(int(i), int(j)), max(int(i), int(j))))
    edges = sorted(edges)
    J = rng.uniform(*j_range, size=len(edges))
    return [(i, j, float(x)) for (i, j), x in zip(edges, J)]
