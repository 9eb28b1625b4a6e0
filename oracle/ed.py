"""Dense exact diagonalization of small spin-1/2 Heisenberg clusters.

TEST INFRASTRUCTURE ONLY (a pin for the oracle, not a path of the product).

The Hamiltonian of Eq. (1), with a coupling J_b per bond, is assembled in
the full 2^N product space from Kronecker products of single-site spin
matrices, with no reference to labels, ranks or lookups:
    H = sum_b J_b (s^x_i s^x_j + s^y_i s^y_j + s^z_i s^z_j).
Site k is bit k of the state index (Eq. 11 at s = 1/2); in the two-state
single-site basis [down, up], s^z = diag(-1/2, +1/2) and s^+ = |up><down|.
"""
import numpy as np
import scipy.sparse as sp

SZ = sp.csr_matrix(np.array([[-0.5, 0.0], [0.0, 0.5]]))
SP = sp.csr_matrix(np.array([[0.0, 0.0], [1.0, 0.0]]))  # |up><down|
SM = SP.T.tocsr()
I2 = sp.identity(2, format="csr")


def site_op(op, k, n_sites):
    """op acting on site k; site N-1 is the most significant Kronecker factor,
    so the full-space index equals the integer label n."""
    out = sp.identity(1, format="csr")
    for site in range(n_sites - 1, -1, -1):
        out = sp.kron(out, op if site == k else I2, format="csr")
    return out


def hamiltonian(n_sites, bonds):
    """Sparse full-space H = sum_b J_b [s^z s^z + (s^+ s^- + s^- s^+)/2]."""
    dim = 1 << n_sites
    h = sp.csr_matrix((dim, dim))
    sz = [site_op(SZ, k, n_sites) for k in range(n_sites)]
    spl = [site_op(SP, k, n_sites) for k in range(n_sites)]
    sm = [site_op(SM, k, n_sites) for k in range(n_sites)]
    for i, j, J in bonds:
        h = h + J * (sz[i] @ sz[j] + 0.5 * (spl[i] @ sm[j] + sm[i] @ spl[j]))
    return h.tocsr()


def total_sz(n_sites):
    """Diagonal of S^z in the full space."""
    n = np.arange(1 << n_sites)
    ups = np.array([bin(int(x)).count("1") for x in n])
    return ups - n_sites / 2.0


def sector_block(h, n_sites, n_up):
    """Dense block of H on the labels with n_up up spins, ascending order."""
    n = np.arange(1 << n_sites)
    ups = np.array([bin(int(x)).count("1") for x in n])
    idx = n[ups == n_up]
    return np.asarray(h[idx][:, idx].todense()), idx


def spectrum_by_sector(n_sites, bonds):
    """{n_up: eigenvalues} for every sector, from numpy's dense eigh."""
    h = hamiltonian(n_sites, bonds)
    out = {}
    for n_up in range(n_sites + 1):
        blk, _ = sector_block(h, n_sites, n_up)
        out[n_up] = np.linalg.eigvalsh(blk)
    return out


def thermo_exact(n_sites, bonds, temps, g=1.0, n_ups=None):
    """Exact E, C, chi, lnZ from the full spectrum (all sectors, both signs
    of M, unless n_ups restricts the trace to the listed sectors)."""
    spec = spectrum_by_sector(n_sites, bonds)
    if n_ups is not None:
        spec = {k: v for k, v in spec.items() if k in set(n_ups)}
    e0 = min(float(v.min()) for v in spec.values())
    temps = np.asarray(temps, dtype=np.float64)
    beta = 1.0 / temps
    z = np.zeros_like(temps)
    h1 = np.zeros_like(temps)
    h2 = np.zeros_like(temps)
    zm2 = np.zeros_like(temps)
    for n_up, ev in spec.items():
        sh = ev - e0
        b = np.exp(-beta[:, None] * sh[None, :])
        zs = b.sum(axis=1)
        z += zs
        h1 += (b * sh).sum(axis=1)
        h2 += (b * sh ** 2).sum(axis=1)
        zm2 += (n_up - n_sites / 2.0) ** 2 * zs
    mean = h1 / z
    return {
        "E": e0 + mean,
        "C": beta ** 2 * (h2 / z - mean ** 2),
        "chi": g ** 2 * beta * zm2 / z,
        "lnZ": np.log(z) - beta * e0,
    }
