"""Dense exact diagonalization of small Heisenberg clusters of local spin s.

TEST INFRASTRUCTURE ONLY (a pin for the general-spin oracle, not a path of
the product).

H = sum_b J_b (S^x_i S^x_j + S^y_i S^y_j + S^z_i S^z_j) is assembled in the
full d^N product space (d = 2s + 1) from Kronecker products of single-site
spin matrices built from their textbook matrix elements, with no reference to
labels, ranks or lookups. Site k is the k-th base-d digit of the state index
(Eq. 11): the single-site basis is ordered a = m + s = 0 .. 2s.
"""
import numpy as np
import scipy.sparse as sp


def spin_matrices(two_s):
    """(S^z, S^+) in the basis m = -s .. s (index a = m + s):
    S^z = diag(m), <m+1|S^+|m> = sqrt(s(s+1) - m(m+1))."""
    s = 0.5 * two_s
    d = two_s + 1
    m = np.arange(d) - s
    sz = np.diag(m)
    spl = np.zeros((d, d))
    for a in range(d - 1):
        spl[a + 1, a] = np.sqrt(s * (s + 1) - m[a] * (m[a] + 1))
    return sp.csr_matrix(sz), sp.csr_matrix(spl)


def site_op(op, k, n_sites, d):
    """op on site k; site N-1 is the most significant Kronecker factor, so
    the full-space index equals the base-d label n of Eq. (11)."""
    out = sp.identity(1, format="csr")
    eye = sp.identity(d, format="csr")
    for site in range(n_sites - 1, -1, -1):
        out = sp.kron(out, op if site == k else eye, format="csr")
    return out


def hamiltonian(n_sites, two_s, bonds):
    """Sparse full-space H = sum_b J_b [S^z S^z + (S^+ S^- + S^- S^+)/2]."""
    d = two_s + 1
    sz1, sp1 = spin_matrices(two_s)
    sm1 = sp1.T.tocsr()
    sz = [site_op(sz1, k, n_sites, d) for k in range(n_sites)]
    spl = [site_op(sp1, k, n_sites, d) for k in range(n_sites)]
    sm = [site_op(sm1, k, n_sites, d) for k in range(n_sites)]
    h = sp.csr_matrix((d ** n_sites, d ** n_sites))
    for i, j, J in bonds:
        h = h + J * (sz[i] @ sz[j] + 0.5 * (spl[i] @ sm[j] + sm[i] @ spl[j]))
    return h.tocsr()


def digit_sums(n_sites, two_s):
    """Digit sum A = sum_k a_k of every full-space index."""
    d = two_s + 1
    n = np.arange(d ** n_sites)
    a = np.zeros_like(n)
    for _ in range(n_sites):
        a += n % d
        n //= d
    return a


def sector_block(h, n_sites, two_s, a_tot):
    """Dense block of H on the labels with digit sum a_tot, ascending."""
    idx = np.nonzero(digit_sums(n_sites, two_s) == a_tot)[0]
    return np.asarray(h[idx][:, idx].todense()), idx
