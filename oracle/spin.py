"""FP64 oracle for the general-spin Heisenberg H.x (local spin s; paper
Sec. 2, Eqs. 10-17) -- TEST INFRASTRUCTURE ONLY, like the rest of oracle/.

Labels are base-d integers n = sum_k a_k d^k with d = 2s + 1 and a_k = m_k
+ s (Eq. 11); the sector with digit sum A (S^z = M = A - N s, Eq. 17) is
ordered by increasing label. ``two_s`` = 2s throughout. The plain
definitions live in spin_oracle.c: the dimension recursion of Eq. (15), a
scan of the label space for the basis, binary search for ranks, H.x row by
row with the ladder coefficients of Eqs. (13)-(14), and a count of the
off-diagonal entries (N_nz of Eq. 10 minus the diagonal).
"""
import ctypes
import math

import numpy as np

from . import lib as _lib_base, _ptr, _bonds, start_vector, lanczos, ritz

NONE = np.uint64(np.iinfo(np.uint64).max)


def lib():
    L = _lib_base()
    if not getattr(L, "_spin_sigs", False):
        u64, i64, i32, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.spn_dim.restype = u64
        L.spn_dim.argtypes = [i32, i32, i32]
        L.spn_enumerate.restype = i64
        L.spn_enumerate.argtypes = [i32, i32, i32, vp, u64]
        L.spn_rank.restype = u64
        L.spn_rank.argtypes = [vp, u64, u64]
        L.spn_hv.restype = None
        L.spn_hv.argtypes = [i32, i32, i32, vp, vp, vp, vp, u64, vp, vp, u64, u64]
        L.spn_neighbors.restype = None
        L.spn_neighbors.argtypes = [i32, i32, vp, vp, vp, u64, u64, u64, vp]
        L.spn_offdiag_count.restype = u64
        L.spn_offdiag_count.argtypes = [i32, i32, i32, i32, vp, vp]
        L.spn_rank_count.restype = None
        L.spn_rank_count.argtypes = [i32, i32, i32, vp, u64, vp]
        L.spn_unrank_count.restype = None
        L.spn_unrank_count.argtypes = [i32, i32, i32, vp, u64, vp]
        L.spn_hv_rows.restype = None
        L.spn_hv_rows.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, u64, vp]
        L._spin_sigs = True
    return L


def dim(m, two_s, a):
    """D(m, A) of Eq. (15)."""
    return int(lib().spn_dim(m, two_s, a))


def a_total(n_sites, two_s, m2):
    """Digit sum of the sector with 2M = m2 (Eq. 17: A = N s + M)."""
    a2 = n_sites * two_s + m2
    assert a2 % 2 == 0, "N s + M must be an integer"
    return a2 // 2


def basis(n_sites, two_s, a):
    """Sector labels with digit sum a, ascending (uint64)."""
    n = dim(n_sites, two_s, a)
    out = np.empty(n, dtype=np.uint64)
    got = lib().spn_enumerate(n_sites, two_s, a, _ptr(out), n)
    assert got == n
    return out


def rank(basis_arr, labels):
    labels = np.atleast_1d(np.asarray(labels, dtype=np.uint64))
    return np.array([lib().spn_rank(_ptr(basis_arr), basis_arr.size, int(x)) for x in labels], dtype=np.uint64)


def hv(n_sites, two_s, bonds, x, basis_arr, row0=0, nrows=None):
    """FP64 rows [row0, row0 + nrows) of H x (x over the whole sector)."""
    bi, bj, J = _bonds(bonds)
    d = basis_arr.size
    nrows = d - row0 if nrows is None else nrows
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(nrows, dtype=np.float64)
    lib().spn_hv(n_sites, two_s, len(bonds), _ptr(bi), _ptr(bj), _ptr(J), _ptr(basis_arr), d, _ptr(x), _ptr(y),
                 row0, nrows)
    return y


def rank_count(n_sites, two_s, a, labels):
    """Indices of labels in the sector with digit sum a, by counting the
    sector labels below each one (Eq. 15 dimensions; no stored basis)."""
    labels = np.ascontiguousarray(np.atleast_1d(labels), dtype=np.uint64)
    out = np.empty(labels.size, dtype=np.uint64)
    lib().spn_rank_count(n_sites, two_s, a, _ptr(labels), labels.size, _ptr(out))
    return out


def unrank_count(n_sites, two_s, a, idx):
    """Labels of sector indices (each < D), by counting."""
    idx = np.ascontiguousarray(np.atleast_1d(idx), dtype=np.uint64)
    out = np.empty(idx.size, dtype=np.uint64)
    lib().spn_unrank_count(n_sites, two_s, a, _ptr(idx), idx.size, _ptr(out))
    return out


def hv_rows(n_sites, two_s, a, bonds, x, rows):
    """FP64 rows `rows` of H x (x over the whole sector), labels and
    partner indices found by counting, so that no basis is stored."""
    bi, bj, J = _bonds(bonds)
    x = np.ascontiguousarray(x, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    y = np.empty(rows.size, dtype=np.float64)
    lib().spn_hv_rows(n_sites, two_s, a, len(bonds), _ptr(bi), _ptr(bj), _ptr(J), _ptr(x), _ptr(rows), rows.size,
                      _ptr(y))
    return y


def neighbors(two_s, bonds, basis_arr, t0, count):
    """[count][2 N_B] partner indices: entry 2b is the state with a_i + 1,
    a_j - 1 for bond b = (i, j), i < j, entry 2b + 1 the one with a_i - 1,
    a_j + 1; NONE where a digit would leave [0, 2s]."""
    bi, bj, _ = _bonds(bonds)
    out = np.empty((count, 2 * len(bonds)), dtype=np.uint64)
    lib().spn_neighbors(two_s, len(bonds), _ptr(bi), _ptr(bj), _ptr(basis_arr), basis_arr.size, t0, count,
                        _ptr(out))
    return out


def clt(basis_arr, n_sites, two_s):
    """Compressed lookup table over the d^N labels (Eqs. 18-21): (mask,
    prefix) per 32-label block, from one pass over the sorted basis."""
    nblocks = max(1, ((two_s + 1) ** n_sites + 31) // 32)
    mask = np.empty(nblocks, dtype=np.uint32)
    prefix = np.empty(nblocks, dtype=np.uint32)
    basis_arr = np.ascontiguousarray(basis_arr, dtype=np.uint64)
    lib().orc_clt(_ptr(basis_arr), basis_arr.size, nblocks, _ptr(mask), _ptr(prefix))
    return mask, prefix


def offdiag_count(n_sites, two_s, a, bonds):
    """Off-diagonal entries of H in the sector (N_nz of Eq. 10 is this + D)."""
    bi, bj, _ = _bonds(bonds)
    return int(lib().spn_offdiag_count(n_sites, two_s, a, len(bonds), _ptr(bi), _ptr(bj)))


def multiplicity(n_sites, two_s, a):
    """Sectors +M and -M share a spectrum: 1 for M = 0, else 2."""
    return 1 if 2 * a == n_sites * two_s else 2


def ftlm_sector(n_sites, two_s, a, bonds, R, M, seed, dist, basis_arr=None, eps=1e-12):
    """R Lanczos samples in the sector with digit sum a; start vectors keyed
    by (seed, a, r) like the spin-1/2 sectors (a = n_up there)."""
    if basis_arr is None:
        basis_arr = basis(n_sites, two_s, a)
    d = basis_arr.size
    samples, raw = [], []
    for r in range(R):
        q1 = start_vector(seed, a, r, dist, d)
        al, be, k = lanczos(lambda v: hv(n_sites, two_s, bonds, v, basis_arr), q1, M, eps)
        samples.append(ritz(al, be, k))
        raw.append((al, be, k))
    return {"a": a, "dim": d, "mult": multiplicity(n_sites, two_s, a), "samples": samples}, raw


def thermo(sectors, temps, n_sites, two_s, g=1.0):
    """Eqs. (6)-(9) over general-spin sector records (keys a, dim, mult,
    samples), E0 shift as in oracle.thermo; M = a - N s."""
    e0 = min(float(np.min(th)) for s in sectors for th, _ in s["samples"])
    temps = np.asarray(temps, dtype=np.float64)
    beta = 1.0 / temps
    z, h1, h2, zm2 = (np.zeros_like(temps) for _ in range(4))
    for s in sectors:
        pref = s["mult"] * s["dim"] / len(s["samples"])
        m_val = s["a"] - 0.5 * n_sites * two_s
        zs = np.zeros_like(temps)
        for th, w in s["samples"]:
            sh = th - e0
            boltz = w[None, :] * np.exp(-beta[:, None] * sh[None, :])
            zs += pref * boltz.sum(axis=1)
            h1 += pref * (boltz * sh[None, :]).sum(axis=1)
            h2 += pref * (boltz * sh[None, :] ** 2).sum(axis=1)
        z += zs
        zm2 += m_val ** 2 * zs
    mean = h1 / z
    return {"E": e0 + mean, "C": beta ** 2 * (h2 / z - mean ** 2), "chi": g ** 2 * beta * zm2 / z,
            "lnZ": np.log(z) - beta * e0}
