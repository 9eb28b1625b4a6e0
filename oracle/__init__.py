"""FP64 CPU oracle for the spin-1/2 Heisenberg FTLM hot path.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no
code with the HIP library and never imports it.

Exact parts (basis, rank, compressed lookup table, neighbour lists, H.x) are
plain definitions in ``ftlm_oracle.c``. The stochastic part (FTLM) runs the
paper's algorithm step by step in FP64:

* start vectors: normalized random vectors (Sec. 2, FTLM; Eq. 2);
* Lanczos without reorthogonalization from q1 = r, keeping alpha and beta
  (Sec. 2, the paragraph after Eq. 3);
* Ritz values theta_k and weights w_k = s_{k,1}^2 of the tridiagonal T, from
  LAPACK's symmetric tridiagonal eigensolver (``stev`` through scipy) as a
  library step;
* Boltzmann sums Eqs. (4)-(8) per S^z sector, C = beta^2 Var(H), and the
  susceptibility of Eq. (9).

Readings of points the paper leaves open:
* the order of operations in a Lanczos step (Paige's ordering: w = Hq -
  beta_{k-1} q_{k-1}, alpha = <q, w>, w -= alpha q, beta = |w|);
* the stopping rule: k = min(M, D), or beta_k <= eps * max_{j<=k}(|alpha_j|,
  beta_{j-1});
* the ground-energy shift E0 = smallest Ritz value of the run in the sums;
* sector multiplicity 1 for M = 0 and 2 for M > 0; the factor g of Eq. (9)
  is a parameter (default 1).
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

NONE = np.uint64(np.iinfo(np.uint64).max)

PM1, GAUSS, UNIT = 0, 1, 2

_lib = None


def lib():
    """Load (building first if needed) the oracle's C library."""
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        u64, i64, i32, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.orc_binom.restype = u64
        L.orc_binom.argtypes = [i32, i32]
        L.orc_sector_dim.restype = u64
        L.orc_sector_dim.argtypes = [i32, i32]
        L.orc_enumerate.restype = i64
        L.orc_enumerate.argtypes = [i32, i32, vp, u64]
        L.orc_count_below.restype = u64
        L.orc_count_below.argtypes = [i32, i32, u64]
        L.orc_rank.restype = u64
        L.orc_rank.argtypes = [i32, i32, u64]
        L.orc_unrank.restype = u64
        L.orc_unrank.argtypes = [i32, i32, u64]
        L.orc_rank_bsearch.restype = u64
        L.orc_rank_bsearch.argtypes = [vp, u64, u64]
        L.orc_rank_many.restype = None
        L.orc_rank_many.argtypes = [i32, i32, vp, u64, vp]
        L.orc_unrank_many.restype = None
        L.orc_unrank_many.argtypes = [i32, i32, vp, u64, vp]
        L.orc_clt.restype = None
        L.orc_clt.argtypes = [vp, u64, u64, vp, vp]
        L.orc_clt_blocks.restype = None
        L.orc_clt_blocks.argtypes = [i32, i32, vp, u64, vp, vp]
        L.orc_clt_lookup.restype = u64
        L.orc_clt_lookup.argtypes = [vp, vp, u64]
        L.orc_neighbors.restype = None
        L.orc_neighbors.argtypes = [i32, i32, i32, vp, vp, vp, u64, u64, vp]
        L.orc_hv.restype = None
        L.orc_hv.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, u64, u64]
        L.orc_full_table.restype = None
        L.orc_full_table.argtypes = [i32, vp, u64, vp]
        L.orc_hv_table.restype = None
        L.orc_hv_table.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, u64, u64]
        L.orc_hv_rows_stream.restype = None
        L.orc_hv_rows_stream.argtypes = [i32, i32, i32, vp, vp, vp, u64, u64, i32, vp, u64, vp]
        L.orc_hv_rows.restype = None
        L.orc_hv_rows.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, u64]
        L.orc_stream_key.restype = u64
        L.orc_stream_key.argtypes = [u64, i32, u64]
        L.orc_splitmix64_output.restype = u64
        L.orc_splitmix64_output.argtypes = [u64, u64]
        L.orc_start_vector.restype = None
        L.orc_start_vector.argtypes = [u64, i32, u64, i32, u64, vp]
        L.orc_moments_stream.restype = None
        L.orc_moments_stream.argtypes = [i32, i32, i32, vp, vp, vp, u64, u64, i32, i32, vp]
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


def set_threads(n):
    """Thread count of the oracle's OpenMP loops (0: leave it); returns the
    count in force."""
    L = lib()
    L.orc_set_threads.restype = ctypes.c_int
    L.orc_set_threads.argtypes = [ctypes.c_int]
    return int(L.orc_set_threads(n))


def binom(n, k):
    """Exact C(n, k) (Eq. 15 at s = 1/2)."""
    return int(lib().orc_binom(n, k))


def sector_dim(n_sites, n_up):
    """D_M = C(N, n_up), n_up = N/2 + M (Eq. 17)."""
    return int(lib().orc_sector_dim(n_sites, n_up))


def basis(n_sites, n_up):
    """Ascending labels with n_up set bits, by a scan of [0, 2^N)."""
    d = sector_dim(n_sites, n_up)
    out = np.empty(d, dtype=np.uint64)
    got = lib().orc_enumerate(n_sites, n_up, _ptr(out), d)
    assert got == d
    return out


def rank(n_sites, n_up, labels):
    """Sector index (count of smaller sector labels); NONE outside the sector."""
    labels = np.ascontiguousarray(labels, dtype=np.uint64)
    out = np.empty_like(labels)
    lib().orc_rank_many(n_sites, n_up, _ptr(labels), labels.size, _ptr(out))
    return out


def rank_bsearch(basis_arr, labels):
    """Position in a stored sorted basis by binary search; NONE if absent."""
    L = lib()
    return np.array([L.orc_rank_bsearch(_ptr(basis_arr), basis_arr.size, int(x))
                     for x in np.asarray(labels, dtype=np.uint64)], dtype=np.uint64)


def unrank(n_sites, n_up, idx):
    """Inverse of rank, by bisection on the count of smaller labels."""
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.empty_like(idx)
    lib().orc_unrank_many(n_sites, n_up, _ptr(idx), idx.size, _ptr(out))
    return out


def clt(basis_arr, n_sites):
    """Compressed lookup table (Eqs. 18-21): (mask, prefix) per 32-label block
    over the whole label space [0, 2^N)."""
    nblocks = max(1, ((1 << n_sites) + 31) // 32)
    mask = np.empty(nblocks, dtype=np.uint32)
    prefix = np.empty(nblocks, dtype=np.uint32)
    basis_arr = np.ascontiguousarray(basis_arr, dtype=np.uint64)
    lib().orc_clt(_ptr(basis_arr), basis_arr.size, nblocks, _ptr(mask), _ptr(prefix))
    return mask, prefix


def clt_blocks(n_sites, n_up, blocks):
    """(mask, prefix) of the listed blocks from the definition (no basis)."""
    blocks = np.ascontiguousarray(blocks, dtype=np.uint64)
    mask = np.empty(blocks.size, dtype=np.uint32)
    prefix = np.empty(blocks.size, dtype=np.uint32)
    lib().orc_clt_blocks(n_sites, n_up, _ptr(blocks), blocks.size, _ptr(mask), _ptr(prefix))
    return mask, prefix


def clt_lookup(mask, prefix, n):
    """Alg. 2 on the oracle's table."""
    return int(lib().orc_clt_lookup(_ptr(mask), _ptr(prefix), int(n)))


def _bonds(bonds):
    bi = np.ascontiguousarray([b[0] for b in bonds], dtype=np.int32)
    bj = np.ascontiguousarray([b[1] for b in bonds], dtype=np.int32)
    J = np.ascontiguousarray([b[2] for b in bonds], dtype=np.float64)
    return bi, bj, J


def neighbors(n_sites, n_up, bonds, t0, count, basis_arr=None):
    """[count][N_B] partner indices (NONE where the bond is parallel)."""
    bi, bj, _ = _bonds(bonds)
    out = np.empty((count, len(bonds)), dtype=np.uint64)
    lib().orc_neighbors(n_sites, n_up, len(bonds), _ptr(bi), _ptr(bj), _ptr(basis_arr),
                        t0, count, _ptr(out))
    return out


def hv(n_sites, n_up, bonds, x, basis_arr=None, row0=0, nrows=None):
    """FP64 H.x (Eq. 12) on rows [row0, row0 + nrows)."""
    bi, bj, J = _bonds(bonds)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if nrows is None:
        nrows = x.size - row0
    y = np.empty(nrows, dtype=np.float64)
    lib().orc_hv(n_sites, n_up, len(bonds), _ptr(bi), _ptr(bj), _ptr(J), _ptr(basis_arr),
                 _ptr(x), _ptr(y), row0, nrows)
    return y


def full_table(n_sites, basis_arr):
    """Full lookup table: uint32 index per label of [0, 2^N), 0xFFFFFFFF
    outside the sector (Sec. 2, the simplest state-to-index map)."""
    table = np.empty(1 << n_sites, dtype=np.uint32)
    lib().orc_full_table(n_sites, _ptr(basis_arr), basis_arr.size, _ptr(table))
    return table


def hv_table(n_sites, n_up, bonds, x, basis_arr, table):
    """FP64 H.x with partner indices from a full lookup table."""
    bi, bj, J = _bonds(bonds)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(x.size, dtype=np.float64)
    lib().orc_hv_table(n_sites, n_up, len(bonds), _ptr(bi), _ptr(bj), _ptr(J), _ptr(basis_arr), _ptr(table),
                       _ptr(x), _ptr(y), 0, x.size)
    return y


def hv_rows(n_sites, n_up, bonds, x, rows, basis_arr=None):
    """FP64 H.x evaluated only at the listed rows."""
    bi, bj, J = _bonds(bonds)
    x = np.ascontiguousarray(x, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    y = np.empty(rows.size, dtype=np.float64)
    lib().orc_hv_rows(n_sites, n_up, len(bonds), _ptr(bi), _ptr(bj), _ptr(J), _ptr(basis_arr),
                      _ptr(x), _ptr(y), _ptr(rows), rows.size)
    return y


def hv_rows_stream(n_sites, n_up, bonds, seed, r, dist, rows):
    """FP64 rows of H.x for x = the unnormalized start vector of sample r,
    generated on demand (no full-length vector)."""
    bi, bj, J = _bonds(bonds)
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    y = np.empty(rows.size, dtype=np.float64)
    lib().orc_hv_rows_stream(n_sites, n_up, len(bonds), _ptr(bi), _ptr(bj), _ptr(J), seed, r, dist, _ptr(rows),
                             rows.size, _ptr(y))
    return y


def first_step_moments(n_sites, n_up, bonds, seed, r0, R, dist):
    """<x|x>, <x|H|x> and <Hx|Hx> of the unnormalized start vectors of samples
    r0 .. r0 + R - 1 over the whole sector, entries generated on demand.
    Returns a [R][3] array."""
    bi, bj, J = _bonds(bonds)
    out = np.empty((R, 3), dtype=np.float64)
    lib().orc_moments_stream(n_sites, n_up, len(bonds), _ptr(bi), _ptr(bj), _ptr(J), seed, r0, R, dist,
                             _ptr(out))
    return out


def first_step(moments):
    """alpha_1 and beta_1 of Lanczos from the normalized start vector, from
    its moments (alpha_1 = <x|H|x>/<x|x>, alpha_1^2 + beta_1^2 =
    <Hx|Hx>/<x|x>)."""
    m = np.asarray(moments, dtype=np.float64)
    a = m[:, 1] / m[:, 0]
    b = np.sqrt(m[:, 2] / m[:, 0] - a * a)
    return a, b


def start_vector(seed, n_up, r, dist, dim, normalize=True):
    """Start vector of sample r (SplitMix64 stream keyed (seed, n_up, r)).

    Normalized in FP64 when ``normalize`` (the paper's |r> are normalized)."""
    out = np.empty(dim, dtype=np.float64)
    lib().orc_start_vector(seed, n_up, r, dist, dim, _ptr(out))
    if normalize:
        out /= math.sqrt(float(np.dot(out, out)))
    return out


def splitmix64_output(s, i):
    """Output i (0-based) of SplitMix64 seeded at s."""
    return int(lib().orc_splitmix64_output(s, i))


def stream_key(seed, n_up, r):
    return int(lib().orc_stream_key(seed, n_up, r))


def lanczos(apply_h, q1, m, eps=1e-12):
    """Lanczos recursion without reorthogonalization from the normalized q1.

    Returns (alpha[steps], beta[steps], steps); T has alpha on its diagonal
    and beta[:steps-1] off it. The run stops after step k when k reaches
    min(m, dim) or when beta_k <= eps * max_{j<=k}(|alpha_j|, beta_{j-1})."""
    dim = q1.size
    m_eff = min(m, dim)
    q = np.array(q1, dtype=np.float64)
    q_prev = np.zeros_like(q)
    beta_prev = 0.0
    scale = 0.0
    alphas, betas = [], []
    for k in range(1, m_eff + 1):
        w = apply_h(q) - beta_prev * q_prev
        a = float(np.dot(q, w))
        w = w - a * q
        b = math.sqrt(float(np.dot(w, w)))
        alphas.append(a)
        betas.append(b)
        scale = max(scale, abs(a), beta_prev)
        if k == m_eff or b <= eps * scale:
            break
        q_prev, q = q, w / b
        beta_prev = b
    return np.array(alphas), np.array(betas), len(alphas)


def ritz(alpha, beta, steps=None):
    """Ritz values theta_k and weights w_k = |s_{k,1}|^2 of T (FP64)."""
    from scipy.linalg import eigh_tridiagonal
    if steps is None:
        steps = len(alpha)
    a = np.asarray(alpha[:steps], dtype=np.float64)
    if steps == 1:
        return a.copy(), np.ones(1)
    b = np.asarray(beta[:steps - 1], dtype=np.float64)
    theta, s = eigh_tridiagonal(a, b, lapack_driver="stev")
    return theta, s[0, :] ** 2


U_FP32 = 2.0 ** -24  # unit roundoff of IEEE single precision


def seed_spread(estimates):
    """Empirical standard deviation of Eq. (22) over N_s independent FTLM
    runs: ``estimates`` is [N_s][...] (one row per seed); returns (mean,
    sigma) with sigma^2 = (1/N_s) sum_s (O_s - mean)^2."""
    x = np.asarray(estimates, dtype=np.float64)
    n_s = x.shape[0]
    mean = x.sum(axis=0) / n_s
    dev = x - mean[None, ...]
    return mean, np.sqrt((dev * dev).sum(axis=0) / n_s)


def ghost_diagnostic(alpha, beta, steps=None, c_tau=1.0, u=U_FP32):
    """Cullum-Willoughby ghost test and Ritz clusters (Sec. 3.2, Eq. 25).

    T is the steps x steps tridiagonal of one chain; T1 is T without its first
    row and column. A Ritz value theta_k of T is a ghost when its deflation
    distance ell_k = min_j |theta_k - theta1_j| (theta1 the eigenvalues of T1)
    is below tau = c_tau * u * (max theta - min theta). Ritz values whose
    distance is <= tau belong to one cluster (joined transitively along the
    sorted spectrum). Returns a dict: theta (ascending), weight, ell, tau,
    ghost (bool), cluster (cluster id per theta_k, ids in ascending order) and
    cluster_weight (total weight per cluster id)."""
    from scipy.linalg import eigvalsh_tridiagonal
    if steps is None:
        steps = len(alpha)
    theta, w = ritz(alpha, beta, steps)
    if steps >= 2:
        a1 = np.asarray(alpha[1:steps], dtype=np.float64)
        if steps >= 3:
            theta1 = eigvalsh_tridiagonal(a1, np.asarray(beta[1:steps - 1], dtype=np.float64),
                                          lapack_driver="stev")
        else:
            theta1 = a1.copy()
        ell = np.array([float(np.min(np.abs(t - theta1))) for t in theta])
    else:
        ell = np.full(1, np.inf)
    tau = c_tau * u * float(theta[-1] - theta[0])
    cluster = np.zeros(steps, dtype=np.int64)
    for k in range(1, steps):
        cluster[k] = cluster[k - 1] + (0 if theta[k] - theta[k - 1] <= tau else 1)
    cw = np.zeros(int(cluster[-1]) + 1)
    for k in range(steps):
        cw[cluster[k]] += w[k]
    return {"theta": theta, "weight": w, "ell": ell, "tau": tau, "ghost": ell < tau, "cluster": cluster,
            "cluster_weight": cw}


def log_temperatures(n=200, t_min=0.05, t_max=10.0):
    """n log-spaced temperatures from t_min to t_max inclusive."""
    k = np.arange(n)
    return t_min * (t_max / t_min) ** (k / (n - 1))


def thermo(sectors, temps, n_sites, g=1.0):
    """Thermal reduction, Eqs. (6)-(9), with every Boltzmann factor shifted by
    E0 = the smallest Ritz value over all sectors and samples.

    ``sectors``: list of dicts with keys n_up, dim, mult, and samples = list
    of (theta, weight) pairs. Returns dict of arrays E, C, chi, lnZ over temps.
    """
    e0 = min(float(np.min(th)) for s in sectors for th, _ in s["samples"])
    temps = np.asarray(temps, dtype=np.float64)
    beta = 1.0 / temps
    z = np.zeros_like(temps)
    h1 = np.zeros_like(temps)
    h2 = np.zeros_like(temps)
    zm2 = np.zeros_like(temps)
    for s in sectors:
        pref = s["mult"] * s["dim"] / len(s["samples"])
        m_val = s["n_up"] - n_sites / 2.0
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
    var = h2 / z - mean ** 2
    return {
        "E": e0 + mean,
        "C": beta ** 2 * var,
        "chi": g ** 2 * beta * zm2 / z,
        "lnZ": np.log(z) - beta * e0,
    }


def multiplicity(n_sites, n_up):
    """Sectors +M and -M share a spectrum: weight 2 for M > 0, 1 for M = 0."""
    return 1 if 2 * n_up == n_sites else 2


def ftlm_sector(n_sites, n_up, bonds, R, M, seed, dist, r0=0, basis_arr=None, eps=1e-12):
    """R Lanczos samples in one sector; returns a thermo() sector record and
    the raw (alpha, beta, steps) per sample."""
    dim = sector_dim(n_sites, n_up)
    if basis_arr is None and n_sites <= 26:
        basis_arr = basis(n_sites, n_up)
    samples, raw = [], []
    for r in range(R):
        q1 = start_vector(seed, n_up, r0 + r, dist, dim)
        a, b, k = lanczos(lambda v: hv(n_sites, n_up, bonds, v, basis_arr), q1, M, eps)
        samples.append(ritz(a, b, k))
        raw.append((a, b, k))
    rec = {"n_up": n_up, "dim": dim, "mult": multiplicity(n_sites, n_up), "samples": samples}
    return rec, raw


def ftlm(n_sites, bonds, n_ups, R, M, seed, dist, temps, g=1.0):
    """Full oracle FTLM over the listed sectors (n_up >= N/2)."""
    recs = [ftlm_sector(n_sites, nu, bonds, R, M, seed, dist)[0] for nu in n_ups]
    return thermo(recs, temps, n_sites, g), recs
