"""Pins for the oracle's stochastic and reduction parts: the start-vector
generator, the Lanczos recursion, Ritz weights and the thermal sums.

The anchors are: SplitMix64's published output sequence; Gauss-quadrature
moment identities of the Lanczos tridiagonal matrix; closed-form thermo of
the dimer and the beta -> 0 limits; exact-trace FTLM (unit start vectors,
N_L = D) against dense ED; and FTLM with random vectors against ED within
the spread over seeds (Eq. 22).
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import ed
from ftlm_inputs import graphs


# ---- start vectors ------------------------------------------------------------

def test_splitmix64_published_sequence():
    # SplitMix64 (Steele, Lea, Flood 2014) seeded with 0.
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [oracle.splitmix64_output(0, i) for i in range(3)] == want


def test_pm1_vectors():
    v = oracle.start_vector(1, 6, 0, oracle.PM1, 100000, normalize=False)
    assert set(np.unique(v)) == {-1.0, 1.0}
    assert abs(v.mean()) < 0.02
    q = oracle.start_vector(1, 6, 0, oracle.PM1, 100000)
    assert abs(np.dot(q, q) - 1.0) < 1e-14


def test_gauss_vectors_are_standard_normal():
    v = oracle.start_vector(2, 15, 3, oracle.GAUSS, 200000, normalize=False)
    assert stats.kstest(v, "norm").pvalue > 1e-3
    assert abs(v.mean()) < 0.01 and abs(v.var() - 1) < 0.02


def test_streams_independent_of_count_and_distinct():
    a = oracle.start_vector(9, 4, 5, oracle.GAUSS, 1000)
    b = oracle.start_vector(9, 4, 5, oracle.GAUSS, 1000)
    np.testing.assert_array_equal(a, b)
    prefix = oracle.start_vector(9, 4, 5, oracle.GAUSS, 10, normalize=False)
    full = oracle.start_vector(9, 4, 5, oracle.GAUSS, 1000, normalize=False)
    np.testing.assert_array_equal(prefix, full[:10])
    keys = {oracle.stream_key(s, n, r) for s in (1, 2) for n in (5, 6) for r in range(20)}
    assert len(keys) == 80
    c = oracle.start_vector(9, 4, 6, oracle.GAUSS, 1000)
    assert abs(np.dot(a, c)) < 0.2


def test_unit_vectors():
    v = oracle.start_vector(0, 3, 7, oracle.UNIT, 20)
    assert v[7] == 1.0 and np.count_nonzero(v) == 1


# ---- Lanczos --------------------------------------------------------------------

def _system(n=12, n_up=6, bonds=None):
    bonds = bonds or graphs.ring(n)
    b = oracle.basis(n, n_up)
    return (lambda v: oracle.hv(n, n_up, bonds, v, b)), len(b)


def test_lanczos_first_coefficients():
    h, d = _system()
    q = oracle.start_vector(1, 6, 0, oracle.PM1, d)
    a, b, k = oracle.lanczos(h, q, 10)
    hq = h(q)
    assert abs(a[0] - q @ hq) < 1e-12
    assert abs(a[0] ** 2 + b[0] ** 2 - hq @ hq) < 1e-10


@pytest.mark.parametrize("n,n_up,dist", [(10, 5, oracle.GAUSS), (12, 6, oracle.PM1), (11, 7, oracle.GAUSS)])
def test_first_step_moments_against_dense_h(n, n_up, dist):
    # the streamed moments (labels walked by next-combination, entries and
    # partner indices generated on demand) against the dense Kronecker-product
    # H restricted to the sector and the stored start vectors
    bonds = graphs.j1j2_ring(n, 1.0, 0.45)
    h, _ = ed.sector_block(ed.hamiltonian(n, bonds), n, n_up)
    m = oracle.first_step_moments(n, n_up, bonds, 7, 2, 3, dist)
    for r in range(3):
        x = oracle.start_vector(7, n_up, 2 + r, dist, h.shape[0], normalize=False)
        hx = h @ x
        np.testing.assert_allclose(m[r], [x @ x, x @ hx, hx @ hx], rtol=1e-12)
    a, b = oracle.first_step(m)
    for r in range(3):
        q = oracle.start_vector(7, n_up, 2 + r, dist, h.shape[0])
        al, be, _ = oracle.lanczos(lambda v: h @ v, q, 2)
        assert abs(a[r] - al[0]) < 1e-12 and abs(b[r] - be[0]) < 1e-11


@pytest.mark.parametrize("m", [4, 12, 40])
def test_gauss_quadrature_moments(m):
    # sum_k w_k theta_k^p = <r|H^p|r> for p <= 2m - 1 (checked to p = 4)
    bonds = graphs.random_cluster(12, np.random.default_rng(3))
    h, d = _system(12, 6, bonds)
    q = oracle.start_vector(4, 6, 1, oracle.GAUSS, d)
    a, b, k = oracle.lanczos(h, q, m)
    th, w = oracle.ritz(a, b, k)
    assert abs(w.sum() - 1.0) < 1e-13
    v = q.copy()
    for p in range(1, 5):
        v = h(v)
        mom = q @ v
        assert abs((w * th ** p).sum() - mom) < 1e-9 * max(1.0, abs(mom))


def test_full_krylov_gives_exact_eigenvalues():
    # In a small sector N_L = D recovers the spectrum; in a larger one the
    # ground state still converges (without reorthogonalization the interior
    # of a long run carries ghosts, Sec. 3.2).
    n = 6
    bonds = graphs.random_cluster(n, np.random.default_rng(8))
    h, d = _system(n, 3, bonds)
    q = oracle.start_vector(2, 3, 0, oracle.GAUSS, d)
    a, b, k = oracle.lanczos(h, q, 10 * d)
    assert k <= d
    th, w = oracle.ritz(a, b, k)
    blk, _ = ed.sector_block(ed.hamiltonian(n, bonds), n, 3)
    ev = np.linalg.eigvalsh(blk)
    big = w > 1e-10
    assert np.all(np.min(np.abs(th[big][:, None] - ev[None, :]), axis=1) < 1e-8)
    n = 10
    bonds = graphs.random_cluster(n, np.random.default_rng(8))
    h, d = _system(n, 5, bonds)
    a, b, k = oracle.lanczos(h, oracle.start_vector(2, 5, 0, oracle.GAUSS, d), 80)
    th, w = oracle.ritz(a, b, k)
    blk, _ = ed.sector_block(ed.hamiltonian(n, bonds), n, 5)
    assert abs(th.min() - np.linalg.eigvalsh(blk).min()) < 1e-10


def test_lanczos_stops_on_breakdown_and_tiny_sectors():
    # D = 1: one step, T = [H_11]
    h, d = _system(12, 12, graphs.ring(12))
    q = oracle.start_vector(1, 12, 0, oracle.PM1, d)
    a, b, k = oracle.lanczos(h, q, 40)
    assert d == 1 and k == 1 and abs(a[0] - 3.0) < 1e-14
    # D = 12 (one flipped spin) with M = 40: stops at k = min(M, D) or before
    h, d = _system(12, 11, graphs.ring(12))
    q = oracle.start_vector(1, 11, 0, oracle.PM1, d)
    a, b, k = oracle.lanczos(h, q, 40)
    assert k <= d
    th, w = oracle.ritz(a, b, k)
    assert abs(w.sum() - 1) < 1e-12
    # an eigenvector start (uniform vector in the ferromagnetic-like
    # translation-invariant sector of the ring) breaks down after one step
    q = np.ones(d) / math.sqrt(d)
    a, b, k = oracle.lanczos(h, q, 40)
    assert k == 1 and b[0] < 1e-12


def test_ritz_matches_dense_tridiagonal_eig():
    rng = np.random.default_rng(0)
    a = rng.standard_normal(30)
    b = rng.random(30) + 0.1
    th, w = oracle.ritz(a, b)
    t = np.diag(a) + np.diag(b[:29], 1) + np.diag(b[:29], -1)
    ev, vec = np.linalg.eigh(t)
    np.testing.assert_allclose(th, ev, atol=1e-12)
    np.testing.assert_allclose(w, vec[0] ** 2, atol=1e-12)
    assert abs(w.sum() - 1) < 1e-13


# ---- thermo ------------------------------------------------------------------------

TEMPS = oracle.log_temperatures()


def test_temperature_grid():
    assert len(TEMPS) == 200
    assert abs(TEMPS[0] - 0.05) < 1e-15 and abs(TEMPS[-1] - 10.0) < 1e-12
    assert np.allclose(np.diff(np.log(TEMPS)), math.log(200) / 199)


def _exact_trace_ftlm(n, bonds, g=1.0, n_ups=None):
    """FTLM with R = D unit vectors and N_L >= D in every sector M >= 0."""
    recs = []
    for n_up in (n_ups or range((n + 1) // 2, n + 1)):
        d = oracle.sector_dim(n, n_up)
        rec, _ = oracle.ftlm_sector(n, n_up, bonds, d, d + 5, 0, oracle.UNIT)
        recs.append(rec)
    return oracle.thermo(recs, TEMPS, n, g)


@pytest.mark.parametrize("n,bonds", [(2, graphs.dimer()), (6, graphs.ring(6)),
                                     (7, graphs.triangle() + [(2, 3, 0.5), (3, 4, 1.0), (4, 5, 0.8), (5, 6, 1.2), (0, 6, 0.3)]),
                                     (8, graphs.j1j2_ring(8, 1.0, 0.4))])
def test_exact_trace_ftlm_equals_ed(n, bonds):
    got = _exact_trace_ftlm(n, bonds, g=2.0)
    want = ed.thermo_exact(n, bonds, TEMPS, g=2.0)
    for key in ("E", "C", "chi", "lnZ"):
        np.testing.assert_allclose(got[key], want[key], rtol=1e-9, atol=1e-10)


def test_dimer_closed_form():
    # Z = 3 e^{-beta/4} + e^{3 beta/4}; E = -dlnZ/dbeta; chi T -> g^2 * ...
    got = _exact_trace_ftlm(2, graphs.dimer())
    beta = 1 / TEMPS
    z = 3 * np.exp(-beta / 4) + np.exp(3 * beta / 4)
    e = (3 * 0.25 * np.exp(-beta / 4) - 0.75 * np.exp(3 * beta / 4)) / z
    # singlet -3/4 and triplet +1/4 are one gap apart: Var(H) = p (1 - p)
    p = 3 * np.exp(-beta / 4) / z
    chi = beta * (2 * 1.0 * np.exp(-beta / 4)) / z  # M = +-1 triplet states
    np.testing.assert_allclose(got["lnZ"], np.log(z), rtol=1e-12)
    np.testing.assert_allclose(got["E"], e, rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(got["C"], beta ** 2 * p * (1 - p), rtol=1e-7, atol=1e-14)
    np.testing.assert_allclose(got["chi"], chi, rtol=1e-11, atol=1e-14)


def test_high_temperature_limits_any_r():
    # beta -> 0 with normalized vectors: Z = sum_G g_G D_G = 2^N and
    # chi T -> g^2 N / 4, for any R; C T^2 -> (3/16) sum J^2, E T -> -(3/16) sum J^2
    n = 10
    bonds = graphs.random_cluster(n, np.random.default_rng(4))
    recs = [oracle.ftlm_sector(n, nu, bonds, 3, 30, 11, oracle.PM1)[0] for nu in range(5, 11)]
    hot = np.array([1e4, 2e4])
    out = oracle.thermo(recs, hot, n, g=1.0)
    np.testing.assert_allclose(np.exp(out["lnZ"]), 2.0 ** n, rtol=1e-3)
    np.testing.assert_allclose(out["chi"] * hot, n / 4, rtol=2e-4)
    # the exact series needs the exact trace; check it with exact-trace FTLM
    hot_out = oracle.thermo([oracle.ftlm_sector(n, nu, bonds, oracle.sector_dim(n, nu), 300, 0, oracle.UNIT)[0]
                             for nu in range(5, 11)], hot, n)
    s2 = sum(J * J for *_, J in bonds)
    sj = sum(J for *_, J in bonds)
    np.testing.assert_allclose(hot_out["C"] * hot ** 2, 3 / 16 * s2, rtol=2e-3)
    np.testing.assert_allclose(hot_out["E"] * hot, -3 / 16 * s2, rtol=2e-3)
    np.testing.assert_allclose(hot_out["chi"] * hot, n / 4 - sj / (8 * hot), rtol=1e-6)


def test_ftlm_ring12_within_stochastic_error():
    # The plain FP64 workload: N = 12 ring, S^z = 0, R = 8 +-1 vectors, M = 40.
    # Its error against ED (same sector) must sit within the spread over seeds.
    n, bonds = 12, graphs.ring(12)
    exact = ed.thermo_exact(n, bonds, TEMPS, n_ups=[6])
    runs = []
    for seed in range(1, 21):
        rec, _ = oracle.ftlm_sector(n, 6, bonds, 8, 40, seed, oracle.PM1)
        runs.append(oracle.thermo([rec], TEMPS, n)["C"])
    runs = np.array(runs)
    sigma = runs.std(axis=0)  # Eq. (22)
    dev = np.abs(runs[0] - exact["C"])
    assert np.all(dev <= 5 * sigma + 1e-9)
    pooled = np.abs(runs.mean(axis=0) - exact["C"])
    assert np.all(pooled <= 5 * sigma / math.sqrt(len(runs)) + 1e-9)
