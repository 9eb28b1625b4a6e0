"""Pins for the oracle's precision diagnostics (Sec. 3.1-3.2): the spread
over seeds of Eq. (22) and the Cullum-Willoughby ghost test of Eq. (25) with
its Ritz clusters.

Anchors: the two-seed closed form of Eq. (22); the high-temperature spread of
the energy estimate, which for normalized +-1 vectors follows from the
variance of a quadratic form; a tridiagonal matrix whose first row is
decoupled (every eigenvalue of T1 is one of T: exact ghosts); Cauchy
interlacing of an unreduced T (no eigenvalue of T1 equals one of T); and an
FP64 Lanczos run far past convergence on a small matrix, whose Ritz clusters
carry the exact projections |<v_i|r>|^2 of the start vector.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import ed
from ftlm_inputs import graphs


def test_seed_spread_two_seeds_closed_form():
    # Eq. (22) with N_s = 2: the deviations are +-(a - b)/2, so sigma = |a - b| / 2
    a = np.array([1.0, -3.0, 0.25])
    b = np.array([2.0, 5.0, 0.25])
    mean, sig = oracle.seed_spread([a, b])
    np.testing.assert_allclose(mean, (a + b) / 2, rtol=0, atol=0)
    np.testing.assert_allclose(sig, np.abs(a - b) / 2, rtol=1e-15, atol=0)


def test_seed_spread_of_the_high_temperature_energy():
    """At T >> W the FTLM energy of one run is the mean of <r|H|r> over its R
    normalized +-1 vectors (sum_k w_k theta_k = alpha_1). For z with i.i.d.
    +-1 entries, z^T H z = Tr H + sum_{i != j} H_ij z_i z_j and |z|^2 = D, so
    Var <r|H|r> = 2 (|H|_F^2 - sum_i H_ii^2) / D^2; over runs of R vectors
    the spread is that / R."""
    n, n_up = 8, 4
    bonds = graphs.ring(n)
    h, _ = ed.sector_block(ed.hamiltonian(n, bonds), n, n_up)
    d = h.shape[0]
    var1 = 2.0 * (np.sum(h * h) - np.sum(np.diag(h) ** 2)) / d ** 2
    R, n_seeds, T = 4, 300, np.array([1e4])
    est = []
    for s in range(n_seeds):
        rec, _ = oracle.ftlm_sector(n, n_up, bonds, R, 20, 1000 + s, oracle.PM1)
        est.append(oracle.thermo([rec], T, n)["E"])
    _, sig = oracle.seed_spread(est)
    want = math.sqrt(var1 / R)
    # sampling error of a standard deviation from 300 runs: ~4 % (1 sigma)
    assert abs(sig[0] / want - 1) < 0.15, (sig[0], want)


def _tridiag(a, b):
    return np.diag(a) + np.diag(b, 1) + np.diag(b, -1)


def test_ghosts_of_a_decoupled_first_row():
    # beta_1 = 0: T = (alpha_1) + T1, so every eigenvalue of T1 is an
    # eigenvalue of T (ell = 0) and only alpha_1 is not a ghost
    a = np.array([0.3, -1.0, 0.5, 2.0, 1.2])
    b = np.array([0.0, 0.7, 0.4, 0.9])
    g = oracle.ghost_diagnostic(a, b, c_tau=1.0)
    k_alpha1 = int(np.argmin(np.abs(g["theta"] - 0.3)))
    assert abs(g["theta"][k_alpha1] - 0.3) < 1e-14
    assert not g["ghost"][k_alpha1]
    others = np.delete(np.arange(5), k_alpha1)
    assert np.all(g["ell"][others] < 1e-13)
    assert np.all(g["ghost"][others])
    # the weight of q1 = e_1 sits on alpha_1 alone
    assert abs(g["weight"][k_alpha1] - 1.0) < 1e-14


def test_no_ghosts_in_an_unreduced_tridiagonal():
    # beta_k != 0: the eigenvalues of T1 strictly interlace those of T. Near
    # a uniform chain every eigenvector has a first component of order
    # sqrt(2 / 13), so no theta_k comes close to an eigenvalue of T1.
    rng = np.random.default_rng(3)
    a = 0.1 * rng.normal(size=12)
    b = 1.0 + 0.1 * rng.uniform(size=11)
    g = oracle.ghost_diagnostic(a, b, c_tau=1.0)
    theta1 = np.linalg.eigvalsh(_tridiag(a[1:], b[1:]))
    theta = np.linalg.eigvalsh(_tridiag(a, b))
    np.testing.assert_allclose(g["theta"], theta, atol=1e-12)
    assert np.all(theta[:-1] < theta1) and np.all(theta1 < theta[1:])
    want_ell = np.array([np.min(np.abs(t - theta1)) for t in theta])
    np.testing.assert_allclose(g["ell"], want_ell, rtol=1e-9)
    assert np.all(want_ell > 1e-3)
    assert not np.any(g["ghost"])
    assert len(g["cluster_weight"]) == 12 and abs(g["cluster_weight"].sum() - 1) < 1e-13


def test_cluster_weights_far_past_convergence():
    """FP64 Lanczos without reorthogonalization, 60 steps on a sector of
    dimension 20: converged Ritz values repeat (ghosts), and the total
    weight of each cluster equals |<v_i|r>|^2 summed over the eigenvalues
    inside it (Gauss quadrature of the spectral measure of r), while the
    spurious copies carry no weight and are flagged by the deflation test."""
    n, n_up = 6, 3
    bonds = [(i, (i + 1) % n, 1.0) for i in range(n)] + [(0, 3, 0.37), (1, 4, 0.61)]
    h, _ = ed.sector_block(ed.hamiltonian(n, bonds), n, n_up)
    d = h.shape[0]
    assert d == 20
    lam, v = np.linalg.eigh(h)
    q1 = oracle.start_vector(5, n_up, 0, oracle.GAUSS, d)
    a, b, k = oracle.lanczos(lambda x: h @ x, q1, 60, eps=0.0)
    assert k == 20  # m_eff = min(M, D)
    # run on past D by hand: the same recursion, no stopping
    al, be = _lanczos_no_stop(h, q1, 60)
    # distinct eigenvalues and the weight of q1 in each eigenspace
    proj_all = (v.T @ q1) ** 2
    lev, proj = [], []
    for i in range(d):
        if lev and lam[i] - lev[-1] < 1e-9:
            proj[-1] += proj_all[i]
        else:
            lev.append(lam[i])
            proj.append(proj_all[i])
    lev, proj = np.array(lev), np.array(proj)
    # tau = 2 u_FP32 W ~ 1e-7 W: above the spread of a ghost copy that is
    # still converging, far below the smallest gap between distinct eigenvalues
    g = oracle.ghost_diagnostic(al, be, c_tau=2.0)
    assert g["tau"] < 0.01 * np.min(np.diff(lev))
    assert np.sum(g["ghost"]) >= 10  # 60 Ritz values, len(lev) distinct eigenvalues
    n_clusters = len(g["cluster_weight"])
    found = []
    for c in range(n_clusters):
        members = g["theta"][g["cluster"] == c]
        if g["cluster_weight"][c] < 1e-12:
            # a spurious copy (weight ~ 0): flagged by the deflation test
            assert np.all(g["ghost"][g["cluster"] == c]), (c, members)
            continue
        i = int(np.argmin(np.abs(lev - members.mean())))
        assert np.max(np.abs(members - lev[i])) < 1e-6, (c, members, lev[i])
        assert abs(g["cluster_weight"][c] - proj[i]) < 1e-8, (c, members)
        found.append(i)
    # every eigenspace the start vector touches has exactly one cluster
    assert sorted(found) == [i for i in range(len(lev)) if proj[i] > 1e-12]


def _lanczos_no_stop(h, q1, m):
    q, q_prev, bp = q1.copy(), np.zeros_like(q1), 0.0
    al, be = [], []
    for _ in range(m):
        w = h @ q - bp * q_prev
        a = float(q @ w)
        w -= a * q
        b = math.sqrt(float(w @ w))
        al.append(a)
        be.append(b)
        q_prev, q, bp = q, w / b, b
    return np.array(al), np.array(be)
