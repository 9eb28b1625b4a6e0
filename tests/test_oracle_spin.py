"""Pins for the general-spin oracle (oracle/spin.py; paper Sec. 2, Eqs.
10-17, Table 1).

Anchors: Table 1's sector dimensions D_0 for the icosahedron at s = 1/2 ..
3 and its N_nz (with the memory column) for s = 1/2 .. 2; brute-force
enumeration of the label space; dense Kronecker-product Hamiltonians
(oracle/ed_spin.py, built from textbook spin matrices) for spin-1, 3/2 and 2
clusters; the closed-form spectrum of the spin-s dimer; the spin-1/2 oracle
(an independent implementation) at s = 1/2; Tr H = 0 over the full space;
and exact-trace FTLM against exact diagonalization at s = 1.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import ed_spin
from oracle import spin as sp
from ftlm_inputs import graphs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def table1():
    return json.load(open(os.path.join(GOLDEN, "paper_values.json")))["table1"]


def test_table1_sector_dimensions(table1):
    for row in table1:
        two_s = row["two_s"]
        a = sp.a_total(12, two_s, 0)
        assert sp.dim(12, two_s, a) == row["D0"], row


def test_table1_nonzeros_and_memory(table1):
    ico = graphs.icosahedron()
    assert len(ico) == 30
    for row in table1:
        if row["two_s"] > 4:
            continue  # 6^12 and 7^12 labels: beyond a unit test's scan
        two_s = row["two_s"]
        a = sp.a_total(12, two_s, 0)
        d0 = sp.dim(12, two_s, a)
        nnz = d0 + sp.offdiag_count(12, two_s, a, ico)
        assert nnz == row["Nnz"], row
        # 64-bit compressed-column storage: 16 bytes per entry + 8 (D + 1)
        mem = 16 * nnz + 8 * (d0 + 1)
        # the printed memory is rounded: within half a unit of its last digit
        assert abs(mem - row["mem_bytes"]) <= row["mem_half_unit"], (row, mem)


@pytest.mark.parametrize("n,two_s", [(5, 2), (4, 3), (3, 4), (6, 1)])
def test_dimensions_by_enumeration(n, two_s):
    total = 0
    for a in range(n * two_s + 1):
        got = sp.basis(n, two_s, a)
        assert len(got) == sp.dim(n, two_s, a)
        assert np.all(np.diff(got.astype(np.int64)) > 0)
        total += len(got)
    assert total == (two_s + 1) ** n


@pytest.mark.parametrize("n,two_s,bonds", [
    (6, 2, graphs.ring(6)),
    (4, 3, [(0, 1, 1.0), (1, 2, 0.7), (2, 3, 1.3), (3, 0, 0.4), (0, 2, -0.6)]),
    (3, 4, graphs.triangle()),
    (5, 2, [(0, 1, 0.3), (1, 2, 1.1), (2, 3, -0.8), (3, 4, 0.5), (0, 4, 1.0), (1, 3, 0.25)]),
])
def test_hv_matches_dense_hamiltonian(n, two_s, bonds):
    h = ed_spin.hamiltonian(n, two_s, bonds)
    assert abs(h - h.T).max() < 1e-14
    rng = np.random.default_rng(n * 10 + two_s)
    for a in range(n * two_s + 1):
        b = sp.basis(n, two_s, a)
        blk, idx = ed_spin.sector_block(h, n, two_s, a)
        np.testing.assert_array_equal(idx, b.astype(np.int64))
        x = rng.standard_normal(len(b))
        np.testing.assert_allclose(sp.hv(n, two_s, bonds, x, b), blk @ x, rtol=0, atol=1e-12)


@pytest.mark.parametrize("two_s", [1, 2, 3, 4, 5])
def test_dimer_closed_form(two_s):
    # two spins s: E(S) = J/2 [S(S+1) - 2 s(s+1)], S = 0 .. 2s, each (2S+1)-fold
    s = 0.5 * two_s
    J = 1.3
    want = []
    for S in range(two_s + 1):
        want += [0.5 * J * (S * (S + 1) - 2 * s * (s + 1))] * (2 * S + 1)
    got = []
    for a in range(2 * two_s + 1):
        b = sp.basis(2, two_s, a)
        m = np.stack([sp.hv(2, two_s, [(0, 1, J)], e, b) for e in np.eye(len(b))], axis=1)
        assert np.allclose(m, m.T, atol=1e-14)
        got += list(np.linalg.eigvalsh(m))
    np.testing.assert_allclose(sorted(got), sorted(want), atol=1e-12)


def test_spin_half_equals_the_spin_half_oracle():
    n, bonds = 10, graphs.random_cluster(10, np.random.default_rng(4))
    rng = np.random.default_rng(5)
    for n_up in range(n + 1):
        b = sp.basis(n, 1, n_up)
        np.testing.assert_array_equal(b, oracle.basis(n, n_up))
        x = rng.standard_normal(len(b))
        np.testing.assert_allclose(sp.hv(n, 1, bonds, x, b), oracle.hv(n, n_up, bonds, x, b), rtol=0, atol=1e-12)


def test_trace_over_the_full_space_is_zero():
    n, two_s = 6, 2
    bonds = graphs.ring(6)
    tr = 0.0
    for a in range(n * two_s + 1):
        b = sp.basis(n, two_s, a)
        tr += sum(sp.hv(n, two_s, bonds, e, b, row0=i, nrows=1)[0] for i, e in enumerate(np.eye(len(b))))
    assert abs(tr) < 1e-10


def test_exact_trace_ftlm_equals_ed_spin1():
    n, two_s = 4, 2
    bonds = [(0, 1, 1.0), (1, 2, 0.8), (2, 3, 1.2), (3, 0, 0.9), (0, 2, 0.35)]
    temps = np.geomspace(0.1, 10, 25)
    h = ed_spin.hamiltonian(n, two_s, bonds)
    recs, eall, sz2 = [], [], []
    # the sectors with M >= 0 (n * two_s is even here: M = 0 is one of them)
    for a in range(n * two_s // 2, n * two_s + 1):
        b = sp.basis(n, two_s, a)
        d = len(b)
        rec, _ = sp.ftlm_sector(n, two_s, a, bonds, d, d, 1, oracle.UNIT, basis_arr=b)
        recs.append(rec)
    th = sp.thermo(recs, temps, n, two_s)
    # exact: every sector (both signs of M, M = A - N s) from the dense spectrum
    for a in range(n * two_s + 1):
        blk, _ = ed_spin.sector_block(h, n, two_s, a)
        ev = np.linalg.eigvalsh(blk)
        eall.append(ev)
        sz2.append(np.full(len(ev), (a - 0.5 * n * two_s) ** 2))
    ev, m2 = np.concatenate(eall), np.concatenate(sz2)
    e0 = ev.min()
    for k, T in enumerate(temps):
        w = np.exp(-(ev - e0) / T)
        z = w.sum()
        E = (w * ev).sum() / z
        C = ((w * ev ** 2).sum() / z - E ** 2) / T ** 2
        chi = (w * m2).sum() / z / T
        assert abs(th["E"][k] - E) < 1e-9 * max(1, abs(E))
        assert abs(th["C"][k] - C) < 1e-8 * max(1, C)
        assert abs(th["chi"][k] - chi) < 1e-9 * max(1, chi)


@pytest.mark.parametrize("n,two_s", [(6, 2), (4, 3), (3, 4)])
def test_neighbor_lists_count_and_symmetry(n, two_s):
    bonds = graphs.ring(n) if n > 3 else graphs.triangle()
    for a in range(n * two_s + 1):
        b = sp.basis(n, two_s, a)
        nb = sp.neighbors(two_s, bonds, b, 0, len(b))
        valid = nb != sp.NONE
        # every valid term is counted once by the off-diagonal count
        assert valid.sum() == sp.offdiag_count(n, two_s, a, bonds)
        # symmetry: t reaches t' through term e of bond b iff t' reaches t
        # through the opposite term of the same bond
        for t in range(len(b)):
            for k in np.nonzero(valid[t])[0]:
                u = int(nb[t, k])
                assert nb[u, k ^ 1] == t


def test_clt_over_base_d_labels():
    n, two_s = 5, 2
    for a in range(n * two_s + 1):
        b = sp.basis(n, two_s, a)
        mask, prefix = sp.clt(b, n, two_s)
        # Alg. 2 on every label of the space equals the rank (binary search)
        for x in range(3 ** n):
            blk, j = x >> 5, x & 31
            hit = (mask[blk] >> j) & 1
            want = sp.rank(b, [x])[0]
            if hit:
                assert prefix[blk] + bin(int(mask[blk]) & ((1 << j) - 1)).count("1") == want
            else:
                assert want == sp.NONE


@pytest.mark.parametrize("n,two_s", [(6, 2), (5, 3), (4, 6), (7, 1)])
def test_counting_rank_equals_the_enumerated_basis(n, two_s):
    # The counting rank (no stored basis) against binary search in the
    # enumerated sector, over every label of [0, d^N) and every digit sum:
    # equal indices in the sector, NONE outside it; unrank inverts it.
    d = two_s + 1
    labels = np.arange(d ** n, dtype=np.uint64)
    for a in range(n * two_s + 1):
        b = sp.basis(n, two_s, a)
        want = np.full(d ** n, sp.NONE, dtype=np.uint64)
        want[b.astype(np.int64)] = np.arange(b.size, dtype=np.uint64)
        np.testing.assert_array_equal(sp.rank_count(n, two_s, a, labels), want)
        np.testing.assert_array_equal(sp.unrank_count(n, two_s, a, np.arange(b.size)), b)


@pytest.mark.parametrize("two_s,a", [(2, 12), (3, 18), (2, 15)])
def test_sampled_rows_by_counting_equal_the_enumerated_hv(two_s, a):
    # icosahedron sectors: rows picked at random, the first and the last row
    bonds = graphs.icosahedron()
    b = sp.basis(12, two_s, a)
    x = np.random.default_rng(1).standard_normal(b.size)
    rows = np.unique(np.concatenate([[0, b.size - 1], np.random.default_rng(2).choice(b.size, 300, replace=False)]))
    y = sp.hv_rows(12, two_s, a, bonds, x, rows)
    np.testing.assert_array_equal(y, sp.hv(12, two_s, bonds, x, b)[rows])
