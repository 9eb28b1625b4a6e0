"""Pins for the oracle's exact parts: sector basis, rank/unrank, the
compressed lookup table, neighbour lists and H.x.

Each check ties the oracle to something other than itself: values printed in
the paper, closed forms, brute force, or the dense Kronecker-product
Hamiltonian of oracle/ed.py (which never uses labels, ranks or lookups).
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import ed
from ftlm_inputs import graphs

NONE = oracle.NONE


# ---- sector basis and dimensions ------------------------------------------

@pytest.mark.parametrize("n", range(1, 17))
def test_sector_dims_are_binomials(n):
    # Eq. (15) at s = 1/2: D(N, A) = C(N, A); the sectors partition 2^N.
    total = 0
    for n_up in range(n + 1):
        b = oracle.basis(n, n_up)
        assert len(b) == math.comb(n, n_up) == oracle.sector_dim(n, n_up)
        assert all(bin(int(x)).count("1") == n_up for x in b)
        assert np.all(np.diff(b.astype(np.int64)) > 0)
        total += len(b)
    assert total == 2 ** n


def test_table1_dimension(golden):
    g = golden["table1_s_half"]
    assert oracle.sector_dim(g["n_sites"], g["n_sites"] // 2) == g["dim"]


def test_icosidodecahedron_dimension(golden):
    d = oracle.sector_dim(30, 15)
    assert d == 155117520
    assert abs(d - golden["sz0_dim_n30"]["dim_approx"]) / d < 0.01


# ---- rank / unrank ----------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 5, 8, 11, 14])
def test_rank_is_position_in_sorted_basis(n):
    for n_up in range(n + 1):
        b = oracle.basis(n, n_up)
        assert np.array_equal(oracle.rank(n, n_up, b), np.arange(len(b), dtype=np.uint64))
        assert np.array_equal(oracle.unrank(n, n_up, np.arange(len(b))), b)


def test_rank_rejects_labels_outside_sector():
    n, n_up = 10, 4
    labels = np.arange(1 << n, dtype=np.uint64)
    r = oracle.rank(n, n_up, labels)
    pop = np.array([bin(int(x)).count("1") for x in labels])
    assert np.all(r[pop != n_up] == NONE)
    assert np.all(r[pop == n_up] != NONE)
    # labels beyond 2^N are outside every sector
    assert oracle.rank(n, n_up, np.array([1 << n | 0b1111], dtype=np.uint64))[0] == NONE


def test_rank_matches_binary_search_and_brute_count():
    rng = np.random.default_rng(7)
    n, n_up = 20, 9
    b = oracle.basis(n, n_up)
    pick = rng.choice(len(b), 300, replace=False)
    assert np.array_equal(oracle.rank_bsearch(b, b[pick]), pick.astype(np.uint64))
    assert np.array_equal(oracle.rank(n, n_up, b[pick]), pick.astype(np.uint64))
    # brute force count of smaller sector labels for a few labels
    for t in pick[:5]:
        x = int(b[t])
        brute = sum(1 for y in range(x) if bin(y).count("1") == n_up)
        assert brute == t


def test_rank_at_n34_sampled():
    # N = 34 cannot be enumerated here; rank and unrank must invert each other
    # and be strictly increasing in the label.
    n, n_up = 34, 17
    d = oracle.sector_dim(n, n_up)
    assert d == 2333606220 and d > 2 ** 31 - 1 and d < 2 ** 32
    rng = np.random.default_rng(3)
    t = np.sort(rng.choice(d, 2000, replace=False).astype(np.uint64))
    t = np.concatenate([np.array([0, 1, d - 2, d - 1], dtype=np.uint64), t])
    t = np.unique(t)
    lab = oracle.unrank(n, n_up, t)
    assert np.all(np.diff(lab.astype(np.uint64)) > 0)
    assert all(bin(int(x)).count("1") == n_up for x in lab)
    assert np.array_equal(oracle.rank(n, n_up, lab), t)
    assert int(lab[0]) == (1 << n_up) - 1
    assert int(lab[-1]) == ((1 << n_up) - 1) << (n - n_up)


# ---- compressed lookup table -------------------------------------------------

def test_clt_worked_example(golden):
    g = golden["clt_worked_example"]
    blk = 5
    earlier = [3, 40, 77, 100]  # some sector labels in earlier blocks
    labels = sorted(earlier + [32 * blk + o for o in g["offsets_in_block"]])
    mask, prefix = oracle.clt(np.array(labels, dtype=np.uint64), 9)
    assert mask[blk] == int(g["mask_binary"], 2)
    got = oracle.clt_lookup(mask, prefix, 32 * blk + g["query_offset"])
    assert got - int(prefix[blk]) == g["index_minus_prefix"]
    assert int(prefix[blk]) == len(earlier)
    assert got == labels.index(32 * blk + g["query_offset"])


@pytest.mark.parametrize("n", [3, 6, 10, 13, 16])
def test_clt_lookup_equals_rank(n):
    for n_up in range(n + 1):
        b = oracle.basis(n, n_up)
        mask, prefix = oracle.clt(b, n)
        assert mask.size == max(1, (2 ** n + 31) // 32)
        xs = np.arange(2 ** n, dtype=np.uint64) if n <= 10 else \
            np.random.default_rng(n).integers(0, 2 ** n, 3000).astype(np.uint64)
        want = oracle.rank(n, n_up, xs)
        got = np.array([oracle.clt_lookup(mask, prefix, int(x)) for x in xs], dtype=np.uint64)
        np.testing.assert_array_equal(got, want)


def test_clt_block_masks_closed_form():
    # Derived: a block b's labels 32b + j share the high bits of b, so its
    # mask is the set of 5-bit j with popcount(j) = n_up - popcount(b).
    n, n_up = 16, 7
    mask, _ = oracle.clt(oracle.basis(n, n_up), n)
    t5 = [sum(1 << j for j in range(32) if bin(j).count("1") == q) for q in range(6)]
    for b in range(mask.size):
        q = n_up - bin(b).count("1")
        assert int(mask[b]) == (t5[q] if 0 <= q <= 5 else 0)


def test_clt_and_table4_sizes(golden):
    # Eq. (21): 8 bytes per block of 32 labels; Table 4 and the CLT paragraph.
    n = 30
    d = oracle.sector_dim(n, 15)
    clt_bytes = 8 * math.ceil(2 ** n / 32)
    assert round(clt_bytes / 1e6) == golden["clt_size_n30"]["clt_mb"]
    assert round(4 * 2 ** n / 1e9, 1) == golden["clt_size_n30"]["full_table_gb"]
    t4 = golden["table4_icosidodecahedron"]
    assert round(clt_bytes / 1e6) == t4["clt_mb"]
    assert round(4 * d / 1e6, -1) == t4["basis_mb"]
    # 7445.6 MB printed as 7440 (truncated to tens)
    assert abs(3 * t4["batch"] * d * 4 / 1e6 - t4["vectors_mb"]) < 10
    assert abs((clt_bytes + 4 * d + 3 * t4["batch"] * d * 4) / 1e6 - t4["total_mb"]) < 10


# ---- neighbour lists ---------------------------------------------------------

def test_table1_nonzero_count(golden):
    g = golden["table1_s_half"]
    bonds = graphs.icosahedron()
    assert len(bonds) == g["n_bonds"]
    n = g["n_sites"]
    nb = oracle.neighbors(n, n // 2, bonds, 0, g["dim"], oracle.basis(n, n // 2))
    nnz = g["dim"] + int(np.count_nonzero(nb != NONE))
    assert nnz == g["nnz"]
    assert round((16 * nnz + 8 * (g["dim"] + 1)) / 1e6, 2) == g["memory_mb"]


@pytest.mark.parametrize("maker,n", [(graphs.ring, 10), (graphs.icosahedron, 12),
                                     (graphs.dodecahedron, 20)])
def test_flip_count_eq10(maker, n):
    # Eq. (10) at s = 1/2: off-diagonal count = 2 N_B C(N-2, n_up-1).
    bonds = maker(n) if maker is graphs.ring else maker()
    for n_up in ([n // 2, n // 2 + 1] if n > 12 else range(n + 1)):
        d = oracle.sector_dim(n, n_up)
        b = oracle.basis(n, n_up)
        nb = oracle.neighbors(n, n_up, bonds, 0, d, b)
        want = 2 * len(bonds) * math.comb(n - 2, n_up - 1) if n_up >= 1 else 0
        assert np.count_nonzero(nb != NONE) == want


def test_neighbors_symmetric_and_valid():
    n, n_up = 12, 5
    bonds = graphs.random_cluster(n, np.random.default_rng(11))
    b = oracle.basis(n, n_up)
    nb = oracle.neighbors(n, n_up, bonds, 0, len(b), b)
    # without a stored basis (count-based rank) the lists are identical
    assert np.array_equal(nb, oracle.neighbors(n, n_up, bonds, 0, len(b)))
    pairs = set()
    for t in range(len(b)):
        for k, (i, j, _) in enumerate(bonds):
            s = nb[t, k]
            up_i, up_j = (int(b[t]) >> i) & 1, (int(b[t]) >> j) & 1
            assert (s == NONE) == (up_i == up_j)
            if s != NONE:
                assert int(b[s]) == int(b[t]) ^ (1 << i) ^ (1 << j)
                pairs.add((t, int(s), k))
    assert all((s, t, k) in pairs for t, s, k in pairs)


# ---- H.x -----------------------------------------------------------------------

def _cases():
    rng = np.random.default_rng(5)
    yield 2, graphs.dimer()
    yield 3, graphs.triangle()
    yield 4, graphs.ring(4)
    yield 9, graphs.ring(9, 0.7)
    yield 10, graphs.j1j2_ring(10, 1.0, 0.45)
    yield 11, graphs.random_cluster(11, rng)
    yield 12, graphs.icosahedron()


@pytest.mark.parametrize("n,bonds", list(_cases()))
def test_hv_matches_dense_kronecker_hamiltonian(n, bonds):
    h = ed.hamiltonian(n, bonds)
    rng = np.random.default_rng(n)
    for n_up in range(n + 1):
        blk, idx = ed.sector_block(h, n, n_up)
        x = rng.standard_normal(len(idx))
        y = oracle.hv(n, n_up, bonds, x, oracle.basis(n, n_up))
        np.testing.assert_allclose(y, blk @ x, rtol=0, atol=1e-12)
        # the count-based rank path gives the same numbers
        np.testing.assert_array_equal(y, oracle.hv(n, n_up, bonds, x, None))


def test_hv_symmetric_and_row_ranges():
    n, n_up = 14, 7
    bonds = graphs.random_cluster(n, np.random.default_rng(2))
    b = oracle.basis(n, n_up)
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal((2, len(b)))
    hu, hv_ = oracle.hv(n, n_up, bonds, u, b), oracle.hv(n, n_up, bonds, v, b)
    assert abs(u @ hv_ - v @ hu) < 1e-10 * np.abs(u @ hv_)
    part = oracle.hv(n, n_up, bonds, v, b, row0=1000, nrows=333)
    np.testing.assert_array_equal(part, hv_[1000:1333])
    rows = np.array([0, 5, 3431, len(b) - 1], dtype=np.uint64)
    np.testing.assert_array_equal(oracle.hv_rows(n, n_up, bonds, v, rows, b), hv_[rows.astype(int)])


def _trace(n, n_up, bonds):
    b = oracle.basis(n, n_up)
    tr = 0.0
    for t in range(len(b)):
        e = np.zeros(len(b))
        e[t] = 1.0
        tr += oracle.hv(n, n_up, bonds, e, b, row0=t, nrows=1)[0]
    return tr


def test_sector_traces_closed_form_and_total_zero():
    # Tr_M H = sum_b (J_b/4)[C(N-2, n-2) + C(N-2, n) - 2 C(N-2, n-1)];
    # summed over all sectors Tr H = 0 (traceless s_i . s_j).
    n = 10
    bonds = graphs.random_cluster(n, np.random.default_rng(1))
    total = 0.0
    for n_up in range(n + 1):
        c = math.comb
        closed = sum(J / 4 for *_, J in bonds) * (
            (c(n - 2, n_up - 2) if n_up >= 2 else 0) + c(n - 2, n_up) - 2 * (c(n - 2, n_up - 1) if n_up >= 1 else 0))
        tr = _trace(n, n_up, bonds)
        assert abs(tr - closed) < 1e-9
        total += tr
    assert abs(total) < 1e-9
    # N = 12 ring, S^z = 0: 12 * (1/4) * (210 + 210 - 2 * 252) = -252
    assert abs(_trace(12, 6, graphs.ring(12)) + 252.0) < 1e-9


def test_trace_h_squared():
    # Tr H^2 / 2^N = (3/16) sum_b J_b^2 over the full space.
    n = 9
    bonds = graphs.random_cluster(n, np.random.default_rng(9))
    acc = 0.0
    for n_up in range(n + 1):
        b = oracle.basis(n, n_up)
        for t in range(len(b)):
            e = np.zeros(len(b))
            e[t] = 1.0
            col = oracle.hv(n, n_up, bonds, e, b)
            acc += col @ col
    assert abs(acc / 2 ** n - 3 / 16 * sum(J * J for *_, J in bonds)) < 1e-10


def _sector_matrix(n, n_up, bonds):
    b = oracle.basis(n, n_up)
    cols = []
    for t in range(len(b)):
        e = np.zeros(len(b))
        e[t] = 1.0
        cols.append(oracle.hv(n, n_up, bonds, e, b))
    return np.array(cols).T


@pytest.mark.parametrize("n,bonds,expected", [
    (2, graphs.dimer(), [-0.75, 0.25, 0.25, 0.25]),
    (3, graphs.triangle(), [-0.75] * 4 + [0.75] * 4),
    (4, graphs.ring(4), [-2.0] + [-1.0] * 3 + [0.0] * 7 + [1.0] * 5),
])
def test_closed_form_spectra(n, bonds, expected):
    ev = np.concatenate([np.linalg.eigvalsh(_sector_matrix(n, k, bonds)) for k in range(n + 1)])
    np.testing.assert_allclose(np.sort(ev), np.sort(expected), atol=1e-12)
    dimer0 = np.linalg.eigvalsh(_sector_matrix(2, 1, graphs.dimer()))
    np.testing.assert_allclose(dimer0, [-0.75, 0.25], atol=1e-12)


def test_ed_pin_itself_closed_forms():
    # the dense Kronecker Hamiltonian reproduces the same closed forms
    for n, bonds, exp in [(2, graphs.dimer(), [-0.75, 0.25, 0.25, 0.25]),
                          (4, graphs.ring(4), [-2.0] + [-1.0] * 3 + [0.0] * 7 + [1.0] * 5)]:
        ev = np.linalg.eigvalsh(ed.hamiltonian(n, bonds).toarray())
        np.testing.assert_allclose(np.sort(ev), np.sort(exp), atol=1e-12)


def test_full_table_and_block_definitions_agree():
    # the full lookup table and the per-block CLT definition (used where the
    # basis is too large to scan) against the basis-based forms
    n, n_up = 18, 8
    bonds = graphs.random_cluster(n, np.random.default_rng(6))
    b = oracle.basis(n, n_up)
    table = oracle.full_table(n, b)
    labels = np.arange(2 ** n, dtype=np.uint64)
    r = oracle.rank(n, n_up, labels)
    np.testing.assert_array_equal(table.astype(np.uint64), np.where(r == NONE, np.uint64(0xFFFFFFFF), r))
    x = np.random.default_rng(1).standard_normal(len(b))
    np.testing.assert_array_equal(oracle.hv_table(n, n_up, bonds, x, b, table), oracle.hv(n, n_up, bonds, x, b))
    mask, prefix = oracle.clt(b, n)
    blocks = np.arange(mask.size)
    m2, p2 = oracle.clt_blocks(n, n_up, blocks)
    np.testing.assert_array_equal(mask, m2)
    np.testing.assert_array_equal(prefix, p2)


def test_hv_rows_on_streamed_vectors():
    # generating x on demand gives the rows of H.x on the stored vector
    n, n_up = 14, 6
    bonds = graphs.random_cluster(n, np.random.default_rng(12))
    b = oracle.basis(n, n_up)
    for dist in (oracle.PM1, oracle.GAUSS):
        x = oracle.start_vector(8, n_up, 3, dist, len(b), normalize=False)
        rows = np.array([0, 17, 1000, len(b) - 1], dtype=np.uint64)
        np.testing.assert_allclose(oracle.hv_rows_stream(n, n_up, bonds, 8, 3, dist, rows),
                                   oracle.hv(n, n_up, bonds, x, b)[rows.astype(int)], rtol=0, atol=1e-12)


def test_paper_cpu_method_equals_the_oracle():
    """The batched B = 8 CLT CPU kernel timed by the CPU baseline (the paper's
    CPU method, not an oracle definition) computes the oracle's H.x."""
    from oracle import paper_cpu
    n, n_up = 16, 7
    bonds = graphs.random_cluster(16, np.random.default_rng(8))
    b = oracle.basis(n, n_up)
    mask, prefix = oracle.clt(b, n)
    x = np.random.default_rng(9).standard_normal((len(b), 8))
    got = paper_cpu.hv_clt_b8(bonds, b, mask, prefix, x)
    for c in range(8):
        np.testing.assert_allclose(got[:, c], oracle.hv(n, n_up, bonds, x[:, c], b), rtol=0, atol=1e-12)
    part = paper_cpu.hv_clt_b8(bonds, b, mask, prefix, x, row0=100, nrows=333)
    np.testing.assert_array_equal(part, got[100:433])
