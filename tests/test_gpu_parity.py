"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bit-exact: rank, unrank, the compressed lookup table and neighbour lists.
H.x: relative l2 error <= 1e-5 in FP32 (each row sums at most ~2 N_B + 1
terms of O(1) magnitude in FP32, so the error is a few units of 6e-8 times
the row norm) and <= 1e-13 in FP64; the CLT and CR kernels visit the bonds
in the same order and must agree bit for bit.
"""
import math

import numpy as np
import pytest

import oracle
from ftlm_inputs import graphs

pytestmark = pytest.mark.gpu

NONE = (1 << 64) - 1


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_26261_amd import ftlm
    return torch, ftlm


def _u64(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def _np_u64(t):
    return t.cpu().numpy().view(np.uint64)


SMALL = [(n, k) for n in (2, 5, 9, 12, 16) for k in range(n + 1)] + [(20, 10), (20, 7), (24, 12), (24, 23)]


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("n,n_up", SMALL)
def test_rank_unrank_exhaustive(env, mode, n, n_up):
    torch, ftlm = env
    sec = ftlm.Sector(n, n_up, mode)
    d = sec.dim
    assert d == math.comb(n, n_up)
    basis = oracle.basis(n, n_up)
    idx = _u64(torch, np.arange(d + 3))  # three indices past the end
    lab = torch.empty_like(idx)
    ftlm.unrank(sec, idx, lab)
    got = _np_u64(lab)
    np.testing.assert_array_equal(got[:d], basis)
    assert np.all(got[d:] == NONE)
    ranks = torch.empty_like(lab[:d])
    ftlm.rank(sec, lab[:d].contiguous(), ranks)
    np.testing.assert_array_equal(_np_u64(ranks), np.arange(d, dtype=np.uint64))
    # arbitrary labels, in and out of the sector and beyond 2^N
    rng = np.random.default_rng(n * 100 + n_up)
    probe = rng.integers(0, 2 ** min(n + 2, 62), size=5000, dtype=np.uint64)
    pl = _u64(torch, probe)
    pr = torch.empty_like(pl)
    ftlm.rank(sec, pl, pr)
    np.testing.assert_array_equal(_np_u64(pr), oracle.rank(n, n_up, probe))


@pytest.mark.parametrize("mode,n,n_up", [(0, 30, 15), (1, 30, 15), (1, 34, 17), (0, 28, 16), (1, 33, 20),
                                         (2, 30, 15), (3, 30, 15), (3, 31, 9)])
def test_rank_unrank_sampled_large(env, mode, n, n_up):
    torch, ftlm = env
    sec = ftlm.Sector(n, n_up, mode)
    d = sec.dim
    rng = np.random.default_rng(n + mode)
    t = np.unique(np.concatenate([rng.integers(0, d, 200000, dtype=np.uint64),
                                  np.array([0, 1, d - 1], dtype=np.uint64)]))
    want = oracle.unrank(n, n_up, t)
    ti = _u64(torch, t)
    lab = torch.empty_like(ti)
    ftlm.unrank(sec, ti, lab)
    np.testing.assert_array_equal(_np_u64(lab), want)
    back = torch.empty_like(ti)
    ftlm.rank(sec, lab, back)
    np.testing.assert_array_equal(_np_u64(back), t)


@pytest.mark.parametrize("n,n_up", [(4, 2), (5, 0), (5, 5), (9, 4), (12, 6), (16, 3), (20, 10), (24, 12)])
def test_clt_tables_exhaustive(env, n, n_up):
    torch, ftlm = env
    sec = ftlm.Sector(n, n_up, 0)
    nb = max(1, 2 ** n // 32)
    mask, prefix = ftlm.clt_export(sec, nb)
    m_o, p_o = oracle.clt(oracle.basis(n, n_up), n)
    np.testing.assert_array_equal(mask, m_o)
    np.testing.assert_array_equal(prefix, p_o)


def test_clt_tables_n30_sampled(env):
    torch, ftlm = env
    n, n_up = 30, 15
    sec = ftlm.Sector(n, n_up, 0)
    nb = 2 ** 25
    mask, prefix = ftlm.clt_export(sec, nb)
    rng = np.random.default_rng(1)
    blocks = np.unique(np.concatenate([rng.integers(0, nb, 300000), [0, nb - 1]]))
    m_o, p_o = oracle.clt_blocks(n, n_up, blocks)
    np.testing.assert_array_equal(mask[blocks], m_o)
    np.testing.assert_array_equal(prefix[blocks], p_o)
    # Eq. 18 as a running sum over all blocks, and the table's total
    pc = np.unpackbits(mask.view(np.uint8)).reshape(-1, 32).sum(axis=1)
    run = np.concatenate([[0], np.cumsum(pc)[:-1]])
    np.testing.assert_array_equal(prefix.astype(np.int64), run)
    assert pc.sum() == math.comb(30, 15)


GRAPHS = [
    (4, graphs.ring(4)),
    (9, graphs.triangle() + [(2, 3, 0.5), (3, 8, 1.1), (4, 8, 0.7), (5, 6, 1.2), (0, 6, 0.3), (7, 1, 0.9)]),
    (12, graphs.icosahedron()),
    (16, graphs.random_cluster(16, np.random.default_rng(16))),
    (20, graphs.dodecahedron()),
]


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("n,bonds", GRAPHS)
def test_neighbors_exhaustive(env, mode, n, bonds):
    torch, ftlm = env
    g = ftlm.Graph(n, bonds)
    for n_up in sorted({0, 1, n // 2, n // 2 + 1, n - 1}):
        sec = ftlm.Sector(n, n_up, mode)
        d = sec.dim
        out = torch.empty(d * g.n_bonds, dtype=torch.int64, device="cuda")
        ftlm.neighbors(sec, g, 0, d, out)
        want = oracle.neighbors(n, n_up, bonds, 0, d, oracle.basis(n, n_up))
        np.testing.assert_array_equal(_np_u64(out).reshape(d, g.n_bonds), want)


@pytest.mark.parametrize("mode,n,bonds", [
    (0, 30, graphs.icosidodecahedron()), (1, 30, graphs.icosidodecahedron()),
    (1, 30, graphs.icosidodecahedron(order="raw")), (1, 34, graphs.j1j2_ring(34, 1.0, 0.3)),
    (0, 24, graphs.square_j1j2()), (1, 24, graphs.square_j1j2()),
    (2, 30, graphs.icosidodecahedron()), (3, 30, graphs.icosidodecahedron())])
def test_neighbors_sampled_windows(env, mode, n, bonds):
    torch, ftlm = env
    n_up = n // 2
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, mode)
    d = sec.dim
    rng = np.random.default_rng(n)
    for t0 in [0, d - 777] + list(rng.integers(0, d - 777, 6)):
        t0 = int(t0)
        out = torch.empty(777 * g.n_bonds, dtype=torch.int64, device="cuda")
        ftlm.neighbors(sec, g, t0, 777, out)
        want = oracle.neighbors(n, n_up, bonds, t0, 777)
        np.testing.assert_array_equal(_np_u64(out).reshape(777, g.n_bonds), want)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("nvec", [1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 32])
@pytest.mark.parametrize("n,bonds", [(12, graphs.icosahedron()), (16, graphs.random_cluster(16, np.random.default_rng(2))),
                                     (20, graphs.dodecahedron())])
def test_hv_parity_multivector(env, nvec, n, bonds):
    torch, ftlm = env
    g = ftlm.Graph(n, bonds)
    n_up = n // 2 - (1 if n == 16 else 0)
    b = oracle.basis(n, n_up)
    d = len(b)
    rng = np.random.default_rng(nvec)
    x64 = rng.standard_normal((d, nvec))
    for dtype, tol in ((torch.float32, 1e-5), (torch.float64, 1e-13)):
        x = torch.from_numpy(x64).to(dtype).cuda().contiguous()
        xs = x.double().cpu().numpy()  # the values the kernel sees
        want = np.stack([oracle.hv(n, n_up, bonds, xs[:, c], b) for c in range(nvec)], axis=1)
        outs = []
        for mode in (0, 1, 2, 3):
            sec = ftlm.Sector(n, n_up, mode)
            y = torch.empty_like(x)
            ftlm.hv(sec, g, x, y)
            got = y.double().cpu().numpy()
            assert _rel_l2(got, want) <= tol, (mode, dtype, _rel_l2(got, want))
            outs.append(got)
        # every index map visits the bonds in the same order: bitwise the same
        for o in outs[1:]:
            np.testing.assert_array_equal(outs[0], o)


@pytest.mark.parametrize("mode", [0, 1])
def test_hv_n30_rows_sampled(env, mode):
    # the headline sector: full H.x on the GPU, exact FP64 rows from the
    # oracle at 20000 sampled rows (valid because the product is row-wise)
    torch, ftlm = env
    n, n_up = 30, 15
    bonds = graphs.icosidodecahedron()
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, mode)
    d = sec.dim
    gen = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn(d, dtype=torch.float32, device="cuda", generator=gen)
    y = torch.empty_like(x)
    ftlm.hv(sec, g, x, y)
    rows = np.unique(np.random.default_rng(0).integers(0, d, 20000).astype(np.uint64))
    xs = x.double().cpu().numpy()
    want = oracle.hv_rows(n, n_up, bonds, xs, rows)
    got = y.double().cpu().numpy()[rows.astype(np.int64)]
    assert _rel_l2(got, want) <= 1e-5
    # symmetry: u.Hv = v.Hu on the full vectors (FP64 sums of FP32 data)
    u = torch.randn(d, dtype=torch.float32, device="cuda", generator=gen)
    hu = torch.empty_like(u)
    ftlm.hv(sec, g, u, hu)
    a = torch.dot(u.double(), y.double()).item()
    bsym = torch.dot(x.double(), hu.double()).item()
    assert abs(a - bsym) <= 1e-5 * (abs(a) + 1.0) * 100


def test_hv_n30_modes_bit_identical(env):
    torch, ftlm = env
    n, n_up = 30, 15
    g = ftlm.Graph(n, graphs.icosidodecahedron())
    gen = torch.Generator(device="cuda").manual_seed(9)
    x = torch.randn(math.comb(30, 15), 4, dtype=torch.float32, device="cuda", generator=gen)
    ys = []
    for mode in (0, 1, 2, 3):
        sec = ftlm.Sector(n, n_up, mode)
        y = torch.empty_like(x)
        ftlm.hv(sec, g, x, y)
        ys.append(y)
        del sec
        torch.cuda.empty_cache()
    for y in ys[1:]:
        assert torch.equal(ys[0], y)


def test_hv_rows_shard(env):
    torch, ftlm = env
    n, n_up = 20, 10
    bonds = graphs.dodecahedron()
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, 1)
    d = sec.dim
    x = torch.randn(d, 2, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    ftlm.hv(sec, g, x, y)
    for row0, nrows in [(0, 1000), (12345, 50001), (d - 333, 333)]:
        part = torch.empty(nrows, 2, dtype=torch.float32, device="cuda")
        ftlm.hv_rows(sec, g, x, part, row0, nrows)
        assert torch.equal(part, y[row0:row0 + nrows])


@pytest.mark.parametrize("mode", [0, 1])
def test_single_vector_buffer_gathers_bitwise(env, mode):
    """A single contiguous vector is gathered through a buffer resource with
    32-bit offsets, a column of a wider block through pointers: the products
    must agree bit for bit (same partner rows, same order), in full and in
    row windows (ftlm_hv_rows), FP32 and FP64. J1-J2 4x6 lattice, S^z = 1:
    D = 2,496,144, 9751 row tiles with a ragged last one."""
    torch, ftlm = env
    n, n_up = 24, 13
    g = ftlm.Graph(n, graphs.square_j1j2())
    sec = ftlm.Sector(n, n_up, mode)
    d = sec.dim
    assert d == math.comb(24, 13) and d % 256 != 0
    gen = torch.Generator(device="cuda").manual_seed(11 + mode)
    for dtype in (torch.float32, torch.float64):
        x2 = torch.randn(d, 2, dtype=dtype, device="cuda", generator=gen)
        x = x2[:, 1].contiguous()
        y2 = torch.empty_like(x2)
        y = torch.empty_like(x)
        ftlm.hv(sec, g, x2, y2)
        ftlm.hv(sec, g, x, y)
        assert torch.equal(y, y2[:, 1]), dtype
        for row0, nrows in [(0, 777), (123457, 50001), (d - 333, 333)]:
            part = torch.empty(nrows, dtype=dtype, device="cuda")
            ftlm.hv_rows(sec, g, x, part, row0, nrows)
            assert torch.equal(part, y[row0:row0 + nrows]), (dtype, row0)


def test_hv_deterministic(env):
    torch, ftlm = env
    n, n_up = 24, 12
    g = ftlm.Graph(n, graphs.square_j1j2())
    sec = ftlm.Sector(n, n_up, 1)
    x = torch.randn(sec.dim, 8, dtype=torch.float32, device="cuda")
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    ftlm.hv(sec, g, x, y1)
    ftlm.hv(sec, g, x, y2)
    assert torch.equal(y1, y2)


@pytest.mark.parametrize("dist", [0, 1, 2])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_start_vectors_match_oracle(env, dist, dtype):
    torch, ftlm = env
    n, n_up, R, seed, r0 = 20, 10, 5, 77, 3
    sec = ftlm.Sector(n, n_up, 1)
    d = sec.dim
    code = ftlm.F32 if dtype == "f32" else ftlm.F64
    tdt = torch.float32 if dtype == "f32" else torch.float64
    work = torch.empty(ftlm.lanczos_workspace_bytes(sec, R, code), dtype=torch.uint8, device="cuda")
    q = torch.empty(d, R, dtype=tdt, device="cuda")
    norms = ftlm.start_vectors(sec, seed, r0, R, dist, q, work)
    got = q.double().cpu().numpy()
    for c in range(R):
        want = oracle.start_vector(seed, n_up, r0 + c, dist, d, normalize=False)
        if dist == 1:
            # Box-Muller through each side's own log/cos: a few ulp in FP64
            np.testing.assert_allclose(got[:, c], want.astype(got.dtype if dtype == "f64" else np.float32),
                                       rtol=4e-15 if dtype == "f64" else 1.2e-7, atol=1e-300)
        else:
            np.testing.assert_array_equal(got[:, c], want)
        assert abs(norms[c] - math.sqrt(float(np.dot(got[:, c], got[:, c])))) <= 1e-12 * norms[c]


def test_hv_n32_single_vector_high_offsets(env):
    # One FP32 vector of the J1-J2 ring N = 32 (J2 = 0.3), S^z = 0: D =
    # 601,080,390 rows, 2.4 GB, so the buffer-resource gathers of a single
    # vector take byte offsets up to 2.4e9, past 2^31. Rows on both sides of
    # row 2^29 (byte offset 2^31) and the last rows are checked against the
    # oracle, and bit for bit against a column of a two-column block (pointer
    # gathers).
    torch, ftlm = env
    n, n_up = 32, 16
    bonds = graphs.j1j2_ring(n, 1.0, 0.3)
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    d = sec.dim
    assert d == math.comb(32, 16) and d * 4 > 2 ** 31
    work = torch.empty(ftlm.lanczos_workspace_bytes(sec, 1, ftlm.F32), dtype=torch.uint8, device="cuda")
    x = torch.empty(d, dtype=torch.float32, device="cuda")
    ftlm.start_vectors(sec, 7, 0, 1, ftlm.PM1, x, work)
    del work
    y = torch.empty_like(x)
    ftlm.hv(sec, g, x, y)
    x2 = torch.empty(d, 2, dtype=torch.float32, device="cuda")
    x2[:, 0].copy_(x)
    x2[:, 1].copy_(x)
    y2 = torch.empty_like(x2)
    ftlm.hv(sec, g, x2, y2)
    del x, x2
    torch.cuda.synchronize()
    rng = np.random.default_rng(32)
    starts = sorted(set([0, 2 ** 29 - 512, 2 ** 29 + 256, d - 1024] +
                        [int(v) for v in rng.integers(0, d - 1024, 12)]))
    rows, got = [], []
    for a in starts:
        w = y.narrow(0, a, 1024)
        assert torch.equal(w, y2.narrow(0, a, 1024)[:, 0]), a
        w = w.cpu().double().numpy()
        pick = np.unique(rng.integers(0, 1024, 64))
        rows.append(a + pick)
        got.append(w[pick])
    rows = np.concatenate(rows).astype(np.uint64)
    got = np.concatenate(got)
    want = oracle.hv_rows_stream(n, n_up, bonds, 7, 0, oracle.PM1, rows)
    assert _rel_l2(got, want) <= 1e-6
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-5)


def test_hv_n34_rows_sampled(env):
    # The largest single sector: J1-J2 ring N = 34 (J1 = 1, J2 = 0.3, 68 bonds),
    # S^z = 0, D = 2,333,606,220 > 2^31, combinatorial ranking only. x is the
    # +-1 start vector of sample 0 (exact in FP32); the oracle evaluates rows
    # of H.x with x generated on demand.
    torch, ftlm = env
    n, n_up = 34, 17
    bonds = graphs.j1j2_ring(n, 1.0, 0.3)
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    d = sec.dim
    assert d == 2333606220
    work = torch.empty(ftlm.lanczos_workspace_bytes(sec, 1, ftlm.F32), dtype=torch.uint8, device="cuda")
    x = torch.empty(d, dtype=torch.float32, device="cuda")
    norms = ftlm.start_vectors(sec, 5, 0, 1, ftlm.PM1, x, work)
    assert abs(norms[0] - math.sqrt(d)) < 1e-6 * math.sqrt(d)
    del work
    y = torch.empty_like(x)
    ftlm.hv(sec, g, x, y)
    torch.cuda.synchronize()
    # Sampled rows come back through contiguous windows (narrow + copy): no
    # torch indexing kernel runs on the 2.3e9-element tensor.
    rng = np.random.default_rng(34)
    starts = sorted(set([0, 2 ** 31 - 512, 2 ** 31 + 4096, d - 1024] +
                        [int(v) for v in rng.integers(0, d - 1024, 24)]))
    rows, got = [], []
    for a in starts:
        w = y.narrow(0, a, 1024).cpu().double().numpy()
        pick = np.unique(rng.integers(0, 1024, 64))
        rows.append(a + pick)
        got.append(w[pick])
    rows = np.concatenate(rows).astype(np.uint64)
    got = np.concatenate(got)
    want = oracle.hv_rows_stream(n, n_up, bonds, 5, 0, oracle.PM1, rows)
    assert _rel_l2(got, want) <= 1e-6
    # the +-1 entries and J in {1, 0.3}: each row is a short sum; FP32 keeps it
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-5)
