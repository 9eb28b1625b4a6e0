"""Edge cases of the GPU entry points, through the C-ABI.

* Argument errors come back as the documented codes and launch nothing:
  widths outside [1, 64], row ranges past the sector, overlapping x and y,
  a graph of another size, bad dtype and distribution codes, Lanczos chain
  and step counts out of range, a workspace that is too small or misaligned.
* An empty row range writes nothing.
* Degenerate sectors: D = 1 (all spins down or all up; every bond parallel,
  so H x = (sum_b J_b / 4) x), and sectors smaller than one 256-row tile,
  at every kernel width, against the FP64 oracle.
* Vector blocks whose base pointer or row stride is not 16-byte aligned run
  on the narrower kernel widths and give the same product.
* The Lanczos update's two paths (rows staged through LDS when a launch
  covers whole rows, per-thread strided rows when it covers part of a wider
  block) give bitwise the same chains, at every staged row size.
"""

import numpy as np
import pytest

import oracle
from ftlm_inputs import graphs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_26261_amd import ftlm
    return torch, ftlm


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _code(ftlm, fn, *args):
    with pytest.raises(ftlm.FtlmError) as e:
        fn(*args)
    return e.value.code


def test_hv_argument_errors(env):
    torch, ftlm = env
    n, n_up = 12, 6
    g = ftlm.Graph(n, graphs.ring(n))
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    d = sec.dim
    x = torch.randn(d, 2, device="cuda")
    y = torch.full_like(x, 7.0)
    lib, st = ftlm._lib, ftlm._stream(None)
    # widths outside [1, 64]
    for nvec in (0, 65, -1):
        rc = lib.ftlm_hv(sec.handle, g.handle, ftlm._dptr(x), ftlm._dptr(y), nvec, ftlm.F32, st)
        assert rc == ftlm.E_RANGE
    # a bad dtype code
    assert lib.ftlm_hv(sec.handle, g.handle, ftlm._dptr(x), ftlm._dptr(y), 2, 7, st) == ftlm.E_INVALID
    # null pointers
    assert lib.ftlm_hv(sec.handle, g.handle, None, ftlm._dptr(y), 2, ftlm.F32, st) == ftlm.E_INVALID
    # rows past the end of the sector
    part = torch.empty(11, 2, device="cuda")
    assert _code(ftlm, ftlm.hv_rows, sec, g, x, part, d - 10, 11) == ftlm.E_RANGE
    assert _code(ftlm, ftlm.hv_rows, sec, g, x, part, d + 1, 0) == ftlm.E_RANGE
    # y overlapping x
    assert _code(ftlm, ftlm.hv, sec, g, x, x) == ftlm.E_INVALID
    both = torch.randn(2 * d * 2, device="cuda")
    assert _code(ftlm, ftlm.hv, sec, g, both[: 2 * d].view(d, 2), both[d: 3 * d].view(d, 2)) == ftlm.E_INVALID
    # a graph on another number of sites
    g10 = ftlm.Graph(10, graphs.ring(10))
    assert _code(ftlm, ftlm.hv, sec, g10, x, y) == ftlm.E_INVALID
    torch.cuda.synchronize()
    # nothing above wrote y
    assert torch.all(y == 7.0)


def test_hv_rows_empty_range_writes_nothing(env):
    torch, ftlm = env
    n, n_up = 14, 7
    g = ftlm.Graph(n, graphs.ring(n))
    for mode in (ftlm.CLT, ftlm.CR):
        sec = ftlm.Sector(n, n_up, mode)
        x = torch.randn(sec.dim, device="cuda")
        y = torch.full((4,), float("nan"), device="cuda")
        for row0 in (0, 1234, sec.dim):
            ftlm.hv_rows(sec, g, x, y, row0, 0)
        torch.cuda.synchronize()
        assert torch.isnan(y).all()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n_up", [0, 12])
def test_single_state_sectors(env, mode, n_up):
    torch, ftlm = env
    n = 12
    bonds = graphs.j1j2_ring(n, 1.0, 0.45)
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, mode)
    assert sec.dim == 1
    jsum4 = sum(J for _, _, J in bonds) / 4.0
    for dtype, tol in ((torch.float32, 1e-6), (torch.float64, 1e-14)):
        for nvec in (1, 3, 8):
            x = torch.randn((1, nvec) if nvec > 1 else (1,), dtype=dtype, device="cuda")
            y = torch.empty_like(x)
            ftlm.hv(sec, g, x, y)
            want = jsum4 * x.double().cpu().numpy()
            np.testing.assert_allclose(y.double().cpu().numpy(), want, rtol=tol, atol=0)
    # the oracle agrees (its diagonal from the bond sum, not from a formula)
    xv = np.array([1.25])
    assert abs(oracle.hv(n, n_up, bonds, xv)[0] - jsum4 * 1.25) < 1e-14
    # Lanczos on one state: one step, alpha_1 = the energy, beta_1 = 0 up to
    # the rounding of the normalisation
    a, b, s = ftlm.lanczos(sec, g, 3, 0, 2, 10, ftlm.GAUSS, ftlm.F64)
    assert list(s) == [1, 1]
    np.testing.assert_allclose(a[:, 0], jsum4, rtol=1e-14)
    assert np.all(np.abs(b[:, 0]) <= 1e-12 * abs(jsum4))


@pytest.mark.parametrize("n,n_up", [(9, 4), (10, 5), (12, 2)])
@pytest.mark.parametrize("mode", [0, 1])
def test_sectors_smaller_than_a_tile(env, n, n_up, mode):
    torch, ftlm = env
    rng = np.random.default_rng(n * 10 + n_up)
    bonds = graphs.random_cluster(n, rng)
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, mode)
    d = sec.dim
    assert d < 256
    b = oracle.basis(n, n_up)
    for nvec in (1, 2, 4, 8, 10, 12, 16, 20, 32):
        dtypes = ((torch.float32, 1e-5), (torch.float64, 1e-13)) if nvec <= 16 else ((torch.float32, 1e-5),)
        x64 = rng.standard_normal((d, nvec))
        for dtype, tol in dtypes:
            x = torch.from_numpy(x64).to(dtype).cuda()
            if nvec == 1:
                x = x[:, 0].contiguous()
            y = torch.full_like(x, float("nan"))
            ftlm.hv(sec, g, x, y)
            xs = x.double().cpu().numpy().reshape(d, nvec)
            want = np.stack([oracle.hv(n, n_up, bonds, xs[:, k], b) for k in range(nvec)], axis=1)
            got = y.double().cpu().numpy().reshape(d, nvec)
            assert np.all(np.isfinite(got))
            assert _rel_l2(got, want) <= tol, (nvec, dtype)


@pytest.mark.parametrize("mode", [0, 1])
def test_misaligned_vector_blocks(env, mode):
    torch, ftlm = env
    n, n_up = 16, 8
    bonds = graphs.random_cluster(n, np.random.default_rng(3))
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, mode)
    d = sec.dim
    b = oracle.basis(n, n_up)
    gen = torch.Generator(device="cuda").manual_seed(9)
    for nvec, shift in ((7, 0), (20, 1), (8, 3), (5, 2)):
        # base pointers shifted by `shift` floats inside a larger buffer
        big_x = torch.randn(d * nvec + 8, device="cuda", generator=gen)
        big_y = torch.full((d * nvec + 8,), float("nan"), device="cuda")
        x = big_x[shift: shift + d * nvec].view(d, nvec)
        y = big_y[shift: shift + d * nvec].view(d, nvec)
        ftlm.hv(sec, g, x, y)
        xs = x.double().cpu().numpy()
        want = np.stack([oracle.hv(n, n_up, bonds, xs[:, k], b) for k in range(nvec)], axis=1)
        got = y.double().cpu().numpy()
        assert _rel_l2(got, want) <= 1e-5, (nvec, shift)
        # the buffer outside the block is untouched
        torch.cuda.synchronize()
        assert torch.isnan(big_y[:shift]).all() and torch.isnan(big_y[shift + d * nvec:]).all()
        # the aligned, contiguous block gives the same product bit for bit
        y2 = torch.empty(d, nvec, device="cuda")
        ftlm.hv(sec, g, x.contiguous().clone(), y2)
        assert torch.equal(y2, y)


def test_lanczos_argument_errors(env):
    torch, ftlm = env
    n, n_up = 12, 6
    g = ftlm.Graph(n, graphs.ring(n))
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    need = ftlm.lanczos_workspace_bytes(sec, 4, ftlm.F32)
    work = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    lz = ftlm.lanczos
    for R in (0, 65):
        assert _code(ftlm, ftlm.lanczos_workspace_bytes, sec, R, ftlm.F32) == ftlm.E_RANGE
    assert _code(ftlm, lz, sec, g, 1, 0, 4, 0, ftlm.PM1, ftlm.F32, work) == ftlm.E_RANGE
    assert _code(ftlm, lz, sec, g, 1, 0, 4, 4097, ftlm.PM1, ftlm.F32, work) == ftlm.E_RANGE
    assert _code(ftlm, lz, sec, g, 1, 0, 4, 10, 9, ftlm.F32, work) == ftlm.E_INVALID
    assert _code(ftlm, lz, sec, g, 1, 0, 4, 10, ftlm.PM1, 5, work) == ftlm.E_INVALID
    assert _code(ftlm, lz, sec, g, 1, 0, 4, 10, ftlm.PM1, ftlm.F32, work[: need - 1]) == ftlm.E_NOSPACE
    assert _code(ftlm, lz, sec, g, 1, 0, 4, 10, ftlm.PM1, ftlm.F32, work[16:]) == ftlm.E_INVALID
    g10 = ftlm.Graph(10, graphs.ring(10))
    assert _code(ftlm, lz, sec, g10, 1, 0, 4, 10, ftlm.PM1, ftlm.F32, work) == ftlm.E_INVALID
    # the workspace as sized works, and gives the chains of a fresh buffer
    a, bt, s = lz(sec, g, 1, 0, 4, 10, ftlm.PM1, ftlm.F32, work[:need])
    a2, b2, s2 = lz(sec, g, 1, 0, 4, 10, ftlm.PM1, ftlm.F32)
    np.testing.assert_array_equal(a, a2)
    np.testing.assert_array_equal(bt, b2)
    np.testing.assert_array_equal(s, s2)


@pytest.mark.parametrize("mode", [0, 1])
def test_rank_outside_sector_is_the_sentinel(env, mode):
    torch, ftlm = env
    n, n_up = 16, 8
    sec = ftlm.Sector(n, n_up, mode)
    labs = np.array([0, 0xFF, 0x1FF, 0x7F, 1 << 16 | 0xFF, (1 << 63) | 0x7F, 0xFFFF, 0x00FF << 8],
                    dtype=np.uint64)
    want = oracle.rank(n, n_up, labs)
    inside = [bin(int(v)).count("1") == n_up and not int(v) >> n for v in labs]
    assert [int(w) != ftlm.NONE for w in want] == inside
    lt = torch.from_numpy(labs.view(np.int64)).cuda()
    idx = torch.empty_like(lt)
    ftlm.rank(sec, lt, idx)
    got = idx.cpu().numpy().view(np.uint64)
    assert [int(v) for v in got] == [int(v) for v in want]


# (dtype, R of the wide block, [(r0, width) of each of its column chunks]):
# inside the wide block every chunk runs the strided update; alone, as a
# block of its own width, it runs the staged one (32- to 128-byte rows:
# 8 FP32 columns 32 B, 10 40 B, 12 48 B, 20 80 B, 32 128 B (half tiles);
# FP64 4 columns 32 B, 16 128 B).
UPDATE_SPLITS = [
    ("f32", 28, [(0, 20), (20, 8)]),
    ("f32", 44, [(0, 32), (32, 12)]),
    ("f32", 30, [(0, 10), (10, 10), (20, 10)]),
    ("f64", 20, [(0, 16), (16, 4)]),
]


@pytest.mark.parametrize("dt,R,chunks", UPDATE_SPLITS)
def test_staged_and_strided_updates_agree(env, dt, R, chunks):
    # N = 24, S^z = 0: D = 2,704,156 rows, several 256-row tiles per
    # workgroup and a ragged last tile of 28 rows. A chain depends on its
    # sample index r0 + r only, so columns [r0, r0 + w) of the wide run equal
    # a w-chain run started at r0, bit for bit.
    torch, ftlm = env
    dtype = ftlm.F32 if dt == "f32" else ftlm.F64
    n, n_up, M, seed = 24, 12, 8, 41
    g = ftlm.Graph(n, graphs.square_j1j2(6, 4, 1.0, 0.5))
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    assert sec.dim % 256 == 28
    a, b, s = ftlm.lanczos(sec, g, seed, 0, R, M, ftlm.GAUSS, dtype)
    assert sum(w for _, w in chunks) == R
    for r0, w in chunks:
        a1, b1, s1 = ftlm.lanczos(sec, g, seed, r0, w, M, ftlm.GAUSS, dtype)
        np.testing.assert_array_equal(a[r0:r0 + w], a1)
        np.testing.assert_array_equal(b[r0:r0 + w], b1)
        np.testing.assert_array_equal(s[r0:r0 + w], s1)
    assert np.all(s == M) and np.all(b[:, : M - 1] > 0)


def test_binding_checks_buffer_shapes(env):
    # the binding refuses buffers the kernels would read or write past
    torch, ftlm = env
    n, n_up = 12, 6
    g = ftlm.Graph(n, graphs.ring(n))
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    d = sec.dim
    x = torch.randn(d, 3, device="cuda")
    for y in (torch.empty(d, 2, device="cuda"), torch.empty(d - 1, 3, device="cuda"),
              torch.empty(d, 3, dtype=torch.float64, device="cuda")):
        with pytest.raises(ValueError):
            ftlm.hv(sec, g, x, y)
    with pytest.raises(ValueError):
        ftlm.hv(sec, g, torch.randn(d + 1, device="cuda"), torch.empty(d + 1, device="cuda"))
    with pytest.raises(ValueError):
        ftlm.hv_rows(sec, g, x, torch.empty(10, 3, device="cuda"), 0, 11)
    with pytest.raises(ValueError):
        ftlm.hv(sec, g, x.half(), x.half())
    labels = torch.zeros(5, dtype=torch.int64, device="cuda")
    for idx in (torch.zeros(5, dtype=torch.int32, device="cuda"), torch.zeros(4, dtype=torch.int64, device="cuda")):
        with pytest.raises(ValueError):
            ftlm.rank(sec, labels, idx)
        with pytest.raises(ValueError):
            ftlm.unrank(sec, idx, labels)
    with pytest.raises(ValueError):
        ftlm.neighbors(sec, g, 0, 4, torch.empty(4 * g.n_bonds - 1, dtype=torch.int64, device="cuda"))
    work = torch.empty(ftlm.lanczos_workspace_bytes(sec, 3, ftlm.F32), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        ftlm.start_vectors(sec, 1, 0, 4, ftlm.PM1, x, work)
    with pytest.raises(ValueError):
        ftlm.start_vectors(sec, 1, 0, 3, ftlm.PM1, x, work[:-1])


def test_non_finite_coefficients_stop_the_chain(env):
    # couplings so large that the FP32 products overflow: every chain's
    # alpha_1 or beta_1 comes out infinite or NaN, the chain stops at step 1
    # and the call reports FTLM_E_NUMERIC (every kernel still runs to its end)
    torch, ftlm = env
    n, n_up = 12, 6
    g = ftlm.Graph(n, [(i, (i + 1) % n, 3e38) for i in range(n)])
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    R, M = 4, 20
    work = torch.empty(ftlm.lanczos_workspace_bytes(sec, R, ftlm.F32), dtype=torch.uint8, device="cuda")
    alpha = np.zeros((R, M))
    beta = np.zeros((R, M))
    steps = np.zeros(R, dtype=np.int32)
    rc = ftlm._lib.ftlm_lanczos(sec.handle, g.handle, 1, 0, R, M, ftlm.PM1, ftlm.F32, ftlm._dptr(work),
                                work.numel(), ftlm._hptr(alpha), ftlm._hptr(beta), ftlm._hptr(steps),
                                ftlm._stream(None))
    assert rc == ftlm.E_NUMERIC
    assert np.all(steps == 1)
    assert not np.all(np.isfinite(alpha[:, 0]) & np.isfinite(beta[:, 0]))
    # a sane graph on the same sector and workspace still runs every step
    g1 = ftlm.Graph(n, graphs.ring(n))
    a, b, s = ftlm.lanczos(sec, g1, 1, 0, R, M, ftlm.PM1, ftlm.F32, work)
    assert np.all(s == M) and np.all(np.isfinite(a)) and np.all(np.isfinite(b))
