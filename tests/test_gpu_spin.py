"""General local spin s on the GPU (Sec. 2, Eqs. 11-17), through the C ABI,
against the general-spin oracle (oracle/spin.py):

* sector dimensions (Eq. 15) and the stored tables (basis, compressed lookup
  table over the d^N labels) bit for bit;
* rank and unrank bit for bit, exhaustively, in both index maps, including
  labels outside the sector and outside [0, d^N);
* neighbour lists (both ladder terms of every bond) bit for bit;
* H.x in FP64 and FP32 for 1, 2, 4 and 8 columns against FP64 rows, on
  sectors spanning many row tiles with a ragged last tile;
* exact-trace FTLM (unit start vectors, R = D) equal to exact
  diagonalization of the dense Kronecker-product Hamiltonian at s = 1;
* the spin-1 icosahedron FTLM over all M >= 0 sectors (R = 4, M = 40)
  against the oracle's FP64 run with the same start vectors
  (tests/golden/icosahedron_s1.json): FP64 to rounding, FP32 well inside
  the oracle's spread over seeds.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import ed_spin
from oracle import spin as sp
from ftlm_inputs import graphs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NONE = np.uint64(np.iinfo(np.uint64).max)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_26261_amd import driver, ftlm
    return torch, ftlm, driver


CASES = [(8, 2), (6, 3), (5, 4), (4, 6)]


@pytest.mark.parametrize("n,two_s", CASES)
@pytest.mark.parametrize("mode", [0, 1])
def test_rank_unrank_tables_exhaustive(env, n, two_s, mode):
    torch, ftlm, _ = env
    d = two_s + 1
    space = np.arange(d ** n, dtype=np.uint64)
    for a in range(n * two_s + 1):
        print(f"spin case N={n} 2s={two_s} A={a} mode={mode}", flush=True)
        want = sp.basis(n, two_s, a)
        assert ftlm.sector_info_spin(n, two_s, a)[0] == len(want)
        sec = ftlm.Sector(n, a, mode, two_s=two_s)
        assert sec.dim == len(want)
        idx = torch.arange(len(want) + 3, dtype=torch.int64, device="cuda")
        lab = torch.empty_like(idx)
        ftlm.unrank(sec, idx, lab)
        got = lab.cpu().numpy().view(np.uint64)
        np.testing.assert_array_equal(got[:len(want)], want)
        assert np.all(got[len(want):] == NONE)
        labels = np.concatenate([space, np.array([d ** n, d ** n + 7, 2 ** 40], dtype=np.uint64)])
        lt = torch.from_numpy(labels.view(np.int64)).cuda()
        out = torch.empty_like(lt)
        ftlm.rank(sec, lt, out)
        r = out.cpu().numpy().view(np.uint64)
        expect = np.full(labels.size, NONE, dtype=np.uint64)
        expect[want.astype(np.int64)] = np.arange(len(want), dtype=np.uint64)
        np.testing.assert_array_equal(r, expect)
        if mode == ftlm.CLT:
            nb = (d ** n + 31) // 32
            mask, prefix = ftlm.clt_export(sec, nb)
            m_o, p_o = sp.clt(want, n, two_s)
            np.testing.assert_array_equal(mask, m_o)
            np.testing.assert_array_equal(prefix, p_o)


@pytest.mark.parametrize("n,two_s", [(8, 2), (6, 3), (5, 4)])
@pytest.mark.parametrize("mode", [0, 1])
def test_neighbors_exhaustive(env, n, two_s, mode):
    torch, ftlm, _ = env
    rng = np.random.default_rng(n + two_s)
    bonds = graphs.random_cluster(n, rng)
    g = ftlm.Graph(n, bonds)
    for a in range(n * two_s + 1):
        b = sp.basis(n, two_s, a)
        sec = ftlm.Sector(n, a, mode, two_s=two_s)
        out = torch.empty(len(b) * 2 * g.n_bonds, dtype=torch.int64, device="cuda")
        ftlm.neighbors(sec, g, 0, len(b), out)
        got = out.cpu().numpy().view(np.uint64).reshape(len(b), 2 * g.n_bonds)
        np.testing.assert_array_equal(got, sp.neighbors(two_s, bonds, b, 0, len(b)))


@pytest.mark.parametrize("n,two_s,a", [(12, 2, 12), (9, 3, 13), (8, 4, 16), (12, 2, 17)])
@pytest.mark.parametrize("mode", [0, 1])
def test_hv_against_oracle(env, n, two_s, a, mode):
    """Many row tiles with a ragged tail: D = 73,789 (spin-1 icosahedron,
    M = 0), 30,276 (9 sites, s = 3/2, A = 13), 38,165 (8 sites, s = 2, A =
    16), 16,236 (spin-1 icosahedron, M = 5)."""
    torch, ftlm, _ = env
    rng = np.random.default_rng(n * 100 + a)
    bonds = graphs.icosahedron() if n == 12 else graphs.random_cluster(n, rng)
    g = ftlm.Graph(n, bonds)
    b = sp.basis(n, two_s, a)
    sec = ftlm.Sector(n, a, mode, two_s=two_s)
    assert sec.dim == len(b) and len(b) % 256 != 0
    for dtype, tol in ((torch.float64, 1e-13), (torch.float32, 1e-5)):
        for nv in (1, 2, 4, 8):
            x = torch.randn((len(b), nv) if nv > 1 else (len(b),), dtype=dtype, device="cuda")
            y = torch.empty_like(x)
            ftlm.hv(sec, g, x, y)
            xs = x.double().cpu().numpy().reshape(len(b), -1)
            got = y.double().cpu().numpy().reshape(len(b), -1)
            for c in range(nv):
                want = sp.hv(n, two_s, bonds, xs[:, c], b)
                rel = np.linalg.norm(got[:, c] - want) / np.linalg.norm(want)
                assert rel <= tol, (dtype, nv, c, rel)


@pytest.mark.parametrize("n,two_s,a", [(12, 2, 12), (8, 4, 16)])
def test_index_maps_agree_bitwise(env, n, two_s, a):
    """Both index maps visit a row's bonds in the same order with the same
    ladder factors (the pipelined ranking pass and the grouped table lookups
    alike), so their products must agree bit for bit at every width; widths
    1 and 8 take groups of three bonds, the others groups of two, and 30 or
    the random cluster's bond count leaves a ragged last group or none."""
    torch, ftlm, _ = env
    rng = np.random.default_rng(7 * n + a)
    bonds = graphs.icosahedron() if n == 12 else graphs.random_cluster(n, rng)
    g = ftlm.Graph(n, bonds)
    cr = ftlm.Sector(n, a, ftlm.CR, two_s=two_s)
    clt = ftlm.Sector(n, a, ftlm.CLT, two_s=two_s)
    d = cr.dim
    assert clt.dim == d and d % 256 != 0
    for dtype in (torch.float32, torch.float64):
        for nv in (1, 2, 4, 8):
            x = torch.randn((d, nv) if nv > 1 else (d,), dtype=dtype, device="cuda")
            y_cr = torch.empty_like(x)
            y_clt = torch.empty_like(x)
            ftlm.hv(cr, g, x, y_cr)
            ftlm.hv(clt, g, x, y_clt)
            np.testing.assert_array_equal(y_cr.cpu().numpy(), y_clt.cpu().numpy(), err_msg=f"{dtype} B={nv}")


def test_exact_trace_ftlm_equals_ed(env):
    torch, ftlm, driver = env
    n, two_s = 5, 2
    bonds = [(0, 1, 1.0), (1, 2, 0.8), (2, 3, 1.2), (3, 4, 0.9), (4, 0, 1.1), (0, 2, 0.35)]
    temps = np.geomspace(0.1, 10, 30)
    recs = []
    for a in range(n * two_s // 2, n * two_s + 1):
        d = ftlm.sector_info_spin(n, two_s, a)[0]
        for mode in (ftlm.CR,):
            th, rr = driver.run(n, bonds, [a], d, d, 1, ftlm.UNIT, dtype=ftlm.F64, mode=mode, temps=temps,
                                two_s=two_s)
            recs += rr
    th = ftlm.thermo(n, recs, temps, 1.0)
    h = ed_spin.hamiltonian(n, two_s, bonds)
    ev, m2 = [], []
    for a in range(n * two_s + 1):
        blk, _ = ed_spin.sector_block(h, n, two_s, a)
        e = np.linalg.eigvalsh(blk)
        ev.append(e)
        m2.append(np.full(len(e), (a - 0.5 * n * two_s) ** 2))
    ev, m2 = np.concatenate(ev), np.concatenate(m2)
    e0 = ev.min()
    for k, T in enumerate(temps):
        w = np.exp(-(ev - e0) / T)
        z = w.sum()
        E = (w * ev).sum() / z
        C = ((w * ev ** 2).sum() / z - E ** 2) / T ** 2
        chi = (w * m2).sum() / z / T
        assert abs(th["E"][k] - E) < 1e-8 * max(1, abs(E))
        assert abs(th["C"][k] - C) < 1e-7 * max(1, C)
        assert abs(th["chi"][k] - chi) < 1e-8 * max(1, chi)


@pytest.mark.parametrize("mode", [0, 1])
def test_chains_same_at_every_launch_width(env, mode):
    """A chain's alpha and beta do not depend on the launch width: every
    column's row terms, epilogue and FP64 sums are taken in the same order
    whether the chain runs alone or with seven others, although the
    8-column Lanczos kernel takes two bonds per ranking slot in CR mode and
    the 1-column one takes one. Chains 0..3 of the 8-chain FP64 run also
    match the oracle's first steps (golden, M = 0 sector of the spin-1
    icosahedron, D = 73,789: many row tiles, 30 bonds)."""
    torch, ftlm, _ = env
    ref = json.load(open(os.path.join(GOLDEN, "icosahedron_s1.json")))
    n, two_s, M, seed = ref["n_sites"], ref["two_s"], ref["M"], ref["seed"]
    assert ref["dist"] == "pm1"
    g = ftlm.Graph(n, [tuple(b) for b in ref["bonds"]])
    sref = ref["sectors"][0]
    sec = ftlm.Sector(n, sref["a"], mode, two_s=two_s)
    assert sec.dim == sref["dim"] == 73789
    for dtype in (ftlm.F64, ftlm.F32):
        a8, b8, s8 = ftlm.lanczos(sec, g, seed, 0, 8, M, ftlm.PM1, dtype)
        for r0, w in ((0, 1), (3, 1), (7, 1), (2, 4), (5, 2)):
            a, b, st = ftlm.lanczos(sec, g, seed, r0, w, M, ftlm.PM1, dtype)
            np.testing.assert_array_equal(st, s8[r0:r0 + w])
            np.testing.assert_array_equal(a, a8[r0:r0 + w], err_msg=f"dtype {dtype} chains {r0}..{r0 + w - 1}")
            np.testing.assert_array_equal(b, b8[r0:r0 + w], err_msg=f"dtype {dtype} chains {r0}..{r0 + w - 1}")
        if dtype == ftlm.F64:
            for smp in sref["samples"]:
                r = smp["r"]
                k = min(10, smp["steps"])
                assert s8[r] == smp["steps"]
                np.testing.assert_allclose(a8[r, :k], smp["alpha"][:k], rtol=0, atol=1e-9)
                np.testing.assert_allclose(b8[r, :k], smp["beta"][:k], rtol=0, atol=1e-9)


@pytest.mark.parametrize("mode", [0, 1])
def test_icosahedron_s1_all_sectors_against_oracle(env, mode):
    torch, ftlm, driver = env
    path = os.path.join(GOLDEN, "icosahedron_s1.json")
    ref = json.load(open(path))
    n, two_s, R, M = ref["n_sites"], ref["two_s"], ref["R"], ref["M"]
    bonds = [tuple(b) for b in ref["bonds"]]
    temps = np.asarray(ref["temps"])
    a_list = [s["a"] for s in ref["sectors"]]
    out = {}
    for dtype in (ftlm.F64, ftlm.F32):
        th, recs = driver.run(n, bonds, a_list, R, M, ref["seed"], ftlm.PM1, dtype=dtype, mode=mode, temps=temps,
                              two_s=two_s)
        out[dtype] = th
        for rec, sref in zip(recs, ref["sectors"]):
            assert rec["dim"] == sref["dim"]
            for smp in sref["samples"]:
                r = smp["r"]
                assert rec["steps"][r] == smp["steps"]
                if dtype == ftlm.F64:
                    # the first steps agree to rounding; later ones drift apart with the
                    # loss of orthogonality (Sec. 3.2)
                    k = min(10, smp["steps"])  # a small sector's chain stops early
                    np.testing.assert_allclose(rec["alpha"][r, :k], smp["alpha"][:k], rtol=0, atol=1e-9)
                    np.testing.assert_allclose(rec["beta"][r, :k], smp["beta"][:k], rtol=0, atol=1e-9)
                else:
                    assert abs(rec["alpha"][r, 0] - smp["alpha"][0]) < 1e-5 * (1 + abs(smp["alpha"][0]))
    # FP64 equals the oracle to rounding. FP32 vectors: after M = 40 steps the
    # low levels of the large sectors are not converged, and the FP32 and FP64
    # chains, which drift apart with the loss of orthogonality (Sec. 3.2),
    # give slightly different quadratures there; an FP32-vector run of the
    # oracle's own Lanczos shows the same 8.5e-4 of max |C| at T = 0.05. The
    # bar is the paper's (Sec. 3.3): far below the stochastic error, here the
    # oracle's sigma_emp over 10 further seeds at the same R = 4 (Eq. 22)
    for k in ("E", "C", "chi"):
        o = np.asarray(ref[k])
        sig = np.asarray(ref["sigma"][k])
        scale = np.abs(o).max()
        assert np.max(np.abs(out[ftlm.F64][k] - o)) <= 1e-8 * scale, k
        d32 = np.abs(out[ftlm.F32][k] - o)
        where = sig >= 1e-3 * sig.max()
        ratio = np.max(d32[where] / sig[where])
        print(f"mode {mode} {k}: FP32 max |d| = {d32.max():.2e} ({d32.max() / scale:.1e} of max), "
              f"max |d|/sigma_emp = {ratio:.1e}", flush=True)
        assert d32.max() <= 2e-3 * scale, k
        assert ratio <= 0.03, k


# The general-spin sectors the benchmark times (icosahedron, M = 0 sectors of
# Table 1 at s = 5/2, D = 144,840,476, and s = 3, D = 786,588,243; the
# compressed table only where the d^N labels fit 32 bits), at both launch
# widths it times. x holds the unnormalized +-1 start vectors of samples
# 0..B-1 (exact in FP32); the oracle rebuilds columns 0 and B-1 in FP64 and
# evaluates sampled rows with labels and partner indices found by counting
# (Eq. 15 dimensions), so no basis of the sector is stored. Rows are read
# back through contiguous windows.
TIMED_SPIN = [(5, 0, 1), (5, 0, 8), (5, 1, 1), (5, 1, 8), (6, 1, 1), (6, 1, 8)]


@pytest.mark.parametrize("two_s,mode,nvec", TIMED_SPIN)
def test_table1_timed_sectors_sampled_rows(env, two_s, mode, nvec):
    torch, ftlm, driver = env
    n, seed, window = 12, 31, 1024
    a = n * two_s // 2
    bonds = graphs.icosahedron()
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, a, mode, two_s=two_s)
    d = sec.dim
    assert d == sp.dim(n, two_s, a)
    work = torch.empty(ftlm.lanczos_workspace_bytes(sec, nvec, ftlm.F32), dtype=torch.uint8, device="cuda")
    x = torch.empty((d, nvec) if nvec > 1 else (d,), dtype=torch.float32, device="cuda")
    ftlm.start_vectors(sec, seed, 0, nvec, ftlm.PM1, x, work)
    del work
    y = torch.empty_like(x)
    ftlm.hv(sec, g, x, y)
    torch.cuda.synchronize()
    del x
    rng = np.random.default_rng(1000 * two_s + 10 * mode + nvec)
    starts = sorted({0, d - window, *(int(v) for v in rng.integers(0, d - window, 10))})
    rows, got = [], []
    for s0 in starts:
        w = y.narrow(0, s0, window).cpu().double().numpy().reshape(window, nvec)
        pick = np.sort(rng.choice(window, 200, replace=False))
        if s0 == d - window:
            pick = np.union1d(pick, [window - 1])  # the last row
        rows.append(s0 + pick)
        got.append(w[pick])
    rows = np.concatenate(rows).astype(np.uint64)
    got = np.concatenate(got)
    del y
    torch.cuda.empty_cache()
    for c in sorted({0, nvec - 1}):
        xc = oracle.start_vector(seed, a, c, oracle.PM1, d, normalize=False)
        want = sp.hv_rows(n, two_s, a, bonds, xc, rows)
        del xc
        diff = np.abs(got[:, c] - want)
        rel = float(np.linalg.norm(got[:, c] - want) / np.linalg.norm(want))
        print(f"2s={two_s} mode {mode} B={nvec} column {c}: {rows.size} rows, rel l2 {rel:.1e}, "
              f"max |d| {diff.max():.1e}", flush=True)
        # each row sums <= 2 N_B + 1 = 61 FP32 terms of size <= J s(s+1) from
        # exact +-1 entries
        assert rel <= 1e-6, (c, rel)
        assert diff.max() <= 1e-4, (c, diff.max(), rows[diff.argmax()])
    del sec
