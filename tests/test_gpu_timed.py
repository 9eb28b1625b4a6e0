"""Oracle parity at the launch configurations the benchmark times.

* The plain multi-vector H.x (ftlm_hv) of the N = 30 icosidodecahedron
  sector (D = 155,117,520) at every block width the benchmark sweeps, in both
  index maps, and of the N = 34 J1-J2 ring sector (D = 2,333,606,220) at four
  columns. x holds the unnormalized start vectors of samples 0..B-1, so the
  oracle evaluates exact FP64 rows of H.x with x generated on demand (the
  product is row-wise, Eq. 12). Every column is compared on >= 20,000 sampled
  rows: relative l2 error <= 1e-5 and an absolute bound per row. Rows are
  read back through contiguous windows (narrow + copy), never by torch
  indexing on tensors above 2^31 elements.
* The Lanczos-epilogue H.x launches of the FTLM pass: every chain of the
  N = 30 workload's 20 (in the block splits the autotuner chooses between)
  against the oracle's first two Lanczos steps, and the four chains of the
  N = 34 workload against the oracle's first step.
"""
import json
import os

import numpy as np
import pytest

import oracle
from ftlm_inputs import graphs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
WINDOW = 1024


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_26261_amd import ftlm
    return torch, ftlm


def _windows(d, rng, n_windows):
    """Window starts: the first and last full windows, one across 2^31 when
    the sector is that large, and random ones (all checked to fit)."""
    starts = {0, d - WINDOW}
    if d > 2 ** 31 + WINDOW:
        starts.add(2 ** 31 - WINDOW // 2)
    starts.update(int(v) for v in rng.integers(0, d - WINDOW, n_windows))
    starts = sorted(starts)
    assert all(0 <= a and a + WINDOW <= d for a in starts)
    return starts


def _sampled_rows(y, d, rng, n_windows, per_window):
    """(rows, values [rows][B]) of y [D] or [D][B] from windows of y."""
    rows, vals = [], []
    for a in _windows(d, rng, n_windows):
        w = y.narrow(0, a, WINDOW).cpu().double().numpy()
        pick = np.sort(rng.choice(WINDOW, per_window, replace=False))
        rows.append(a + pick)
        vals.append(w[pick])
    return np.concatenate(rows).astype(np.uint64), np.concatenate(vals)


def _check_columns(got, rows, n, n_up, bonds, seed, dist):
    got = got.reshape(len(rows), -1)
    for c in range(got.shape[1]):
        want = oracle.hv_rows_stream(n, n_up, bonds, seed, c, dist, rows)
        d = np.abs(got[:, c] - want)
        rel = float(np.linalg.norm(got[:, c] - want) / np.linalg.norm(want))
        assert rel <= 1e-5, (c, rel)
        # each row sums <= 2 N_B + 1 terms of O(1) in FP32 from FP32-rounded x
        assert d.max() <= 1e-4, (c, d.max(), rows[d.argmax()])


@pytest.mark.parametrize("mode,nvec", [(m, b) for m in (0, 1) for b in (1, 4, 8, 10, 12, 16, 20, 32)]
                         + [(m, b) for m in (2, 3) for b in (1, 8, 12)])
def test_hv_n30_every_column(env, mode, nvec):
    torch, ftlm = env
    n, n_up, seed = 30, 15, 2
    bonds = graphs.icosidodecahedron()
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, mode)
    d = sec.dim
    work = torch.empty(ftlm.lanczos_workspace_bytes(sec, nvec, ftlm.F32), dtype=torch.uint8, device="cuda")
    x = torch.empty((d, nvec) if nvec > 1 else (d,), dtype=torch.float32, device="cuda")
    ftlm.start_vectors(sec, seed, 0, nvec, ftlm.GAUSS, x, work)
    del work
    y = torch.empty_like(x)
    ftlm.hv(sec, g, x, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(100 * mode + nvec)
    rows, got = _sampled_rows(y, d, rng, 40, 600)
    assert len(rows) >= 20000
    _check_columns(got, rows, n, n_up, bonds, seed, oracle.GAUSS)
    del x, y, sec
    torch.cuda.empty_cache()


def test_hv_n34_four_columns(env):
    torch, ftlm = env
    n, n_up, seed = 34, 17, 5
    bonds = graphs.j1j2_ring(n, 1.0, 0.3)
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    d = sec.dim
    assert d == 2333606220
    work = torch.empty(ftlm.lanczos_workspace_bytes(sec, 4, ftlm.F32), dtype=torch.uint8, device="cuda")
    x = torch.empty(d, 4, dtype=torch.float32, device="cuda")
    ftlm.start_vectors(sec, seed, 0, 4, ftlm.GAUSS, x, work)
    del work
    y = torch.empty_like(x)
    ftlm.hv(sec, g, x, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(34)
    rows, got = _sampled_rows(y, d, rng, 40, 600)
    assert len(rows) >= 20000
    _check_columns(got, rows, n, n_up, bonds, seed, oracle.GAUSS)
    del x, y, sec
    torch.cuda.empty_cache()


# The launch splits of the 20 chains between which the autotuner chooses
# (its pick is a fixed-width batch loop over r0 = 0, b, 2b, ...).
SPLITS = {20: [(0, 20)], 12: [(0, 12), (12, 8)], 10: [(0, 10), (10, 10)], 8: [(0, 8), (8, 8), (16, 4)],
          4: [(r, 4) for r in range(0, 20, 4)]}


@pytest.mark.parametrize("batch", [20, 12, 10, 8, 4])
def test_icosidodecahedron_every_chain_first_steps(env, batch):
    path = os.path.join(GOLDEN, "icosidodecahedron_first_steps.json")
    torch, ftlm = env
    ref = json.load(open(path))
    n, n_up = ref["n_sites"], ref["n_up"]
    g = ftlm.Graph(n, [tuple(b) for b in ref["bonds"]])
    # the stored-map variants (full table, Lin's tables) at the autotuned split
    modes = (ftlm.CLT, ftlm.CR) + ((ftlm.FULL, ftlm.LIN) if batch == 12 else ())
    for mode in modes:
        sec = ftlm.Sector(n, n_up, mode)
        alpha = np.zeros((20, 3))
        beta = np.zeros((20, 3))
        for r0, b in SPLITS[batch]:
            a, bt, s = ftlm.lanczos(sec, g, ref["seed"], r0, b, 3, ftlm.GAUSS, ftlm.F32)
            assert np.all(s == 3)
            alpha[r0:r0 + b], beta[r0:r0 + b] = a, bt
        for smp in ref["samples"]:
            r = smp["r"]
            for k in range(ref["steps"]):
                # FP32 vectors, FP64 sums: a few FP32 roundoffs of the scale
                assert abs(alpha[r, k] - smp["alpha"][k]) <= 2e-6, (mode, r, k, alpha[r, k], smp["alpha"][k])
                assert abs(beta[r, k] - smp["beta"][k]) <= 2e-6 * smp["beta"][k], (mode, r, k)
        del sec
        torch.cuda.empty_cache()


def test_ring34_four_chains_first_step(env):
    path = os.path.join(GOLDEN, "ring34_first_step.json")
    if not os.path.exists(path):
        pytest.skip("reference not generated")
    torch, ftlm = env
    ref = json.load(open(path))
    n, n_up = ref["n_sites"], ref["n_up"]
    g = ftlm.Graph(n, graphs.j1j2_ring(n, 1.0, ref["j2"]))
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    a, b, s = ftlm.lanczos(sec, g, ref["seed"], 0, 4, 2, ftlm.PM1, ftlm.F32)
    assert np.all(s == 2)
    # +-1 entries are exact in FP32 and the sums over 2.3e9 rows run in FP64,
    # but every row of H.x is summed in FP32 from terms of size up to
    # sum|J|/2; that rounding does not average out (the diagonal of a row is
    # the same FP32 sum for every row with the same bond pattern), so alpha_1
    # carries a bias of a few units of 2^-24 sum|J|
    tol_a = 2 * 2.0 ** -24 * sum(abs(J) for _, _, J in graphs.j1j2_ring(n, 1.0, ref["j2"]))
    for smp in ref["samples"]:
        r = smp["r"]
        assert abs(a[r, 0] - smp["alpha"][0]) <= tol_a, (r, a[r, 0], tol_a)
        assert abs(b[r, 0] - smp["beta"][0]) <= 1e-6 * smp["beta"][0], (r, b[r, 0])
    del sec
    torch.cuda.empty_cache()
