"""ftlm_lanczos_noalloc (the entry point for callers that cannot allocate
device memory) against ftlm_lanczos: two calls in a row, the second on a
smaller sector with fewer chains, each bitwise equal to ftlm_lanczos on a
caller-allocated workspace (same kernels, same fixed reduction order). Runs
through the C ABI.
"""
import numpy as np
import pytest

from ftlm_inputs import graphs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_26261_amd import ftlm
    return torch, ftlm


def _both(ftlm, n, n_up, bonds, mode, R, M, dist, dtype, seed):
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, n_up, mode)
    print(f"noalloc case N={n} n_up={n_up} mode={mode} R={R} M={M} dtype={dtype}", flush=True)
    want = ftlm.lanczos(sec, g, seed, 0, R, M, dist, dtype)
    got = ftlm.lanczos_noalloc(sec, g, seed, 0, R, M, dist, dtype)
    return want, got


def test_noalloc_equals_lanczos_two_calls(env):
    torch, ftlm = env
    rng = np.random.default_rng(7)
    # first call: N = 18 random cluster, 8 FP32 chains (workspace ~13 MB)
    cases = [(18, 9, graphs.random_cluster(18, rng), ftlm.CR, 8, 40, ftlm.GAUSS, ftlm.F32, 11),
             # second, smaller: N = 12 ring, 3 FP64 chains, CLT
             (12, 6, graphs.ring(12), ftlm.CLT, 3, 30, ftlm.PM1, ftlm.F64, 12)]
    for n, n_up, bonds, mode, R, M, dist, dtype, seed in cases:
        (a0, b0, s0), (a1, b1, s1) = _both(ftlm, n, n_up, bonds, mode, R, M, dist, dtype, seed)
        assert np.array_equal(s0, s1)
        assert np.all(s1 >= 1)
        assert np.array_equal(a0, a1)
        assert np.array_equal(b0, b1)
    torch.cuda.synchronize()


def test_noalloc_rejects_a_workspace_beyond_the_scratch(env):
    torch, ftlm = env
    n, n_up = 24, 12  # D = 2,704,156: 8 FP32 chains need ~173 MB
    g = ftlm.Graph(n, graphs.ring(n))
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    assert ftlm.lanczos_workspace_bytes(sec, 8, ftlm.F32) > ftlm.NOALLOC_SCRATCH_BYTES
    with pytest.raises(ftlm.FtlmError) as e:
        ftlm.lanczos_noalloc(sec, g, 1, 0, 8, 10, ftlm.PM1, ftlm.F32)
    assert e.value.code == ftlm.E_RANGE
    # the scratch is still usable afterwards
    n, n_up = 14, 7
    g = ftlm.Graph(n, graphs.ring(n))
    sec = ftlm.Sector(n, n_up, ftlm.CR)
    a0, b0, s0 = ftlm.lanczos(sec, g, 3, 0, 2, 20, ftlm.PM1, ftlm.F32)
    a1, b1, s1 = ftlm.lanczos_noalloc(sec, g, 3, 0, 2, 20, ftlm.PM1, ftlm.F32)
    assert np.array_equal(a0, a1) and np.array_equal(b0, b1) and np.array_equal(s0, s1)
