"""The continuous-batching request server on the GPU.

* A served request gives exactly (bit for bit) the thermodynamics of the
  same job run directly through ftlm_lanczos + ftlm_ritz + ftlm_thermo.
* The same requests give identical results alone and in a mix that overlaps
  on the device, also when admission is throttled by a small arena (memory
  pressure) or by max_active.
* A request that can never fit is rejected at submission.
* Served thermodynamics agree with the FP64 oracle.
"""
import math
import time

import numpy as np
import pytest

import oracle
from ftlm_inputs import graphs
from ftlm_inputs.requests import exchange_fit_stream

pytestmark = pytest.mark.gpu

TEMPS = oracle.log_temperatures(40)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_26261_amd import driver, ftlm
    return torch, ftlm, driver


def _small_stream(count, seed):
    return exchange_fit_stream(count, seed=seed, rate=400.0, n_range=(10, 17), R=8, M=40)


def _wait_all(server, ids, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(ids):
        for rid in ids:
            if rid not in out:
                r = server.poll(rid)
                if r is not None:
                    out[rid] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.001)
    return out


def _direct(ftlm, driver, req, mode, dtype):
    g = ftlm.Graph(req["n_sites"], req["bonds"])
    sec = ftlm.Sector(req["n_sites"], req["n_up"], mode)
    rec = driver.sector_samples(sec, g, req["R"], req["M"], req["seed"], ftlm.PM1, dtype)
    return ftlm.thermo(req["n_sites"], [rec], TEMPS, 1.0)


@pytest.mark.parametrize("mode,steps_per_round", [(0, 0), (1, 0), (1, 1), (1, 7)])
def test_served_equals_direct(env, mode, steps_per_round):
    # several Lanczos steps per round: requests finish inside a round and
    # their remaining launches must leave them untouched
    torch, ftlm, driver = env
    reqs = _small_stream(8, seed=11)
    srv = ftlm.Server(1 << 30, mode=mode, dtype=ftlm.F32, steps_per_round=steps_per_round)
    ids = [srv.submit(q["n_sites"], q["bonds"], q["n_up"], q["R"], q["M"], q["seed"], ftlm.PM1, TEMPS) for q in reqs]
    res = _wait_all(srv, ids)
    for q, rid in zip(reqs, ids):
        want = _direct(ftlm, driver, q, mode, ftlm.F32)
        for key in ("E", "C", "chi", "lnZ"):
            np.testing.assert_array_equal(res[rid][key], want[key])
        assert res[rid]["t_submit"] <= res[rid]["t_admit"] <= res[rid]["t_done"]
        assert res[rid]["dim"] == math.comb(q["n_sites"], q["n_up"])
    srv.close()


def test_alone_and_in_the_mix_identical(env):
    torch, ftlm, driver = env
    reqs = _small_stream(20, seed=12)
    # alone: one request on the server at a time
    srv = ftlm.Server(1 << 30, mode=ftlm.CR, dtype=ftlm.F32)
    alone = {}
    for k, q in enumerate(reqs):
        rid = srv.submit(q["n_sites"], q["bonds"], q["n_up"], q["R"], q["M"], q["seed"], ftlm.PM1, TEMPS)
        alone[k] = _wait_all(srv, [rid])[rid]
    srv.close()
    # in the mix: arrivals while others run; an arena that holds only a few
    # requests at once (memory-based admission) and a cap on active requests
    sizes = [ftlm.server_request_bytes(q["n_sites"], q["bonds"], q["n_up"], q["R"], q["M"], ftlm.CR, ftlm.F32)
             for q in reqs]
    for arena, cap in ((int(2.5 * max(sizes)) + (1 << 20), 0), (1 << 30, 3)):
        srv = ftlm.Server(arena, mode=ftlm.CR, dtype=ftlm.F32, max_active=cap)
        t0 = srv.clock()
        ids = []
        for q in reqs:
            while srv.clock() - t0 < q["t"]:
                time.sleep(0.0002)
            ids.append(srv.submit(q["n_sites"], q["bonds"], q["n_up"], q["R"], q["M"], q["seed"], ftlm.PM1, TEMPS))
        res = _wait_all(srv, ids)
        overlapped = any(res[ids[i + 1]]["t_admit"] < res[ids[i]]["t_done"] for i in range(len(ids) - 1))
        assert overlapped, "requests never overlapped on the device"
        for k, rid in enumerate(ids):
            for key in ("E", "C", "chi", "lnZ"):
                np.testing.assert_array_equal(res[rid][key], alone[k][key])
        assert srv.stats()["peak_bytes"] <= arena
        srv.close()


def test_request_too_big_is_rejected(env):
    torch, ftlm, driver = env
    srv = ftlm.Server(64 << 20, mode=ftlm.CR, dtype=ftlm.F32)
    bonds = graphs.ring(24)
    with pytest.raises(ftlm.FtlmError) as e:
        srv.submit(24, bonds, 12, 16, 80, 1, ftlm.PM1, TEMPS)
    assert e.value.code == ftlm.E_REJECTED
    # a small request still goes through afterwards
    rid = srv.submit(10, graphs.ring(10), 5, 4, 20, 1, ftlm.PM1, TEMPS)
    assert _wait_all(srv, [rid])[rid]["steps"] > 0
    srv.close()


def test_served_against_oracle(env):
    torch, ftlm, driver = env
    reqs = _small_stream(3, seed=13)
    srv = ftlm.Server(1 << 30, mode=ftlm.CLT, dtype=ftlm.F32)
    ids = [srv.submit(q["n_sites"], q["bonds"], q["n_up"], q["R"], q["M"], q["seed"], ftlm.PM1, TEMPS) for q in reqs]
    res = _wait_all(srv, ids)
    for q, rid in zip(reqs, ids):
        rec, _ = oracle.ftlm_sector(q["n_sites"], q["n_up"], q["bonds"], q["R"], q["M"], q["seed"], oracle.PM1)
        want = oracle.thermo([rec], TEMPS, q["n_sites"])
        for key in ("E", "C"):
            scale = np.max(np.abs(want[key]))
            assert np.all(np.abs(res[rid][key] - want[key]) <= 1e-4 * scale + 1e-12)
    srv.close()


def test_binding_imported_before_torch(env):
    # a fresh process that loads the binding before anything imports torch:
    # the library must still share torch's HIP runtime (a server is the
    # first object whose setup calls HIP directly)
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2605_26261_amd import ftlm\n"
            "from ftlm_inputs import graphs\n"
            "s = ftlm.Server(1 << 28, mode=ftlm.CR, dtype=ftlm.F32)\n"
            "rid = s.submit(10, graphs.ring(10), 5, 4, 20, 1, ftlm.PM1, [1.0])\n"
            "import time\n"
            "t0 = time.time()\n"
            "while s.poll(rid) is None:\n"
            "    assert time.time() - t0 < 60\n"
            "    time.sleep(0.001)\n"
            "s.close()\n"
            "print('served')\n") % root
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=110)
    assert r.returncode == 0 and "served" in r.stdout, r.stderr[-2000:]
