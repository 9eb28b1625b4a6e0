"""Benchmark of the FTLM hot path on one MI355X.

Workload: the spin-1/2 Heisenberg icosidodecahedron (N = 30, 60 bonds, J = 1),
S^z = 0 sector (D = C(30,15) = 155,117,520), R = 20 Gaussian start vectors
(seed 2), M = 100 Lanczos steps, FP32 vectors with FP64 alpha/beta, run with
both index maps (compressed lookup table and combinatorial ranking).

One step = one full FTLM pass over the batch: start vectors, M batched
Lanczos steps (multi-vector H.x with fused alpha, update with fused beta),
the host Ritz solves and the thermal reduction. Sector tables are built once
before timing (inputs resident in HBM). The headline value is H.x
states.bonds/s over the whole job (D * N_B per vector-H.x) for the faster
index map; the line also carries FTLM samples/s, the H.x kernel's roofline
and the FP64 CPU oracle timed on a bounded sample of the same product.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H·v states·bonds/s + HBM GB/s (N=30 S^z=0); FTLM samples/s, p50/p99 latency"
HBM_PEAK_GBS = 8000.0
N_SITES, N_UP, R, M, SEED = 30, 15, 20, 100, 2


# block widths of one FP32 Lanczos-epilogue H.x launch
LAUNCH_WIDTHS_F32 = (1, 2, 4, 8, 10, 12, 16, 20, 32)

# Bytes between the L2 and the memory side per steady-state launch of the
# dominant kernel (Lanczos-epilogue H.x over a block of FP32 columns, per
# index map and block width), from rocprofv3 FETCH_SIZE and WRITE_SIZE runs
# scaled by the counts of a 2 GiB copy and checked against request-size
# counters (profiles/hv_lanczos_n30_r20_counters.md). The memory side
# includes the Infinity Cache, so this bounds the HBM traffic from above.
# They describe the kernel sources with this hash and are dropped otherwise.
KERNEL_SOURCES = ["layout.hpp", "device.hpp", "kernels.hpp", "rowloop.hpp", "hv_impl.hpp", "hv_f32.hip"]
MEASURED_TRAFFIC = {"sources": "1123cd4f9861cbbe", "bytes": {
    "clt": {1: 19.44e9, 2: 34.19e9, 4: 65.48e9, 8: 125.77e9, 10: 160.94e9, 12: 197.3e9, 16: 272.91e9, 20: 340.19e9},
    "cr": {1: 13.41e9, 2: 26.88e9, 4: 55.84e9, 8: 112.51e9, 10: 153.01e9, 12: 190.25e9, 16: 250.94e9, 20: 338.26e9},
    "full": {1: 99.57e9, 2: 111.91e9, 4: 147.91e9, 8: 210.6e9, 10: 253.37e9, 12: 286.72e9, 16: 367.8e9, 20: 433.01e9},
    "lin": {1: 14.4e9, 2: 28.82e9, 4: 59.68e9, 8: 119.64e9, 10: 155.34e9, 12: 190.45e9, 16: 264.38e9, 20: 332.48e9}}}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_26261_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def clt_touched_bytes(n, n_up):
    """Bytes of the non-empty compressed-lookup-table blocks: block b holds
    sector labels iff 0 <= n_up - popcount(b) <= 5."""
    blocks = sum(math.comb(n - 5, k) for k in range(max(0, n_up - 5), min(n - 5, n_up) + 1))
    return 8 * blocks


def map_bytes(mode, dim, n, n_up):
    """Bytes of the stored index map a launch must read at least once: the
    basis (4 D) and the touched part of the map: the non-empty CLT blocks,
    the D sector entries of the full table, or both Lin tables."""
    if mode == "cr":
        return 0
    b = 4 * dim
    if mode == "clt":
        b += clt_touched_bytes(n, n_up)
    elif mode == "full":
        b += 4 * dim
    elif mode == "lin":
        lo = n // 2
        b += 4 * ((1 << (n - lo)) + (1 << lo))
    return b


def hv_alg_bytes(mode, dim, nvec, n, n_up):
    """Algorithmic HBM bytes of one Lanczos-epilogue H.x launch over nvec FP32
    columns: read x (u_k) and z (u_{k-1}), write w, plus the stored map."""
    return 12 * dim * nvec + map_bytes(mode, dim, n, n_up)


def timed_hv(ftlm, torch, sec, g, x, y, reps):
    """Median of `reps` H.x launches, each bracketed by HIP events on the
    stream the library launches on (torch's current stream)."""
    ftlm.hv(sec, g, x, y)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        ftlm.hv(sec, g, x, y)
        e1.record(st)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def run_gpu(args):
    import numpy as np
    import torch

    from ftlm_inputs import graphs
    from paper_2605_26261_amd import driver, ftlm

    dev = torch.device("cuda:0")
    bonds = graphs.icosidodecahedron()
    g = ftlm.Graph(N_SITES, bonds)
    n_bonds = g.n_bonds
    temps = driver.log_temperatures()
    results = {}
    all_modes = {"clt": ftlm.CLT, "cr": ftlm.CR, "full": ftlm.FULL, "lin": ftlm.LIN}
    for mode_name in args.modes.split(","):
        mode = all_modes[mode_name]
        sec = ftlm.Sector(N_SITES, N_UP, mode, device=dev)
        dim = sec.dim
        work = torch.empty(ftlm.lanczos_workspace_bytes(sec, R, ftlm.F32), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        if args.batch == "auto":
            tune = ftlm.autotune(sec, g, R, ftlm.F32, work=work)
            B = int(tune["batch"])
            tuned = {str(w): round(t, 3) for w, t in tune["candidates"].items()}
        else:
            B, tuned = int(args.batch), None
        batches = [(r0, min(B, R - r0)) for r0 in range(0, R, B)]

        def step():
            parts = [driver.sector_samples(sec, g, b, M, SEED, ftlm.GAUSS, ftlm.F32, r0=r0, work=work)
                     for r0, b in batches]
            rec = {k: parts[0][k] for k in ("n_up", "dim", "mult")}
            for k in ("theta", "weight", "steps", "alpha", "beta"):
                rec[k] = np.concatenate([p[k] for p in parts])
            th = ftlm.thermo(N_SITES, [rec], temps, 1.0)
            return rec, th

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ftlm.stats_reset()
        ftlm.stats_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hv_count = 0
        for _ in range(args.steps):
            rec, th = step()
            hv_count += int(rec["steps"].sum())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ftlm.stats_enable(False)
        launches, hv_ms = ftlm.stats_read()
        # every batch launches M = min(M, D) steps
        job_alg = args.steps * M * sum(hv_alg_bytes(mode_name, dim, b, N_SITES, N_UP) for _, b in batches)
        # the H.x of one batch of B chains alone: the roofline's launch
        ftlm.lanczos(sec, g, SEED, 0, B, 2, ftlm.GAUSS, ftlm.F32, work=work)
        torch.cuda.synchronize()
        ftlm.stats_reset()
        ftlm.stats_enable(True)
        ftlm.lanczos(sec, g, SEED, 0, B, 12, ftlm.GAUSS, ftlm.F32, work=work)
        torch.cuda.synchronize()
        ftlm.stats_enable(False)
        nb, msb = ftlm.stats_read()
        avg_ms = msb / nb
        alg = hv_alg_bytes(mode_name, dim, B, N_SITES, N_UP)
        results[mode_name] = {
            "batch": B,
            "autotune_ms": tuned,
            "seconds": dt,
            "ms_per_step": 1e3 * dt / args.steps,
            "states_bonds_per_s": dim * n_bonds * hv_count / dt,
            "samples_per_s": R * args.steps / dt,
            "hv_launches": launches,
            "hv_job_alg_gbs": job_alg / (hv_ms * 1e-3) / 1e9,
            "hv_avg_ms": avg_ms,
            "hv_kernel_states_bonds_per_s": dim * n_bonds * B / (avg_ms * 1e-3),
            "hv_alg_bytes": alg,
            "hv_alg_gbs": alg / (avg_ms * 1e-3) / 1e9,
            "E0": float(rec["theta"][rec["theta"] != 0].min()),
        }
        log(mode_name, json.dumps(results[mode_name]))
        # plain H.x (ftlm_hv) at several block widths: median of 20 launches
        del work
        torch.cuda.empty_cache()
        sweep = {}
        for nv in (1, 4, 8, 10, 12, 16, 20, 32):
            x = torch.randn((dim, nv) if nv > 1 else (dim,), dtype=torch.float32, device=dev)
            y = torch.empty_like(x)
            ms = timed_hv(ftlm, torch, sec, g, x, y, 20)
            a = 8 * dim * nv + map_bytes(mode_name, dim, N_SITES, N_UP)  # read x, write y, read the map
            sweep[str(nv)] = {"ms": ms, "states_bonds_per_s": dim * n_bonds * nv / (ms * 1e-3),
                              "alg_gbs": a / (ms * 1e-3) / 1e9}
            del x, y
            torch.cuda.empty_cache()
        results[mode_name]["hv_width_sweep"] = sweep
        log(mode_name, "hv sweep", json.dumps(sweep))
        del sec
        torch.cuda.empty_cache()
    return results, n_bonds


def plan_vs_plain():
    """The batched all-sector workload (6x4 J1-J2 lattice, 13 sectors, R = 32
    +-1 chains per sector, M = 80): one hipGraph-captured plan (one launch per
    kernel per step over all sectors, its column split chosen by
    ftlm_plan_tune) against the plain form (one sector and one chain at a
    time, eager). FTLM samples/s each."""
    import numpy as np
    import torch

    from ftlm_inputs import graphs
    from paper_2605_26261_amd import driver, ftlm

    n, R, M, seed = 24, 32, 80, 3
    bonds = graphs.square_j1j2(6, 4, 1.0, 0.5)
    g = ftlm.Graph(n, bonds)
    n_ups = list(range(12, 25))
    plan = ftlm.Plan(g, n_ups, ftlm.CR, R, M, ftlm.F32)
    tuning = plan.tune()  # split of the 32 columns into launches
    plan.run(seed, ftlm.PM1, use_graph=True)  # capture + warm up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = driver.plan_records(plan, n, seed, ftlm.PM1, use_graph=True)
    ftlm.thermo(n, recs, driver.log_temperatures(), 1.0)
    t_plan = time.perf_counter() - t0
    del plan
    torch.cuda.empty_cache()
    # plain: every chain alone (B = 1), sector by sector, eager launches, all
    # 416 samples, each with its Ritz solve
    t0 = time.perf_counter()
    for nu in n_ups:
        sec = ftlm.Sector(n, nu, ftlm.CR)
        work = torch.empty(ftlm.lanczos_workspace_bytes(sec, 1, ftlm.F32), dtype=torch.uint8, device="cuda")
        for r in range(R):
            driver.sector_samples(sec, g, 1, M, seed, ftlm.PM1, ftlm.F32, r0=r, work=work)
        del sec, work
    log(f"plan: plain form of {R * len(n_ups)} samples done")
    t_plain = time.perf_counter() - t0
    samples = R * len(n_ups)
    return {"workload": "6x4 J1-J2 lattice (N=24, J2=0.5), all 13 sectors, R=32 +-1, M=80, FP32",
            "plan_graph_s": t_plan, "plan_samples_per_s": samples / t_plan,
            "plan_max_width": tuning["max_width"],
            "plan_tuning_ms": {str(w): round(ms, 3) for w, (_, ms) in tuning["candidates"].items()},
            "plain_s": t_plain, "plain_samples_per_s": samples / t_plain,
            "plain_protocol": f"one chain per launch, sector by sector, eager; all {R} chains of every sector "
                              f"with their Ritz solves (the thermal reduction, ~10 ms, not included)"}


def serving(n_warm=200, n_meas=2000, rate=50.0, max_active=0, plain=True, steps_per_round=0, n_plain=200):
    """Poisson-arriving exchange-fit requests (N in 16..28, random clusters,
    J in [0.2, 1.5], one random sector, R = 16, M = 80) through the
    continuous-batching server; p50/p99 latency (arrival to result) and
    samples/s, and the plain form (FIFO, one request at a time, one chain per
    launch) on the same arrivals. At 50 requests/s both forms are overloaded,
    so latencies grow along the stream: the two are compared on the same
    requests (the first n_plain measured ones, behind the same warm-up
    backlog)."""
    import numpy as np
    import torch

    from ftlm_inputs.requests import exchange_fit_stream
    from paper_2605_26261_amd import driver, ftlm

    reqs = exchange_fit_stream(n_warm + n_meas, seed=4, rate=rate)
    temps = driver.log_temperatures()
    srv = ftlm.Server(48 << 30, mode=ftlm.CR, dtype=ftlm.F32, max_active=max_active, steps_per_round=steps_per_round)
    t0 = srv.clock()
    pending, done, k = {}, {}, 0
    while len(done) < len(reqs):
        now = srv.clock() - t0
        while k < len(reqs) and reqs[k]["t"] <= now:
            q = reqs[k]
            pending[srv.submit(q["n_sites"], q["bonds"], q["n_up"], q["R"], q["M"], q["seed"], ftlm.PM1, temps)] = k
            k += 1
        for rid in list(pending):
            r = srv.poll(rid)
            if r is not None:
                done[pending.pop(rid)] = r
                if len(done) % 200 == 0:
                    log(f"serving: {len(done)} of {len(reqs)} requests done")
        time.sleep(0.0005)
    stats = srv.stats()
    srv.close()
    meas = [done[i] for i in range(n_warm, len(reqs))]
    lat = np.array([r["t_done"] - r["t_submit"] for r in meas]) * 1e3
    span = max(r["t_done"] for r in meas) - min(r["t_submit"] for r in meas)
    served_sps = 16 * len(meas) / span
    out = {"workload": f"Poisson {rate:g}/s exchange-fit stream, N in 16..28, R=16, M=80, FP32; "
                       f"{n_warm} warm-up + {n_meas} measured requests",
           "max_active": max_active or 16, "steps_per_round": steps_per_round or 4,
           "arrivals_per_s": rate, "served_requests_per_s": len(meas) / span,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "samples_per_s": served_sps, "peak_arena_bytes": stats["peak_bytes"], "rounds": stats["rounds"]}
    if not plain:
        return out
    # plain FIFO on the same arrivals: each warm-up request and each of the
    # first n_plain measured ones served alone, one chain per launch; their
    # FIFO latencies follow from the measured service times and the arrival
    # times, and are compared with the served latencies of the same requests
    service = []
    for i, q in enumerate(reqs[:n_warm + n_plain]):
        if i % 50 == 0:
            log(f"plain FIFO: request {i} of {n_warm + n_plain}")
        t1 = time.perf_counter()
        driver.run(q["n_sites"], q["bonds"], [q["n_up"]], q["R"], q["M"], q["seed"], ftlm.PM1, batch=1, temps=temps)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t1)
    finish, lat_plain = 0.0, []
    for q, sv in zip(reqs[:n_warm + n_plain], service):
        finish = max(finish, q["t"]) + sv
        lat_plain.append((finish - q["t"]) * 1e3)
    lat_plain = lat_plain[n_warm:]
    first = lat[:len(lat_plain)]
    out.update({"first_n": len(lat_plain),
                "first_p50_ms": float(np.percentile(first, 50)), "first_p99_ms": float(np.percentile(first, 99)),
                "plain_p50_ms": float(np.percentile(lat_plain, 50)),
                "plain_p99_ms": float(np.percentile(lat_plain, 99)),
                "plain_samples_per_s": 16 * len(service) / sum(service),
                "plain_protocol": f"FIFO, one request at a time, one chain per launch, from measured service "
                                  f"times of the {n_warm} warm-up and first {len(lat_plain)} measured requests; "
                                  f"latencies of those {len(lat_plain)}, to compare with first_p50/p99_ms"})
    return out


def _precision_summary(ftlm, got, ref, runs, temps, keys):
    """FP32-vs-FP64 differences of one run against a stored FP64 oracle
    reference and the spread over seeds (Eq. 22) at the same R."""
    import numpy as np
    out = {}
    for k in keys:
        o64 = np.asarray(ref[k])
        d = np.abs(np.asarray(got[k]) - o64)
        _, sig = ftlm.seed_spread(np.array([r[k] for r in runs]))
        where = sig >= 1e-3 * sig.max()
        out[k] = {"max_abs_diff": float(d.max()), "max_rel_to_max": float(d.max() / np.abs(o64).max()),
                  "max_sigma_emp": float(sig.max()),
                  "max_diff_over_sigma": float(np.max(d[where] / sig[where]))}
    return out


def precision(n_seeds=10):
    """The precision pattern: FTLM with FP32 vectors and FP64 reductions
    against the FP64 oracle's stored results for the same start vectors
    (tests/golden, written by scripts that call only the oracle), and the
    stochastic error sigma_emp over n_seeds further seeds at the same R."""
    import numpy as np

    from ftlm_inputs import graphs
    from paper_2605_26261_amd import driver, ftlm

    gold = os.path.join(ROOT, "tests", "golden")
    out = {"n_seeds": n_seeds, "seeds": f"{1000}..{1000 + n_seeds - 1}"}
    # N = 12 ring, S^z = 0, R = 8 +-1, M = 40 (the FP64 workload): FP32 and FP64 on the GPU
    ref = json.load(open(os.path.join(gold, "ring12_r8.json")))
    temps = np.asarray(ref["temps"])
    rec = {}
    for name, dt in (("f32", ftlm.F32), ("f64", ftlm.F64)):
        th, _ = driver.run(12, graphs.ring(12), [6], 8, 40, ref["seed"], ftlm.PM1, dtype=dt, temps=temps)
        runs = [driver.run(12, graphs.ring(12), [6], 8, 40, 1000 + s, ftlm.PM1, dtype=dt, temps=temps)[0]
                for s in range(n_seeds)]
        rec[name] = _precision_summary(ftlm, th, ref, runs, temps, ("E", "C"))
    out["ring12_R8_M40"] = rec
    # icosidodecahedron N = 30, S^z = 0, the first 2 Gaussian chains of seed 2, M = 100, both index maps
    ref = json.load(open(os.path.join(gold, "icosidodecahedron_r2.json")))
    temps = np.asarray(ref["temps"])
    bonds = [tuple(b) for b in ref["bonds"]]
    rec = {}
    for name, mode in (("clt", ftlm.CLT), ("cr", ftlm.CR)):
        th, _ = driver.run(30, bonds, [15], 2, 100, ref["seed"], ftlm.GAUSS, mode=mode, temps=temps)
        if name == "cr":
            runs = [driver.run(30, bonds, [15], 2, 100, 1000 + s, ftlm.GAUSS, mode=mode, temps=temps)[0]
                    for s in range(n_seeds)]
        rec[name] = th
    out["icosidodecahedron_R2_M100"] = {k: _precision_summary(ftlm, rec[k], ref, runs, temps, ("E", "C"))
                                        for k in rec}
    # 6x4 J1-J2 lattice, all 13 sectors, R = 2 +-1, M = 80, one plan
    ref = json.load(open(os.path.join(gold, "square4x6_r2.json")))
    temps = np.asarray(ref["temps"])
    g = ftlm.Graph(24, [tuple(b) for b in ref["bonds"]])
    plan = ftlm.Plan(g, [sct["n_up"] for sct in ref["sectors"]], ftlm.CR, 2, ref["M"], ftlm.F32)
    th = ftlm.thermo(24, driver.plan_records(plan, 24, ref["seed"], ftlm.PM1), temps, 1.0)
    runs = [ftlm.thermo(24, driver.plan_records(plan, 24, 1000 + s, ftlm.PM1), temps, 1.0) for s in range(n_seeds)]
    out["square4x6_R2_M80"] = _precision_summary(ftlm, th, ref, runs, temps, ("E", "C", "chi"))
    del plan
    out["ghosts"] = ghost_study()
    return out


def ghost_study(n_chains=8, M=100):
    """Sec. 3.2 on the GPU: Cullum-Willoughby ghosts (Eq. 25, C_tau = 1) of
    FP32 and FP64 chains from the same start vectors in the M = 0 sector of
    the spin-1 icosahedron (D = 73,789), N_L = 100, and how far the total
    weights of matching Ritz clusters move between the precisions."""
    import numpy as np

    from ftlm_inputs import graphs
    from paper_2605_26261_amd import ftlm

    g = ftlm.Graph(12, graphs.icosahedron())
    sec = ftlm.Sector(12, 12, ftlm.CR, two_s=2)
    res = {}
    for name, dt in (("f32", ftlm.F32), ("f64", ftlm.F64)):
        a, b, st = ftlm.lanczos(sec, g, 11, 0, n_chains, M, ftlm.GAUSS, dt)
        res[name] = [ftlm.ghosts(a[r], b[r], int(st[r]), c_tau=1.0) for r in range(n_chains)]
    # converged, repeated eigenvalues: FP64 clusters with a ghost-flagged
    # member; the FP32 Ritz values around them carry the same total weight
    dw, n_conv = 0.0, 0
    for g64, g32 in zip(res["f64"], res["f32"]):
        win = max(1e-5, 10 * g64["tau"])
        for c, w in enumerate(g64["cluster_weight"]):
            members = g64["cluster"] == c
            if w < 1e-6 or not g64["ghost"][members].any():
                continue
            th = g64["theta"][members]
            near = (g32["theta"] >= th.min() - win) & (g32["theta"] <= th.max() + win)
            dw = max(dw, abs(g32["weight"][near].sum() - w))
            n_conv += 1
    return {"workload": f"spin-1 icosahedron M=0 (D={sec.dim}), {n_chains} Gaussian chains, N_L={M}, C_tau=1",
            "ghosts_f32": [int(x["ghost"].sum()) for x in res["f32"]],
            "ghosts_f64": [int(x["ghost"].sum()) for x in res["f64"]],
            "converged_clusters": n_conv, "max_cluster_weight_shift": dw}


def general_spin(reps=3):
    """General local spin (Sec. 2, Eqs. 11-17) on the icosahedron (N = 12,
    30 bonds, J = 1), the M = 0 sectors of Table 1 at s = 2, 5/2 and 3
    (digit sum A = N s): plain H.x at 1 and 8 FP32 columns with both index
    maps (the compressed table only while d^N labels fit 32 bits, so not at
    s = 3), and one Lanczos run of 8 Gaussian chains, M = 100 steps, in the
    s = 5/2 sector. A state-bond counts each bond once per row (its two
    ladder terms together)."""
    import torch

    from ftlm_inputs import graphs
    from paper_2605_26261_amd import ftlm

    n = 12
    g = ftlm.Graph(n, graphs.icosahedron())
    out = {"workload": "icosahedron N=12 (30 bonds, J=1), M=0 sectors of Table 1 at s=2, 5/2, 3; FP32"}
    for two_s in (4, 5, 6):
        a = n * two_s // 2
        for name, mode in (("cr", ftlm.CR), ("clt", ftlm.CLT)):
            if mode == ftlm.CLT and (two_s + 1) ** n > 2 ** 32:
                continue
            sec = ftlm.Sector(n, a, mode, two_s=two_s)
            d = sec.dim
            rec = {"dim": d}
            for B in (1, 8):
                x = torch.empty((d, B) if B > 1 else (d,), dtype=torch.float32, device="cuda").fill_(0.5)
                y = torch.empty_like(x)
                ms = timed_hv(ftlm, torch, sec, g, x, y, reps)
                alg = 8 * d * B + (4 * d if name == "clt" else 0)
                rec[f"hv_B{B}_ms"] = ms
                rec[f"hv_B{B}_states_bonds_per_s"] = d * g.n_bonds * B / (ms * 1e-3)
                rec[f"hv_B{B}_alg_gbs"] = alg / (ms * 1e-3) / 1e9
                del x, y
                torch.cuda.empty_cache()
            if two_s == 5 and name == "cr":
                ftlm.lanczos(sec, g, 3, 0, 8, 2, ftlm.GAUSS, ftlm.F32)  # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, st = ftlm.lanczos(sec, g, 3, 0, 8, 100, ftlm.GAUSS, ftlm.F32)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                rec["lanczos_R8_M100_s"] = dt
                rec["lanczos_states_bonds_per_s"] = d * g.n_bonds * float(st.sum()) / dt
            out[f"2s={two_s} {name}"] = rec
            log("spin", two_s, name, json.dumps(rec))
            del sec
            torch.cuda.empty_cache()
    return out


def largest_sector():
    """J1-J2 ring N = 34 (J2 = 0.3), S^z = 0, D = 2,333,606,220, CR only: H.x
    at B = 1 and B = 4, and the whole FTLM run of the workload (R = 4
    Gaussian chains, seed 5, M = 60, FP32 vectors) with its samples/s."""
    import torch

    from ftlm_inputs import graphs
    from paper_2605_26261_amd import driver, ftlm

    n, R, M, seed = 34, 4, 60, 5
    bonds = graphs.j1j2_ring(n, 1.0, 0.3)
    g = ftlm.Graph(n, bonds)
    sec = ftlm.Sector(n, 17, ftlm.CR)
    d = sec.dim
    out = {"workload": "J1-J2 ring N=34 S^z=0 (D=2333606220, 68 bonds), CR, FP32; FTLM R=4 Gaussian seed 5, M=60"}
    for B in (1, 4):
        x = torch.empty((d, B) if B > 1 else (d,), dtype=torch.float32, device="cuda").fill_(0.5)
        y = torch.empty_like(x)
        ms = timed_hv(ftlm, torch, sec, g, x, y, 3)
        out[f"hv_B{B}_ms"] = ms
        out[f"hv_B{B}_states_bonds_per_s"] = d * g.n_bonds * B / (ms * 1e-3)
        out[f"hv_B{B}_alg_gbs"] = 8 * d * B / (ms * 1e-3) / 1e9
        del x, y
        torch.cuda.empty_cache()
    work = torch.empty(ftlm.lanczos_workspace_bytes(sec, R, ftlm.F32), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec = driver.sector_samples(sec, g, R, M, seed, ftlm.GAUSS, ftlm.F32, work=work)
    th = ftlm.thermo(n, [rec], driver.log_temperatures(), 1.0)
    dt = time.perf_counter() - t0
    out["ftlm_s"] = dt
    out["ftlm_samples_per_s"] = R / dt
    out["ftlm_states_bonds_per_s"] = d * g.n_bonds * int(rec["steps"].sum()) / dt
    out["E0"] = float(rec["theta"][rec["theta"] != 0].min())
    out["E_per_site_T0.5"] = float(th["E"][int(abs(driver.log_temperatures() - 0.5).argmin())] / n)
    del work, sec
    torch.cuda.empty_cache()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(target_s=10.0):
    """The FP64 oracle (plain definitions, never tuned) on the host cores, at
    all cores and at one thread, each case on a bounded sample:

    * the N = 30 S^z = 0 H.x on a row range (states.bonds/s; the headline
      figure, also the value of the line);
    * the N = 12 ring FTLM (R = 8 +-1 chains, M = 40, FP64) whole, repeated
      to fill the time (samples/s);
    * the 6x4 J1-J2 lattice: Lanczos steps of one chain in the largest sector
      (D = 2,704,156), from which the whole all-sector run (416 chains of 80
      steps) is priced in proportion to D x bonds (samples/s, extrapolated);
    * the N = 30 R = 2 reference run (200 FP64 H.x), priced from the H.x rate."""
    import numpy as np

    import oracle
    from ftlm_inputs import graphs

    ncores = len(os.sched_getaffinity(0))
    out = {"cpu_model": _cpu_model(), "cores_available": ncores, "cases": {}}
    bonds = graphs.icosidodecahedron()
    dim = math.comb(N_SITES, N_UP)
    x = np.random.default_rng(0).standard_normal(dim)
    for threads in (ncores, 1):
        used = oracle.set_threads(threads)
        tag = f"{used}t"
        # N = 30 H.x on rows [0, n)
        probe = 1 << 14
        t0 = time.perf_counter()
        oracle.hv(N_SITES, N_UP, bonds, x, None, row0=0, nrows=probe)
        tp = time.perf_counter() - t0
        nrows = int(min(dim, max(probe, probe * target_s / max(tp, 1e-6))))
        t0 = time.perf_counter()
        oracle.hv(N_SITES, N_UP, bonds, x, None, row0=0, nrows=nrows)
        dt = time.perf_counter() - t0
        rate = nrows * len(bonds) / dt
        out["cases"][f"hv_n30_{tag}"] = {"value": rate, "unit": "states·bonds/s", "threads": used,
                                         "sample": f"rows [0, {nrows}) of D = {dim}, {dt:.1f} s"}
        if threads == ncores:
            out.update({"value": rate, "unit": "states·bonds/s", "cores": used, "kind": "oracle",
                        "sample": f"FP64 oracle H.x on rows [0, {nrows}) of the N=30 S^z=0 icosidodecahedron "
                                  f"sector (count-based ranks, no stored basis), {dt:.1f} s, {used} threads"})
            # the R = 2 reference run: 2 chains x 100 steps of the full sector
            out["cases"]["ftlm_n30_R2_priced"] = {"seconds": 200 * dim * len(bonds) / rate, "threads": used,
                                                  "sample": "200 FP64 H.x at the measured H.x rate"}
        # N = 12 ring FTLM, whole
        temps = oracle.log_temperatures()
        t0, runs = time.perf_counter(), 0
        while True:
            oracle.ftlm(12, graphs.ring(12), [6], 8, 40, 1, oracle.PM1, temps)
            runs += 1
            if time.perf_counter() - t0 > 2.0:
                break
        dt = time.perf_counter() - t0
        out["cases"][f"ftlm_ring12_{tag}"] = {"value": 8 * runs / dt, "unit": "samples/s", "threads": used,
                                              "sample": f"{runs} whole runs (R=8, M=40, D=924), {dt:.1f} s"}
        # 6x4 lattice: the H.x of the largest sector on a row range, from which
        # the whole all-sector run is priced in proportion to rows x bonds
        n, nu = 24, 12
        sq = graphs.square_j1j2(6, 4, 1.0, 0.5)
        d24 = math.comb(n, nu)
        b24 = oracle.basis(n, nu)
        q = np.random.default_rng(1).standard_normal(d24)
        rows = 1 << 14
        t0 = time.perf_counter()
        oracle.hv(n, nu, sq, q, b24, row0=0, nrows=rows)
        tp = time.perf_counter() - t0
        rows = int(min(d24, max(rows, rows * 0.3 * target_s / max(tp, 1e-6))))
        t0 = time.perf_counter()
        oracle.hv(n, nu, sq, q, b24, row0=0, nrows=rows)
        dt = time.perf_counter() - t0
        total_rows = sum(math.comb(n, k) for k in range(12, 25))
        whole = dt / rows * 32 * 80 * total_rows
        out["cases"][f"ftlm_square4x6_{tag}"] = {
            "value": 416 / whole, "unit": "samples/s (extrapolated)", "threads": used,
            "sample": f"H.x on rows [0, {rows}) of the D = {d24} sector, {dt:.1f} s; the all-sector run "
                      f"(13 sectors, R = 32 chains of M = 80 steps) priced as {whole:.0f} s of H.x in proportion to "
                      f"rows"}
        del b24
    oracle.set_threads(ncores)
    out["cases"].update(paper_cpu_method(target_s))
    return out


def _mem_available_bytes():
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemAvailable:"):
                    return int(line.split()[1]) * 1024
    except OSError:
        pass
    return 0


def paper_cpu_method(target_s=10.0):
    """The paper's own CPU method on the same host (Sec. 2, "Computational
    setup": a batched B = 8 FP64 H.x with the compressed lookup table and
    OpenMP over rows; its CPU column of Table 3): the N = 30 S^z = 0 product
    on a row sample, at all cores and at one thread. Needs ~12 GB of host
    memory (basis, table and an [D][8] FP64 block); skipped below that."""
    import numpy as np

    import oracle
    from oracle import paper_cpu
    from ftlm_inputs import graphs

    dim = math.comb(N_SITES, N_UP)
    need = dim * (8 * 8 + 8) + (1 << 25) * 8
    if _mem_available_bytes() < 1.5 * need:
        return {"paper_cpu_clt_b8_n30": {"skipped": f"needs ~{need / 1e9:.0f} GB of host memory"}}
    bonds = graphs.icosidodecahedron()
    basis = oracle.basis(N_SITES, N_UP)
    mask, prefix = oracle.clt(basis, N_SITES)
    x = np.empty((dim, 8), dtype=np.float64)
    x.fill(0.5)
    res = {}
    ncores = len(os.sched_getaffinity(0))
    for threads in (ncores, 1):
        used = oracle.set_threads(threads)
        probe = 1 << 15
        t0 = time.perf_counter()
        paper_cpu.hv_clt_b8(bonds, basis, mask, prefix, x, 0, probe)
        tp = time.perf_counter() - t0
        rows = int(min(dim, max(probe, probe * (target_s if threads > 1 else 0.5 * target_s) / max(tp, 1e-6))))
        t0 = time.perf_counter()
        paper_cpu.hv_clt_b8(bonds, basis, mask, prefix, x, 0, rows)
        dt = time.perf_counter() - t0
        res[f"paper_cpu_clt_b8_n30_{used}t"] = {
            "value": rows * len(bonds) * 8 / dt, "unit": "states·bonds/s (8 vectors per row)", "threads": used,
            "sample": f"rows [0, {rows}) of D = {dim}, {dt:.1f} s; the paper's CPU reference kernel "
                      f"(batched B = 8 FP64 CLT H.x, OpenMP over rows)"}
    oracle.set_threads(ncores)
    del x, basis, mask, prefix
    return res


def profile_kernels(batch=None):
    """Short run for hardware-counter passes: per index map, a 3-step Lanczos
    run over `batch` chains (when None, one at every FP32 launch width up to
    R, so that whichever width the autotuner picks, the last two
    Lanczos-epilogue H.x launches of its run are steady-state launches of the
    FTLM pass) and 3 single-vector H.x launches; then an elementwise kernel
    that reads 2 GiB and writes 2 GiB, to calibrate the byte counters."""
    import torch

    from ftlm_inputs import graphs
    from paper_2605_26261_amd import ftlm

    dev = torch.device("cuda:0")
    g = ftlm.Graph(N_SITES, graphs.icosidodecahedron())
    for mode in (ftlm.CLT, ftlm.CR, ftlm.FULL, ftlm.LIN):
        sec = ftlm.Sector(N_SITES, N_UP, mode, device=dev)
        for B in ([batch] if batch else [w for w in LAUNCH_WIDTHS_F32 if w <= R]):
            log("profile: batch", B)
            ftlm.lanczos(sec, g, SEED, 0, B, 3, ftlm.GAUSS, ftlm.F32)
        x = torch.randn(sec.dim, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            ftlm.hv(sec, g, x, y)
        torch.cuda.synchronize()
        del sec, x, y
        torch.cuda.empty_cache()
    # calibration: an elementwise kernel that reads 2 GiB and writes 2 GiB
    a = torch.empty(512 << 20, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.add(a, 1.0, out=b)
    torch.cuda.synchronize()
    log("profile run done")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-headline", action="store_true", help="skip the plan, serving and N=34 measurements")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="measured requests of the serving stream (after 200 warm-up)")
    ap.add_argument("--batch", default="auto", help="chains per Lanczos batch ('auto': the autotuner's choice)")
    ap.add_argument("--modes", default="clt,cr,full,lin",
                    help="index maps of the headline workload (compressed table, ranking, full table, Lin)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="short kernel-only run for rocprofv3 counter passes")
    ap.add_argument("--only", choices=["plan", "serving", "largest", "precision", "spin"],
                    help="run one secondary measurement alone and print its JSON (for kernel traces)")
    args = ap.parse_args()
    if args.profile_kernels:
        profile_kernels(None if args.batch == "auto" else int(args.batch))
        return
    if args.only:
        run = {"plan": plan_vs_plain, "largest": largest_sector, "precision": precision, "spin": general_spin,
               "serving": lambda: serving(n_warm=200 if args.serve_requests >= 200 else 10,
                                          n_meas=args.serve_requests)}[args.only]
        print(json.dumps({args.only: run()}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    results, n_bonds = run_gpu(args)
    best = max(results, key=lambda k: results[k]["states_bonds_per_s"])
    r = results[best]
    dom = results[best]
    traffic = None
    if kernel_source_hash() == MEASURED_TRAFFIC["sources"]:
        traffic = MEASURED_TRAFFIC["bytes"].get(best, {}).get(dom["batch"])
    roof = {"bound": "hbm", "achieved": dom["hv_alg_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dom["hv_alg_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "bytes per launch between L2 and the memory side (2 x FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated; includes Infinity Cache hits)",
            "kernel": f"hv_lanczos_kernel<uint32, {best.upper()}, float, {dom['batch']}> (Lanczos-epilogue H.x "
                      f"over {dom['batch']} FP32 columns)",
            "alg_bytes_per_launch": dom["hv_alg_bytes"], "avg_launch_ms": dom["hv_avg_ms"]}
    # counted HBM traffic of the same launch over its measured duration
    counted_gbs = traffic / (dom["hv_avg_ms"] * 1e-3) / 1e9 if traffic else None
    roof["counted_gbs"] = counted_gbs
    roof["counted_frac"] = counted_gbs / HBM_PEAK_GBS if counted_gbs else None
    # the plain H.x (ftlm_hv, no Lanczos epilogue) of the same map: one vector
    # and the block width with the best per-vector rate
    sweep = dom["hv_width_sweep"]
    best_w = max(sweep, key=lambda w: sweep[w]["states_bonds_per_s"])
    roof["plain_hv"] = {w: {"ms": sweep[w]["ms"], "achieved_gbs": sweep[w]["alg_gbs"],
                            "frac": sweep[w]["alg_gbs"] / HBM_PEAK_GBS,
                            "states_bonds_per_s": sweep[w]["states_bonds_per_s"]}
                        for w in sorted({"1", best_w}, key=int)}
    out = {
        "metric": METRIC,
        "value": r["states_bonds_per_s"],
        "unit": "states·bonds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "icosidodecahedron N=30 S^z=0 (D=155117520, 60 bonds, J=1), R=20 Gaussian seed 2, "
                               "M=100, FP32 vectors / FP64 alpha-beta; one step = one full FTLM pass",
                   "index_mode": best},
        "samples_per_s": r["samples_per_s"],
        "hbm_gbs_alg": dom["hv_alg_gbs"],
        "hbm_gbs_counted": counted_gbs,
        "modes": results,
        "roofline": roof,
    }
    if not args.only_headline:
        import torch
        torch.cuda.empty_cache()
        out["batched_all_sector"] = plan_vs_plain()
        log("plan", json.dumps(out["batched_all_sector"]))
        torch.cuda.empty_cache()
        out["serving"] = serving(n_warm=200 if args.serve_requests >= 200 else 10, n_meas=args.serve_requests)
        log("serving", json.dumps(out["serving"]))
        torch.cuda.empty_cache()
        out["largest_sector"] = largest_sector()
        log("n34", json.dumps(out["largest_sector"]))
        torch.cuda.empty_cache()
        out["precision"] = precision()
        log("precision", json.dumps(out["precision"]))
        torch.cuda.empty_cache()
        out["general_spin"] = general_spin()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
