"""FTLM runs through libftlm: per sector, R Lanczos chains on the device,
Ritz values on the host, then the thermal reduction (paper Sec. 2, Eqs. 4-9).

Orchestration only; every numerical step is a library call.
"""
import numpy as np

from . import ftlm


def multiplicity(n_sites, n_up):
    """The sector's weight in the thermal sums (ftlm_sector_info)."""
    return ftlm.sector_info(n_sites, n_up)[1]


def log_temperatures(n=200, t_min=0.05, t_max=10.0):
    k = np.arange(n)
    return t_min * (t_max / t_min) ** (k / (n - 1))


def records_from_coefficients(n_sites, n_up, dim, alpha, beta, steps, two_s=1):
    """Host Ritz solves of R chains -> a thermo record of the sector (n_up:
    the digit sum A when two_s > 1)."""
    theta, weight = ftlm.ritz_batch(alpha, beta, steps)
    return {"n_up": n_up, "two_s": two_s, "dim": dim, "mult": ftlm.sector_info_spin(n_sites, two_s, n_up)[1],
            "theta": theta, "weight": weight, "steps": np.asarray(steps), "alpha": alpha, "beta": beta}


def sector_samples(sector, graph, R, M, seed, dist, dtype, r0=0, work=None, stream=None):
    """Runs R chains in one batch; returns the thermo record of the sector."""
    alpha, beta, steps = ftlm.lanczos(sector, graph, seed, r0, R, M, dist, dtype, work=work, stream=stream)
    return records_from_coefficients(sector.n_sites, sector.n_up, sector.dim, alpha, beta, steps,
                                     getattr(sector, "two_s", 1))


def run(n_sites, bonds, n_ups, R, M, seed, dist, dtype=ftlm.F32, mode=ftlm.CR, temps=None, g=1.0,
        batch=None, device="cuda", two_s=1):
    """Full FTLM over the listed sectors (n_ups: digit sums A when two_s =
    2s > 1). Chains run in batches of `batch` (default: all R at once;
    "auto": the autotuned width). Returns (thermo dict, per-sector records)."""
    temps = log_temperatures() if temps is None else temps
    graph = ftlm.Graph(n_sites, bonds)
    recs = []
    for n_up in n_ups:
        sec = ftlm.Sector(n_sites, n_up, mode, device=device, two_s=two_s)
        if batch == "auto":
            b = ftlm.autotune(sec, graph, R, dtype)["batch"]
        else:
            b = R if batch is None else batch
        parts = []
        for r0 in range(0, R, b):
            parts.append(sector_samples(sec, graph, min(b, R - r0), M, seed, dist, dtype, r0=r0))
        rec = {k: parts[0][k] for k in ("n_up", "two_s", "dim", "mult")}
        for k in ("theta", "weight", "steps", "alpha", "beta"):
            rec[k] = np.concatenate([p[k] for p in parts])
        recs.append(rec)
    return ftlm.thermo(n_sites, recs, temps, g), recs


def plan_records(plan, n_sites, seed, dist, r0=0, use_graph=True):
    """One run of an all-sector plan -> per-sector thermo records."""
    alpha, beta, steps = plan.run(seed, dist, r0=r0, use_graph=use_graph)
    return [records_from_coefficients(n_sites, nu, ftlm.sector_info(n_sites, nu)[0], alpha[i], beta[i], steps[i])
            for i, nu in enumerate(plan.n_ups)]


def run_plan(n_sites, bonds, n_ups, R, M, seed, dist, dtype=ftlm.F32, mode=ftlm.CR, temps=None, g=1.0,
             use_graph=True, device="cuda", tune=True):
    """Full FTLM over the listed sectors as one batched plan (its split of the
    R columns into launches timed and chosen by ftlm_plan_tune unless
    tune=False; the chains do not depend on it)."""
    temps = log_temperatures() if temps is None else temps
    graph = ftlm.Graph(n_sites, bonds)
    plan = ftlm.Plan(graph, n_ups, mode, R, M, dtype, device=device)
    if tune:
        plan.tune()
    recs = plan_records(plan, n_sites, seed, dist, use_graph=use_graph)
    return ftlm.thermo(n_sites, recs, temps, g), recs
