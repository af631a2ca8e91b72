#!/usr/bin/env python3
"""Benchmark of the DM-gas pair interaction step on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
dmb_build_cells (Morton sort, tiles, candidate lists) followed by
dmb_interact_step (gas mean-field pass, DM Monte Carlo pass, decision and
partner resolve).  Inputs are resident in HBM before timing starts.

Default workload: isolated galaxy, 1 000 000 gas in an exponential disk and
4 000 000 DM in an NFW halo, 64-neighbour kernels, one interaction step with
binary32 pair math and binary64 accumulation.

Prints ONE JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks used for the roofline fractions.
HBM_PEAK_GBS = 8000.0
# Vector ALU: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz lane-instructions per second.
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
# Algorithmic VALU lane-instructions per pair (the method's own work, not the
# kernels' issue count): DM pass = distance and test 25 + overlap 25 +
# Philox4x32-10 100 + Box-Muller 30 + P_ij and its sums 15; gas pass =
# distance and test 25 + overlap 25 + closed-form rate terms 60 + binary64
# accumulation 8.
PAIR_ALGO_VALU = {"pass_dm": 195, "pass_gas": 118}
# Algorithmic HBM bytes per particle of build_cells: position and h read
# (32), Morton key and index written (12), four 8-bit radix passes over key
# and index (4 x 24), sorted position and h written (32), less the reuse of the
# key pass by the sub-tile cut: about 150 bytes.
BUILD_ALGO_BYTES_PER_PARTICLE = 150


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def src_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_24688_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def make_workload(name: str, scale: float, seed: int, n_pow: int = 0):
    import workloads
    sig = workloads.sigma0_for_npow(n_pow)
    if name == "galaxy":
        cfg = workloads.galaxy(n_gas=int(1_000_000 * scale), n_dm=int(4_000_000 * scale), seed=(2, seed),
                               n_pow=n_pow, sigma0_cm2=sig)
        desc = {"workload": "isolated galaxy: exponential gas disk + NFW halo",
                "n_gas": len(cfg["gas"]["mass"]), "n_dm": len(cfg["dm"]["mass"]), "n_ngb": 64,
                "sigma0_cm2": sig, "m_chi_over_mp": 2.0, "n_pow": n_pow, "dt_myr": 1.0,
                "pair_math": "binary32", "accumulation": "binary64"}
    elif name == "milky_way":
        cfg = workloads.milky_way(n_gas=int(8_000_000 * scale), n_dm=int(32_000_000 * scale), seed=(3, seed),
                                  n_pow=n_pow, sigma0_cm2=sig)
        desc = {"workload": "Milky-Way-scale disk + halo, h over 3 decades, 10% active per species",
                "n_gas": len(cfg["gas"]["mass"]), "n_dm": len(cfg["dm"]["mass"]), "n_ngb": 64,
                "sigma0_cm2": sig, "m_chi_over_mp": 2.0, "n_pow": n_pow, "dt_myr": 0.1,
                "pair_math": "binary32", "accumulation": "binary64"}
    elif name == "box":
        cfg = workloads.box(seed=(1, seed), n_pow=n_pow, sigma0_cm2=sig)
        desc = {"workload": "periodic test box", "n_gas": 4096, "n_dm": 4096, "n_ngb": 32,
                "sigma0_cm2": sig, "m_chi_over_mp": 2.0, "n_pow": n_pow, "dt_myr": 0.05,
                "pair_math": "binary64", "accumulation": "binary64"}
    else:
        raise SystemExit(f"unknown workload {name}")
    return cfg, desc


def train_network(ctx, dev, log_fn) -> dict:
    """The rate-closure network trained on the GPU (2 000 000 samples labelled
    by binary64 quadrature, 200 epochs of Adam)."""
    import torch
    import workloads
    t0 = time.time()
    X = torch.from_numpy(workloads.mlp_samples(2_000_000, seed=(4, 1))).to(dev)
    Y = ctx.mlp_labels(X)
    torch.cuda.synchronize()
    t1 = time.time()
    losses = ctx.mlp_train(X, Y, epochs=200, batch=4096, lr0=2e-3, lr_min=1e-5, seed=1, init=True, use_graph=True)
    t2 = time.time()
    del X, Y
    log_fn(f"bench: network trained: labels {t1 - t0:.2f} s, 200 epochs {t2 - t1:.2f} s, loss {losses[-1]:.3e}")
    return {"samples": 2_000_000, "epochs": 200, "batch": 4096, "label_s": round(t1 - t0, 3),
            "train_s": round(t2 - t1, 3), "final_loss": float(losses[-1])}


def host_cpu() -> dict:
    """The host CPU model and the logical cores the process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 0
    return {"model": model, "logical_cores_usable": usable}


def cpu_baseline(cfg, seconds: float, pairs_per_step: int, seed: int = 0):
    """The CPU oracle, as it stands, with its uniform-grid candidate search,
    timed on a bounded random sample of the owners of the same workload and
    scaled to a whole step: grid build + per-owner time x (all owners /
    sampled owners).  Returns pairs per second of the extrapolated step."""
    import numpy as np
    import oracle
    oracle.lib()
    gas, dm, par = cfg["gas"], cfg["dm"], cfg["params"]
    r = np.random.default_rng(seed)
    ng, nd = len(gas["mass"]), len(dm["mass"])
    none = np.zeros(0, dtype=np.int64)
    t0 = time.perf_counter()
    oracle.step(gas, dm, par, gas_sel=none, dm_sel=none, grid=True)    # the two grids, no owners
    t_build = time.perf_counter() - t0
    k = max(1, min(ng, 2000))
    t_own = 0.0
    while True:
        gs = np.sort(r.choice(ng, size=min(k, ng), replace=False))
        ds = np.sort(r.choice(nd, size=min(k * max(1, nd // max(ng, 1)), nd), replace=False))
        t0 = time.perf_counter()
        res = oracle.step(gas, dm, par, gas_sel=gs, dm_sel=ds, grid=True)
        dt = time.perf_counter() - t0
        t_own = max(dt - t_build, 1e-9)
        if dt >= 0.5 * seconds or (len(gs) == ng and len(ds) == nd):
            break
        k = int(min(ng, k * max(2.0, 0.6 * seconds / max(dt, 1e-3))))
    frac = 0.5 * (len(gs) / max(ng, 1) + len(ds) / max(nd, 1))
    t_full = t_build + t_own / frac
    c = res["counters"]
    return {"value": pairs_per_step / t_full, "unit": "pair interactions/s", "cores": oracle.num_threads(),
            "cpu": host_cpu(), "kind": "oracle", "neighbours": "uniform grids (the oracle's own candidate search)",
            "sample": f"{len(gs)} random gas owners and {len(ds)} random DM owners of the benchmark workload "
                      f"({c['pairs_gas']} + {c['pairs_dm']} pairs in {dt:.1f} s including the grid build of "
                      f"{t_build:.1f} s); a whole step is estimated as the build plus the per-owner time scaled "
                      f"to all owners: {t_full:.1f} s for {pairs_per_step} pairs"}


def build_roofline(n_particles: int, build_ms) -> dict:
    """build_cells against HBM: algorithmic bytes per step over the measured
    build time (event-timed, both species, all stages)."""
    if not build_ms:
        return {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None}
    b = n_particles * BUILD_ALGO_BYTES_PER_PARTICLE
    achieved = b / (build_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "build_ms": build_ms,
            "algorithmic_bytes": b, "bytes_per_particle": BUILD_ALGO_BYTES_PER_PARTICLE}


def surrogate_compare(ctx, cfg, dev, steps: int, log_fn) -> dict:
    """Network rates vs quadrature on the galaxy workload with sigma ~ v^n,
    n in {-4, -2, 2} (sigma0 with sigma(200 km/s) = 1e-24 cm^2): pairs per
    second of the interaction step and gas-pass time for the closed forms,
    quadrature at K = 32 (the 1e-10 judge) and K = 12 (the smallest K at the
    1e-3 level) and the network; the network is trained first on the GPU.
    Rate errors are measured against the binary64 closed forms."""
    import numpy as np
    import torch
    import paper_2603_24688_amd as dmb
    import workloads
    res = {"train": train_network(ctx, dev, log_fn)}
    ctx.set_pass_overlap(False)     # gas-pass times are then the pass's own
    G = dmb.to_device(cfg["gas"], dev)
    D = dmb.to_device(cfg["dm"], dev)
    out = dmb.alloc_out(len(cfg["gas"]["mass"]), len(cfg["dm"]["mass"]), dev)
    modes = [("exact", dmb.DMB_RATES_EXACT, 0), ("quad32", dmb.DMB_RATES_QUAD, 32),
             ("quad12", dmb.DMB_RATES_QUAD, 12), ("mlp", dmb.DMB_RATES_MLP, 32)]
    # rate accuracy over the range of w / vs met in the workload (one DM velocity per pair)
    w = torch.linspace(0.0, 1000.0, 200_001, dtype=torch.float64, device=dev)
    vs = torch.full_like(w, 9.085)
    for n_pow in (-4, -2, 2):
        par = dict(cfg["params"])
        par["n_pow"] = n_pow
        par["sigma0_cm2"] = workloads.sigma0_for_npow(n_pow)
        A0, B0 = ctx.rates_eval(w, vs, n_pow, precision=dmb.DMB_FP64, rates=dmb.DMB_RATES_EXACT)
        ok = A0 > 0
        row = {}
        ctx.build_cells(G, D, par, precision=dmb.DMB_FP32)
        for name, rates, K in modes:
            A1, B1 = ctx.rates_eval(w, vs, n_pow, precision=dmb.DMB_FP32, rates=rates, quad_nodes=K)
            err = torch.maximum((A1[ok] / A0[ok] - 1).abs(), (B1[ok] / B0[ok] - 1).abs()).max().item()
            par["rates"], par["quad_nodes"] = rates, K
            ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP32)
            torch.cuda.synchronize()
            ctx.profile_enable(True)
            ctx.profile_read(reset=True)
            ta = time.perf_counter()
            for _ in range(steps):
                ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP32)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            ph = ctx.profile_read(reset=True)
            ctx.profile_enable(False)
            pairs = dmb.counters_dict(out["counters"])["pairs_gas"]
            ms = (tb - ta) * 1e3 / steps
            row[name] = {"pairs_per_s": pairs / (ms * 1e-3), "interact_ms": round(ms, 4),
                         "pass_gas_ms": round(ph["pass_gas"][0] / max(ph["pass_gas"][1], 1), 4),
                         "max_rel_rate_err": err}
        # speed ratios (> 1: the network's gas pass is faster)
        row["mlp_vs_quad12"] = row["quad12"]["pass_gas_ms"] / row["mlp"]["pass_gas_ms"]
        row["mlp_vs_quad32"] = row["quad32"]["pass_gas_ms"] / row["mlp"]["pass_gas_ms"]
        row["network_faster_than_quad12_at_equal_accuracy"] = bool(row["mlp_vs_quad12"] > 1.0)
        res[f"n={n_pow}"] = row
        log_fn(f"bench: surrogate n={n_pow}: " + ", ".join(
            f"{k} {v['pass_gas_ms']:.3f} ms (err {v['max_rel_rate_err']:.1e})" for k, v in row.items()
            if isinstance(v, dict)))
    ctx.set_pass_overlap(True)
    return res


def closure_compare(ctx, cfg, dev, steps: int, log_fn) -> dict:
    """Per-gas Maxwellian closure (rates mode 3) against the per-pair mean field
    on the galaxy workload in binary32: gas-pass time of each (passes in
    sequence, so the time is the pass's own) and how far the closure's dp and
    dE lie from the per-pair sums (the DM around a gas particle is not one
    Maxwellian, so they differ by more than rounding)."""
    import numpy as np
    import torch
    import paper_2603_24688_amd as dmb
    G = dmb.to_device(cfg["gas"], dev)
    D = dmb.to_device(cfg["dm"], dev)
    out = dmb.alloc_out(len(cfg["gas"]["mass"]), len(cfg["dm"]["mass"]), dev)
    par = dict(cfg["params"])
    ctx.build_cells(G, D, par, precision=dmb.DMB_FP32)
    ctx.set_pass_overlap(False)
    res, got = {}, {}
    for name, rates in (("pair", dmb.DMB_RATES_EXACT), ("closure", dmb.DMB_RATES_CLOSURE)):
        par["rates"] = rates
        ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP32)
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        ctx.profile_read(reset=True)
        ta = time.perf_counter()
        for _ in range(steps):
            ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP32)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ph = ctx.profile_read(reset=True)
        ctx.profile_enable(False)
        got[name] = (out["dp_gas"].cpu().numpy(), out["de_gas"].cpu().numpy())
        res[name] = {"interact_serial_ms": round((tb - ta) * 1e3 / steps, 4),
                     "pass_gas_ms": round(ph["pass_gas"][0] / max(ph["pass_gas"][1], 1), 4)}
    ctx.set_pass_overlap(True)
    (p0, e0), (p1, e1) = got["pair"], got["closure"]
    live = np.abs(e0) > 0
    dpr = np.linalg.norm(p1 - p0, axis=1)[live] / np.maximum(np.linalg.norm(p0, axis=1)[live], 1e-300)
    der = np.abs(e1 - e0)[live] / np.abs(e0)[live]
    res["gas_pass_speedup"] = res["pair"]["pass_gas_ms"] / res["closure"]["pass_gas_ms"]
    res["dp_rel_diff_median"] = float(np.median(dpr)) if dpr.size else None
    res["de_rel_diff_median"] = float(np.median(der)) if der.size else None
    log_fn(f"bench: closure: gas pass {res['closure']['pass_gas_ms']:.3f} ms vs per-pair "
           f"{res['pair']['pass_gas_ms']:.3f} ms; median |ddp|/|dp| {res['dp_rel_diff_median']:.2e}, "
           f"|ddE|/|dE| {res['de_rel_diff_median']:.2e}")
    return res


def galaxy_binary64(ctx, cfg, dev, steps: int, log_fn) -> dict:
    """The same galaxy step in binary64 throughout (exact overlap, binary64
    rates and draws): build + interaction step per step, passes overlapped as
    in the headline."""
    import torch
    import paper_2603_24688_amd as dmb
    G = dmb.to_device(cfg["gas"], dev)
    D = dmb.to_device(cfg["dm"], dev)
    out = dmb.alloc_out(len(cfg["gas"]["mass"]), len(cfg["dm"]["mass"]), dev)
    par = dict(cfg["params"])
    ctx.build_cells(G, D, par, precision=dmb.DMB_FP64)
    ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP64)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for s in range(steps):
        par["step"] = s
        ctx.build_cells(G, D, par, precision=dmb.DMB_FP64)
        ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP64)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    cnt = dmb.counters_dict(out["counters"])
    ms = (tb - ta) * 1e3 / steps
    log_fn(f"bench: galaxy in binary64: {ms:.2f} ms per step, {cnt['pairs_dm']} pairs")
    return {"ms_per_step": round(ms, 4), "pairs_per_step": cnt["pairs_dm"], "pairs_per_s": cnt["pairs_dm"] / (ms * 1e-3),
            "pair_math": "binary64", "overlap": "exact (piecewise Gauss-Legendre)", "steps": steps}


def rb_compare(ctx, cfg, dev, steps: int, log_fn) -> dict:
    """Rao-Blackwellised DM sampling against the paper's per-pair sampling on
    the galaxy workload in binary32: DM-pass and resolve times (passes in
    sequence, so each time is the kernel's own), and the interaction step's
    time and pairs per second with the passes overlapped, as in the headline."""
    import torch
    import paper_2603_24688_amd as dmb
    G = dmb.to_device(cfg["gas"], dev)
    D = dmb.to_device(cfg["dm"], dev)
    out = dmb.alloc_out(len(cfg["gas"]["mass"]), len(cfg["dm"]["mass"]), dev)
    par = dict(cfg["params"])
    ctx.build_cells(G, D, par, precision=dmb.DMB_FP32)
    res = {}
    for name, mode in (("per_pair", dmb.DMB_SAMPLE_PAIR), ("rao_blackwell", dmb.DMB_SAMPLE_RB)):
        par["dm_sampling"] = mode
        # the kernels' own times, passes in sequence
        ctx.set_pass_overlap(False)
        ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP32)
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        ctx.profile_read(reset=True)
        for _ in range(steps):
            ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP32)
        torch.cuda.synchronize()
        ph = ctx.profile_read(reset=True)
        ctx.profile_enable(False)
        own = {f"{k}_ms": round(ph[k][0] / max(ph[k][1], 1), 4) for k in ("pass_dm", "combine_dm", "resolve")}
        # the interaction step as the headline runs it
        ctx.set_pass_overlap(True)
        ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP32)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(steps):
            ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP32)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        cnt = dmb.counters_dict(out["counters"])
        ms = (tb - ta) * 1e3 / steps
        res[name] = {"interact_ms": round(ms, 4), "pairs_per_s": cnt["pairs_dm"] / (ms * 1e-3),
                     "scatters": cnt["scatters"], **own}
    res["dm_pass_speedup"] = res["per_pair"]["pass_dm_ms"] / res["rao_blackwell"]["pass_dm_ms"]
    log_fn(f"bench: rao-blackwell: DM pass {res['rao_blackwell']['pass_dm_ms']:.3f} ms vs per-pair "
           f"{res['per_pair']['pass_dm_ms']:.3f} ms; interaction {res['rao_blackwell']['interact_ms']:.3f} vs "
           f"{res['per_pair']['interact_ms']:.3f} ms")
    return res


def batch_sweep(dev, steps: int, log_fn) -> dict:
    """Parameter sweep of 64 periodic boxes of uneven size (10^4 .. 5 10^5
    particles per species, sigma0 1e-28 .. 1e-24 cm^2, m_chi/m_p in
    {0.5, 1, 2, 5}; the test box's densities and temperatures): autotune,
    then `steps` replays of one captured step of all boxes."""
    import torch
    import paper_2603_24688_amd as dmb
    import workloads
    t0 = time.time()
    bx = workloads.batch(n_box=64, n_min=10_000, n_max=500_000, seed=(5, 1))
    G = [dmb.to_device(b["gas"], dev) for b in bx]
    D = [dmb.to_device(b["dm"], dev) for b in bx]
    P = [dict(b["params"]) for b in bx]
    O = [dmb.alloc_out(len(b["gas"]["mass"]), len(b["dm"]["mass"]), dev) for b in bx]
    ng = sum(len(b["gas"]["mass"]) for b in bx)
    nd = sum(len(b["dm"]["mass"]) for b in bx)
    del bx
    log_fn(f"bench: batch of 64 boxes generated in {time.time() - t0:.1f} s: {ng} gas, {nd} DM")
    ctx = dmb.Context(0)
    try:
        t1 = time.time()
        choice = ctx.batch_tune(G, D, P, O, precision=dmb.DMB_FP32)
        t2 = time.time()
        log_fn(f"bench: batch autotune {t2 - t1:.1f} s -> {choice}")
        ctx.batch_step(G, D, P, O, precision=dmb.DMB_FP32, nsteps=1, graph=True)   # warm-up replay
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ctx.batch_step(G, D, P, O, precision=dmb.DMB_FP32, nsteps=steps, graph=True)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        pairs = sum(dmb.counters_dict(o["counters"])["pairs_gas"] for o in O)
        scat = sum(dmb.counters_dict(o["counters"])["scatters"] for o in O)
        ms = (tb - ta) * 1e3 / steps
        log_fn(f"bench: batch {steps} graph replays: {ms:.3f} ms per step, {pairs} pairs per step")
        return {"workload": "64 periodic boxes, 1e4..5e5 particles per species each, sigma0 1e-28..1e-24 cm^2, "
                            "m_chi/m_p in {0.5,1,2,5}", "n_gas": ng, "n_dm": nd, "pairs_per_step": pairs,
                "scatters_per_step": scat, "ms_per_step": ms, "pairs_per_s": pairs / (ms * 1e-3),
                "graph_replays": steps, "tuned": choice, "tune_s": round(t2 - t1, 2),
                "pair_math": "binary32", "accumulation": "binary64"}
    finally:
        ctx.close()


def milky_way_loop(dev, steps: int, warmup: int, log_fn, scale: float = 1.0) -> dict:
    """Milky-Way-scale disk + halo (8M gas + 32M DM, h over 3 decades) advanced
    `steps` steps of 0.1 Myr by the library's time loop with hierarchical
    timesteps: each step draws an independent 10 % of each species as active
    (Philox tag 3); binary32 pair math, binary64 totals.  Pairs counted are
    those touching an active particle (gas pass + DM pass)."""
    import torch
    import paper_2603_24688_amd as dmb
    import workloads
    t0 = time.time()
    cfg = workloads.milky_way(n_gas=int(8_000_000 * scale), n_dm=int(32_000_000 * scale))
    for sp in ("gas", "dm"):
        cfg[sp].pop("active", None)
    ng, nd = len(cfg["gas"]["mass"]), len(cfg["dm"]["mass"])
    log_fn(f"bench: milky way generated in {time.time() - t0:.1f} s: {ng} gas, {nd} DM")
    par = dict(cfg["params"])
    ctx = dmb.Context(0)
    try:
        G, D = dmb.to_device(cfg["gas"], dev), dmb.to_device(cfg["dm"], dev)
        del cfg
        if warmup > 0:
            ctx.run(G, D, par, warmup, dt_max=par["dt"], precision=dmb.DMB_FP32, active_frac=0.1)
        par["step"] = warmup
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        diag = ctx.run(G, D, par, steps, dt_max=par["dt"], precision=dmb.DMB_FP32, active_frac=0.1)
        t2 = time.perf_counter()
    finally:
        ctx.close()
    col = dmb.DIAG_NAMES.index
    pairs = float(diag[1:, col("pairs")].sum() + diag[1:, col("pairs_gas")].sum())
    ms = (t2 - t1) * 1e3 / max(steps, 1)
    p0 = diag[0, col("p_dm_x")] + diag[0, col("p_gas_x")]
    p1 = diag[-1, col("p_dm_x")] + diag[-1, col("p_gas_x")]
    log_fn(f"bench: milky way loop: {steps} steps in {(t2 - t1):.2f} s, {pairs / max(steps, 1):.3e} active-touching "
           f"pairs per step, {int(diag[1:, col('scatters')].sum())} scatters")
    return {"workload": "Milky-Way-scale disk + NFW halo, 8M gas + 32M DM, h log-uniform over 3 decades (top-anchored "
                        "at the 64-neighbour maximum), 10% of each species active per step, dt 0.1 Myr",
            "n_gas": ng, "n_dm": nd, "steps": steps, "ms_per_step": ms, "s_for_steps": t2 - t1,
            "active_pair_visits_per_step": pairs / max(steps, 1), "active_pair_visits_per_s": pairs / max(t2 - t1, 1e-12),
            "pair_count": "gas-pass visits (active gas) + DM-pass visits (active DM); a pair with both ends active is evaluated by both passes and counts twice",
            "scatters": int(diag[1:, col("scatters")].sum()), "pair_math": "binary32", "totals": "binary64",
            "total_px_change_rel": float(abs(p1 - p0) / max(abs(diag[0, col("p_dm_x")]), 1e-300))}


def box_time_loop(dev, steps: int, warmup: int, log_fn) -> dict:
    """The periodic test box (4096 gas + 4096 DM, binary64) advanced `steps`
    steps by the library's time loop (rebuild, interaction step, kicks and
    transfers, drift, per-step diagnostics) in one dmb_run call, after
    `warmup` untimed steps on a copy of the same state."""
    import torch
    import paper_2603_24688_amd as dmb
    import workloads
    cfg = workloads.box(seed=(1, 1))
    par = dict(cfg["params"])
    ctx = dmb.Context(0)
    try:
        if warmup > 0:
            Gw, Dw = dmb.to_device(cfg["gas"], dev), dmb.to_device(cfg["dm"], dev)
            ctx.run(Gw, Dw, par, warmup, dt_max=par["dt"], precision=dmb.DMB_FP64)
            del Gw, Dw
        G, D = dmb.to_device(cfg["gas"], dev), dmb.to_device(cfg["dm"], dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        diag = ctx.run(G, D, par, steps, dt_max=par["dt"], dt_control=False, precision=dmb.DMB_FP64)
        t1 = time.perf_counter()
    finally:
        ctx.close()
    col = dmb.DIAG_NAMES.index
    pairs = float(diag[1:, col("pairs")].sum())
    ms = (t1 - t0) * 1e3 / max(steps, 1)
    log_fn(f"bench: box time loop: {steps} steps in {(t1 - t0) * 1e3:.2f} ms, {pairs / max(steps, 1):.0f} pairs per "
           f"step, max JB {diag[:, col('jb_dm')].max():.4f}")
    return {"workload": "periodic test box L = 1 kpc, 4096 gas + 4096 DM, Maxwellian gas T = 1e4 K, DM T = 1e5 K "
                        "drifting at 50 km/s, m_chi = 2 m_p, sigma0 = 1e-24 cm^2, 32 neighbours, dt = 0.05 Myr",
            "steps": steps, "ms_for_steps": (t1 - t0) * 1e3, "ms_per_step": ms, "pairs_per_step": pairs / max(steps, 1),
            "pairs_per_s": pairs / max(t1 - t0, 1e-12), "precision": "binary64",
            "scatters": int(diag[1:, col("scatters")].sum()), "max_jb": float(diag[:, col("jb_dm")].max())}


def pmc_from_profile(kernel: str):
    """Counters of one launch of `kernel` from the rocprofv3 PMC runs committed
    under profiles/ (HBM bytes from FETCH_SIZE / WRITE_SIZE scaled by a plain
    copy of known size, and SQ_INSTS_VALU), if they were taken for the current
    kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("src_hash") != src_hash():
        return None
    return d.get("kernels", {}).get(kernel)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="galaxy", choices=["galaxy", "box", "milky_way", "batch"])
    ap.add_argument("--rates", default="exact", choices=["exact", "quad", "mlp", "closure"],
                    help="rate integrals: closed forms, quadrature (--quad-nodes), the trained network "
                         "or the per-gas Maxwellian closure")
    ap.add_argument("--quad-nodes", type=int, default=12)
    ap.add_argument("--dm-sampling", default="pair", choices=["pair", "rb"],
                    help="DM Monte Carlo: one gas-velocity sample per pair (the paper's) or Rao-Blackwellised")
    ap.add_argument("--n-pow", type=int, default=0, choices=[-4, -2, 0, 2])
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the workload's particle counts")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-box batched sweep")
    ap.add_argument("--no-box", action="store_true", help="skip the 100-step time loop of the periodic test box")
    ap.add_argument("--no-milky-way", action="store_true",
                    help="skip the 200-step hierarchical-timestep run at Milky-Way scale")
    ap.add_argument("--no-fp64", action="store_true", help="skip the binary64 run of the galaxy step")
    ap.add_argument("--no-rb", action="store_true",
                    help="skip the Rao-Blackwellised vs per-pair DM sampling comparison")
    ap.add_argument("--no-closure", action="store_true",
                    help="skip the per-gas closure vs per-pair mean-field comparison")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the network-vs-quadrature comparison (sigma ~ v^n on the galaxy workload)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this size (for PMC counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not part of this "
                                   "build (see the sharding notes in the design doc)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2603_24688_amd as dmb

    dev = torch.device("cuda:0")
    if args.workload == "box":
        b = box_time_loop(dev, args.steps, args.warmup, log)
        line = {"metric": "DM-gas pair interactions/sec per step", "value": b["pairs_per_s"],
                "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                "ms_per_step": b["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f64", "data": "synthetic", "config": b}
        print(json.dumps(line), flush=True)
        return
    if args.workload == "milky_way":
        b = milky_way_loop(dev, args.steps, args.warmup, log, args.scale)
        line = {"metric": "DM-gas pair interactions/sec per step (pairs touching an active particle)",
                "value": b["active_pair_visits_per_s"], "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": b["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": b}
        print(json.dumps(line), flush=True)
        return
    if args.workload == "batch":
        b = batch_sweep(dev, args.steps, log)
        line = {"metric": "DM-gas pair interactions/sec per step", "value": b["pairs_per_s"],
                "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
                "ms_per_step": b["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f32", "data": "synthetic", "config": b}
        print(json.dumps(line), flush=True)
        return
    t0 = time.time()
    cfg, desc = make_workload(args.workload, args.scale, args.seed, args.n_pow)
    log(f"bench: workload generated in {time.time() - t0:.1f} s: {desc['n_gas']} gas, {desc['n_dm']} DM")
    precision = dmb.DMB_FP32 if desc["pair_math"] == "binary32" else dmb.DMB_FP64
    G = dmb.to_device(cfg["gas"], dev)
    D = dmb.to_device(cfg["dm"], dev)
    out = dmb.alloc_out(desc["n_gas"], desc["n_dm"], dev)
    ctx = dmb.Context(0)
    par = dict(cfg["params"])
    rates = {"exact": dmb.DMB_RATES_EXACT, "quad": dmb.DMB_RATES_QUAD, "mlp": dmb.DMB_RATES_MLP,
             "closure": dmb.DMB_RATES_CLOSURE}[args.rates]
    par["rates"], par["quad_nodes"] = rates, args.quad_nodes
    desc["rates"] = args.rates if args.rates != "quad" else f"quad{args.quad_nodes}"
    par["dm_sampling"] = dmb.DMB_SAMPLE_RB if args.dm_sampling == "rb" else dmb.DMB_SAMPLE_PAIR
    desc["dm_sampling"] = "rao_blackwell" if args.dm_sampling == "rb" else "per_pair"
    if args.rates == "mlp":
        precision = dmb.DMB_FP32
        desc["pair_math"] = "binary32"
        desc["network"] = train_network(ctx, dev, log)

    def one_step(s):
        par["step"] = s
        ctx.build_cells(G, D, par, precision=precision)
        ctx.interact_step(G, D, par, out, precision=precision)

    for s in range(args.warmup):
        one_step(s)
        torch.cuda.synchronize()
        log(f"bench: warmup step {s} done")
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        one_step(args.warmup + s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ph = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    cnt = dmb.counters_dict(out["counters"])
    bst = ctx.build_stats()
    log(f"bench: build stats {bst}")
    log(f"bench: timed {args.steps} steps in {t1 - t0:.3f} s; counters {cnt}")
    log("bench: phases (ms per step) " + ", ".join(f"{k}={v[0] / max(v[1], 1):.3f}" for k, v in ph.items()))
    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: copy probe of {args.copy_probe_mb} MiB done")

    ms_step = (t1 - t0) * 1e3 / args.steps
    pairs = max(cnt["pairs_gas"], cnt["pairs_dm"])
    value = pairs / (ms_step * 1e-3)
    per_kernel = {k: v[0] / max(v[1], 1) for k, v in ph.items()}
    # the dominant pass: the one with the most algorithmic work per step (the DM pass for the
    # closed-form rates); with other rate modes the gas pass's work grows, so take the longer span
    if args.rates == "exact" and precision == dmb.DMB_FP32:
        dom = ("pass_dm" if PAIR_ALGO_VALU["pass_dm"] * cnt["pairs_dm"] >= PAIR_ALGO_VALU["pass_gas"] * cnt["pairs_gas"]
               else "pass_gas")
    else:
        dom = "pass_dm" if per_kernel["pass_dm"] >= per_kernel["pass_gas"] else "pass_gas"
    t_dom = per_kernel[dom] * 1e-3
    units = cnt["pairs_dm"] if dom == "pass_dm" else cnt["pairs_gas"]
    counted = (precision == dmb.DMB_FP32 and args.n_pow == 0 and args.dm_sampling == "pair"
               and (dom == "pass_dm" or args.rates == "exact"))
    kname = "k_pass_dm" if dom == "pass_dm" else "k_pass_gas"
    pmc = pmc_from_profile(kname)
    if counted:
        achieved = units * PAIR_ALGO_VALU[dom] / t_dom / 1e9
        roof = {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": VALU_PEAK_GOPS,
                "unit": "Gop/s (VALU lane-instructions)", "frac": achieved / VALU_PEAK_GOPS,
                "traffic": None if pmc is None else pmc.get("hbm_bytes"),
                "kernel_ms": per_kernel[dom], "algorithmic_ops_per_pair": PAIR_ALGO_VALU[dom],
                "pairs_per_launch": units,
                "kernel_ms_note": "span of the pass in the timed steps; the other pass runs beside it on a "
                                  "second stream (the DM pass, enqueued first, takes the time it takes alone: "
                                  "compare rao_blackwell.per_pair.pass_dm_ms)",
                "issued_valu_per_pair": None if pmc is None else pmc.get("valu_lane_instr") / units}
    else:
        roof = {"bound": "alu", "kernel": kname, "achieved": None, "peak": VALU_PEAK_GOPS, "unit": "Gop/s",
                "frac": None, "traffic": None, "kernel_ms": per_kernel[dom],
                "note": "algorithmic counts are stated for binary32 closed-form rates with n = 0 and per-pair "
                        "DM sampling"}
    # algorithmic HBM bytes of the step: each particle read once (sorted copies),
    # outputs written once (see the design doc for the per-particle byte counts)
    bytes_step = desc["n_gas"] * (40 + 32) + desc["n_dm"] * (32 + 36)
    line = {
        "metric": "DM-gas pair interactions/sec per step",
        "value": value, "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if precision == dmb.DMB_FP32 else "f64", "data": "synthetic",
        "config": dict(desc, pairs_per_step=pairs, scatters_per_step=cnt["scatters"]),
        "phases_ms": {k: round(v, 4) for k, v in per_kernel.items()},
        # the step's kernels overlap on two streams: the interaction time is the step less its build
        "interact_only_pairs_per_s": pairs / ((ms_step - per_kernel.get("build", 0.0)) * 1e-3),
        "hbm_algorithmic_GBps": bytes_step / (ms_step * 1e-3) / 1e9,
        "roofline": roof,
        "build_roofline": build_roofline(desc["n_gas"] + desc["n_dm"], per_kernel.get("build")),
        "build_stats": bst,
        "hit_fraction": {"gas": pairs / max(1, bst["cand_pairs_gas"] * 4096),
                         "dm": pairs / max(1, bst["cand_pairs_dm"] * 4096)},
    }
    default_run = args.workload == "galaxy" and args.rates == "exact" and args.n_pow == 0 and args.dm_sampling == "pair"
    if default_run and not args.no_fp64:
        line["galaxy_binary64"] = galaxy_binary64(ctx, cfg, dev, 5, log)
    if default_run and not args.no_rb:
        line["rao_blackwell"] = rb_compare(ctx, cfg, dev, 3, log)
    if default_run and not args.no_closure:
        line["closure"] = closure_compare(ctx, cfg, dev, 3, log)
    if default_run and not args.no_surrogate:
        line["surrogate"] = surrogate_compare(ctx, cfg, dev, 3, log)
    if default_run and not args.no_batch:
        line["batch"] = batch_sweep(dev, 10, log)
    if default_run and not args.no_box:
        line["box_time_loop"] = box_time_loop(dev, 100, 2, log)
    if default_run and not args.no_milky_way:
        line["milky_way_loop"] = milky_way_loop(dev, 200, 2, log)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds, pairs)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
