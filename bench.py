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
# VALU instructions per pair in the pair-body basic blocks of the built
# kernels (binary32 path, n = 0), counted from the gfx950 assembly.
PAIR_BODY_VALU = {"pass_dm": 281, "pass_gas": 207}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def src_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_24688_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def make_workload(name: str, scale: float, seed: int):
    import workloads
    if name == "galaxy":
        cfg = workloads.galaxy(n_gas=int(1_000_000 * scale), n_dm=int(4_000_000 * scale), seed=(2, seed))
        desc = {"workload": "isolated galaxy: exponential gas disk + NFW halo",
                "n_gas": len(cfg["gas"]["mass"]), "n_dm": len(cfg["dm"]["mass"]), "n_ngb": 64,
                "sigma0_cm2": cfg["params"]["sigma0_cm2"], "m_chi_over_mp": 2.0, "n_pow": 0, "dt_myr": 1.0,
                "pair_math": "binary32", "accumulation": "binary64"}
    elif name == "box":
        cfg = workloads.box(seed=(1, seed))
        desc = {"workload": "periodic test box", "n_gas": 4096, "n_dm": 4096, "n_ngb": 32,
                "sigma0_cm2": 1e-24, "m_chi_over_mp": 2.0, "n_pow": 0, "dt_myr": 0.05,
                "pair_math": "binary64", "accumulation": "binary64"}
    else:
        raise SystemExit(f"unknown workload {name}")
    return cfg, desc


def cpu_baseline(cfg, seconds: float, seed: int = 0):
    """The CPU oracle, as it stands, on a bounded random sample of owners of
    the same workload (both passes, brute-force neighbours over the full other
    species), scaled to pairs per second."""
    import numpy as np
    import oracle
    oracle.lib()
    gas, dm, par = cfg["gas"], cfg["dm"], cfg["params"]
    r = np.random.default_rng(seed)
    ng, nd = len(gas["mass"]), len(dm["mass"])
    k = 16
    done_pairs, done_t, n_gs, n_ds = 0, 0.0, 0, 0
    while done_t < seconds and (n_gs < ng or n_ds < nd):
        gs = np.sort(r.choice(ng, size=min(k, ng), replace=False))
        ds = np.sort(r.choice(nd, size=min(4 * k, nd), replace=False))
        t0 = time.perf_counter()
        res = oracle.step(gas, dm, par, gas_sel=gs, dm_sel=ds)
        dt = time.perf_counter() - t0
        done_pairs += res["counters"]["pairs_gas"] + res["counters"]["pairs_dm"]
        done_t += dt
        n_gs += len(gs)
        n_ds += len(ds)
        if dt < 0.25 * seconds:
            k *= 2
    # pairs processed by both passes count once per pass; the metric counts each pair once
    rate = 0.5 * done_pairs / max(done_t, 1e-9)
    return {"value": rate, "unit": "pair interactions/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n_gs} random gas owners and {n_ds} random DM owners of the benchmark workload "
                      f"(brute-force neighbours over all particles of the other species), {done_t:.1f} s of "
                      f"oracle time, {done_pairs} pair evaluations over both passes"}


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
    t0 = time.time()
    X = torch.from_numpy(workloads.mlp_samples(2_000_000, seed=(4, 1))).to(dev)
    Y = ctx.mlp_labels(X)
    torch.cuda.synchronize()
    t1 = time.time()
    losses = ctx.mlp_train(X, Y, epochs=200, batch=4096, lr0=2e-3, lr_min=1e-5, seed=1, init=True, use_graph=True)
    t2 = time.time()
    del X, Y
    log_fn(f"bench: network trained: labels {t1 - t0:.2f} s, 200 epochs {t2 - t1:.2f} s, loss {losses[-1]:.3e}")
    res = {"train": {"samples": 2_000_000, "epochs": 200, "batch": 4096, "label_s": round(t1 - t0, 3),
                     "train_s": round(t2 - t1, 3), "final_loss": float(losses[-1])}}
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
        row["mlp_vs_quad12"] = row["quad12"]["pass_gas_ms"] / row["mlp"]["pass_gas_ms"]
        row["mlp_vs_quad32"] = row["quad32"]["pass_gas_ms"] / row["mlp"]["pass_gas_ms"]
        res[f"n={n_pow}"] = row
        log_fn(f"bench: surrogate n={n_pow}: " + ", ".join(
            f"{k} {v['pass_gas_ms']:.3f} ms (err {v['max_rel_rate_err']:.1e})" for k, v in row.items()
            if isinstance(v, dict)))
    return res


def traffic_from_profile(kernel: str):
    """HBM bytes per launch measured with rocprofv3 PMC runs, if they were
    taken for the current kernel sources; else None."""
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
    ap.add_argument("--workload", default="galaxy", choices=["galaxy", "box"])
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the workload's particle counts")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    t0 = time.time()
    cfg, desc = make_workload(args.workload, args.scale, args.seed)
    log(f"bench: workload generated in {time.time() - t0:.1f} s: {desc['n_gas']} gas, {desc['n_dm']} DM")
    precision = dmb.DMB_FP32 if desc["pair_math"] == "binary32" else dmb.DMB_FP64
    dev = torch.device("cuda:0")
    G = dmb.to_device(cfg["gas"], dev)
    D = dmb.to_device(cfg["dm"], dev)
    out = dmb.alloc_out(desc["n_gas"], desc["n_dm"], dev)
    ctx = dmb.Context(0)
    par = dict(cfg["params"])

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
    dom = "pass_dm" if per_kernel["pass_dm"] >= per_kernel["pass_gas"] else "pass_gas"
    t_dom = per_kernel[dom] * 1e-3
    units = cnt["pairs_dm"] if dom == "pass_dm" else cnt["pairs_gas"]
    ops = units * PAIR_BODY_VALU[dom] if precision == dmb.DMB_FP32 else None
    if ops is not None:
        achieved = ops / t_dom / 1e9
        roof = {"bound": "alu", "kernel": "k_pass_dm" if dom == "pass_dm" else "k_pass_gas",
                "achieved": achieved, "peak": VALU_PEAK_GOPS, "unit": "Gop/s (VALU lane-instructions)",
                "frac": achieved / VALU_PEAK_GOPS, "traffic": traffic_from_profile(dom),
                "kernel_ms": per_kernel[dom],
                "ops_per_pair": PAIR_BODY_VALU[dom], "pairs_per_launch": units}
    else:
        roof = {"bound": "alu", "kernel": dom, "achieved": None, "peak": VALU_PEAK_GOPS, "unit": "Gop/s",
                "frac": None, "traffic": None, "kernel_ms": per_kernel[dom]}
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
        "interact_only_pairs_per_s": pairs / (sum(v for k, v in per_kernel.items() if k != "build") * 1e-3),
        "hbm_algorithmic_GBps": bytes_step / (ms_step * 1e-3) / 1e9,
        "roofline": roof,
        "build_stats": bst,
        "hit_fraction": {"gas": pairs / max(1, bst["cand_pairs_gas"] * 4096),
                         "dm": pairs / max(1, bst["cand_pairs_dm"] * 4096)},
    }
    if args.workload == "galaxy" and not args.no_surrogate:
        line["surrogate"] = surrogate_compare(ctx, cfg, dev, 3, log)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
