"""Full-size workloads on the GPU, checked on sampled owners against the CPU
oracle (which evaluates the sampled owners one by one, brute force over the
whole other species) and through properties that hold at any size.

- galaxy, 1 000 000 gas + 4 000 000 DM, binary32 pair math (the benchmark's
  configuration and launch);
- Milky-Way scale, 8 000 000 gas + 32 000 000 DM, h spread over 3 decades,
  10 % of each species active, binary32 pair math.
Bars as in the small parity tests: per gas owner the mean field within 1e-5
condition-aware, or, for owners whose neighbours all sit near the support
edge (where the binary32 overlap table is accurate to ~1e-7 of the pair's
peak, not of its value), within 1e-6 peak-scaled; exact decisions away from
thresholds; inactive owners receive nothing; with every particle active the
gas and DM passes visit the same pairs.
"""
from __future__ import annotations

import time

import numpy as np
import pytest

import workloads
from parity_util import decision_report, kick_error, mean_field_errors, run_gpu

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2603_24688_amd as dmb
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dmb.Context(0)
    yield c
    c.close()


def _sampled_check(ctx, cfg, label, n_gas_s=192, n_dm_s=192, precision=1):
    import oracle
    t0 = time.time()
    gpu = run_gpu(ctx, cfg, precision)
    t1 = time.time()
    ga = cfg["gas"].get("active")
    da = cfg["dm"].get("active")
    ng, nd = len(cfg["gas"]["mass"]), len(cfg["dm"]["mass"])
    gpool = np.arange(ng) if ga is None else np.nonzero(ga)[0]
    dpool = np.arange(nd) if da is None else np.nonzero(da)[0]
    r = np.random.default_rng(17)
    gsel = np.sort(r.choice(gpool, min(n_gas_s, gpool.size), replace=False))
    dsel = np.sort(r.choice(dpool, min(n_dm_s, dpool.size), replace=False))
    ref = oracle.step(cfg["gas"], cfg["dm"], cfg["params"], gas_sel=gsel, dm_sel=dsel, peak_scale=True)
    t2 = time.time()
    cond, peak = mean_field_errors(gpu, ref, gsel)
    ok = (cond <= 1e-5) | (peak <= 1e-6)
    edge = int(np.sum((cond > 1e-5) & (peak <= 1e-6)))
    dec = decision_report(gpu, ref, dsel)
    ke = kick_error(gpu, ref, dsel)
    c = gpu["counters"]
    _log(f"[{label}] gpu step {t1 - t0:.1f} s (incl. upload), oracle on {len(gsel)}+{len(dsel)} owners "
         f"{t2 - t1:.1f} s; pairs {c['pairs_gas']} / {c['pairs_dm']}; mean field: max condition-aware "
         f"{cond.max():.2e}, {edge} edge-only owners within {peak[cond > 1e-5].max(initial=0):.1e} peak-scaled; decisions "
         f"{dec['compared']} (excluded {dec['excluded']}, scatters {dec['scatters']}) mismatch {dec['mismatch']}; "
         f"kick {ke:.2e}")
    assert np.all(ok)
    assert dec["mismatch"] == 0
    assert ke <= 2e-5
    if ga is None and da is None:
        assert c["pairs_gas"] == c["pairs_dm"]
    if ga is not None:
        idle = ga == 0
        assert np.all(gpu["dp_gas"][idle] == 0.0) and np.all(gpu["de_gas"][idle] == 0.0)
    if da is not None:
        idle = da == 0
        assert np.all(gpu["partner"][idle] == -1) and np.all(gpu["dv_dm"][idle] == 0.0)
    return gpu, ref


def test_galaxy_full_size_sampled(ctx):
    cfg = workloads.galaxy(n_gas=1_000_000, n_dm=4_000_000, seed=(2, 1))
    _sampled_check(ctx, cfg, "galaxy 1M+4M")


def test_milky_way_full_size_sampled(ctx):
    t0 = time.time()
    cfg = workloads.milky_way()
    _log(f"[milky way] generated in {time.time() - t0:.1f} s")
    _sampled_check(ctx, cfg, "milky way 8M+32M, 10% active, h over 3 decades", n_gas_s=96, n_dm_s=96)
