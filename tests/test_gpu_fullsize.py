"""Full-size workloads on the GPU, checked on sampled owners against the CPU
oracle (which evaluates the sampled owners one by one, brute force over the
whole other species) and through properties that hold at any size.

- galaxy, 1 000 000 gas + 4 000 000 DM, binary32 pair math (the benchmark's
  configuration and launch);
- Milky-Way scale, 8 000 000 gas + 32 000 000 DM, h spread over 3 decades
  (top-anchored at each species' 64-neighbour maximum), 10 % of each species
  active, binary32 pair math.
Bars as in the small parity tests: per gas owner the mean field within 1e-5
condition-aware; exact decisions away from thresholds; inactive owners
receive nothing; with every particle active the gas and DM passes visit the
same pairs.  Where the pair lists fit in memory, every sampled owner's
neighbour set (count, sum of partner indices and of their squares) equals the
oracle's brute-force set.
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


def _owner_stats(pairs, owner_col, sel):
    """Per owner in `sel`: partner count, sum of partner indices and of their
    squares, from a device pair list [n, 2] of (DM index, gas index)."""
    import torch
    own = pairs[:, owner_col]
    oth = pairs[:, 1 - owner_col]
    n = int(max(int(own.max().item()) + 1, int(sel.max()) + 1)) if pairs.shape[0] else int(sel.max()) + 1
    cnt = torch.bincount(own, minlength=n)
    s1 = torch.zeros(n, dtype=torch.int64, device=pairs.device).index_add_(0, own, oth)
    s2 = torch.zeros(n, dtype=torch.int64, device=pairs.device).index_add_(0, own, oth * oth)
    idx = torch.from_numpy(np.asarray(sel)).to(pairs.device)
    return (cnt[idx].cpu().numpy(), s1[idx].cpu().numpy().astype(np.uint64),
            s2[idx].cpu().numpy().astype(np.uint64))


def _sampled_check(ctx, cfg, label, n_gas_s=192, n_dm_s=192, precision=1, pair_sets=False):
    import torch
    import oracle
    import paper_2603_24688_amd as dmb
    t0 = time.time()
    if pair_sets:
        G, D = dmb.to_device(cfg["gas"]), dmb.to_device(cfg["dm"])
        out = dmb.alloc_out(len(cfg["gas"]["mass"]), len(cfg["dm"]["mass"]))
        ctx.build_cells(G, D, cfg["params"], precision=precision)
        pg, pd = ctx.pair_list(G, D, cfg["params"], out, precision=precision, cap=450_000_000)
        torch.cuda.synchronize()
        gpu = {k: v.cpu().numpy() for k, v in out.items() if k != "counters"}
        gpu["counters"] = dmb.counters_dict(out["counters"])
        del G, D, out
    else:
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
    ref = oracle.step(cfg["gas"], cfg["dm"], cfg["params"], gas_sel=gsel, dm_sel=dsel)
    t2 = time.time()
    cond = mean_field_errors(gpu, ref, gsel)
    dec = decision_report(gpu, ref, dsel)
    ke = kick_error(gpu, ref, dsel)
    c = gpu["counters"]
    _log(f"[{label}] gpu step {t1 - t0:.1f} s (incl. upload), oracle on {len(gsel)}+{len(dsel)} owners "
         f"{t2 - t1:.1f} s; pairs {c['pairs_gas']} / {c['pairs_dm']}; mean field: max condition-aware "
         f"{cond.max():.2e}; decisions {dec['compared']} (excluded {dec['excluded']}, scatters {dec['scatters']}) "
         f"mismatch {dec['mismatch']}; kick {ke:.2e}")
    tol = 1e-12 if precision == 0 else 1e-5
    assert np.all(cond <= tol), (gsel[cond > tol], cond[cond > tol])
    assert dec["mismatch"] == 0
    assert ke <= (1e-12 if precision == 0 else 2e-5)
    if pair_sets:
        for col, sel, owner_dm, lst, name in ((1, gsel, False, pg, "gas pass"), (0, dsel, True, pd, "DM pass")):
            g_cnt, g_s1, g_s2 = _owner_stats(lst, col, sel)
            o_cnt, o_s1, o_s2 = oracle.pair_stats(cfg["gas"], cfg["dm"], cfg["params"], sel, owner_dm)
            bad = (g_cnt != o_cnt) | (g_s1 != o_s1) | (g_s2 != o_s2)
            _log(f"[{label}] {name}: neighbour sets of {sel.size} sampled owners, {int(o_cnt.sum())} pairs, "
                 f"{int(bad.sum())} differ")
            assert not bad.any(), sel[bad][:10]
        del pg, pd
        torch.cuda.empty_cache()
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
    _sampled_check(ctx, cfg, "galaxy 1M+4M", pair_sets=True)


def test_galaxy_full_size_binary64(ctx):
    """The galaxy at full size in binary64 (exact overlap, binary64 rates and
    draws): sampled owners against the oracle at the binary64 bars."""
    cfg = workloads.galaxy(n_gas=1_000_000, n_dm=4_000_000, seed=(2, 1))
    _sampled_check(ctx, cfg, "galaxy 1M+4M binary64", precision=0)


def test_milky_way_full_size_sampled(ctx):
    t0 = time.time()
    cfg = workloads.milky_way()
    _log(f"[milky way] generated in {time.time() - t0:.1f} s")
    _sampled_check(ctx, cfg, "milky way 8M+32M, 10% active, h over 3 decades", n_gas_s=96, n_dm_s=96,
                   pair_sets=True)


def test_galaxy_full_size_closure_and_rao_blackwell(ctx):
    """The galaxy at full size with the per-gas Maxwellian closure on the gas
    side and Rao-Blackwellised sampling on the DM side (each variant touches
    one side only), on sampled owners against the oracle's same modes."""
    import paper_2603_24688_amd as dmb
    cfg = workloads.galaxy(n_gas=1_000_000, n_dm=4_000_000, seed=(2, 1))
    cfg["params"]["rates"] = dmb.DMB_RATES_CLOSURE
    cfg["params"]["dm_sampling"] = dmb.DMB_SAMPLE_RB
    _sampled_check(ctx, cfg, "galaxy 1M+4M closure + Rao-Blackwellised")
