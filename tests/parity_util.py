"""Comparison helpers for HIP-vs-oracle parity tests."""
from __future__ import annotations

import numpy as np


def run_gpu(ctx, cfg, precision, device="cuda"):
    import torch
    import paper_2603_24688_amd as dmb
    gas, dm, par = cfg["gas"], cfg["dm"], cfg["params"]
    G, D = dmb.to_device(gas, device), dmb.to_device(dm, device)
    out = dmb.alloc_out(len(gas["mass"]), len(dm["mass"]), device)
    ctx.build_cells(G, D, par, precision=precision)
    ctx.interact_step(G, D, par, out, precision=precision)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items() if k != "counters"}
    res["counters"] = dmb.counters_dict(out["counters"])
    return res


def mean_field_error(gpu, ref, gas_sel=None):
    """Condition-aware error per gas particle and component:
    |gpu - oracle| / max(|oracle|, sum_i |term_ij|)."""
    sel = slice(None) if gas_sel is None else gas_sel
    dp_scale = np.maximum(np.abs(ref["dp_gas"][sel]), ref["dp_abs"][sel])
    de_scale = np.maximum(np.abs(ref["de_gas"][sel]), ref["de_abs"][sel])
    dp_err = np.abs(gpu["dp_gas"][sel] - ref["dp_gas"][sel])
    de_err = np.abs(gpu["de_gas"][sel] - ref["de_gas"][sel])
    with np.errstate(invalid="ignore", divide="ignore"):
        e1 = np.where(dp_scale > 0, dp_err / dp_scale, dp_err)
        e2 = np.where(de_scale > 0, de_err / de_scale, de_err)
    return float(np.max(e1, initial=0.0)), float(np.max(e2, initial=0.0))


def mean_field_errors(gpu, ref, gas_sel=None):
    """Per gas owner: the condition-aware error of mean_field_error, the larger
    over the momentum components and the energy."""
    sel = slice(None) if gas_sel is None else gas_sel
    dp_err = np.abs(gpu["dp_gas"][sel] - ref["dp_gas"][sel])                 # [n, 3]
    de_err = np.abs(gpu["de_gas"][sel] - ref["de_gas"][sel])
    dp_scale = np.maximum(np.abs(ref["dp_gas"][sel]), ref["dp_abs"][sel])    # per component
    de_scale = np.maximum(np.abs(ref["de_gas"][sel]), ref["de_abs"][sel])
    with np.errstate(invalid="ignore", divide="ignore"):
        cond = np.maximum(np.where(dp_scale > 0, dp_err / dp_scale, dp_err).max(axis=1),
                          np.where(de_scale > 0, de_err / de_scale, de_err))
    return cond


def decision_report(gpu, ref, dm_sel=None):
    """Partner choices on DM not flagged near-threshold by the oracle."""
    sel = np.arange(len(ref["partner"])) if dm_sel is None else np.asarray(dm_sel)
    flags = ref["flags"][sel]
    ok = flags == 0
    g = gpu["partner"][sel]
    r = ref["partner"][sel]
    mism = np.nonzero(ok & (g != r))[0]
    return {"compared": int(ok.sum()), "excluded": int((~ok).sum()), "mismatch": int(mism.size),
            "mismatch_idx": sel[mism], "scatters": int((r >= 0).sum())}


def kick_error(gpu, ref, dm_sel=None):
    """Max |dv_gpu - dv_oracle| / max(|dv_oracle|, 1) over DM with equal partners."""
    sel = np.arange(len(ref["partner"])) if dm_sel is None else np.asarray(dm_sel)
    same = (gpu["partner"][sel] == ref["partner"][sel])
    a = gpu["dv_dm"][sel][same]
    b = ref["dv_dm"][sel][same]
    if a.size == 0:
        return 0.0
    den = np.maximum(np.linalg.norm(b, axis=1), 1.0)
    return float(np.max(np.linalg.norm(a - b, axis=1) / den))
