"""Batched boxes through the C ABI (dmb_batch_build / dmb_batch_step / dmb_batch_tune).

- every box of a batched step equals the single-box call on that box, bit for
  bit (same work items, same accumulation order);
- boxes agree with the CPU oracle to the single-box bars (FP64 1e-12, FP32
  1e-5; scatter decisions exact away from thresholds);
- nsteps replays of a captured hipGraph equal an eager step at the last
  Philox step, bit for bit, and so do nsteps eager steps;
- the autotuner picks a setting from its candidate set and results stay
  identical to single-box calls under that setting.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads
from parity_util import decision_report, kick_error, mean_field_error, run_gpu

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


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


@pytest.fixture(scope="module")
def boxes():
    # uneven sizes, sigma0 log-spaced over 4 decades, m_chi from {0.5, 1, 2, 5} m_p
    return workloads.batch(n_box=6, n_min=1200, n_max=6000, seed=(5, 2))


def _to_dev(bx, rates=0, sampling=0, aniso=False):
    import paper_2603_24688_amd as dmb
    G = [dmb.to_device(b["gas"]) for b in bx]
    D = [dmb.to_device(b["dm"]) for b in bx]
    # anisotropic scattering: a different Henyey-Greenstein g per box
    P = [dict(b["params"], rates=rates, dm_sampling=sampling, aniso_g=(0.4 * (-1) ** k if aniso else 0.0))
         for k, b in enumerate(bx)]
    O = [dmb.alloc_out(len(b["gas"]["mass"]), len(b["dm"]["mass"])) for b in bx]
    return G, D, P, O


def _host(o):
    import paper_2603_24688_amd as dmb
    r = {k: v.cpu().numpy() for k, v in o.items() if k != "counters"}
    r["counters"] = dmb.counters_dict(o["counters"])
    return r


def _same(a, b):
    for k in ("dp_gas", "de_gas", "dv_dm", "partner", "p_sum", "p_max"):
        if not np.array_equal(a[k], b[k]):
            return k
    if a["counters"] != b["counters"]:
        return "counters"
    return None


# rates 3: the per-gas Maxwellian closure; sampling 1: Rao-Blackwellised DM sampling;
# aniso: a Henyey-Greenstein g of +-0.4 per box
@pytest.mark.parametrize("precision,rates,sampling,aniso", [(0, 0, 0, False), (1, 0, 0, False), (0, 3, 0, False),
                                                            (1, 3, 0, False), (0, 0, 1, False), (1, 0, 1, False),
                                                            (1, 0, 0, True), (1, 3, 1, True)])
def test_batch_equals_single_boxes(ctx, boxes, precision, rates, sampling, aniso):
    import torch
    G, D, P, O = _to_dev(boxes, rates, sampling, aniso)
    ctx.batch_build(G, D, P, precision=precision)
    ctx.batch_step(G, D, P, O, precision=precision)
    torch.cuda.synchronize()
    for b, bx in enumerate(boxes):
        single = run_gpu(ctx, dict(bx, params=P[b]), precision)
        got = _host(O[b])
        bad = _same(got, single)
        _log(f"[batch p={precision} rates={rates} sampling={sampling} aniso={aniso}] box {b}: n={len(bx['gas']['mass'])} pairs {got['counters']['pairs_gas']} "
             f"scatters {got['counters']['scatters']} {'identical' if bad is None else 'differs in ' + bad}")
        assert bad is None


@pytest.mark.parametrize("precision,rates,sampling,aniso", [(0, 0, 0, False), (1, 0, 0, False), (1, 3, 0, False),
                                                            (1, 0, 1, False), (0, 3, 1, True)])
def test_batch_oracle_parity(ctx, boxes, precision, rates, sampling, aniso):
    import oracle
    import torch
    G, D, P, O = _to_dev(boxes, rates, sampling, aniso)
    ctx.batch_build(G, D, P, precision=precision)
    ctx.batch_step(G, D, P, O, precision=precision)
    torch.cuda.synchronize()
    for b in (0, len(boxes) - 1):
        bx = boxes[b]
        ng, nd = len(bx["gas"]["mass"]), len(bx["dm"]["mass"])
        gsel = np.sort(np.random.default_rng(b).choice(ng, min(ng, 600), replace=False))
        dsel = np.sort(np.random.default_rng(b + 10).choice(nd, min(nd, 600), replace=False))
        ref = oracle.step(bx["gas"], bx["dm"], P[b], gas_sel=gsel, dm_sel=dsel)
        got = _host(O[b])
        ep, ee = mean_field_error(got, ref, gsel)
        dec = decision_report(got, ref, dsel)
        ke = kick_error(got, ref, dsel)
        _log(f"[batch oracle p={precision} rates={rates} sampling={sampling} aniso={aniso}] box {b}: dp {ep:.2e} dE {ee:.2e} decisions {dec['compared']} "
             f"mismatch {dec['mismatch']} kick {ke:.2e}")
        assert ep <= TOL[precision] and ee <= TOL[precision]
        assert dec["mismatch"] == 0
        assert ke <= (1e-12 if precision == 0 else 2e-5)


def test_batch_graph_replay(ctx, boxes):
    import torch
    G, D, P, O = _to_dev(boxes)
    ctx.batch_build(G, D, P, precision=1)
    ctx.batch_step(G, D, P, O, precision=1, nsteps=3, graph=True)
    torch.cuda.synchronize()
    g = [_host(o) for o in O]
    ctx.batch_step(G, D, P, O, precision=1, nsteps=3, graph=False)
    torch.cuda.synchronize()
    e3 = [_host(o) for o in O]
    P2 = [dict(p, step=int(p.get("step", 0)) + 2) for p in P]
    ctx.batch_step(G, D, P2, O, precision=1, nsteps=1)
    torch.cuda.synchronize()
    e1 = [_host(o) for o in O]
    for b in range(len(boxes)):
        assert _same(g[b], e1[b]) is None, b
        assert _same(e3[b], e1[b]) is None, b
    _log(f"[batch graph] 3 replays == 3 eager steps == one step at step+2 for {len(boxes)} boxes; scatters "
         f"{[x['counters']['scatters'] for x in e1]}")


def test_batch_errors(ctx, boxes):
    import paper_2603_24688_amd as dmb
    G, D, P, O = _to_dev(boxes)
    ctx.batch_build(G, D, P, precision=1)
    bad = [dict(p) for p in P]
    bad[1]["n_pow"] = -2
    with pytest.raises(dmb.DmbError, match="DMB_EINVAL"):
        ctx.batch_step(G, D, bad, O, precision=1)
    with pytest.raises(dmb.DmbError, match="DMB_ESTALE"):
        ctx.batch_step(G[:3], D[:3], P[:3], O[:3], precision=1)
    O2 = [dict(o) for o in O]
    O2[0]["counters"] = None
    with pytest.raises(dmb.DmbError, match="DMB_EINVAL"):
        ctx.batch_step(G, D, P, O2, precision=1)


def test_batch_tune(boxes):
    """Own context: the tuned setting stays in the context it was found for."""
    import torch
    import paper_2603_24688_amd as dmb
    c = dmb.Context(0)
    try:
        G, D, P, O = _to_dev(boxes)
        ch = c.batch_tune(G, D, P, O, precision=1)
        _log(f"[batch tune] {ch}")
        assert ch["work_item"] in (32, 64, 128) and ch["subtile_delta"] in (0, 1, 2) and ch["grid_pct"] in (50, 100)
        c.batch_step(G, D, P, O, precision=1)
        torch.cuda.synchronize()
        for b in (0, len(boxes) - 1):
            assert _same(_host(O[b]), run_gpu(c, boxes[b], 1)) is None
    finally:
        c.close()
