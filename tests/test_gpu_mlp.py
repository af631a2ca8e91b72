"""HIP kernels of the learned rate closure vs the FP64 reference (oracle/mlp.py).

- labels (binary64 quadrature on the GPU) vs the exact 1F1 terms: 1e-10;
- forward (bfloat16 MFMA, binary32 accumulation) vs the reference with the
  same rounding points: 99 % of outputs within 1e-5, all within 2e-3 (a
  bfloat16 rounding of an activation can land on the other side of a
  rounding boundary when binary32 and binary64 sums straddle it);
- gradient vs the reference backward: 1e-3 relative per parameter tensor;
- Adam steps vs the reference optimiser; graph replay bit-identical to eager;
- trained on 2 000 000 GPU-made samples: relative rate error <= 1e-3 on a
  held-out set of 200 000 (the accuracy bar of the closure);
- the interaction step with network rates vs the oracle, and its pass time
  against the quadrature it replaces.
"""
from __future__ import annotations

import time

import numpy as np
import pytest

import workloads
from parity_util import decision_report, kick_error, mean_field_error, run_gpu

pytestmark = pytest.mark.gpu

TRAIN_EPOCHS = 200


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2603_24688_amd as dmb
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dmb.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _log(msg):
    print(msg, flush=True)


def test_mlp_labels(ctx):
    from oracle import mlp
    x = workloads.mlp_samples(20000, seed=(4, 20))
    got = ctx.mlp_labels(_dev(x)).cpu().numpy()
    ref = mlp.labels(x)
    err = np.max(np.abs(got - ref))
    _log(f"[labels] max |y_gpu - y_ref| = {err:.2e}")
    assert err < 1e-10


def test_mlp_params_roundtrip(ctx):
    p = workloads.mlp_params(seed=(4, 30))
    ctx.mlp_set_params(p)
    assert np.array_equal(ctx.mlp_get_params(), p)


def test_mlp_forward(ctx):
    from oracle import mlp
    p = workloads.mlp_params()
    ctx.mlp_set_params(p)
    x = workloads.mlp_samples(4096 + 37, seed=(4, 21))      # several waves and a ragged tail
    got = ctx.mlp_eval(_dev(x)).cpu().numpy()
    ref = mlp.predict_log_rates(p.astype(np.float64), x)
    err = np.abs(got - ref)
    _log(f"[forward] p99 {np.quantile(err, 0.99):.2e} max {err.max():.2e} (output scale {np.abs(ref).max():.2f})")
    assert np.quantile(err, 0.99) < 1e-5
    assert err.max() < 2e-3


def test_mlp_grad(ctx):
    from oracle import mlp
    p = workloads.mlp_params()
    ctx.mlp_set_params(p)
    x = workloads.mlp_samples(1000, seed=(4, 22))
    y = mlp.labels(x) + 0.05 * np.random.default_rng(3).normal(size=(1000, 2))
    g, L = ctx.mlp_grad(_dev(x), _dev(y))
    Lr, gr = mlp.backward(p.astype(np.float64), x, y, quant=True)
    _log(f"[grad] loss gpu {L:.8e} oracle {Lr:.8e}")
    assert abs(L - Lr) <= 1e-5 * Lr
    o = 0
    for name, shp in mlp.SHAPES:
        k = int(np.prod(shp))
        a, b = g[o:o + k].astype(np.float64), gr[o:o + k]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        _log(f"[grad] {name}: relative error {rel:.2e}")
        assert rel <= 1e-3, name
        o += k


def test_mlp_adam_steps(ctx):
    """Two full-batch Adam steps (constant learning rate) against the
    reference gradient and optimiser."""
    from oracle import mlp
    p0 = workloads.mlp_params(seed=(4, 31), scale=0.5).astype(np.float32)
    x = workloads.mlp_samples(512, seed=(4, 23))
    y = mlp.labels(x)
    ctx.mlp_set_params(p0)
    lr = 1e-3
    losses = ctx.mlp_train(_dev(x), _dev(y), epochs=2, batch=512, lr0=lr, lr_min=lr, seed=3, init=False,
                           use_graph=False)
    p2 = ctx.mlp_get_params().astype(np.float64)
    p, m, v = p0.astype(np.float64), 0.0, 0.0
    g_hist = []
    for t in (1, 2):
        L, g = mlp.backward(p.astype(np.float32).astype(np.float64), x, y, quant=True)
        assert abs(losses[t - 1] - L) <= 1e-4 * L
        g_hist.append(g)
        p, m, v = mlp.adam(p, g, m, v, t, lr)
    # where the gradient is not tiny, Adam's early steps are ~lr sign(g)
    robust = (np.abs(g_hist[0]) > 1e-5) & (np.abs(g_hist[1]) > 1e-5)
    d = np.abs(p2 - p)[robust]
    _log(f"[adam] {robust.sum()} parameters compared, max |dp| {d.max():.2e} (lr {lr})")
    assert d.max() <= 0.05 * lr
    assert np.abs(p2 - p).max() <= 2.5 * lr


def test_mlp_graph_replay_matches_eager(ctx):
    from oracle import mlp
    x = workloads.mlp_samples(8192, seed=(4, 24))
    y = mlp.labels(x)
    X, Y = _dev(x), _dev(y)
    la = ctx.mlp_train(X, Y, epochs=3, batch=1024, seed=5, init=True, use_graph=False)
    pa = ctx.mlp_get_params()
    lb = ctx.mlp_train(X, Y, epochs=3, batch=1024, seed=5, init=True, use_graph=True)
    pb = ctx.mlp_get_params()
    _log(f"[graph] losses eager {la} graph {lb}")
    assert np.array_equal(la, lb)
    assert np.array_equal(pa, pb)
    assert la[-1] < la[0]


@pytest.fixture(scope="module")
def trained(ctx):
    """The closure trained on the GPU: 2 000 000 samples labelled by binary64
    quadrature on the GPU, Adam with a cosine schedule."""
    x = workloads.mlp_samples(2_000_000, seed=(4, 1))
    X = _dev(x)
    t0 = time.time()
    Y = ctx.mlp_labels(X)
    t1 = time.time()
    losses = ctx.mlp_train(X, Y, epochs=TRAIN_EPOCHS, batch=4096, lr0=2e-3, lr_min=1e-5, seed=1, init=True,
                           use_graph=True)
    t2 = time.time()
    _log(f"[train] labels {t1 - t0:.2f} s, {TRAIN_EPOCHS} epochs {t2 - t1:.2f} s, loss {losses[0]:.3e} -> "
         f"{losses[-1]:.3e}")
    return {"params": ctx.mlp_get_params(), "losses": losses}


def _rel_rate_err(got, ref):
    return np.max(np.abs(np.expm1(got - ref)), axis=1)


def test_mlp_trained_accuracy(ctx, trained):
    from oracle import mlp
    ctx.mlp_set_params(trained["params"])
    xh = workloads.mlp_samples(200_000, seed=(4, 2))
    e = _rel_rate_err(ctx.mlp_eval(_dev(xh)).cpu().numpy(), mlp.exact_log_rates(xh))
    box = xh[:, 0] <= 10.0
    xs = workloads.mlp_samples(50_000, seed=(4, 3), ext=0.0, x2_zero=True)
    es = _rel_rate_err(ctx.mlp_eval(_dev(xs)).cpu().numpy(), mlp.exact_log_rates(xs))
    _log(f"[accuracy] held-out: max {e.max():.2e} p99 {np.quantile(e, 0.99):.2e}; x1<=10: max {e[box].max():.2e}; "
         f"x1>10: max {e[~box].max():.2e}; one DM velocity (x2=0): max {es.max():.2e}")
    assert e.max() <= 1e-3
    assert es.max() <= 1e-3


def test_mlp_rates_eval(ctx, trained, ):
    """Rates of the network path of the interaction step against the closed
    forms (binary64), including u beyond the trained range (quadrature) and
    cold gas."""
    ctx.mlp_set_params(trained["params"])
    r = np.random.default_rng(9)
    n = 50000
    w = r.uniform(0.0, 600.0, n)
    vs = np.full(n, 9.085)
    vs[:100] = 0.2          # u > 1000: quadrature fallback
    vs[100:110] = 0.0       # cold gas
    for n_pow in (-4, -2, 0, 2):
        A0, B0 = ctx.rates_eval(_dev(w), _dev(vs), n_pow, precision=0, rates=0)
        A1, B1 = ctx.rates_eval(_dev(w), _dev(vs), n_pow, precision=1, rates=2)
        A0, B0, A1, B1 = (t.cpu().numpy() for t in (A0, B0, A1, B1))
        ok = A0 > 0
        e = np.maximum(np.abs(A1[ok] / A0[ok] - 1), np.abs(B1[ok] / B0[ok] - 1))
        _log(f"[rates n={n_pow}] max relative error {e.max():.2e}")
        assert e.max() <= 1.2e-3


@pytest.mark.parametrize("n_pow", [-4, -2, 2])
def test_mlp_step_small_galaxy(ctx, trained, n_pow):
    """Interaction step with network rates (binary32) vs the oracle: the gas
    transfers within the rate accuracy, the DM side (which does not use the
    rates) to the FP32 bar."""
    import oracle
    ctx.mlp_set_params(trained["params"])
    cfg = workloads.galaxy(n_gas=20000, n_dm=80000, seed=(2, 7), n_pow=n_pow,
                           sigma0_cm2=workloads.sigma0_for_npow(n_pow))
    cfg["params"]["rates"] = 2
    gsel = np.sort(np.random.default_rng(4).choice(20000, 2000, replace=False))
    dsel = np.sort(np.random.default_rng(5).choice(80000, 4000, replace=False))
    ref = oracle.step(cfg["gas"], cfg["dm"], cfg["params"], gas_sel=gsel, dm_sel=dsel)
    gpu = run_gpu(ctx, cfg, 1)
    ep, ee = mean_field_error(gpu, ref, gsel)
    dec = decision_report(gpu, ref, dsel)
    ke = kick_error(gpu, ref, dsel)
    _log(f"[mlp step n={n_pow}] dp err {ep:.2e} dE err {ee:.2e} decisions {dec['compared']} mismatch "
         f"{dec['mismatch']} kick err {ke:.2e}")
    assert ep <= 2e-3 and ee <= 2e-3
    assert dec["mismatch"] == 0
    assert ke <= 2e-5


def test_surrogate_cost_against_quadrature(ctx, trained):
    """Gas-pass time on a 250 000 gas + 1 000 000 DM galaxy with sigma ~ v^-2:
    network rates against quadrature at K = 32 (1e-10 level) and at K = 12
    (the smallest K at the network's 1e-3 level), and the closed forms for
    reference.  The network is cheaper than the K = 32 quadrature but not than
    the K = 12 one that meets the same 1e-3 bar: at equal accuracy it brings
    no speed gain here, which the log line records (network / K = 12 time
    above 1).  Only the K = 32 ordering is asserted."""
    import torch
    import paper_2603_24688_amd as dmb
    ctx.mlp_set_params(trained["params"])
    cfg = workloads.galaxy(n_gas=250_000, n_dm=1_000_000, seed=(2, 8), n_pow=-2,
                           sigma0_cm2=workloads.sigma0_for_npow(-2))
    G, D = dmb.to_device(cfg["gas"]), dmb.to_device(cfg["dm"])
    out = dmb.alloc_out(len(cfg["gas"]["mass"]), len(cfg["dm"]["mass"]))
    par = dict(cfg["params"])
    ctx.build_cells(G, D, par, precision=1)
    ctx.set_pass_overlap(False)     # each pass's own time
    res = {}
    for name, rates, K in [("exact", 0, 0), ("quad32", 1, 32), ("quad12", 1, 12), ("mlp", 2, 32)]:
        par["rates"], par["quad_nodes"] = rates, K
        ctx.interact_step(G, D, par, out, precision=1)
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        ctx.profile_read(reset=True)
        for _ in range(3):
            ctx.interact_step(G, D, par, out, precision=1)
        ph = ctx.profile_read(reset=True)
        ctx.profile_enable(False)
        res[name] = ph["pass_gas"][0] / max(ph["pass_gas"][1], 1)
    ctx.set_pass_overlap(True)
    pairs = dmb.counters_dict(out["counters"])["pairs_gas"]
    _log("[surrogate cost] gas pass ms: " + ", ".join(f"{k} {v:.3f}" for k, v in res.items()) +
         f"; pairs {pairs}; network time / K=32 quadrature {res['mlp'] / res['quad32']:.2f}, "
         f"/ K=12 quadrature {res['mlp'] / res['quad12']:.2f}")
    assert res["mlp"] < res["quad32"]
