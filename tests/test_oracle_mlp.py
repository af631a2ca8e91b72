"""Pins of the FP64 reference of the learned rate closure (oracle/mlp.py).

Each check compares the reference with something it does not share code
with: torch's bfloat16 conversion, mpmath's 1F1, a Gauss-Hermite average over
a Maxwellian DM population of the per-pair rates of the C oracle, torch
autograd (with its own straight-through quantisers), central differences,
and torch.optim.Adam.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
import workloads



def test_bf16_rounding_matches_torch():
    r = np.random.default_rng(11)
    a = np.concatenate([r.normal(size=20000) * 10.0 ** r.uniform(-8, 8, 20000),
                        1.0 + np.array([2.0 ** -8, 3 * 2.0 ** -8, -(2.0 ** -9), 5 * 2.0 ** -9]), [0.0, -0.0]])
    ref = torch.tensor(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(a), ref)
    # ties go to even: 1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_n_index_and_layout():
    assert list(mlp.n_index([-4, -2, 0, 2])) == [0, 1, 2, 3]
    with pytest.raises(ValueError):
        mlp.n_index([1])
    assert mlp.N_PARAMS == 8834
    p = np.arange(mlp.N_PARAMS, dtype=np.float64)
    assert np.array_equal(mlp.pack(mlp.unpack(p)), p)


def test_labels_against_mpmath():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    for n in (-4, -2, 0, 2):
        al = oracle.alpha_n(n)
        u = np.array([0.0, 0.3, 1.7, 4.2, 9.9, 37.0, 800.0])
        x = np.stack([u, np.zeros_like(u), np.zeros_like(u), np.full_like(u, n)], axis=1)
        y = mlp.labels(x)
        bA, bB = mlp.base_logs(u, n)
        for k, uk in enumerate(u):
            z = -0.5 * mpmath.mpf(uk) ** 2
            fA = al / 3 * mpmath.hyp1f1(-(n + 1) / 2, 2.5, z)
            fB = al * mpmath.hyp1f1(-(n + 3) / 2, 1.5, z)
            assert abs(y[k, 0] + bA[k] - float(mpmath.log(fA))) < 1e-12
            assert abs(y[k, 1] + bB[k] - float(mpmath.log(fB))) < 1e-12


def test_labels_limits():
    """The residual vanishes at u = 0 (the base functions equal the 1F1 terms
    there, both alpha_n/3 and alpha_n), decays like 1/u^2 at large u (the base
    shares the leading power u^{n+1}, u^{n+3} of the rates, whose large-w
    limits are sigma(w) w and sigma(w) w^3, Appendix B), and stays small in
    between."""
    for n in (-4, -2, 0, 2):
        al = oracle.alpha_n(n)
        bA, bB = mlp.base_logs(np.array([0.0]), n)
        assert abs(bA[0] - np.log(al / 3)) < 1e-14 and abs(bB[0] - np.log(al)) < 1e-14
        x0 = np.array([[0.0, 0.0, 0.0, n]])
        assert np.max(np.abs(mlp.labels(x0))) < 1e-14
        u = np.array([200.0, 400.0, 800.0])
        y = mlp.labels(np.stack([u, 0 * u, 0 * u, np.full(3, n)], axis=1))
        assert np.max(np.abs(y)) < 1e-3
        # 1/u^2 decay: doubling u divides the residual by ~4
        ratio = y[0] / np.where(y[1] == 0, 1, y[1])
        assert np.all((np.abs(y[1]) < 1e-9) | ((ratio > 3.5) & (ratio < 4.5)))
        uu = np.linspace(0.0, 30.0, 3001)
        yy = mlp.labels(np.stack([uu, 0 * uu, 0 * uu, np.full_like(uu, n)], axis=1))
        assert np.max(np.abs(yy)) < 0.09


def test_similarity_reduction_is_the_maxwellian_average():
    """With DM velocities drawn from a Maxwellian of dispersion vs_chi about
    the gas-frame drift w, the average of the per-pair rate terms A(|w'|) w'
    and B(|w'|) (C oracle, Appendix B) equals one evaluation at dispersion
    vth = sqrt(vs^2 + vs_chi^2): the reduction behind the inputs x2, x3."""
    zh, wh = np.polynomial.hermite_e.hermegauss(40)
    wh = wh / np.sqrt(2 * np.pi)
    for n in (-2, 0, 2):
        for (x1, x2, x3) in [(1.3, 5.0, 0.3), (4.0, 3.0, 0.0), (0.4, 2.0, 1.0)]:
            vs = 7.0
            vchi = vs * math.sqrt(x2 * 10.0 ** (-x3))
            w = np.array([x1 * vs, 0.0, 0.0])
            accA, accB = 0.0, 0.0
            for i, zi in enumerate(zh):
                for j, zj in enumerate(zh):
                    for k, zk in enumerate(zh):
                        wp = w + vchi * np.array([zi, zj, zk])
                        A, B = oracle.rates(n, float(np.linalg.norm(wp)), vs)
                        ww = wh[i] * wh[j] * wh[k]
                        accA += ww * A * wp[0]
                        accB += ww * B
            lr = mlp.exact_log_rates(np.array([[x1, x2, x3, n]]))[0]
            # A(w; vth) w_x and B(w; vth) from the closure's log-rates (units of vs^{n+1}, vs^{n+3})
            A_red = math.exp(lr[0]) * vs ** (n + 1) * w[0]
            B_red = math.exp(lr[1]) * vs ** (n + 3)
            assert abs(accA / A_red - 1) < 1e-6, (n, x1, x2, x3, accA, A_red)
            assert abs(accB / B_red - 1) < 1e-6, (n, x1, x2, x3, accB, B_red)


def _torch_net(p: np.ndarray, x: np.ndarray, quant: bool):
    """Independent torch implementation of the network (autograd graph).
    Quantisers: straight-through bfloat16 rounding of values (Q) and of
    incoming gradients (GQ) at the points the kernels round them."""
    class Q(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            return t.to(torch.float32).to(torch.bfloat16).to(torch.float64) if quant else t

        @staticmethod
        def backward(ctx, g):
            return g

    class GQ(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            return t

        @staticmethod
        def backward(ctx, g):
            return g.to(torch.float32).to(torch.bfloat16).to(torch.float64) if quant else g

    W = {}
    o = 0
    for name, shp in mlp.SHAPES:
        k = int(np.prod(shp))
        W[name] = torch.tensor(p[o:o + k].astype(np.float64).reshape(shp), requires_grad=True)
        o += k
    u = x[:, 0] / np.sqrt(1.0 + x[:, 1] * 10.0 ** (-x[:, 2]))
    s = 2.0 * u / (u + 2.0) - 1.0
    if quant:
        s = s.astype(np.float32).astype(np.float64)
        hi = torch.tensor(s).to(torch.float32).to(torch.bfloat16).to(torch.float64)
        lo = (torch.tensor(s) - hi).to(torch.float32).to(torch.bfloat16).to(torch.float64)
        st = hi + lo
    else:
        st = torch.tensor(s)
    onehot = torch.zeros(len(x), 4, dtype=torch.float64)
    idx = {-4: 0, -2: 1, 0: 2, 2: 3}
    for r, nv in enumerate(x[:, 3]):
        onehot[r, idx[int(nv)]] = 1.0
    f = torch.cat([st[:, None], onehot], dim=1)
    h = torch.relu(f @ Q.apply(W["W1"]).T + W["b1"])
    h = Q.apply(h)
    h = torch.relu(GQ.apply(h @ Q.apply(W["W2"]).T) + W["b2"])
    h = Q.apply(h)
    h = torch.relu(GQ.apply(h @ Q.apply(W["W3"]).T) + W["b3"])
    h = Q.apply(h)
    out = h @ Q.apply(W["W4"]).T + W["b4"]
    return out, W


def _torch_grad(p, x, y, quant):
    out, W = _torch_net(p, x, quant)
    L = mlp.LOSS_SCALE ** 2 * ((out - torch.tensor(y)) ** 2).sum() / (2 * len(y))
    L.backward()
    return float(L.detach()), np.concatenate([W[name].grad.numpy().ravel() for name, _ in mlp.SHAPES])


@pytest.mark.parametrize("quant", [False, True])
def test_forward_matches_torch(quant):
    p = workloads.mlp_params()
    x = workloads.mlp_samples(300, seed=(4, 3))
    ref, _ = _torch_net(p, x, quant)
    got = mlp.forward(p, x, quant)["o"]
    assert np.max(np.abs(got - ref.detach().numpy())) < 1e-12


@pytest.mark.parametrize("quant", [False, True])
def test_backward_matches_autograd(quant):
    p = workloads.mlp_params()
    x = workloads.mlp_samples(256, seed=(4, 4))
    y = 0.05 * np.random.default_rng(5).normal(size=(256, 2))
    L, g = mlp.backward(p, x, y, quant)
    Lt, gt = _torch_grad(p, x, y, quant)
    assert abs(L - Lt) <= 1e-12 * abs(Lt)
    assert np.max(np.abs(g - gt)) <= 1e-11 * np.max(np.abs(gt))


def test_backward_central_differences():
    p = workloads.mlp_params().astype(np.float64)
    x = workloads.mlp_samples(64, seed=(4, 5))
    y = 0.05 * np.random.default_rng(6).normal(size=(64, 2))
    _, g = mlp.backward(p, x, y, quant=False)
    r = np.random.default_rng(7)
    picks = np.concatenate([r.choice(mlp.N_PARAMS, 40, replace=False), [0, 320, 8832, 8833]])
    for i in picks:
        eps = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        Lp = mlp.loss(mlp.forward(pp, x, quant=False)["o"], y)
        Lm = mlp.loss(mlp.forward(pm, x, quant=False)["o"], y)
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_matches_torch():
    r = np.random.default_rng(8)
    p0 = r.normal(size=50)
    grads = [r.normal(size=50) for _ in range(3)]
    t = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads):
        opt.zero_grad()
        t.grad = torch.tensor(g)
        opt.step()
        p, m, v = mlp.adam(p, g, m, v, k + 1, 1e-3)
    assert np.max(np.abs(p - t.detach().numpy())) < 1e-14


def test_cosine_schedule():
    assert mlp.lr_at(1, 100, 2e-3, 1e-5) == pytest.approx(2e-3)
    assert mlp.lr_at(51, 100, 2e-3, 1e-5) == pytest.approx(0.5 * (2e-3 + 1e-5))
    assert mlp.lr_at(101, 100, 2e-3, 1e-5) == pytest.approx(1e-5)
