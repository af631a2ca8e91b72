"""FP64 reference of the learned rate closure (test infrastructure only).

The closure replaces the rate integrals of eq. scrA / scrB (Appendix B) for a
power-law cross section sigma-bar = sigma0 (v/c)^n by a small network.  It is
an extension of the paper's method, not part of it; everything here is the
plain definition, written for checking the HIP kernels:

  inputs   x1 = w / vs_gas, x2 = T_DM / T_gas, x3 = log10(m_chi / mu), n.
  With a Maxwellian DM population the relative velocity is Gaussian with
  dispersion vth = vs_gas r, r = sqrt(1 + x2 10^{-x3}), so (Appendix B)
      Ahat / vs^{n+1} = r^{n+1} (alpha_n/3) 1F1(-(n+1)/2, 5/2, -u^2/2),
      Bhat / vs^{n+3} = r^{n+3}  alpha_n    1F1(-(n+3)/2, 3/2, -u^2/2),
  u = x1 / r.  The network learns the residual of the two 1F1 terms over
  base functions a_A(u), a_B(u) that are exact at u = 0 and share the
  large-u power (`base_logs`), as a function of s = 2 u/(u + 2) - 1 and a
  one-hot encoding of n.

  network  z1 = W1 [s, onehot(n)] + b1, then ReLU; two 64x64 ReLU layers; a
  64 -> 2 output layer.  Quantisation points (bfloat16, round to nearest
  even) are those of the MFMA kernels: every weight, the activations that
  enter layers 2-4, and the error signals that enter the two MFMA products
  of the backward pass; the input s is carried as a bfloat16 hi/lo pair.
  Biases, accumulations and the optimiser are FP32 on the GPU, FP64 here.

Parameter vector (float32 on the GPU, this order, row-major W[out][in]):
  W1[64][5], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[2][64], b4[2].
"""
from __future__ import annotations

import math

import numpy as np

from . import alpha_n, hyp1f1_negx_v

N_VALUES = (-4, -2, 0, 2)
HIDDEN = 64
N_IN = 5                 # s and the one-hot of n
T_SCALE = 2.0            # s = 2 u / (u + T_SCALE) - 1
LOSS_SCALE = 10.0       # L = LOSS_SCALE^2 sum_{b,k} (o_bk - y_bk)^2 / (2 B)
U_MAX = 1000.0           # trained range of u; beyond it the kernels use quadrature

SHAPES = [("W1", (HIDDEN, N_IN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (HIDDEN, HIDDEN)), ("b3", (HIDDEN,)), ("W4", (2, HIDDEN)), ("b4", (2,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    The value is first rounded to binary32, as the GPU holds it."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64).reshape(np.shape(a))


# ----------------------------------------------------------------------------- features and labels
def similarity(x: np.ndarray):
    """u = x1 / r and r = sqrt(1 + x2 10^{-x3}) for samples x[:, 0:4]."""
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt(1.0 + x[:, 1] * 10.0 ** (-x[:, 2]))
    return x[:, 0] / r, r


def n_index(nv) -> np.ndarray:
    nv = np.asarray(nv)
    idx = np.full(nv.shape, -1, dtype=np.int64)
    for k, v in enumerate(N_VALUES):
        idx[nv == v] = k
    if np.any(idx < 0):
        raise ValueError("n must be one of -4, -2, 0, 2")
    return idx


def net_input(u: np.ndarray) -> np.ndarray:
    """s = 2u/(u+2) - 1 as the kernels carry it: binary32, then a bfloat16
    hi/lo pair whose sum enters the first layer."""
    s = (2.0 * u / (u + T_SCALE) - 1.0).astype(np.float32).astype(np.float64)
    hi = bf16(s)
    return hi + bf16(s - hi)


# Shape constants c1 of the base functions, per n (rows -4, -2, 0, 2) and
# term (A, B): the value (to 3 decimals) that minimises the largest |residual|
# over 0 <= u <= 1000.  Any positive value gives a valid base; this choice
# keeps the residual the network has to represent small (largest 0.087).
C1 = {-4: (0.833, 0.694), -2: (4.327, 4.114), 0: (8.061, 7.967), 2: (11.981, 12.089)}


def base_logs(u: np.ndarray, n: int):
    """ln a_A(u), ln a_B(u) with a = (c0 + c1 u^2 + u^4)^{p/4}, p = n+1 (A),
    n+3 (B), and c0 = (alpha_n/3)^{4/p} (A), alpha_n^{4/p} (B): each equals its
    1F1 term of Appendix B at u = 0 and shares its leading power u^p at large u."""
    al = alpha_n(n)
    pA, pB = n + 1, n + 3
    c0A, c0B = (al / 3.0) ** (4.0 / pA), al ** (4.0 / pB)
    c1A, c1B = C1[n]
    u2 = u * u
    return 0.25 * pA * np.log(c0A + u2 * (c1A + u2)), 0.25 * pB * np.log(c0B + u2 * (c1B + u2))


def exact_logs(u: np.ndarray, n: int):
    """ln[(alpha_n/3) 1F1(-(n+1)/2, 5/2, -u^2/2)], ln[alpha_n 1F1(-(n+3)/2, 3/2, -u^2/2)]."""
    al = alpha_n(n)
    x = 0.5 * u * u
    fA = al / 3.0 * hyp1f1_negx_v(-0.5 * (n + 1), 2.5, x)
    fB = al * hyp1f1_negx_v(-0.5 * (n + 3), 1.5, x)
    return np.log(fA), np.log(fB)


def labels(x: np.ndarray) -> np.ndarray:
    """Residual targets y = (ln fA - ln a_A, ln fB - ln a_B) for samples x."""
    u, _ = similarity(x)
    nv = np.asarray(x)[:, 3]
    y = np.zeros((len(u), 2))
    for v in N_VALUES:
        m = nv == v
        if not np.any(m):
            continue
        eA, eB = exact_logs(u[m], v)
        bA, bB = base_logs(u[m], v)
        y[m, 0] = eA - bA
        y[m, 1] = eB - bB
    return y


def log_rates(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """(ln Ahat/vs^{n+1}, ln Bhat/vs^{n+3}) from residuals y."""
    u, r = similarity(x)
    nv = np.asarray(x)[:, 3]
    out = np.zeros((len(u), 2))
    for v in N_VALUES:
        m = nv == v
        if not np.any(m):
            continue
        bA, bB = base_logs(u[m], v)
        out[m, 0] = (v + 1) * np.log(r[m]) + bA + y[m, 0]
        out[m, 1] = (v + 3) * np.log(r[m]) + bB + y[m, 1]
    return out


def exact_log_rates(x: np.ndarray) -> np.ndarray:
    return log_rates(x, labels(x))


# ----------------------------------------------------------------------------- network
def forward(p: np.ndarray, x: np.ndarray, quant: bool = True) -> dict:
    """Network output o (residual estimate) and the intermediates the
    backward pass needs.  quant=False drops every bfloat16 rounding."""
    q = bf16 if quant else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(p)
    u, _ = similarity(x)
    s = net_input(u) if quant else 2.0 * u / (u + T_SCALE) - 1.0
    ni = n_index(np.asarray(x)[:, 3])
    oh = np.zeros((len(u), 4))
    oh[np.arange(len(u)), ni] = 1.0
    f = np.concatenate([s[:, None], oh], axis=1)
    z1 = f @ q(P["W1"]).T + P["b1"]
    a1 = q(np.maximum(z1, 0.0))
    z2 = a1 @ q(P["W2"]).T + P["b2"]
    a2 = q(np.maximum(z2, 0.0))
    z3 = a2 @ q(P["W3"]).T + P["b3"]
    a3 = q(np.maximum(z3, 0.0))
    o = a3 @ q(P["W4"]).T + P["b4"]
    return {"f": f, "a1": a1, "a2": a2, "a3": a3, "o": o, "P": P, "q": q}


def loss(o: np.ndarray, y: np.ndarray) -> float:
    """L = LOSS_SCALE^2 sum_{b,k} (o_bk - y_bk)^2 / (2 B)."""
    return float(LOSS_SCALE ** 2 * np.sum((o - y) ** 2) / (2 * len(o)))


def backward(p: np.ndarray, x: np.ndarray, y: np.ndarray, quant: bool = True):
    """(loss, gradient in the parameter layout) for one batch.  The error
    signals that enter the two MFMA products (layers 3 -> 2 and 2 -> 1) and
    the weight-gradient products of layers 2 and 3 are rounded to bfloat16
    first; the output error and the layer-1 error stay unrounded.
    Quantisers pass gradients straight through."""
    F = forward(p, x, quant)
    q, P = F["q"], F["P"]
    B = len(y)
    e = LOSS_SCALE ** 2 * (F["o"] - y) / B
    g = {}
    g["W4"] = e.T @ F["a3"]
    g["b4"] = e.sum(0)
    d3 = (e @ q(P["W4"])) * (F["a3"] > 0)
    g3 = q(d3)
    g["W3"] = g3.T @ F["a2"]
    g["b3"] = d3.sum(0)
    d2 = (g3 @ q(P["W3"])) * (F["a2"] > 0)
    g2 = q(d2)
    g["W2"] = g2.T @ F["a1"]
    g["b2"] = d2.sum(0)
    d1 = (g2 @ q(P["W2"])) * (F["a1"] > 0)
    g["W1"] = d1.T @ F["f"]
    g["b1"] = d1.sum(0)
    return loss(F["o"], y), pack(g)


def lr_at(t: int, total: int, lr0: float, lr_min: float) -> float:
    """Cosine schedule from lr0 (t = 1) towards lr_min (t = total + 1)."""
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * (t - 1) / total))


def adam(p, g, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) on parameters p with gradient g.
    Returns the new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def predict_log_rates(p: np.ndarray, x: np.ndarray, quant: bool = True) -> np.ndarray:
    return log_rates(x, forward(p, x, quant)["o"])
