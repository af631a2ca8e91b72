"""Pins of the CPU oracle against what the paper and mathematics fix.

Every test here checks the oracle against something other than itself:
closed forms derived independently (sympy), the defining integrals evaluated
by generic quadrature, an independent library (mpmath, numpy's Philox4x64,
scipy's k-d tree), physical invariants, or statistics of the Monte Carlo
against the mean field.  No GPU.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
PAPER = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))


# --------------------------------------------------------------------------- kernel
def test_kernel_normalisation_and_centre(orc):
    """Sec. 2.4: W integrates to 1, support [0,h); W(0,h) = 8/(pi h^3)."""
    from scipy.integrate import quad
    for h in (0.3, 1.0, 2.5):
        v = quad(lambda r: 4 * math.pi * r * r * orc.W(r, h), 0, h, points=[0.5 * h], epsabs=0, epsrel=1e-13)[0]
        assert abs(v - PAPER["kernel_normalisation"]["value"]) < 1e-13
        assert orc.W(0.0, h) == pytest.approx(8.0 / (math.pi * h ** 3), rel=1e-15)
        assert orc.W(h, h) == 0.0 and orc.W(1.0001 * h, h) == 0.0


def test_kernel_plummer_equivalence(orc):
    """Sec. 2.4: the spline softening equals Plummer softening with eps = h/2.8.
    The central potential of a unit mass with density W(r,h) is
    -G int W/r d^3x = -4 pi G int r W dr; Plummer gives -G/eps."""
    from scipy.integrate import quad
    h = 1.0
    phi0 = quad(lambda r: 4 * math.pi * r * orc.W(r, h), 0, h, points=[0.5], epsabs=0, epsrel=1e-13)[0]
    assert phi0 * h == pytest.approx(PAPER["plummer_h_over_eps"]["value"], rel=1e-13)


# --------------------------------------------------------------------------- overlap
def _g_cylindrical(d, h1, h2):
    """Overlap by generic 2-D quadrature in cylindrical coordinates (an
    independent route: the oracle integrates in spherical coordinates with a
    closed-form inner integral)."""
    from scipy.integrate import quad
    import oracle as orc
    lo, hi = max(-h1, d - h2), min(h1, d + h2)
    if hi <= lo:
        return 0.0

    def inner(z):
        rmax2 = min(h1 * h1 - z * z, h2 * h2 - (z - d) ** 2)
        if rmax2 <= 0:
            return 0.0
        f = lambda rho: 2 * math.pi * rho * orc.W(math.hypot(rho, z), h1) * orc.W(math.hypot(rho, z - d), h2)
        br = [x for x in (math.sqrt(max(0.0, (0.5 * h1) ** 2 - z * z)),
                          math.sqrt(max(0.0, (0.5 * h2) ** 2 - (z - d) ** 2))) if 0 < x < math.sqrt(rmax2)]
        return quad(f, 0, math.sqrt(rmax2), points=br or None, epsabs=1e-13, epsrel=1e-11, limit=200)[0]

    pts = sorted({x for x in (-0.5 * h1, 0.5 * h1, d - 0.5 * h2, d + 0.5 * h2, 0.0, d) if lo < x < hi})
    return quad(inner, lo, hi, points=pts or None, epsabs=1e-13, epsrel=1e-10, limit=200)[0]


@pytest.mark.parametrize("d,h1,h2", [(0.0, 1.0, 1.0), (0.3, 1.0, 1.0), (0.9, 1.0, 0.5), (1.2, 0.7, 1.0),
                                     (0.05, 1.0, 0.1), (0.95, 1.0, 0.1), (1.45, 1.0, 0.5)])
def test_overlap_vs_cylindrical_quadrature(orc, d, h1, h2):
    """Appendix D definition g = int W W d^3x evaluated independently."""
    ref = _g_cylindrical(d, h1, h2)
    assert orc.overlap(d, h1, h2) == pytest.approx(ref, rel=2e-8, abs=1e-11)


@pytest.mark.parametrize("h1,h2", [(1.0, 1.0), (1.0, 0.3), (0.7, 1.0), (1.0, 0.05)])
def test_overlap_normalisation(orc, h1, h2):
    """int d^3d g(d) = (int W)(int W) = 1: the overlap is the convolution of
    two unit-mass kernels."""
    from scipy.integrate import quad
    hb, hs = max(h1, h2), min(h1, h2)
    pts = sorted({p for p in (0.5 * hb - hs, 0.5 * hb - 0.5 * hs, 0.5 * hb, 0.5 * hb + 0.5 * hs, 0.5 * hb + hs,
                              hb - hs, hb - 0.5 * hs, hb, hb + 0.5 * hs, 0.5 * hs, hs) if 0 < p < h1 + h2})
    v = quad(lambda d: 4 * math.pi * d * d * orc.overlap(d, h1, h2), 0, h1 + h2, points=pts, limit=400,
             epsabs=0, epsrel=1e-13)[0]
    assert abs(v - 1.0) < 1e-11


def test_overlap_centre_closed_form(orc):
    """g(0; h, h) = int W^2 d^3x, computed symbolically from the kernel of Sec. 2.4."""
    import sympy as sp
    q = sp.symbols("q", positive=True)
    w1 = 8 / sp.pi * (1 - 6 * q ** 2 + 6 * q ** 3)
    w2 = 8 / sp.pi * 2 * (1 - q) ** 3
    exact = 4 * sp.pi * (sp.integrate(q ** 2 * w1 ** 2, (q, 0, sp.Rational(1, 2)))
                         + sp.integrate(q ** 2 * w2 ** 2, (q, sp.Rational(1, 2), 1)))
    exact = float(sp.nsimplify(exact))
    for h in (1.0, 0.37):
        assert orc.overlap(0.0, h, h) == pytest.approx(exact / h ** 3, rel=1e-14)
    assert exact == pytest.approx(982.0 / (315.0 * math.pi), rel=1e-15)


def test_overlap_limits_and_support(orc):
    """Narrow second kernel: g -> W(d; h_big) (Appendix D, eta -> 0); zero for
    d >= h_i + h_j; symmetric in (h_i, h_j); continuous at d -> 0."""
    for d in (0.1, 0.3, 0.6, 0.8):
        assert orc.overlap(d, 1.0, 1e-4) == pytest.approx(orc.W(d, 1.0), rel=1e-6)
    assert orc.overlap(1.5, 1.0, 0.5) == 0.0
    assert orc.overlap(1.5000001, 1.0, 0.5) == 0.0
    assert orc.overlap(1.4999, 1.0, 0.5) > 0.0
    for d in (0.0, 0.2, 0.7, 1.1):
        assert orc.overlap(d, 0.4, 0.9) == orc.overlap(d, 0.9, 0.4)
    assert orc.overlap(1e-9, 1.0, 0.6) == pytest.approx(orc.overlap(0.0, 1.0, 0.6), rel=1e-12)
    assert orc.overlap(1e-5, 1.0, 0.6) == pytest.approx(orc.overlap(0.0, 1.0, 0.6), rel=1e-9)


def _H_shell_closed(delta, eta):
    """h_b^3 g within h_s/2 of contact, rho = (1 + eta - delta)/eta <= 1/2: only
    the outer branch 2(1 - q)^3 of both kernels takes part, and the Appendix D
    integral is one polynomial piece with the closed form
    eta^3 rho^8 512/(pi delta) [1/1120 - (1 + eta) rho/2520 + eta rho^2/6300]."""
    import mpmath as mp
    rho = (1 + eta - delta) / eta
    return eta ** 3 * rho ** 8 * 512 / (mp.pi * delta) * (mp.mpf(1) / 1120 - (1 + eta) * rho / 2520
                                                         + eta * rho ** 2 / 6300)


def test_overlap_near_contact_closed_form_and_conditioning(orc):
    """Near contact the overlap goes as rho^8 and, for small eta, its integrand
    sits on a window of width ~eta: a quadrature in s carries a relative
    rounding error of order eps (1/nu + 1/eta), nu = 1 - d/(h_b + h_s).  At
    rho = 0.2 ... 0.45 the oracle equals the closed form to 1e-13 (2e-14/eta for
    small eta); nearer contact (nu down to 1e-7) its error, against the closed
    form at 50 digits for the same rounded delta and eta, stays below
    4 eps (1/nu + 1/eta)."""
    import mpmath as mp
    mp.mp.dps = 50
    for hb, hs, rho in [(1.0, 0.5, 0.3), (1.0, 1.0, 0.2), (1.3, 0.7, 0.45), (1.0, 0.01, 0.4)]:
        d = hb + hs - rho * hs
        ref = float(_H_shell_closed(mp.mpf(d / hb), mp.mpf(hs / hb)))
        assert orc.overlap(d, hb, hs) * hb ** 3 == pytest.approx(ref, rel=1e-13 + 2e-14 * hb / hs)
    r = np.random.default_rng(11)
    eps, worst, n = 1.11e-16, 0.0, 0
    for _ in range(200):
        hb = r.uniform(0.1, 2.0)
        eta = 10 ** r.uniform(-4, 0)
        hs = eta * hb
        d = (1 - 10 ** r.uniform(-7, -2)) * (hb + hs)
        delta, et = d / hb, hs / hb
        if (1 + et - delta) / et > 0.5:
            continue
        ref = float(_H_shell_closed(mp.mpf(delta), mp.mpf(et)))
        nu = 1 - d / (hb + hs)
        worst = max(worst, abs(orc.overlap(d, hb, hs) * hb ** 3 / ref - 1) / (eps * (1 / nu + 1 / et)))
        n += 1
    assert n > 100
    assert worst < 4.0


# --------------------------------------------------------------------------- 1F1 and the rates
AB_PAIRS = [(-0.5 * (n + 1), 2.5) for n in (-4, -2, 0, 2)] + [(-0.5 * (n + 3), 1.5) for n in (-4, -2, 0, 2)]


@pytest.mark.parametrize("a,b", AB_PAIRS)
def test_hyp1f1_vs_mpmath(orc, a, b):
    """Sec. 2.4: 1F1(a,b;-x) for small a, b; series below x = 50 and the
    paper's five-term expansion above it, with the paper's < 1e-14 claim."""
    import mpmath
    mpmath.mp.dps = 40
    worst_lo = worst_hi = 0.0
    for x in list(np.linspace(0, 49.9, 120)) + [1e-8, 1e-3, 0.5]:
        ref = float(mpmath.hyp1f1(a, b, -mpmath.mpf(float(x))))
        worst_lo = max(worst_lo, abs(orc.hyp1f1_negx(a, b, x) / ref - 1))
    for x in list(np.geomspace(50, 1e6, 80)):
        ref = float(mpmath.hyp1f1(a, b, -mpmath.mpf(float(x))))
        worst_hi = max(worst_hi, abs(orc.hyp1f1_negx(a, b, x) / ref - 1))
    assert worst_lo < 2e-14
    assert worst_hi < PAPER["asymptotic_max_rel_err"]["value"]


def _closed_forms(n, x):
    """Erf/exp closed forms of the two 1F1 for integer n (derived with sympy
    from the power series; independent of the oracle's series)."""
    E = math.erf(math.sqrt(x))
    sp_ = math.sqrt(math.pi)
    ex = math.exp(-x)
    rx = math.sqrt(x)
    if n == -4:
        FA = -1.5 * ex / x + 0.75 * sp_ * E / x ** 1.5
        FB = sp_ * E / (2 * rx)
    elif n == -2:
        FA = 0.75 * ex / x + 0.75 * sp_ * E / rx - 3 * sp_ * E / (8 * x ** 1.5)
        FB = 0.5 * sp_ * rx * E + 0.5 * ex + sp_ * E / (4 * rx)
    elif n == 0:
        FA = 3.0 / 32.0 * (sp_ * (4 * x * x + 4 * x - 1) * E / x ** 1.5 + 2 * (2 * x + 1) * ex / x)
        FB = (sp_ * (4 * x * x + 12 * x + 3) * E + 2 * rx * (2 * x + 5) * ex) / (16 * rx)
    elif n == 2:
        FA = (sp_ * x * (8 * x ** 3 + 36 * x * x + 18 * x - 3) * E + 2 * x ** 1.5 * (4 * x * x + 16 * x + 3) * ex) / (
            64 * x ** 2.5)
        FB = (sp_ * (8 * x ** 3 + 60 * x * x + 90 * x + 15) * E + 2 * rx * (4 * x * x + 28 * x + 33) * ex) / (96 * rx)
    return FA, FB


def test_closed_forms_are_1f1():
    """The closed forms used as a pin are themselves checked against sympy's
    hyper() expansion symbolically at a rational point."""
    import mpmath
    mpmath.mp.dps = 30
    for n in (-4, -2, 0, 2):
        for x in (0.7, 3.0, 20.0):
            FA, FB = _closed_forms(n, x)
            assert FA == pytest.approx(float(mpmath.hyp1f1(-(n + 1) / 2, 2.5, -x)), rel=1e-12)
            assert FB == pytest.approx(float(mpmath.hyp1f1(-(n + 3) / 2, 1.5, -x)), rel=1e-12)


@pytest.mark.parametrize("n", [-4, -2, 0, 2])
def test_rates_vs_closed_forms(orc, n):
    """Appendix B power-law forms of A and B against the erf/exp closed forms."""
    vs = 9.085
    al = 2 ** ((n + 5) / 2) * math.gamma(3 + n / 2) / math.sqrt(math.pi)
    for w in (2.0, 9.0, 30.0, 80.0, 200.0):
        x = w * w / (2 * vs * vs)
        FA, FB = _closed_forms(n, x)
        A, B = orc.rates(n, w, vs)
        assert A == pytest.approx(al / 3 * vs ** (n + 1) * FA, rel=1e-12)
        assert B == pytest.approx(al * vs ** (n + 3) * FB, rel=1e-12)


def _rates_by_definition(n, w, vs):
    """eq. scrA / scrB evaluated directly: d^3u over a Gaussian G(w-u, vs^2)
    with sigma-bar(u) = u^n, in spherical coordinates about w (2-D quadrature)."""
    from scipy.integrate import dblquad
    norm = (2 * math.pi * vs * vs) ** -1.5

    def gauss(u, c):
        return norm * math.exp(-(u * u + w * w - 2 * u * w * c) / (2 * vs * vs))

    umax = w + 12 * vs
    A = dblquad(lambda c, u: 2 * math.pi * u * u * gauss(u, c) * u * (u * c / w) * u ** n, 0, umax, -1, 1,
                epsabs=0, epsrel=1e-10)[0]
    B = dblquad(lambda c, u: 2 * math.pi * u * u * gauss(u, c) * u ** 3 * u ** n, 0, umax, -1, 1,
                epsabs=0, epsrel=1e-10)[0]
    return A, B


@pytest.mark.parametrize("n", [-2, 0, 2])
def test_rates_vs_definition(orc, n):
    """alpha_n, the 1F1 parameters and the vs powers against the defining
    integrals (eq. scrA, scrB) with sigma-bar = (v/c)^n folded out."""
    for w, vs in ((15.0, 9.0), (3.0, 9.0), (50.0, 22.0)):
        Ad, Bd = _rates_by_definition(n, w, vs)
        A, B = orc.rates(n, w, vs)
        assert A == pytest.approx(Ad, rel=1e-8)
        assert B == pytest.approx(Bd, rel=1e-8)


@pytest.mark.parametrize("n", [-4, -2, 0, 2])
def test_rates_limits(orc, n):
    """w -> 0: A = alpha_n vs^{n+1}/3, B = alpha_n vs^{n+3}; w >> vs: A -> w^{n+1}
    (deterministic drag sigma-bar(w) w), B -> w^{n+3}; cold gas takes that limit."""
    vs = 5.0
    al = 2 ** ((n + 5) / 2) * math.gamma(3 + n / 2) / math.sqrt(math.pi)
    A0, B0 = orc.rates(n, 0.0, vs)
    assert A0 == pytest.approx(al / 3 * vs ** (n + 1), rel=1e-14)
    assert B0 == pytest.approx(al * vs ** (n + 3), rel=1e-14)
    w = 5e4
    A, B = orc.rates(n, w, vs)
    assert A == pytest.approx(w ** (n + 1), rel=1e-6)
    assert B == pytest.approx(w ** (n + 3), rel=1e-6)
    Ac, Bc = orc.rates(n, 40.0, 0.0)
    assert Ac == pytest.approx(40.0 ** (n + 1), rel=1e-15)


def _gauss_expect(f, V, s, nh=64, nl=64):
    """E[f(v)] for v ~ N((V,0,0), s^2 I) where f depends on (v_x, |v_perp|):
    Gauss-Hermite in v_x, Gauss-Laguerre in |v_perp|^2/(2 s^2)."""
    xh, wh = np.polynomial.hermite.hermgauss(nh)
    tl, wl = np.polynomial.laguerre.laggauss(nl)
    tot = 0.0
    for a in range(nh):
        vx = V + s * math.sqrt(2) * xh[a]
        for b in range(nl):
            tot += wh[a] * wl[b] * f(vx, s * math.sqrt(2 * tl[b]))
    return tot / math.sqrt(math.pi)


@pytest.mark.parametrize("n", [-2, 0, 2])
def test_mean_field_averages_to_app_f_rates(orc, n):
    """Appendix F: averaging the per-pair gas rates (eq. gas-dVdt, gas-dTdt)
    over a Maxwellian DM population gives the two-population rates with
    v_th^2 = T_B/m_B + T_chi/m_chi.  The temperature equation is read with the
    left side d/dt[(3/2) T_B/m_B] (same convention as eq. gas-dTdt)."""
    m, mu = 2.0, 1.0
    sB, sX, V = 9.0, 20.0, 50.0
    def fp(vx, vp):
        A, _ = orc.rates(n, math.hypot(vx, vp), sB)
        return A * vx
    def fe(vx, vp):
        w = math.hypot(vx, vp)
        A, B = orc.rates(n, w, sB)
        return w * w * A - mu / (m + mu) * B
    lhs_p = _gauss_expect(fp, V, sX)
    lhs_e = _gauss_expect(fe, V, sX)
    vth = math.sqrt(sB * sB + sX * sX)
    Ath, Bth = orc.rates(n, V, vth)
    TX, TB = m * sX * sX, mu * sB * sB
    assert lhs_p == pytest.approx(Ath * V, rel=1e-9)
    assert lhs_e == pytest.approx((Bth * (TX - TB) / (m + mu) + Ath * TB / mu * V * V) / vth ** 2, rel=1e-9)


# --------------------------------------------------------------------------- Philox, uniforms, normals
def test_philox4x32_known_answers(orc):
    """Philox4x32-10 against the published known-answer vectors of its authors
    (tests/golden/philox4x32_10_kat.json): pins the multipliers, the Weyl key
    increments, the round count and the word order."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.json")
    with open(path) as f:
        kat = json.load(f)["vectors"]
    for v in kat:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        want = [int(x, 16) for x in v["out"]]
        assert [int(x) for x in orc.philox4x32(ctr, key)] == want


def test_philox_round_structure_vs_numpy(orc):
    """The 64-bit-word instance of the oracle's Philox round structure equals
    numpy's Philox4x64-10 (an independent implementation); numpy generates the
    block at counter+1."""
    r = np.random.default_rng(7)
    for _ in range(20):
        key = r.integers(0, 2 ** 63, size=2, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        ctr = r.integers(0, 2 ** 62, size=4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr)
        ref = bg.random_raw(4)
        c1 = ctr.copy()
        c1[0] += np.uint64(1)
        assert np.array_equal(orc.philox4x64(c1, key), ref)


def test_philox32_statistics(orc):
    """Counter-based 4x32 outputs: bytes uniform (chi^2), words of adjacent
    counters uncorrelated, 24-bit uniforms exact and inside (0,1)."""
    from scipy.stats import chi2
    outs = np.array([orc.philox4x32([i, 17, 3, 0], [0xDEADBEEF, 0x12345678]) for i in range(20000)],
                    dtype=np.uint64)
    by = np.concatenate([(outs >> np.uint64(s)) & np.uint64(255) for s in (0, 8, 16, 24)]).ravel()
    cnt = np.bincount(by.astype(np.int64), minlength=256)
    e = by.size / 256
    stat = ((cnt - e) ** 2 / e).sum()
    assert chi2.sf(stat, 255) > 1e-4
    u = (outs[:, 0] >> np.uint64(8)).astype(np.float64)
    c = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(c) < 0.03
    assert orc.u24(0) == 0.5 / 2 ** 24 and orc.u24(0xFFFFFFFF) == 1 - 0.5 / 2 ** 24
    assert np.float32(orc.u24(0x12345678)) == orc.u24(0x12345678)


def test_box_muller_normals(orc):
    from scipy.stats import kstest
    r = np.random.default_rng(3)
    z = np.array([orc.normals3(r.uniform(0, 1, 4)) for _ in range(20000)])
    for k in range(3):
        assert kstest(z[:, k], "norm").pvalue > 1e-4
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.03


# --------------------------------------------------------------------------- pair set
@pytest.mark.parametrize("periodic", [True, False])
def test_pair_set_vs_kdtree(orc, periodic):
    """Pair set {d_ij < h_i + h_j} (minimum image when periodic) against an
    independent k-d tree search."""
    from scipy.spatial import cKDTree
    cfg = workloads.box(n_gas=700, n_dm=500, seed=(9, 2))
    if not periodic:
        cfg["params"]["box"] = None
    gas, dm = cfg["gas"], cfg["dm"]
    got = {tuple(p) for p in orc.pairs(gas, dm, cfg["params"]).tolist()}
    L = 1.0 if periodic else None
    tg = cKDTree(gas["pos"], boxsize=L)
    td = cKDTree(dm["pos"], boxsize=L)
    rmax = gas["h"].max() + dm["h"].max()
    sm = td.sparse_distance_matrix(tg, rmax, output_type="ndarray")
    ref = {(int(i), int(j)) for i, j, d in zip(sm["i"], sm["j"], sm["v"]) if d < dm["h"][i] + gas["h"][j]}
    assert got == ref
    assert len(ref) > 1000


# --------------------------------------------------------------------------- kinematics
def test_kick_is_elastic(orc):
    """eq. scatter_chi / scatter_B: in the centre-of-mass frame of (chi, sampled
    baryon) the DM speed is unchanged by the kick, and the implied baryon kick
    conserves momentum and kinetic energy exactly."""
    cfg = workloads.box(n_gas=600, n_dm=600, seed=(4, 4), sigma0_cm2=3e-21)
    gas, dm, par = cfg["gas"], cfg["dm"], cfg["params"]
    res = orc.step(gas, dm, par)
    sc = np.nonzero(res["partner"] >= 0)[0]
    assert sc.size > 50
    mchi = par["m_chi_g"]
    key = [par["seed"] & 0xFFFFFFFF, par["seed"] >> 32]
    for i in sc[:200]:
        j = int(res["partner"][i])
        u = [orc.u24(x) for x in orc.philox4x32([i, j, par["step"], 0], key)]
        vB = gas["vel"][j] + math.sqrt(2 * gas["u"][j] / 3) * orc.normals3(u)
        mu = gas["mu"][j]
        v0 = dm["vel"][i]
        v1 = v0 + res["dv_dm"][i]
        vcm = (mchi * v0 + mu * vB) / (mchi + mu)
        assert np.linalg.norm(v1 - vcm) == pytest.approx(np.linalg.norm(v0 - vcm), rel=1e-12)
        dvB = -mchi / mu * res["dv_dm"][i]
        vB1 = vB + dvB
        ke0 = mchi * v0 @ v0 + mu * vB @ vB
        ke1 = mchi * v1 @ v1 + mu * vB1 @ vB1
        assert ke1 == pytest.approx(ke0, rel=1e-12)
        assert np.linalg.norm(v1 - vB1) == pytest.approx(np.linalg.norm(v0 - vB), rel=1e-12)


# --------------------------------------------------------------------------- Monte Carlo vs mean field
def _pair_system(sigma0, dmv=(60.0, -10.0, 5.0), n_gas=1, seed=0):
    r = np.random.default_rng(seed)
    gas = {"pos": np.array([[0.5, 0.5, 0.5]]) + r.uniform(-0.02, 0.02, (n_gas, 3)),
           "vel": r.normal(0, 5, (n_gas, 3)), "mass": np.full(n_gas, 2.0e6), "h": r.uniform(0.08, 0.12, n_gas),
           "u": r.uniform(80, 160, n_gas), "mu": np.full(n_gas, workloads.M_P)}
    dm = {"pos": np.array([[0.51, 0.49, 0.5]]), "vel": np.array([dmv]), "mass": np.array([3.0e6]),
          "h": np.array([0.1])}
    par = workloads.params(sigma0_cm2=sigma0, dt_myr=0.05, box=(1.0, 1.0, 1.0))
    return gas, dm, par


def test_categorical_draw_frequencies(orc):
    """eq. dm-update-vels: one draw per DM from the mixture; over many steps
    partner j occurs with frequency E[P_ij] and no scatter with 1 - E[P_i]."""
    from scipy.stats import chi2
    gas, dm, par = _pair_system(1.2e-22, n_gas=5, seed=1)
    S = 6000
    counts = np.zeros(6)
    psum = 0.0
    for s in range(S):
        par["step"] = s
        res = orc.step(gas, dm, par)
        j = res["partner"][0]
        counts[j if j >= 0 else 5] += 1
        psum += res["p_sum"][0]
    pbar = psum / S
    assert 0.2 < pbar < 0.8
    # expected partner frequencies from per-pair P averaged over the same steps
    exp = np.zeros(6)
    for j in range(5):
        g1 = {k: (v[j:j + 1] if isinstance(v, np.ndarray) else v) for k, v in gas.items()}
        ps = 0.0
        for s in range(0, S, 3):
            par["step"] = s
            ps += orc.step(g1, dm, par)["p_sum"][0]
        exp[j] = ps / len(range(0, S, 3)) * S
    exp[5] = S - exp[:5].sum()
    stat = ((counts - exp) ** 2 / exp).sum()
    assert chi2.sf(stat, 5) > 1e-4


@pytest.mark.parametrize("n_pow,sigma0,g", [(0, 6e-23, 0.0), (-2, 6e-23 * (299792.458 / 60) ** -2, 0.0),
                                            (0, 6e-23, 0.6), (0, 6e-23, -0.5)])
def test_mc_matches_mean_field_in_expectation(orc, n_pow, sigma0, g):
    """Appendix C: per pair, M_i E[dv_i] + dp_j = 0 and E[dE_i] + dE_j + V_j.dp_j
    = 0.  The Monte Carlo mean over many Philox steps agrees with the
    deterministic mean field within 4 standard errors.  With anisotropic
    scattering (g != 0) the Monte Carlo draws with the total cross section
    and angles from p(Omega), the mean field uses sigma-bar = (1 - g) sigma
    (Sec. 2.3); the mean field built on sigma instead is rejected."""
    gas, dm, par = _pair_system(sigma0, seed=2)
    par["n_pow"] = n_pow
    par["aniso_g"] = g
    S = 20000
    dvs = np.zeros((S, 3))
    dEs = np.zeros(S)
    v0 = dm["vel"][0]
    Mi = dm["mass"][0]
    for s in range(S):
        par["step"] = s
        res = orc.step(gas, dm, par)
        dv = res["dv_dm"][0]
        dvs[s] = Mi * dv
        dEs[s] = 0.5 * Mi * ((v0 + dv) @ (v0 + dv) - v0 @ v0)
    dp = res["dp_gas"][0]
    dE = res["de_gas"][0] + gas["vel"][0] @ dp
    m = dvs.mean(0)
    se = dvs.std(0) / math.sqrt(S)
    assert np.all(np.abs(m + dp) < 4 * se + 1e-12 * np.abs(dp).max())
    assert abs(dEs.mean() + dE) < 4 * dEs.std() / math.sqrt(S)
    assert res["counters"]["scatters"] in (0, 1)
    if g != 0.0:
        # the test has the power to see a mean field on the total cross section
        iso = orc.step(gas, dm, dict(par, aniso_g=0.0))["dp_gas"][0]
        assert np.abs(m + iso).max() > 8 * se.max()


@pytest.mark.parametrize("g", [0.7, -0.4, 0.05])
def test_anisotropic_scattering_angles(orc, g):
    """Sec. 2.2-2.3, dsigma/dOmega = sigma p(Omega) with the Henyey-Greenstein
    p of mean cos theta = g: every scatter turns the relative velocity by an
    angle whose cosine follows the law's CDF (Kolmogorov-Smirnov) with mean g,
    and keeps its magnitude (eq. scatter_chi).  Cold gas, so the incoming
    relative velocity is known; a cross section that makes every step scatter."""
    from scipy.stats import kstest
    gas, dm, par = _pair_system(1e-15, seed=3)
    gas["u"] = np.zeros(1)
    par["aniso_g"] = g
    mu = workloads.M_P
    fr = mu / (par["m_chi_g"] + mu)
    u_in = dm["vel"][0] - gas["vel"][0]
    v = np.linalg.norm(u_in)
    cos = []
    for s in range(3000):
        par["step"] = s
        res = orc.step(gas, dm, par)
        assert res["partner"][0] == 0
        u_out = u_in + res["dv_dm"][0] / fr          # dv = fr (|u| n - u)
        assert abs(np.linalg.norm(u_out) / v - 1) < 1e-12
        cos.append(u_out @ u_in / (v * v))
    cos = np.array(cos)
    cdf = lambda c: (1 - g * g) / (2 * g) * (1 / np.sqrt(1 + g * g - 2 * g * c) - 1 / (1 + g))
    assert kstest(cos, cdf).pvalue > 1e-3
    assert abs(cos.mean() - g) < 4 * cos.std() / np.sqrt(len(cos))


def test_step_outputs_structure(orc):
    """Full step on the 4096+4096 periodic box: pair counts match on both
    sides, at most one scatter per DM, crit and P>=1 diagnostics consistent."""
    cfg = workloads.box()
    res = orc.step(cfg["gas"], cfg["dm"], cfg["params"])
    c = res["counters"]
    assert c["pairs_gas"] == c["pairs_dm"] > 900_000
    assert c["scatters"] == int((res["partner"] >= 0).sum())
    assert np.all(res["p_max"] <= res["p_sum"] + 1e-300)
    assert np.all(np.isfinite(res["dp_gas"])) and np.all(np.isfinite(res["de_gas"]))
    none = res["partner"] < 0
    assert np.all(res["dv_dm"][none] == 0.0)


# --------------------------------------------------------------------------- two-population relaxation
@pytest.mark.parametrize("n", [-2, 0, 2])
def test_relaxation_rhs_is_the_maxwellian_average(orc, n):
    """The relaxation rates of oracle/relax.py equal the average, over a
    Maxwellian DM population, of the per-pair mean-field terms of eq.
    gas-dVdt / gas-dTdt (rates at the gas dispersion, relative velocity
    w = v - V_B), and conserve momentum and total energy."""
    from oracle import relax
    rho_b, rho_x, sig, m_x, mu = 1e10, 2e10, 1e-24 * (299792.458 / 200.0) ** n, 2 * 1.67262192369e-24, 1.67262192369e-24
    VX, VB, sx, sb = 50.0, 3.0, 20.0, 9.0
    d = relax.rhs([VX, VB, sx * sx, sb * sb], rho_b, rho_x, sig, n, m_x, mu)
    k = relax.coupling(sig, n, m_x, mu)

    def fp(vx, vp):
        A, _ = orc.rates(n, math.hypot(vx - VB, vp), sb)
        return A * (vx - VB)

    def fe(vx, vp):
        w = math.hypot(vx - VB, vp)
        A, B = orc.rates(n, w, sb)
        return w * w * A - mu / (m_x + mu) * B
    dVB = k * rho_x * _gauss_expect(fp, VX, sx)
    duB = k * rho_x * _gauss_expect(fe, VX, sx)
    assert d[1] == pytest.approx(dVB, rel=1e-9)
    assert 1.5 * d[3] == pytest.approx(duB, rel=1e-9)
    # conservation of momentum and of internal + bulk kinetic energy per volume
    assert abs(rho_x * d[0] + rho_b * d[1]) <= 1e-12 * rho_b * abs(d[1])
    dE = rho_x * (1.5 * d[2] + VX * d[0]) + rho_b * (1.5 * d[3] + VB * d[1])
    assert abs(dE) <= 1e-10 * rho_b * abs(1.5 * d[3])


def test_relaxation_equilibrium_is_stationary(orc):
    from oracle import relax
    m_x, mu = 2 * 1.67262192369e-24, 1.67262192369e-24
    sb2 = 80.0
    sx2 = sb2 * mu / m_x          # equal temperatures, no drift
    d = relax.rhs([7.0, 7.0, sx2, sb2], 1e10, 1e10, 1e-24, 0, m_x, mu)
    assert np.max(np.abs(d)) < 1e-12 * sb2


@pytest.mark.parametrize("name", ["box", "galaxy", "galaxy_h_spread"])
def test_grid_candidates_give_the_brute_force_step(orc, name):
    """The oracle's uniform-grid candidate search only filters: every output of
    the step (and every counter) is bit-identical to the brute-force scan over
    all particles, for a periodic box, an open galaxy and h spread over three
    decades; so are per-owner neighbour statistics."""
    import workloads
    if name == "box":
        cfg = workloads.box(n_gas=1500, n_dm=1300, seed=(18, 1), sigma0_cm2=2e-22)
    else:
        cfg = workloads.galaxy(n_gas=3000, n_dm=9000, seed=(2, 18), sigma0_cm2=1e-20)
        if name == "galaxy_h_spread":
            for sp in ("gas", "dm"):
                cfg[sp]["h"] = workloads.spread_h_log(cfg[sp]["h"], 3.0)
    a = orc.step(cfg["gas"], cfg["dm"], cfg["params"])
    b = orc.step(cfg["gas"], cfg["dm"], cfg["params"], grid=True)
    for k in ("dv_dm", "dp_gas", "de_gas", "dp_abs", "de_abs", "partner", "p_sum", "p_max", "flags"):
        assert np.array_equal(a[k], b[k]), k
    assert a["counters"] == b["counters"]
    assert a["counters"]["pairs_gas"] > 0
    r = np.random.default_rng(3)
    for owner_dm, n in ((False, len(cfg["gas"]["mass"])), (True, len(cfg["dm"]["mass"]))):
        sel = np.sort(r.choice(n, 200, replace=False))
        x = orc.pair_stats(cfg["gas"], cfg["dm"], cfg["params"], sel, owner_dm)
        y = orc.pair_stats(cfg["gas"], cfg["dm"], cfg["params"], sel, owner_dm, grid=True)
        for u, v in zip(x, y):
            assert np.array_equal(u, v)


def test_active_flags_fraction_and_independence(orc):
    """Drawn active sets (hierarchical timesteps): each species' active fraction
    is binomial about the requested value; species and steps are independent
    (Philox counters differ in the species and step words)."""
    n, f = 200_000, 0.1
    a = orc.active_flags(n, 0, 5, 0x2603246880000001, 0, f)
    b = orc.active_flags(n, 1, 5, 0x2603246880000001, 0, f)
    c = orc.active_flags(n, 0, 6, 0x2603246880000001, 0, f)
    sd = np.sqrt(f * (1 - f) / n)
    for x in (a, b, c):
        assert abs(x.mean() - f) < 5 * sd
    # joint activity of two independent draws: f^2
    for x, y in ((a, b), (a, c)):
        assert abs((x & y).mean() - f * f) < 5 * np.sqrt(f * f * (1 - f * f) / n)
    assert orc.active_flags(10, 0, 5, 1, 0, 0.0).sum() == 0 and orc.active_flags(10, 0, 5, 1, 0, 1.0).sum() == 10


# --------------------------------------------------------------------------- per-gas Maxwellian closure
def _crowded_gas(dm_vel, seed):
    """One gas particle among many DM inside its kernel reach."""
    r = np.random.default_rng(seed)
    n = len(dm_vel)
    x = r.normal(size=(n, 3))
    x *= (0.14 * r.uniform(size=n) ** (1 / 3) / np.linalg.norm(x, axis=1))[:, None]
    gas = {"pos": np.array([[0.5, 0.5, 0.5]]), "vel": np.array([[3.0, -2.0, 1.0]]), "mass": np.array([1.0e6]),
           "h": np.array([0.1]), "u": np.array([workloads.u_from_T(1e4)]), "mu": np.array([workloads.M_P])}
    dm = {"pos": 0.5 + x, "vel": dm_vel, "mass": np.full(n, 2.0e3), "h": np.full(n, 0.05)}
    par = workloads.params(sigma0_cm2=1e-24, dt_myr=0.05)
    return gas, dm, par


@pytest.mark.parametrize("n_pow,tol", [(0, 0.02), (-2, 0.02), (2, 0.06)])
def test_gas_closure_equals_pair_sum_for_maxwellian_dm(orc, n_pow, tol):
    """Per-gas Maxwellian closure (Appendix F rates with the kernel-weighted DM
    density, drift and dispersion around the gas particle): for DM drawn from
    one Maxwellian it agrees with the per-pair mean field of eq. gas-dVdt /
    gas-dTdt within the sampling noise of 80 000 neighbours (about 5 standard
    deviations, measured over seeds; sigma ~ v^2 weights the tails and is
    noisier); for two cold DM streams, far from Maxwell-Boltzmann, its energy
    transfer is off by more than 5 % for n = 0 and -2."""
    N = 80_000
    r = np.random.default_rng(40 + n_pow)
    W, sx = np.array([40.0, 0.0, 0.0]), 30.0
    gas, dm, par = _crowded_gas(W + sx * r.normal(size=(N, 3)), 41)
    par["n_pow"] = n_pow
    pair = orc.step(gas, dm, par)
    clos = orc.step(gas, dm, dict(par, rates=3))
    assert pair["counters"]["pairs_gas"] == clos["counters"]["pairs_gas"] == N
    ep = np.abs(clos["dp_gas"][0] - pair["dp_gas"][0]).max() / np.abs(pair["dp_gas"][0]).max()
    ee = abs(clos["de_gas"][0] / pair["de_gas"][0] - 1)
    assert ep < tol and ee < tol, (ep, ee)
    streams = np.where(r.uniform(size=(N, 1)) < 0.5, 1.0, -1.0) * np.array([60.0, 0.0, 0.0]) + \
        5.0 * r.normal(size=(N, 3))
    gas, dm, par = _crowded_gas(streams, 42)
    par["n_pow"] = n_pow
    pair = orc.step(gas, dm, par)
    clos = orc.step(gas, dm, dict(par, rates=3))
    ee = abs(clos["de_gas"][0] / pair["de_gas"][0] - 1)
    if n_pow in (0, -2):
        assert ee > 0.05, ee


@pytest.mark.parametrize("T", [1e4, 0.0])
@pytest.mark.parametrize("n_pow", [-4, -2, 0, 2])
def test_gas_closure_single_velocity_reduces_to_pair_sum(orc, n_pow, T):
    """When every DM neighbour moves with one velocity the closure's dispersion
    s_X vanishes, vth = varsigma, and the Maxwellian average is the per-pair
    mean field itself: dp and dE agree to rounding, for warm gas and in the
    cold limit (u = 0, where both sides take A = w^{n+1}, B = w^{n+3})."""
    N = 40
    gas, dm, par = _crowded_gas(np.tile([[25.0, -7.0, 12.0]], (N, 1)), 43)
    gas["u"] = np.array([workloads.u_from_T(T)]) if T > 0 else np.zeros(1)
    dm["mass"] = np.linspace(1e3, 3e3, N)
    par["n_pow"] = n_pow
    pair = orc.step(gas, dm, par)
    clos = orc.step(gas, dm, dict(par, rates=3))
    assert pair["counters"]["pairs_gas"] == clos["counters"]["pairs_gas"] == N
    np.testing.assert_allclose(clos["dp_gas"][0], pair["dp_gas"][0], rtol=1e-11)
    np.testing.assert_allclose(clos["de_gas"][0], pair["de_gas"][0], rtol=1e-11)


# --------------------------------------------------------------------------- Rao-Blackwellised DM sampling
@pytest.mark.parametrize("n_pow", [-2, 0, 2])
def test_rb_expected_probability_is_the_mean_of_P(orc, n_pow):
    """Pbar_ij uses E|w - varsigma z|^{n+1} = Bhat of power n - 2.  Checked
    against a 4M-sample numpy average, against the textbook means of the
    noncentral chi distribution with 3 degrees of freedom (E 1/|u| =
    erf(a/sqrt2)/(a vs), E|u| = vs [sqrt(2/pi) e^{-a^2/2} + (a + 1/a)
    erf(a/sqrt2)]), and at the step level: the Rao-Blackwellised P_i equals
    the mean over Philox steps of the per-pair P_i (5 standard errors)."""
    from scipy.special import erf
    r = np.random.default_rng(7)
    z = r.normal(size=(4_000_000, 3))
    for w, vs in ((3.0, 2.0), (0.4, 1.5), (12.0, 1.0)):
        v = np.linalg.norm(np.array([w, 0.0, 0.0]) - vs * z, axis=1) ** (n_pow + 1)
        got = orc.rates(n_pow - 2, w, vs)[1]
        assert abs(got - v.mean()) < 5 * v.std() / math.sqrt(len(v)), (w, vs, got, v.mean())
        a = w / vs
        if n_pow == -2:
            assert got == pytest.approx(erf(a / math.sqrt(2)) / (a * vs), rel=1e-13)
        if n_pow == 0:
            ref = vs * (math.sqrt(2 / math.pi) * math.exp(-a * a / 2) + (a + 1 / a) * erf(a / math.sqrt(2)))
            assert got == pytest.approx(ref, rel=1e-13)
    gas, dm, par = _pair_system(3e-23, n_gas=4, seed=3)
    par["n_pow"] = n_pow
    par["sigma0_cm2"] = workloads.sigma0_for_npow(n_pow, 60.0, 3e-23)
    rb = orc.step(gas, dm, dict(par, dm_sampling=1))["p_sum"][0]
    S = 3000
    ps = np.empty(S)
    for s in range(S):
        par["step"] = s
        ps[s] = orc.step(gas, dm, par)["p_sum"][0]
    assert abs(ps.mean() - rb) < 5 * ps.std() / math.sqrt(S), (ps.mean(), rb)


def _tilted_radial_cdf(m, a, r):
    """CDF of |u| for the law |u|^m N(u; a e_x, I), from the 3-D definition:
    the density on the sphere |u| = t is t^{m+2} times the angular integral of
    the Gaussian, both integrated numerically."""
    from scipy import integrate

    def shell(t):
        ang = integrate.quad(lambda c: math.exp(-0.5 * (t * t + a * a - 2 * t * a * c)), -1.0, 1.0,
                             epsabs=0, epsrel=1e-13)[0]
        return t ** (m + 2) * ang
    lo, hi = max(0.0, a - 12.0), a + 12.0
    Z = integrate.quad(shell, lo, hi, epsabs=0, epsrel=1e-12, limit=200)[0]
    return integrate.quad(shell, lo, min(max(r, lo), hi), epsabs=0, epsrel=1e-12, limit=200)[0] / Z


@pytest.mark.parametrize("m", [-1, 1, 3])
def test_rb_radius_inverts_the_tilted_radial_law(orc, m):
    """The tilted radius at uniform u has CDF value u under the radial law
    built numerically from the 3-D density |u|^m N(u; w, I)."""
    for a in (0.0, 0.05, 1.3, 7.0):
        for u in (1e-3, 0.2, 0.5, 0.8, 0.999):
            r = orc.rb_radius(m, a, u)
            F = _tilted_radial_cdf(m, a, r)
            assert abs(F - u) < 1e-9 * max(min(u, 1 - u), 1e-3), (m, a, u, r, F)


@pytest.mark.parametrize("n_pow", [-2, 0, 2])
def test_rb_urel_follows_the_tilted_law(orc, n_pow):
    """Moments of the tilted draw (orc_rb_urel with independent uniforms)
    against importance-weighted moments of plain Gaussian samples (weights
    |u|^{n+1}): mean vector, E|u|^2 and E u_k^2, within 5 standard errors."""
    r = np.random.default_rng(11 + n_pow)
    w, vs = np.array([30.0, -20.0, 10.0]), 25.0
    N = 6000
    U = r.uniform(size=(N, 3))
    S = np.array([orc.rb_urel(n_pow, w, vs, U[k]) for k in range(N)])
    z = r.normal(size=(4_000_000, 3))
    u = w - vs * z
    wt = np.linalg.norm(u, axis=1) ** (n_pow + 1)
    wt /= wt.sum()
    for f in (lambda x: x[:, 0], lambda x: x[:, 1], lambda x: x[:, 2], lambda x: (x * x).sum(1),
              lambda x: x[:, 0] ** 2, lambda x: x[:, 2] ** 2):
        ref = (wt * f(u)).sum()
        got = f(S)
        assert abs(got.mean() - ref) < 5 * got.std() / math.sqrt(N), (got.mean(), ref)
    # cold gas: u = w exactly
    assert np.array_equal(orc.rb_urel(n_pow, w, 0.0, U[0]), w)


@pytest.mark.parametrize("n_pow,g", [(0, 0.0), (-2, 0.0), (0, 0.5)])
def test_rb_scheme_is_exact_in_law(orc, n_pow, g):
    """With P_i <= 1 the Rao-Blackwellised scheme gives the per-pair scheme's
    joint law of (partner, kick): over many Philox steps the partner
    frequencies agree (chi-square on the two-sample table) and so do the
    mean kick vector and mean |dv|^2 per partner (5 standard errors); also
    with a Henyey-Greenstein angle (g = 0.5) about the relative velocity."""
    from scipy.stats import chi2_contingency
    gas, dm, par = _pair_system(3e-23, n_gas=3, seed=5)
    par["n_pow"] = n_pow
    par["aniso_g"] = g
    par["sigma0_cm2"] = workloads.sigma0_for_npow(n_pow, 60.0, 2.5e-22)
    S = 8000
    res = {}
    for mode in (0, 1):
        parts = np.empty(S, np.int64)
        dv = np.empty((S, 3))
        pmax = 0.0
        for s in range(S):
            out = orc.step(gas, dm, dict(par, step=s, dm_sampling=mode))
            parts[s] = out["partner"][0]
            dv[s] = out["dv_dm"][0]
            pmax = max(pmax, out["p_sum"][0])
        assert pmax < 1.0
        res[mode] = (parts, dv)
    (p0, d0), (p1, d1) = res[0], res[1]
    tab = np.array([[np.sum(p == j) for j in (-1, 0, 1, 2)] for p in (p0, p1)])
    assert tab[:, 1:].sum() > 0.2 * S
    assert chi2_contingency(tab)[1] > 1e-4, tab
    for j in (0, 1, 2):
        a, b = d0[p0 == j], d1[p1 == j]
        if min(len(a), len(b)) < 200:
            continue
        for fa, fb in ((a, b), ((a * a).sum(1, keepdims=True), (b * b).sum(1, keepdims=True))):
            se = np.sqrt(fa.var(0) / len(fa) + fb.var(0) / len(fb))
            assert np.all(np.abs(fa.mean(0) - fb.mean(0)) < 5 * se), (j, fa.mean(0), fb.mean(0), se)
