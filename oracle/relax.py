"""Two-population relaxation (Appendix F), FP64 reference (test infrastructure).

Uniform gas (mass density rho_B, bulk velocity V_B, 1-D dispersion s_B, so
T_B = mu s_B^2 and u_B = 3/2 s_B^2) and DM (rho_X, V_X, s_X, T_X = m_X s_X^2)
exchanging momentum and energy through a cross section sigma0 (v/c)^n.
Averaging the per-pair gas rates of eq. gas-dVdt / gas-dTdt over a
Maxwellian DM population gives rates with the combined dispersion
vth^2 = s_B^2 + s_X^2 evaluated at the drift V = V_X - V_B (Appendix F; the
temperature equation read with d/dt[(3/2) T_B / mu] on the left, the
convention of eq. gas-dTdt):
    dV_B/dt = k rho_X A(V; vth) V,
    du_B/dt = k rho_X [B(V; vth) (T_X - T_B)/(m_X + mu) + A(V; vth) T_B V^2 / mu] / vth^2,
with k = sigma0 c^-n / (m_X + mu) and A, B of eq. scrA / scrB without the
sigma0 c^-n factor.  The DM follows from conservation of momentum and of
total (internal + bulk kinetic) energy per unit volume.

Units as in the library: kpc, km/s, Msun, time kpc/(km/s), masses m_X, mu in
grams; sigma0 in cm^2.
"""
from __future__ import annotations

import math

import numpy as np

from . import rates

MSUN_G = 1.988409870698051e33
KPC_CM = 3.0856775814913673e21
C_KMS = 299792.458


def coupling(sigma0_cm2: float, n_pow: int, m_chi_g: float, mu_g: float) -> float:
    """k = sigma0 c^-n / (m_X + mu) in kpc^2 (km/s)^-n per Msun."""
    return sigma0_cm2 / KPC_CM ** 2 * C_KMS ** (-n_pow) * MSUN_G / (m_chi_g + mu_g)


def rhs(state, rho_b: float, rho_x: float, sigma0_cm2: float, n_pow: int, m_chi_g: float, mu_g: float):
    """d/dt of (V_X, V_B, s_X^2, s_B^2) (drift along one axis)."""
    VX, VB, sx2, sb2 = state
    V = VX - VB
    vth = math.sqrt(max(sx2 + sb2, 0.0))
    A, B = rates(n_pow, abs(V), vth)
    k = coupling(sigma0_cm2, n_pow, m_chi_g, mu_g)
    dVB = k * rho_x * A * V
    TX, TB = m_chi_g * sx2, mu_g * sb2
    duB = k * rho_x * (B * (TX - TB) / (m_chi_g + mu_g) + A * TB / mu_g * V * V) / (vth * vth)
    dVX = -rho_b / rho_x * dVB
    # total energy per volume: rho_x (3/2 sx2 + VX^2/2) + rho_b (uB + VB^2/2) is conserved
    dEb = rho_b * (duB + VB * dVB)
    dux = (-dEb - rho_x * VX * dVX) / rho_x
    return np.array([dVX, dVB, dux / 1.5, duB / 1.5])


def evolve(state0, t_end: float, rho_b, rho_x, sigma0_cm2, n_pow, m_chi_g, mu_g, t_eval=None):
    """Integrate with scipy's DOP853 (rtol 1e-10); returns (t, states)."""
    from scipy.integrate import solve_ivp
    sol = solve_ivp(lambda t, y: rhs(y, rho_b, rho_x, sigma0_cm2, n_pow, m_chi_g, mu_g), (0.0, t_end),
                    np.asarray(state0, dtype=np.float64), method="DOP853", rtol=1e-10, atol=1e-12,
                    t_eval=t_eval)
    return sol.t, sol.y.T
