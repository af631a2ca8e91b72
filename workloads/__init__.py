"""Seeded synthetic inputs for the DM-gas interaction step.

This module only builds particle sets (positions, velocities, masses, kernel
radii, internal energies) and run parameters; it contains none of the
interaction method's arithmetic.  Both the HIP path's tests and the CPU oracle
draw their inputs from here.

Units: kpc, km/s, Msun; time in kpc/(km/s); gas specific internal energy u in
(km/s)^2 (u = 3/2 k_B T / mu); sigma0 in cm^2; m_chi and mu in grams.

Workloads (stand-ins for the paper's periodic test box, Appendix F, and for the
AGORA isolated disk galaxy of Table 1, whose initial-condition files are not
available):
  box      periodic box, uniform random positions, Maxwellian gas and drifting
           Maxwellian DM (the paper's test problem, Appendix F / Table 3)
  galaxy   exponential gas disk + NFW halo with isotropic Jeans dispersion
  batch    many independent periodic boxes of log-uniform sizes
"""
from __future__ import annotations

import math

import numpy as np

# Physical constants (CGS) for initial-condition generation.
K_B = 1.380649e-16
M_P = 1.67262192369e-24
MSUN_G = 1.988409870698051e33
KPC_CM = 3.0856775814913673e21
G_KPC = 4.30091e-6            # kpc (km/s)^2 / Msun
MYR_IN_TUNIT = 1.0 / 977.7922216807891   # 1 Myr in kpc/(km/s)
H_FLOOR_KPC = 0.0448          # interaction-softening floor of the galaxy runs (Sec. 4)


def rng(*key) -> np.random.Generator:
    return np.random.default_rng(list(int(k) for k in key))


def u_from_T(T_K: float, mu_g: float = M_P) -> float:
    """Specific internal energy (3/2) k_B T / mu in (km/s)^2."""
    return 1.5 * K_B * T_K / mu_g / 1e10


def sigma1d_from_T(T_K: float, m_g: float) -> float:
    """1-D Maxwellian velocity dispersion sqrt(k_B T / m) in km/s."""
    return math.sqrt(K_B * T_K / m_g) / 1e5


def knn_h(pos: np.ndarray, k: int, box: float | None = None) -> np.ndarray:
    """Distance to the k-th nearest same-species neighbour (kernel support radius)."""
    from scipy.spatial import cKDTree
    tree = cKDTree(pos, boxsize=box) if box else cKDTree(pos)
    d, _ = tree.query(pos, k=k + 1, workers=-1)
    return np.ascontiguousarray(d[:, -1])


def params(sigma0_cm2=1e-24, n_pow=0, m_chi_over_mp=2.0, dt_myr=0.05, seed=0x2603246880000001,
           step=0, box_id=0, box=None) -> dict:
    return {"sigma0_cm2": float(sigma0_cm2), "n_pow": int(n_pow), "m_chi_g": float(m_chi_over_mp) * M_P,
            "dt": float(dt_myr) * MYR_IN_TUNIT, "seed": int(seed), "step": int(step), "box_id": int(box_id),
            "box": None if box is None else tuple(float(b) for b in box)}


# --------------------------------------------------------------------------- periodic box
def box(n_gas=4096, n_dm=4096, L=1.0, rho_gas=1e10, rho_dm=1e10, T_gas=1e4, T_dm=1e5,
        V_dm=(50.0, 0.0, 0.0), m_chi_over_mp=2.0, sigma0_cm2=1e-24, n_pow=0, n_ngb=32, dt_myr=0.05,
        seed=(1, 1), h_mode="knn", philox_seed=None) -> dict:
    """Periodic test box (Appendix F, Table 3 layout): gas at rest with
    temperature T_gas, DM Maxwellian at T_dm drifting with V_dm, equal-mass
    particles, uniform random positions for both species."""
    r = rng(*seed)
    Lv = float(L)
    vol = Lv ** 3
    gas_pos = r.uniform(0.0, Lv, size=(n_gas, 3))
    dm_pos = r.uniform(0.0, Lv, size=(n_dm, 3))
    m_chi = m_chi_over_mp * M_P
    s_dm = sigma1d_from_T(T_dm, m_chi)
    dm_vel = np.asarray(V_dm, dtype=np.float64)[None, :] + s_dm * r.standard_normal((n_dm, 3))
    gas_vel = np.zeros((n_gas, 3))
    if h_mode == "knn":
        h_gas = knn_h(gas_pos, n_ngb, Lv)
        h_dm = knn_h(dm_pos, n_ngb, Lv)
    else:  # radius holding n_ngb particles at the mean density
        h_gas = np.full(n_gas, (3.0 * n_ngb * vol / (4.0 * math.pi * n_gas)) ** (1.0 / 3.0))
        h_dm = np.full(n_dm, (3.0 * n_ngb * vol / (4.0 * math.pi * n_dm)) ** (1.0 / 3.0))
    gas = {"pos": gas_pos, "vel": gas_vel, "mass": np.full(n_gas, rho_gas * vol / n_gas), "h": h_gas,
           "u": np.full(n_gas, u_from_T(T_gas)), "mu": np.full(n_gas, M_P)}
    dm = {"pos": dm_pos, "vel": dm_vel, "mass": np.full(n_dm, rho_dm * vol / n_dm), "h": h_dm}
    ps = 0x2603246880000000 + int(seed[-1]) if philox_seed is None else philox_seed
    par = params(sigma0_cm2, n_pow, m_chi_over_mp, dt_myr, ps, 0, 0, (Lv, Lv, Lv))
    return {"gas": gas, "dm": dm, "params": par}


# --------------------------------------------------------------------------- galaxy
NFW_M200 = 1.074e12
NFW_R200 = 205.5
NFW_RS = 20.0
DISK_MASS = 4.297e10
GAS_FRAC = 0.2
DISK_RD = 3.0
DISK_ZD = 0.3


def _nfw_m(x):
    return np.log1p(x) - x / (1.0 + x)


def nfw_rho(r, rs=NFW_RS, m200=NFW_M200, r200=NFW_R200):
    c = r200 / rs
    rho_s = m200 / (4.0 * math.pi * rs ** 3 * _nfw_m(c))
    x = np.maximum(r, 1e-6) / rs
    return rho_s / (x * (1.0 + x) ** 2)


def nfw_menc(r, rs=NFW_RS, m200=NFW_M200, r200=NFW_R200):
    c = r200 / rs
    return m200 * _nfw_m(np.minimum(r, r200) / rs) / _nfw_m(c)


def _nfw_sigma_r(rs=NFW_RS, m200=NFW_M200, r200=NFW_R200, n=4000):
    """Isotropic Jeans dispersion sigma_r(r) of the truncated NFW halo (zero
    pressure at R200), tabulated on a log grid."""
    rg = np.geomspace(1e-4, r200, n)
    rho = nfw_rho(rg, rs, m200, r200)
    integrand = rho * G_KPC * nfw_menc(rg, rs, m200, r200) / rg ** 2
    # cumulative integral from r to r200 (trapezoid in log r)
    lr = np.log(rg)
    f = integrand * rg
    seg = 0.5 * (f[1:] + f[:-1]) * np.diff(lr)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    return rg, np.sqrt(np.maximum(tail / rho, 0.0))


def _sample_nfw_radii(r: np.random.Generator, n, rs=NFW_RS, r200=NFW_R200):
    grid = np.geomspace(1e-5, r200, 20000)
    cdf = _nfw_m(grid / rs) / _nfw_m(r200 / rs)
    return np.interp(r.uniform(0.0, 1.0, n), cdf, grid)


def _iso_dirs(r: np.random.Generator, n):
    ct = r.uniform(-1.0, 1.0, n)
    ph = r.uniform(0.0, 2.0 * math.pi, n)
    st = np.sqrt(1.0 - ct * ct)
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)


def _density_h(rho, mass_per_particle, n_ngb, floor=H_FLOOR_KPC):
    """Radius of the sphere holding n_ngb particles at the local profile density."""
    return np.maximum(floor, (3.0 * n_ngb * mass_per_particle / (4.0 * math.pi * rho)) ** (1.0 / 3.0))


def galaxy(n_gas=1_000_000, n_dm=4_000_000, n_ngb=64, seed=(2, 1), sigma0_cm2=1e-24, n_pow=0,
           m_chi_over_mp=2.0, dt_myr=1.0, T_gas=1e4, disp_gas=10.0, h_mode="density") -> dict:
    """Isolated disk galaxy stand-in: exponential gas disk (R_d = 3 kpc, z_d =
    0.3 kpc, truncated R < 30, |z| < 3) with circular velocity from the NFW
    halo plus a 10 km/s dispersion; NFW halo (r_s = 20 kpc, M200 = 1.074e12,
    R200 = 205.5 kpc) with isotropic Jeans velocities.  Masses from Table 1
    (gas = 0.2 x 4.297e10 Msun)."""
    r = rng(*seed)
    # gas disk
    R = r.gamma(2.0, DISK_RD, size=int(n_gas * 1.2) + 100)
    R = R[R < 10.0 * DISK_RD][:n_gas]
    while R.shape[0] < n_gas:
        extra = r.gamma(2.0, DISK_RD, size=n_gas)
        R = np.concatenate([R, extra[extra < 10.0 * DISK_RD]])[:n_gas]
    z = r.laplace(0.0, DISK_ZD, size=int(n_gas * 1.2) + 100)
    z = z[np.abs(z) < 10.0 * DISK_ZD][:n_gas]
    while z.shape[0] < n_gas:
        extra = r.laplace(0.0, DISK_ZD, size=n_gas)
        z = np.concatenate([z, extra[np.abs(extra) < 10.0 * DISK_ZD]])[:n_gas]
    phi = r.uniform(0.0, 2.0 * math.pi, n_gas)
    gas_pos = np.stack([R * np.cos(phi), R * np.sin(phi), z], axis=1)
    vc = np.sqrt(G_KPC * nfw_menc(np.sqrt(R * R + z * z)) / np.maximum(np.sqrt(R * R + z * z), 1e-3))
    gas_vel = np.stack([-vc * np.sin(phi), vc * np.cos(phi), np.zeros(n_gas)], axis=1)
    gas_vel += disp_gas * r.standard_normal((n_gas, 3))
    m_gas = DISK_MASS * GAS_FRAC / n_gas
    # halo
    rr = _sample_nfw_radii(r, n_dm)
    dm_pos = rr[:, None] * _iso_dirs(r, n_dm)
    rg, sg = _nfw_sigma_r()
    sr = np.interp(rr, rg, sg)
    dm_vel = sr[:, None] * r.standard_normal((n_dm, 3))
    m_dm = NFW_M200 / n_dm
    if h_mode == "knn":
        h_gas = np.maximum(H_FLOOR_KPC, knn_h(gas_pos, n_ngb))
        h_dm = np.maximum(H_FLOOR_KPC, knn_h(dm_pos, n_ngb))
    else:
        rho_gas = DISK_MASS * GAS_FRAC / (4.0 * math.pi * DISK_RD ** 2 * DISK_ZD) * np.exp(
            -R / DISK_RD - np.abs(z) / DISK_ZD)
        h_gas = _density_h(rho_gas, m_gas, n_ngb)
        h_dm = _density_h(nfw_rho(rr), m_dm, n_ngb)
    gas = {"pos": gas_pos, "vel": gas_vel, "mass": np.full(n_gas, m_gas), "h": h_gas,
           "u": np.full(n_gas, u_from_T(T_gas)), "mu": np.full(n_gas, M_P)}
    dm = {"pos": dm_pos, "vel": dm_vel, "mass": np.full(n_dm, m_dm), "h": h_dm}
    par = params(sigma0_cm2, n_pow, m_chi_over_mp, dt_myr, 0x2603246880000000 + int(seed[-1]), 0, 0, None)
    return {"gas": gas, "dm": dm, "params": par}


def spread_h_log(h: np.ndarray, decades: float = 3.0, h_top: float | None = None) -> np.ndarray:
    """Rank-matched log-uniform kernel radii over `decades`, anchored at h_top
    (default: the largest input radius): h_k = h_top 10^{-decades (1 - (k+1/2)/N)}
    for the particle of rank k in h."""
    n = h.shape[0]
    order = np.argsort(h, kind="stable")
    out = np.empty_like(h)
    top = h.max() if h_top is None else float(h_top)
    out[order] = top * 10.0 ** (-decades * (1.0 - (np.arange(n) + 0.5) / n))
    return out


def knn_max(pos: np.ndarray, h_rank: np.ndarray, k: int, n_cand: int = 50_000) -> float:
    """Largest distance to the k-th nearest same-species neighbour, searched
    among the n_cand particles with the largest h_rank (the sparsest ones)."""
    from scipy.spatial import cKDTree
    tree = cKDTree(pos, leafsize=32, balanced_tree=False, compact_nodes=False)
    cand = np.argpartition(h_rank, -min(n_cand, len(h_rank)))[-min(n_cand, len(h_rank)):]
    d, _ = tree.query(pos[cand], k=k + 1, workers=-1)
    return float(d[:, -1].max())


def sigma0_for_npow(n_pow: int, v_ref_kms: float = 200.0, sigma_ref_cm2: float = 1e-24) -> float:
    """sigma0 such that sigma(v_ref) = sigma_ref for sigma = sigma0 (v/c)^n."""
    return sigma_ref_cm2 * (299792.458 / v_ref_kms) ** n_pow


# --------------------------------------------------------------------------- batch of boxes
def batch(n_box=64, n_min=10_000, n_max=500_000, seed=(5, 1), n_ngb=32, h_mode="density",
          scale=1.0) -> list:
    """Independent periodic boxes: N_b = floor(10^U(log10 n_min, log10 n_max))
    per species (times `scale`), side L_b = (N_b/4096)^{1/3} kpc at the box
    workload's density; sigma_b log-spaced 1e-28..1e-24 cm^2; m_chi/m_p drawn
    from {0.5, 1, 2, 5}."""
    r = rng(*seed)
    sizes = np.floor(10.0 ** r.uniform(math.log10(n_min), math.log10(n_max), n_box)).astype(np.int64)
    sizes = np.maximum(64, (sizes * scale).astype(np.int64))
    mchi = r.choice(np.array([0.5, 1.0, 2.0, 5.0]), n_box)
    out = []
    for b in range(n_box):
        nb = int(sizes[b])
        L = (nb / 4096.0) ** (1.0 / 3.0)
        sig = 10.0 ** (-28.0 + 4.0 * b / max(1, n_box - 1))
        cfg = box(n_gas=nb, n_dm=nb, L=L, m_chi_over_mp=float(mchi[b]), sigma0_cm2=sig, n_ngb=n_ngb,
                  seed=(seed[0], seed[1], b), h_mode=h_mode, philox_seed=0x2603246880000000 + int(seed[-1]))
        cfg["params"]["box_id"] = b
        out.append(cfg)
    return out


# --------------------------------------------------------------------------- rate-closure samples
MLP_N_VALUES = (-4.0, -2.0, 0.0, 2.0)


def mlp_samples(n: int, seed=(4, 1), ext: float = 0.25, x2_zero: bool = False) -> np.ndarray:
    """Inputs x[n][4] = (w/vs_gas, T_DM/T_gas, log10(m_chi/mu), n) of the rate
    closure: x1 uniform on [0, 10] (a fraction `ext` log-uniform on
    [10, 1000] instead), x2 uniform on [0, 100] (0 with x2_zero: one DM
    velocity per pair, as in the interaction step), x3 uniform on [-2, 1.3]
    (10 MeV .. 10 GeV for mu = m_p), n uniform over {-4, -2, 0, 2}."""
    r = rng(*seed)
    x = np.empty((n, 4))
    x[:, 0] = r.uniform(0.0, 10.0, n)
    m = r.random(n) < ext
    x[m, 0] = 10.0 ** r.uniform(1.0, 3.0, int(m.sum()))
    x[:, 1] = 0.0 if x2_zero else r.uniform(0.0, 100.0, n)
    x[:, 2] = r.uniform(-2.0, 1.3, n)
    x[:, 3] = r.choice(np.array(MLP_N_VALUES), n)
    return x


def mlp_params(seed=(4, 9), scale: float = 1.0) -> np.ndarray:
    """A random parameter vector of the rate-closure network (He-uniform
    weights times `scale`, small random biases) for checking its kernels."""
    r = rng(*seed)
    shapes = [(64, 5), (64,), (64, 64), (64,), (64, 64), (64,), (2, 64), (2,)]
    out = []
    for s in shapes:
        if len(s) == 2:
            b = math.sqrt(6.0 / s[1])
            out.append(scale * r.uniform(-b, b, s).ravel())
        else:
            out.append(r.uniform(-0.1, 0.1, s))
    return np.concatenate(out).astype(np.float32)


# --------------------------------------------------------------------------- Milky-Way-scale step
def milky_way(n_gas=8_000_000, n_dm=32_000_000, seed=(3, 1), active_frac=0.1, step=0, decades=3.0,
              dt_myr=0.1, n_pow=0, sigma0_cm2=1e-24) -> dict:
    """Disk + halo with the galaxy profiles at Milky-Way particle counts, for
    one step of a hierarchical-timestep run: h spread log-uniformly over
    `decades` decades per species, rank-matched to the profile-density h and
    top-anchored at the largest 64-neighbour distance of the species (its kNN
    maximum, found among the 50 000 sparsest particles), and an independent
    `active_frac` of each species active (drawn per step)."""
    cfg = galaxy(n_gas=n_gas, n_dm=n_dm, n_ngb=64, seed=seed, sigma0_cm2=sigma0_cm2, n_pow=n_pow, dt_myr=dt_myr)
    for sp in ("gas", "dm"):
        top = knn_max(cfg[sp]["pos"], cfg[sp]["h"], 64)
        cfg[sp]["h"] = spread_h_log(cfg[sp]["h"], decades, top)
    r = rng(seed[0], seed[1], 100 + int(step))
    cfg["gas"]["active"] = (r.random(n_gas) < active_frac).astype(np.uint8)
    cfg["dm"]["active"] = (r.random(n_dm) < active_frac).astype(np.uint8)
    cfg["params"]["step"] = int(step)
    return cfg
