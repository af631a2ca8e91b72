"""CPU FP64 oracle for the DM-gas pair interaction step (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library:
``dmb_oracle.c`` is plain C compiled with gcc, wrapped here with ctypes.

Functions follow Hainje & Farrar (arXiv 2603.24688); each C function cites the
section / equation it writes out.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dmb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

N_COUNTERS = 8
COUNTER_NAMES = ["pairs_gas", "pairs_dm", "scatters", "near_boundary", "near_decision",
                 "crit_viol", "p_ge_1", "nonfinite"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("vel", C.c_void_p), ("mass", C.c_void_p),
                ("h", C.c_void_p), ("u", C.c_void_p), ("mu", C.c_void_p), ("active", C.c_void_p),
                ("dt", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("sigma0_cm2", C.c_double), ("n_pow", C.c_int), ("m_chi_g", C.c_double),
                ("dt", C.c_double), ("seed", C.c_uint64), ("step", C.c_uint32), ("box_id", C.c_uint32),
                ("box", C.c_double * 3), ("aniso_g", C.c_double), ("gas_closure", C.c_int), ("dm_rb", C.c_int)]


class Out(C.Structure):
    _fields_ = [("dv_dm", C.c_void_p), ("dp_gas", C.c_void_p), ("de_gas", C.c_void_p),
                ("dp_abs", C.c_void_p), ("de_abs", C.c_void_p), ("pk_abs", C.c_void_p), ("partner", C.c_void_p),
                ("p_sum", C.c_void_p), ("p_max", C.c_void_p), ("flags", C.c_void_p),
                ("counters", C.c_uint64 * N_COUNTERS)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        d, i, u32, u64, p = C.c_double, C.c_int, C.c_uint32, C.c_uint64, C.c_void_p
        L.orc_w.restype = d; L.orc_w.argtypes = [d]
        L.orc_W.restype = d; L.orc_W.argtypes = [d, d]
        L.orc_overlap.restype = d; L.orc_overlap.argtypes = [d, d, d]
        L.orc_overlap_G.restype = d; L.orc_overlap_G.argtypes = [d, d]
        L.orc_hyp1f1_negx.restype = d; L.orc_hyp1f1_negx.argtypes = [d, d, d]
        L.orc_hyp1f1_negx_v.restype = None; L.orc_hyp1f1_negx_v.argtypes = [C.c_long, d, d, p, p]
        L.orc_alpha_n.restype = d; L.orc_alpha_n.argtypes = [i]
        L.orc_rates.restype = None; L.orc_rates.argtypes = [i, d, d, C.POINTER(d), C.POINTER(d)]
        L.orc_philox4x32_10.restype = None; L.orc_philox4x32_10.argtypes = [p, p, p]
        L.orc_philox4x64_10.restype = None; L.orc_philox4x64_10.argtypes = [p, p, p]
        L.orc_u24.restype = d; L.orc_u24.argtypes = [u32]
        L.orc_normals3.restype = None; L.orc_normals3.argtypes = [p, p]
        L.orc_rb_radius.restype = d; L.orc_rb_radius.argtypes = [i, d, d]
        L.orc_rb_urel.restype = None; L.orc_rb_urel.argtypes = [i, p, d, p, p]
        L.orc_step.restype = i
        L.orc_step.argtypes = [C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params), C.POINTER(Out)]
        L.orc_step_sel.restype = i
        L.orc_step_sel.argtypes = [C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params),
                                   C.POINTER(Out), p, C.c_int64, p, C.c_int64]
        L.orc_pairs.restype = C.c_int64
        L.orc_pairs.argtypes = [C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params), p, p, C.c_int64]
        L.orc_num_threads.restype = i; L.orc_num_threads.argtypes = []
        L.orc_pair_stats.restype = None
        L.orc_pair_stats.argtypes = [C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params), p, C.c_int64,
                                     i, i, p, p, p]
        L.orc_active_flags.restype = None
        L.orc_active_flags.argtypes = [C.c_int64, u32, u32, u64, u32, d, p]
        L.orc_step_sel_grid.restype = i
        L.orc_step_sel_grid.argtypes = [C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params),
                                        C.POINTER(Out), p, C.c_int64, p, C.c_int64]
        _lib = L
    return _lib


# --------------------------------------------------------------------------- scalar helpers
def w(q: float) -> float:
    return lib().orc_w(float(q))


def W(r: float, h: float) -> float:
    return lib().orc_W(float(r), float(h))


def overlap(d: float, h1: float, h2: float) -> float:
    return lib().orc_overlap(float(d), float(h1), float(h2))


def overlap_G(delta: float, eta: float) -> float:
    return lib().orc_overlap_G(float(delta), float(eta))


def hyp1f1_negx(a: float, b: float, x: float) -> float:
    return lib().orc_hyp1f1_negx(float(a), float(b), float(x))


def hyp1f1_negx_v(a: float, b: float, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_hyp1f1_negx_v(x.size, float(a), float(b), x.ctypes.data, out.ctypes.data)
    return out


def alpha_n(n: int) -> float:
    return lib().orc_alpha_n(int(n))


def rb_radius(m: int, a: float, u0: float) -> float:
    """|u|/varsigma of the tilted law |u|^m N(u; w, varsigma^2 I) at uniform u0, a = |w|/varsigma."""
    return lib().orc_rb_radius(int(m), float(a), float(u0))


def rb_urel(n: int, w_, vs: float, u) -> np.ndarray:
    """Tilted relative velocity (Rao-Blackwellised partner draw) for w, varsigma and uniforms u[0..2]."""
    w_ = np.ascontiguousarray(w_, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_rb_urel(int(n), w_.ctypes.data, float(vs), u.ctypes.data, out.ctypes.data)
    return out


def rates(n: int, w_: float, vs: float) -> tuple[float, float]:
    A, B = C.c_double(), C.c_double()
    lib().orc_rates(int(n), float(w_), float(vs), C.byref(A), C.byref(B))
    return A.value, B.value


def philox4x32(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def philox4x64(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def u24(r: int) -> float:
    return lib().orc_u24(int(r) & 0xFFFFFFFF)


def normals3(u) -> np.ndarray:
    uu = np.ascontiguousarray(u, dtype=np.float64)
    z = np.zeros(3)
    lib().orc_normals3(uu.ctypes.data, z.ctypes.data)
    return z


def num_threads() -> int:
    return lib().orc_num_threads()


# --------------------------------------------------------------------------- full step
def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _particles(d: dict, keep: list) -> Particles:
    n = int(np.asarray(d["mass"]).shape[0])
    arrs = {
        "pos": _f64(d["pos"], (n, 3)), "vel": _f64(d["vel"], (n, 3)), "mass": _f64(d["mass"]),
        "h": _f64(d["h"]), "u": _f64(d.get("u")), "mu": _f64(d.get("mu")), "dt": _f64(d.get("dt")),
    }
    act = d.get("active")
    arrs["active"] = None if act is None else np.ascontiguousarray(act, dtype=np.uint8)
    keep.extend(a for a in arrs.values() if a is not None)
    ptr = {k: (None if a is None else a.ctypes.data) for k, a in arrs.items()}
    return Particles(n, ptr["pos"], ptr["vel"], ptr["mass"], ptr["h"], ptr["u"], ptr["mu"],
                     ptr["active"], ptr["dt"])


def _params(p: dict) -> Params:
    box = p.get("box") or (0.0, 0.0, 0.0)
    return Params(float(p["sigma0_cm2"]), int(p.get("n_pow", 0)), float(p["m_chi_g"]), float(p["dt"]),
                  int(p["seed"]) & 0xFFFFFFFFFFFFFFFF, int(p.get("step", 0)) & 0xFFFFFFFF,
                  int(p.get("box_id", 0)), (C.c_double * 3)(*[float(b) for b in box]),
                  float(p.get("aniso_g", 0.0)), 1 if p.get("rates") == 3 else 0,
                  1 if p.get("dm_sampling") == 1 else 0)


def step(gas: dict, dm: dict, params: dict, gas_sel=None, dm_sel=None, peak_scale=False, grid=False) -> dict:
    """Run the oracle step.  gas/dm: dicts of numpy arrays (pos, vel, mass, h,
    u, mu, active, dt); params: sigma0_cm2, n_pow, m_chi_g, dt, seed, step,
    box_id, box.  gas_sel / dm_sel: optional owner index subsets.  peak_scale
    also returns pk_abs: per gas, the sum of |terms| with each overlap
    replaced by its value at zero separation.  grid: neighbour candidates from
    uniform grids instead of every particle (bit-identical results)."""
    keep: list = []
    G = _particles(gas, keep)
    D = _particles(dm, keep)
    P = _params(params)
    ng, nd = G.n, D.n
    res = {
        "dv_dm": np.zeros((nd, 3)), "dp_gas": np.zeros((ng, 3)), "de_gas": np.zeros(ng),
        "dp_abs": np.zeros((ng, 3)), "de_abs": np.zeros(ng), "pk_abs": np.zeros(ng),
        "partner": np.full(nd, -1, np.int32),
        "p_sum": np.zeros(nd), "p_max": np.zeros(nd), "flags": np.zeros(nd, np.uint8),
    }
    if not peak_scale:
        res["pk_abs"] = None
    O = Out(*(None if res[k] is None else res[k].ctypes.data
              for k in ["dv_dm", "dp_gas", "de_gas", "dp_abs", "de_abs", "pk_abs", "partner", "p_sum", "p_max",
                        "flags"]))
    gs = None if gas_sel is None else np.ascontiguousarray(gas_sel, dtype=np.int64)
    ds = None if dm_sel is None else np.ascontiguousarray(dm_sel, dtype=np.int64)
    keep.extend(a for a in (gs, ds) if a is not None)
    fn = lib().orc_step_sel_grid if grid else lib().orc_step_sel
    rc = fn(C.byref(G), C.byref(D), C.byref(P), C.byref(O),
                            None if gs is None else gs.ctypes.data, 0 if gs is None else len(gs),
                            None if ds is None else ds.ctypes.data, 0 if ds is None else len(ds))
    if rc != 0:
        raise RuntimeError(f"orc_step failed: {rc}")
    res["counters"] = dict(zip(COUNTER_NAMES, [int(c) for c in O.counters]))
    return res


def pairs(gas: dict, dm: dict, params: dict, cap: int | None = None) -> np.ndarray:
    """Brute-force pair set as an (n, 2) int64 array of (dm index, gas index)."""
    keep: list = []
    G = _particles(gas, keep)
    D = _particles(dm, keep)
    P = _params(params)
    if cap is None:
        cap = int(G.n) * 512 + 1024
    oi = np.zeros(cap, np.int64)
    oj = np.zeros(cap, np.int64)
    n = lib().orc_pairs(C.byref(G), C.byref(D), C.byref(P), oi.ctypes.data, oj.ctypes.data, cap)
    if n > cap:
        return pairs(gas, dm, params, cap=int(n))
    return np.stack([oi[:n], oj[:n]], axis=1)


def pair_stats(gas: dict, dm: dict, params: dict, sel, owner_is_dm: bool, grid: bool = False):
    """For owners `sel` (gas indices, or DM indices when owner_is_dm): number of
    partners, sum of partner indices and sum of their squares (uint64), brute
    force over the other species (or over the uniform grids' candidates)."""
    keep: list = []
    G = _particles(gas, keep)
    D = _particles(dm, keep)
    P = _params(params)
    s = np.ascontiguousarray(sel, dtype=np.int64)
    cnt = np.zeros(s.size, np.int64)
    s1 = np.zeros(s.size, np.uint64)
    s2 = np.zeros(s.size, np.uint64)
    lib().orc_pair_stats(C.byref(G), C.byref(D), C.byref(P), s.ctypes.data, s.size, int(bool(owner_is_dm)),
                         int(bool(grid)), cnt.ctypes.data, s1.ctypes.data, s2.ctypes.data)
    return cnt, s1, s2


def active_flags(n: int, species: int, step: int, seed: int, box: int, frac: float) -> np.ndarray:
    """Active flags (uint8) of one species (0 gas, 1 DM) at one step of a
    hierarchical-timestep run: tag-3 uniform below frac."""
    out = np.zeros(int(n), np.uint8)
    lib().orc_active_flags(int(n), int(species), int(step) & 0xFFFFFFFF, int(seed) & 0xFFFFFFFFFFFFFFFF,
                           int(box), float(frac), out.ctypes.data)
    return out
