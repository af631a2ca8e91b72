"""MI355X (gfx950) DM-gas pair interaction step of Hainje & Farrar (arXiv 2603.24688).

Thin ctypes binding over the C ABI of ``libdmb.so`` (declared in
``include/dmb.h``).  Every step of the computation runs in the HIP kernels of
the library; this module only marshals torch device tensors into the C
structs.  Importing works without a GPU; calling needs the built library and a
HIP device and raises otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdmb.so")

DMB_FP64, DMB_FP32 = 0, 1
DMB_RATES_EXACT, DMB_RATES_QUAD, DMB_RATES_MLP, DMB_RATES_CLOSURE = 0, 1, 2, 3
DMB_SAMPLE_PAIR, DMB_SAMPLE_RB = 0, 1
MLP_PARAMS = 8834
COUNTER_NAMES = ["pairs_gas", "pairs_dm", "scatters", "near_boundary", "near_decision",
                 "crit_viol", "p_ge_1", "nonfinite"]
N_COUNTERS = len(COUNTER_NAMES)
STATUS = {0: "DMB_OK", -1: "DMB_EINVAL", -2: "DMB_ENOMEM", -3: "DMB_EHIP", -4: "DMB_ERANGE", -5: "DMB_ESTALE"}

# Symbols declared in include/dmb.h.
EXPORTS = ["dmb_create", "dmb_destroy", "dmb_set_stream", "dmb_build_cells", "dmb_interact_step",
           "dmb_overlap_eval", "dmb_rates_eval", "dmb_philox_eval", "dmb_profile_enable", "dmb_profile_read",
           "dmb_build_stats", "dmb_last_error", "dmb_mlp_labels", "dmb_mlp_init", "dmb_mlp_set_params",
           "dmb_mlp_get_params", "dmb_mlp_grad", "dmb_mlp_train", "dmb_mlp_eval", "dmb_batch_build",
           "dmb_batch_step", "dmb_batch_tune", "dmb_set_search_groups", "dmb_set_pass_overlap", "dmb_pair_list",
           "dmb_sort_pairs", "dmb_step_static", "dmb_run"]
BUILD_STATS = ["active_gas", "active_dm", "gas_tiles", "dm_tiles", "gas_owner_tiles", "dm_owner_tiles",
               "cand_pairs_gas", "cand_pairs_dm", "items_gas", "items_dm"]
PHASES = ["build", "gather", "pass_gas", "combine_gas", "pass_dm", "combine_dm", "resolve"]


class DmbError(RuntimeError):
    pass


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("vel", C.c_void_p), ("mass", C.c_void_p),
                ("h", C.c_void_p), ("u", C.c_void_p), ("mu", C.c_void_p), ("active", C.c_void_p),
                ("dt", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("sigma0_cm2", C.c_double), ("n_pow", C.c_int32), ("m_chi_g", C.c_double), ("dt", C.c_double),
                ("seed", C.c_uint64), ("step", C.c_uint32), ("box_id", C.c_uint32), ("box", C.c_double * 3),
                ("precision", C.c_int32), ("rates", C.c_int32), ("quad_nodes", C.c_int32), ("aniso_g", C.c_double),
                ("dm_sampling", C.c_int32)]


class Out(C.Structure):
    _fields_ = [("dv_dm", C.c_void_p), ("dp_gas", C.c_void_p), ("de_gas", C.c_void_p), ("partner", C.c_void_p),
                ("p_sum", C.c_void_p), ("p_max", C.c_void_p), ("counters", C.c_void_p)]


class RunCfg(C.Structure):
    _fields_ = [("nsteps", C.c_int32), ("dt_control", C.c_int32), ("dt_max", C.c_double), ("safety", C.c_double),
                ("active_frac", C.c_double)]


DIAG_NAMES = ["time", "dt", "p_dm_x", "p_dm_y", "p_dm_z", "p_gas_x", "p_gas_y", "p_gas_z", "e_dm", "e_gas",
              "v_dm_x", "v_dm_y", "v_dm_z", "v_gas_x", "v_gas_y", "v_gas_z", "s2_dm", "s2_gas", "jb_dm", "scatters",
              "crit_viol", "p_max", "pairs", "pairs_gas"]
N_DIAG = len(DIAG_NAMES)


class MlpTrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr0", C.c_double), ("lr_min", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double), ("seed", C.c_uint64),
                ("init", C.c_int32), ("use_graph", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdmb.so and declare the C signatures.  Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise DmbError(f"{path} is not built; run paper_2603_24688_amd.build.build()")
    # torch ships its own HIP runtime; load it first so that libdmb.so binds to
    # the same runtime instance (one device context per process).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    L.dmb_create.restype = C.c_int; L.dmb_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    L.dmb_destroy.restype = C.c_int; L.dmb_destroy.argtypes = [vp]
    L.dmb_set_stream.restype = C.c_int; L.dmb_set_stream.argtypes = [vp, vp]
    L.dmb_build_cells.restype = C.c_int
    L.dmb_build_cells.argtypes = [vp, C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params)]
    L.dmb_interact_step.restype = C.c_int
    L.dmb_interact_step.argtypes = [vp, C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params), C.POINTER(Out)]
    L.dmb_pair_list.restype = C.c_int
    L.dmb_pair_list.argtypes = [vp, C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params), C.POINTER(Out),
                                i64, vp, vp, vp]
    L.dmb_run.restype = C.c_int
    L.dmb_run.argtypes = [vp, C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params), C.POINTER(RunCfg), vp]
    L.dmb_step_static.restype = C.c_int
    L.dmb_step_static.argtypes = [vp, C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params), C.POINTER(Out)]
    L.dmb_sort_pairs.restype = C.c_int; L.dmb_sort_pairs.argtypes = [vp, i64, vp, vp, i32, i32, vp, vp]
    L.dmb_overlap_eval.restype = C.c_int; L.dmb_overlap_eval.argtypes = [vp, i64, vp, vp, vp, i32, vp]
    L.dmb_rates_eval.restype = C.c_int; L.dmb_rates_eval.argtypes = [vp, i64, vp, vp, i32, i32, i32, i32, vp, vp]
    L.dmb_philox_eval.restype = C.c_int; L.dmb_philox_eval.argtypes = [vp, i64, vp, u64, vp]
    L.dmb_profile_enable.restype = C.c_int; L.dmb_profile_enable.argtypes = [vp, i32]
    L.dmb_set_search_groups.restype = C.c_int; L.dmb_set_search_groups.argtypes = [vp, i32]
    L.dmb_set_pass_overlap.restype = C.c_int; L.dmb_set_pass_overlap.argtypes = [vp, i32]
    L.dmb_profile_read.restype = C.c_int; L.dmb_profile_read.argtypes = [vp, vp, vp, i32]
    L.dmb_build_stats.restype = C.c_int; L.dmb_build_stats.argtypes = [vp, vp]
    L.dmb_last_error.restype = C.c_char_p; L.dmb_last_error.argtypes = [vp]
    L.dmb_mlp_labels.restype = C.c_int; L.dmb_mlp_labels.argtypes = [vp, i64, vp, i32, vp]
    L.dmb_mlp_init.restype = C.c_int; L.dmb_mlp_init.argtypes = [vp, u64]
    L.dmb_mlp_set_params.restype = C.c_int; L.dmb_mlp_set_params.argtypes = [vp, vp, i64]
    L.dmb_mlp_get_params.restype = C.c_int; L.dmb_mlp_get_params.argtypes = [vp, vp, i64]
    L.dmb_mlp_grad.restype = C.c_int; L.dmb_mlp_grad.argtypes = [vp, i64, vp, vp, vp, vp]
    L.dmb_mlp_train.restype = C.c_int
    L.dmb_mlp_train.argtypes = [vp, i64, vp, vp, C.POINTER(MlpTrainCfg), vp]
    L.dmb_mlp_eval.restype = C.c_int; L.dmb_mlp_eval.argtypes = [vp, i64, vp, vp]
    L.dmb_batch_build.restype = C.c_int
    L.dmb_batch_build.argtypes = [vp, i32, C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params)]
    L.dmb_batch_step.restype = C.c_int
    L.dmb_batch_step.argtypes = [vp, i32, C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params),
                                 C.POINTER(Out), i32, i32]
    L.dmb_batch_tune.restype = C.c_int
    L.dmb_batch_tune.argtypes = [vp, i32, C.POINTER(Particles), C.POINTER(Particles), C.POINTER(Params),
                                 C.POINTER(Out), vp]
    _lib = L
    return L


def _ptr(t):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise DmbError("tensors passed to the HIP library must live on the GPU")
    if not t.is_contiguous():
        raise DmbError("tensors passed to the HIP library must be contiguous")
    return t.data_ptr()


def _particles(d: dict) -> Particles:
    return Particles(int(d["mass"].shape[0]), _ptr(d["pos"]), _ptr(d.get("vel")), _ptr(d.get("mass")),
                     _ptr(d["h"]), _ptr(d.get("u")), _ptr(d.get("mu")), _ptr(d.get("active")), _ptr(d.get("dt")))


def _params(p: dict, precision: int) -> Params:
    box = p.get("box") or (0.0, 0.0, 0.0)
    return Params(float(p["sigma0_cm2"]), int(p.get("n_pow", 0)), float(p["m_chi_g"]), float(p["dt"]),
                  int(p["seed"]) & 0xFFFFFFFFFFFFFFFF, int(p.get("step", 0)) & 0xFFFFFFFF, int(p.get("box_id", 0)),
                  (C.c_double * 3)(*[float(b) for b in box]), int(precision), int(p.get("rates", DMB_RATES_EXACT)),
                  int(p.get("quad_nodes", 0)), float(p.get("aniso_g", 0.0)), int(p.get("dm_sampling", 0)))


class Context:
    """One library context bound to a HIP device and stream (torch's current
    stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise DmbError("no HIP device visible")
        self.device = device
        s = torch.cuda.current_stream(device) if stream is None else stream
        self.stream = s
        h = C.c_void_p()
        rc = self.lib.dmb_create(C.byref(h), int(device), C.c_void_p(s.cuda_stream))
        if rc != 0:
            msg = self.lib.dmb_last_error(None).decode(errors="replace")
            raise DmbError(f"dmb_create failed: {STATUS.get(rc, rc)}: {msg}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.dmb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc != 0:
            msg = self.lib.dmb_last_error(self.h).decode(errors="replace")
            raise DmbError(f"{what}: {STATUS.get(rc, rc)}: {msg}")

    # -- the two calls of the hot path ---------------------------------------------------------
    def build_cells(self, gas: dict, dm: dict, params: dict, precision: int = DMB_FP32):
        G, D, P = _particles(gas), _particles(dm), _params(params, precision)
        self._check(self.lib.dmb_build_cells(self.h, C.byref(G), C.byref(D), C.byref(P)), "dmb_build_cells")

    def interact_step(self, gas: dict, dm: dict, params: dict, out: dict, precision: int = DMB_FP32):
        G, D, P = _particles(gas), _particles(dm), _params(params, precision)
        O = Out(_ptr(out["dv_dm"]), _ptr(out["dp_gas"]), _ptr(out["de_gas"]), _ptr(out["partner"]),
                _ptr(out.get("p_sum")), _ptr(out.get("p_max")), _ptr(out.get("counters")))
        self._check(self.lib.dmb_interact_step(self.h, C.byref(G), C.byref(D), C.byref(P), C.byref(O)),
                    "dmb_interact_step")

    def pair_list(self, gas: dict, dm: dict, params: dict, out: dict, precision: int = DMB_FP32, cap: int = 0):
        """One step (outputs into `out`) that also returns the pairs each pass visited:
        (pairs_gas, pairs_dm) as int64 [n, 2] device tensors of (DM index, gas index)."""
        import torch
        G, D, P = _particles(gas), _particles(dm), _params(params, precision)
        O = Out(_ptr(out["dv_dm"]), _ptr(out["dp_gas"]), _ptr(out["de_gas"]), _ptr(out["partner"]),
                _ptr(out.get("p_sum")), _ptr(out.get("p_max")), _ptr(out.get("counters")))
        dev = out["dv_dm"].device
        for _ in range(2):
            lg = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=dev)
            ld = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=dev)
            cnt = (C.c_int64 * 2)()
            self._check(self.lib.dmb_pair_list(self.h, C.byref(G), C.byref(D), C.byref(P), C.byref(O), int(cap),
                                               _ptr(lg), _ptr(ld), cnt), "dmb_pair_list")
            if max(cnt[0], cnt[1]) <= cap:
                break
            cap = int(max(cnt[0], cnt[1]))
        to64 = lambda t, n: t[:n].to(torch.int64) & 0xFFFFFFFF
        return to64(lg, int(cnt[0])), to64(ld, int(cnt[1]))

    def sort_pairs(self, keys, vals, lo_bit: int, passes: int):
        """Stable radix sort of (keys uint64-as-int64, vals int32) device tensors by key
        bits [lo_bit, lo_bit + 8 passes); returns the sorted (keys, vals)."""
        import torch
        ko, vo = torch.empty_like(keys), torch.empty_like(vals)
        self._check(self.lib.dmb_sort_pairs(self.h, keys.numel(), _ptr(keys), _ptr(vals), int(lo_bit), int(passes),
                                            _ptr(ko), _ptr(vo)), "dmb_sort_pairs")
        return ko, vo

    def run(self, gas: dict, dm: dict, params: dict, nsteps: int, dt_max: float, dt_control: bool = False,
            safety: float = 0.5, precision: int = DMB_FP64, active_frac: float = 0.0):
        """nsteps steps of the time loop on device (pos, vel, u of the tensors updated in place);
        returns the diagnostics as a numpy array [nsteps + 1, N_DIAG] (columns DIAG_NAMES)."""
        import numpy as np
        G, D, P = _particles(gas), _particles(dm), _params(params, precision)
        cfg = RunCfg(int(nsteps), int(bool(dt_control)), float(dt_max), float(safety), float(active_frac))
        diag = np.zeros((int(nsteps) + 1, N_DIAG), dtype=np.float64)
        self._check(self.lib.dmb_run(self.h, C.byref(G), C.byref(D), C.byref(P), C.byref(cfg), diag.ctypes.data),
                    "dmb_run")
        return diag

    def step_static(self, gas: dict, dm: dict, params: dict, out: dict, precision: int = DMB_FP32):
        """build_cells + interact_step in one call that allocates no device memory (static scratch)."""
        G, D, P = _particles(gas), _particles(dm), _params(params, precision)
        O = Out(_ptr(out["dv_dm"]), _ptr(out["dp_gas"]), _ptr(out["de_gas"]), _ptr(out["partner"]),
                _ptr(out.get("p_sum")), _ptr(out.get("p_max")), _ptr(out.get("counters")))
        self._check(self.lib.dmb_step_static(self.h, C.byref(G), C.byref(D), C.byref(P), C.byref(O)),
                    "dmb_step_static")

    def build_stats(self) -> dict:
        v = (C.c_int64 * len(BUILD_STATS))()
        self._check(self.lib.dmb_build_stats(self.h, v), "dmb_build_stats")
        return dict(zip(BUILD_STATS, [int(x) for x in v]))

    # -- phase timing ---------------------------------------------------------------------------
    def set_search_groups(self, cap: int):
        """Candidate-search group list capacity (0: no group pass); outputs do not depend on it."""
        self._check(self.lib.dmb_set_search_groups(self.h, int(cap)), "dmb_set_search_groups")

    def set_pass_overlap(self, on: bool = True):
        """Gas and DM passes on two streams (True, default) or in sequence (for per-pass timing)."""
        self._check(self.lib.dmb_set_pass_overlap(self.h, int(bool(on))), "dmb_set_pass_overlap")

    def profile_enable(self, on: bool = True):
        self._check(self.lib.dmb_profile_enable(self.h, int(bool(on))), "dmb_profile_enable")

    def profile_read(self, reset: bool = True) -> dict:
        ms = (C.c_double * len(PHASES))()
        calls = (C.c_int64 * len(PHASES))()
        self._check(self.lib.dmb_profile_read(self.h, ms, calls, int(bool(reset))), "dmb_profile_read")
        return {p: (ms[k], int(calls[k])) for k, p in enumerate(PHASES)}

    # -- evaluation helpers -------------------------------------------------------------------
    def overlap_eval(self, d, h1, h2, precision: int = DMB_FP32):
        import torch
        g = torch.empty_like(d)
        self._check(self.lib.dmb_overlap_eval(self.h, d.numel(), _ptr(d), _ptr(h1), _ptr(h2), precision, _ptr(g)),
                    "dmb_overlap_eval")
        return g

    def rates_eval(self, w, vs, n_pow: int, precision: int = DMB_FP32, rates: int = DMB_RATES_EXACT,
                   quad_nodes: int = 0):
        import torch
        A, B = torch.empty_like(w), torch.empty_like(w)
        self._check(self.lib.dmb_rates_eval(self.h, w.numel(), _ptr(w), _ptr(vs), int(n_pow), precision, int(rates),
                                            int(quad_nodes), _ptr(A), _ptr(B)), "dmb_rates_eval")
        return A, B

    # -- batched boxes -------------------------------------------------------------------------
    @staticmethod
    def _batch_structs(gas_list, dm_list, par_list, precision, out_list=None):
        nb = len(gas_list)
        if not (len(dm_list) == nb and len(par_list) == nb and (out_list is None or len(out_list) == nb)):
            raise ValueError("batch lists differ in length")
        G = (Particles * nb)(*[_particles(g) for g in gas_list])
        D = (Particles * nb)(*[_particles(d) for d in dm_list])
        P = (Params * nb)(*[_params(p, precision) for p in par_list])
        O = None
        if out_list is not None:
            O = (Out * nb)(*[Out(_ptr(o["dv_dm"]), _ptr(o["dp_gas"]), _ptr(o["de_gas"]), _ptr(o["partner"]),
                                 _ptr(o.get("p_sum")), _ptr(o.get("p_max")), _ptr(o["counters"])) for o in out_list])
        return nb, G, D, P, O

    def batch_build(self, gas_list, dm_list, par_list, precision: int = DMB_FP32):
        nb, G, D, P, _ = self._batch_structs(gas_list, dm_list, par_list, precision)
        self._check(self.lib.dmb_batch_build(self.h, nb, G, D, P), "dmb_batch_build")

    def batch_step(self, gas_list, dm_list, par_list, out_list, precision: int = DMB_FP32, nsteps: int = 1,
                   graph: bool = False):
        nb, G, D, P, O = self._batch_structs(gas_list, dm_list, par_list, precision, out_list)
        self._check(self.lib.dmb_batch_step(self.h, nb, G, D, P, O, int(nsteps), int(bool(graph))), "dmb_batch_step")

    def batch_tune(self, gas_list, dm_list, par_list, out_list, precision: int = DMB_FP32) -> dict:
        nb, G, D, P, O = self._batch_structs(gas_list, dm_list, par_list, precision, out_list)
        ch = (C.c_int64 * 4)()
        self._check(self.lib.dmb_batch_tune(self.h, nb, G, D, P, O, ch), "dmb_batch_tune")
        return {"work_item": int(ch[0]), "subtile_delta": int(ch[1]), "grid_pct": int(ch[2]),
                "us_per_step": int(ch[3])}

    # -- learned rate closure ----------------------------------------------------------------
    def mlp_labels(self, x, quad_nodes: int = 0):
        """Residual targets [n, 2] (float64, device) for inputs x [n, 4] (float64, device)."""
        import torch
        y = torch.empty((x.shape[0], 2), dtype=torch.float64, device=x.device)
        self._check(self.lib.dmb_mlp_labels(self.h, x.shape[0], _ptr(x), int(quad_nodes), _ptr(y)), "dmb_mlp_labels")
        return y

    def mlp_init(self, seed: int):
        self._check(self.lib.dmb_mlp_init(self.h, int(seed) & 0xFFFFFFFFFFFFFFFF), "dmb_mlp_init")

    def mlp_set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self.lib.dmb_mlp_set_params(self.h, p.ctypes.data, p.size), "dmb_mlp_set_params")

    def mlp_get_params(self):
        import numpy as np
        p = np.empty(MLP_PARAMS, dtype=np.float32)
        self._check(self.lib.dmb_mlp_get_params(self.h, p.ctypes.data, p.size), "dmb_mlp_get_params")
        return p

    def mlp_grad(self, x, y):
        """(gradient [MLP_PARAMS] float32 numpy, loss) of the n samples as one batch."""
        import numpy as np
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        loss = C.c_double()
        self._check(self.lib.dmb_mlp_grad(self.h, x.shape[0], _ptr(x), _ptr(y), g.ctypes.data, C.byref(loss)),
                    "dmb_mlp_grad")
        return g, loss.value

    def mlp_train(self, x, y, epochs: int, batch: int = 4096, lr0: float = 2e-3, lr_min: float = 1e-5,
                  beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, seed: int = 1, init: bool = True,
                  use_graph: bool = True):
        """Train on (x, y) (device tensors); returns the mean loss of each epoch."""
        import numpy as np
        cfg = MlpTrainCfg(int(epochs), int(batch), float(lr0), float(lr_min), float(beta1), float(beta2), float(eps),
                          int(seed) & 0xFFFFFFFFFFFFFFFF, int(bool(init)), int(bool(use_graph)))
        losses = np.zeros(int(epochs), dtype=np.float64)
        self._check(self.lib.dmb_mlp_train(self.h, x.shape[0], _ptr(x), _ptr(y), C.byref(cfg), losses.ctypes.data),
                    "dmb_mlp_train")
        return losses

    def mlp_eval(self, x):
        """Network (ln Ahat/vs^{n+1}, ln Bhat/vs^{n+3}) [n, 2] for inputs x [n, 4]."""
        import torch
        out = torch.empty((x.shape[0], 2), dtype=torch.float64, device=x.device)
        self._check(self.lib.dmb_mlp_eval(self.h, x.shape[0], _ptr(x), _ptr(out)), "dmb_mlp_eval")
        return out

    def philox_eval(self, ctr, seed: int):
        import torch
        out = torch.empty_like(ctr)
        self._check(self.lib.dmb_philox_eval(self.h, ctr.shape[0], _ptr(ctr), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                             _ptr(out)), "dmb_philox_eval")
        return out


def alloc_out(n_gas: int, n_dm: int, device="cuda"):
    """Output buffers for interact_step (torch tensors on `device`)."""
    import torch
    return {
        "dv_dm": torch.empty((n_dm, 3), dtype=torch.float64, device=device),
        "dp_gas": torch.empty((n_gas, 3), dtype=torch.float64, device=device),
        "de_gas": torch.empty((n_gas,), dtype=torch.float64, device=device),
        "partner": torch.empty((n_dm,), dtype=torch.int32, device=device),
        "p_sum": torch.empty((n_dm,), dtype=torch.float64, device=device),
        "p_max": torch.empty((n_dm,), dtype=torch.float64, device=device),
        "counters": torch.zeros((N_COUNTERS,), dtype=torch.int64, device=device),
    }


def to_device(species: dict, device="cuda") -> dict:
    """numpy particle dict -> contiguous torch tensors on `device`."""
    import numpy as np
    import torch
    out = {}
    for k, v in species.items():
        if v is None:
            continue
        a = np.ascontiguousarray(v)
        t = torch.from_numpy(a)
        if k == "active":
            t = t.to(torch.uint8)
        out[k] = t.to(device).contiguous()
    return out


def counters_dict(t) -> dict:
    vals = t.cpu().tolist()
    return {k: int(v) for k, v in zip(COUNTER_NAMES, vals)}
