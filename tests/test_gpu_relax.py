"""100 steps of the periodic test box (4096 gas + 4096 DM, binary64) against
the closed-form two-population relaxation (Appendix F, oracle/relax.py).

Between steps the DM velocities take their kicks, the gas its momentum and
internal-energy transfers, and both species drift (periodic wrap); cells are
rebuilt every step.  The gas side is a deterministic mean field and tracks
the relaxation closely (bulk velocity and dispersion within 3 % of their
change); the DM side is a Monte Carlo process and is held to four standard
errors of its own scatter noise.  Total momentum is conserved within that
noise too.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

MU = 1.67262192369e-24


def _log(msg):
    print(msg, flush=True)


def test_box_relaxation_100_steps():
    import torch
    import paper_2603_24688_amd as dmb
    from oracle import relax
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = workloads.box()
    g, d, par = cfg["gas"], cfg["dm"], dict(cfg["params"])
    L = par["box"][0]
    dt = par["dt"]
    nsteps = 100
    rho_b, rho_x = g["mass"].sum() / L ** 3, d["mass"].sum() / L ** 3
    ctx = dmb.Context(0)
    G, D = dmb.to_device(g), dmb.to_device(d)
    out = dmb.alloc_out(len(g["mass"]), len(d["mass"]))
    mg = G["mass"][:, None]

    def state():
        vx = D["vel"][:, 0].mean().item()
        vb = G["vel"][:, 0].mean().item()
        sx2 = ((D["vel"] - D["vel"].mean(0)) ** 2).sum(1).mean().item() / 3.0
        spread = ((G["vel"] - G["vel"].mean(0)) ** 2).sum(1).mean().item()
        sb2 = (2.0 / 3.0) * (G["u"].mean().item() + 0.5 * spread)
        return np.array([vx, vb, sx2, sb2])

    hist = [state()]
    var_v = 0.0        # sum over steps and DM of |dv_x|^2 (scatter noise of the DM mean velocity)
    var_e = 0.0        # same for the change of |v|^2
    scat = 0
    for k in range(nsteps):
        par["step"] = k
        ctx.build_cells(G, D, par, precision=dmb.DMB_FP64)
        ctx.interact_step(G, D, par, out, precision=dmb.DMB_FP64)
        dv = out["dv_dm"]
        var_v += (dv[:, 0] ** 2).sum().item()
        de2 = 2.0 * (D["vel"] * dv).sum(1) + (dv ** 2).sum(1)
        var_e += (de2 ** 2).sum().item()
        scat += dmb.counters_dict(out["counters"])["scatters"]
        D["vel"].add_(dv)
        G["vel"].add_(out["dp_gas"] / mg)
        G["u"].add_(out["de_gas"] / G["mass"])
        D["pos"].copy_(torch.remainder(D["pos"] + D["vel"] * dt, L))
        G["pos"].copy_(torch.remainder(G["pos"] + G["vel"] * dt, L))
        if (k + 1) % 10 == 0:
            hist.append(state())
    torch.cuda.synchronize()
    ctx.close()
    hist = np.array(hist)
    t_eval = np.arange(0, nsteps + 1, 10) * dt
    _, ode = relax.evolve(hist[0], nsteps * dt, rho_b, rho_x, par["sigma0_cm2"], par["n_pow"], par["m_chi_g"], MU,
                          t_eval=t_eval)
    n_dm = len(d["mass"])
    sig_vx = np.sqrt(var_v) / n_dm
    sig_sx2 = np.sqrt(var_e) / n_dm / 3.0
    for j in range(len(t_eval)):
        _log(f"[relax] step {10 * j:3d}: V_X {hist[j, 0]:.3f} (ode {ode[j, 0]:.3f})  V_B {hist[j, 1]:.4f} "
             f"(ode {ode[j, 1]:.4f})  s_X^2 {hist[j, 2]:.2f} (ode {ode[j, 2]:.2f})  s_B^2 {hist[j, 3]:.3f} "
             f"(ode {ode[j, 3]:.3f})")
    _log(f"[relax] {scat} scatters; DM noise: V_X {sig_vx:.3f} km/s, s_X^2 {sig_sx2:.2f} (km/s)^2")
    dVB = ode[-1, 1] - ode[0, 1]
    dSB = ode[-1, 3] - ode[0, 3]
    assert np.all(np.abs(hist[:, 1] - ode[:, 1]) <= 0.03 * abs(dVB))
    assert np.all(np.abs(hist[:, 3] - ode[:, 3]) <= 0.03 * abs(dSB))
    assert np.all(np.abs(hist[:, 0] - ode[:, 0]) <= 4 * sig_vx + 0.03 * abs(dVB))
    assert np.all(np.abs(hist[:, 2] - ode[:, 2]) <= 4 * sig_sx2 + 0.03 * abs(ode[-1, 2] - ode[0, 2]))
    # momentum: what the gas gained, the DM lost (within the scatter noise)
    p_gain = rho_b * (hist[-1, 1] - hist[0, 1])
    p_loss = rho_x * (hist[0, 0] - hist[-1, 0])
    assert abs(p_gain - p_loss) <= 4 * rho_x * sig_vx
