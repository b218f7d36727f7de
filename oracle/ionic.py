"""Ionic models and their time integrator (FP64, CPU).  Test infrastructure.

The paper writes every ionic model as du/dt + I_ion(u, w) = I_app,
dw/dt = H(u, w) (eq. of the ionic model ODEs) and ships four of them; the
equations themselves are only cited.  Here, written from the original
publications:

  ap      Aliev-Panfilov (1996): u dimensionless, u_mV = 100 u - 80 (paper,
          Section "Idealized left atrium"); one unit of model time is
          12.9 ms, so the reaction terms carry a 1/12.9 ms factor.
  bo      Bueno-Orovio minimal model (2008), EPI parameter set;
          u_mV = 85.7 u - 84 (paper, Section "Idealized left ventricle").
  ttp06   ten Tusscher-Panfilov (2006), endo / mid / epi cells; initial
          conditions printed in the paper (Section "Slab benchmark").
  passive I_ion = 0, no state (used by closed-form pins).

Integrator (one ionic step, paper eq. of the time-discrete ionic model with
the reading stated in the design notes): gating variables advance by
Rush-Larsen at the extrapolated potential u*, i.e. y <- y_inf(u*) +
(y - y_inf(u*)) exp(-dt/tau(u*)); all other variables take one forward-Euler
step with rates evaluated at (u*, new gates, old concentrations); TTP06
calcium buffering is handled with total concentrations (explicit step) and
the exact rapid-buffer inversion.  I_ion is then evaluated at (u*, w_{n+1})
as in the time-discrete monodomain equation.

Second integrator, the paper's own (eq. of the time-discrete ionic model,
`*_step_bdf`): (alpha w_{n+1} - w_BDF)/dt = H(u_EXT, w_EXT, w_{n+1}) with the
BDF combination and extrapolation of the potential's order.  Variables that
enter their own rate linearly are taken implicitly, the rest explicitly, so
the step is solved by direct inversion: each gate y' = (y_inf - y)/tau gives
y_{n+1} = (y_BDF + dt y_inf/tau)/(alpha + dt/tau) with y_inf, tau at
(u_EXT, w_EXT); the Aliev-Panfilov recovery variable is implicit in its
linear -v term with the rate factor eps(u_EXT, v_EXT); TTP06 concentrations
(calcium as buffered totals, Na, K, RR) are explicit,
x_{n+1} = (x_BDF + dt F(u_EXT, gates_{n+1}, c_EXT))/alpha.

Parity status.  Pinned on the CPU: the rest-state fixed points (AP, BO
exact; TTP06 drift bound), the uniform-state reduction, the AP excitation
term by the bistable-front speed, the Rush-Larsen and BDF gate updates
(brute-force and closed-form integration of frozen gate ODEs), the
rapid-buffer inversion, the rewritten I_CaL against its GHK form, and the
TTP06 concentration bookkeeping of both integrators (`ttp06_step`,
`ttp06_step_bdf`) by charge conservation: the membrane currents equal the
valence- and volume-weighted change of Na, K and total Ca; and the
steady states of the TTP06 gates m, xr2, s (epicardial), r and d against
the paper's printed rest state (those gates relax within milliseconds, so
y_inf(-85.23 mV) must give the printed values).

Parity unpinned (the publications' equations and traces are not available
here, and no closed form or invariant fixes them):
  ap_dv                 the Aliev-Panfilov recovery rate away from rest;
  bo_gate_targets       the Bueno-Orovio gate targets and time constants;
  bo_iion               the Bueno-Orovio currents J_fi, J_so, J_si;
  ttp06_gate_targets    the TTP06 time constants and the steady states of
                        h, j, xr1, xs, f, f2, fcass (those of m, xr2, s,
                        r, d are pinned, above);
  ttp06_currents        the TTP06 current and flux formulas (except I_CaL's
                        rewrite and the stoichiometry the conservation pin fixes).
TTP06 is pinned end to end by the N-version slab activation time through the
GPU path (the paper's 42.0 / 41.8 ms), which must match this oracle.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Model metadata
# ---------------------------------------------------------------------------

MV_PER_UNIT = {"passive": 1.0, "ap": 100.0, "bo": 85.7, "ttp06": 1.0}
MV_OFFSET = {"passive": 0.0, "ap": -80.0, "bo": -84.0, "ttp06": 0.0}
# potential (model units) above which a node counts as activated
ACT_THRESHOLD = {"passive": 0.5, "ap": 0.5, "bo": 0.5, "ttp06": -40.0}
N_VARS = {"passive": 0, "ap": 1, "bo": 3, "ttp06": 18}


def to_mv(model, u):
    return MV_PER_UNIT[model] * np.asarray(u) + MV_OFFSET[model]


# ---------------------------------------------------------------------------
# Aliev-Panfilov
# ---------------------------------------------------------------------------

AP_DEFAULT = dict(k=8.0, a=0.15, eps0=0.002, mu1=0.2, mu2=0.3, T=12.9)


def ap_iion(u, w, p=AP_DEFAULT):
    v = w[0]
    return (p["k"] * u * (u - p["a"]) * (u - 1.0) + u * v) / p["T"]


def ap_dv(u, v, p=AP_DEFAULT):
    eps = p["eps0"] + p["mu1"] * v / (u + p["mu2"])
    return eps * (-v - p["k"] * u * (u - p["a"] - 1.0)) / p["T"]


def ap_step(u_star, w, dt, p=AP_DEFAULT):
    """v is not a gate: one forward-Euler step at (u*, v_n)."""
    v = w[0]
    return np.stack([v + dt * ap_dv(u_star, v, p)])


def ap_step_bdf(u_ext, w_bdf, w_ext, dt, alpha, p=AP_DEFAULT):
    """Recovery variable implicit in its -v term, eps(u, v) at (u_EXT, v_EXT)."""
    eps = (p["eps0"] + p["mu1"] * w_ext[0] / (u_ext + p["mu2"])) / p["T"]
    drive = p["k"] * u_ext * (u_ext - p["a"] - 1.0)
    return np.stack([(w_bdf[0] - dt * eps * drive) / (alpha + dt * eps)])


def gate_bdf(y_bdf, y_inf, tau, dt, alpha):
    """BDF step of y' = (y_inf - y)/tau, implicit in y."""
    return (y_bdf + dt * y_inf / tau) / (alpha + dt / tau)


def ap_initial(n):
    return np.zeros(n), np.zeros((1, n))


# ---------------------------------------------------------------------------
# Bueno-Orovio minimal model, EPI parameters
# ---------------------------------------------------------------------------

BO_EPI = dict(u_o=0.0, u_u=1.55, theta_v=0.3, theta_w=0.13, theta_vm=0.006, theta_o=0.006,
              tau_v1m=60.0, tau_v2m=1150.0, tau_vp=1.4506, tau_w1m=60.0, tau_w2m=15.0,
              k_wm=65.0, u_wm=0.03, tau_wp=200.0, tau_fi=0.11, tau_o1=400.0, tau_o2=6.0,
              tau_so1=30.0181, tau_so2=0.9957, k_so=2.0458, u_so=0.65, tau_s1=2.7342,
              tau_s2=16.0, k_s=2.0994, u_s=0.9087, tau_si=1.8875, tau_winf=0.07,
              winf_star=0.94)


def _H(x):
    """Heaviside step with H(0) = 0."""
    return (np.asarray(x) > 0.0).astype(np.float64)


def bo_gate_targets(u, p=BO_EPI):
    """(y_inf, tau) of v, w, s at potential u; each gate obeys
    dy/dt = (y_inf - y)/tau piecewise in u."""
    Hv = _H(u - p["theta_v"])
    Hvm = _H(u - p["theta_vm"])
    Hw = _H(u - p["theta_w"])
    Ho = _H(u - p["theta_o"])
    v_inf = (1.0 - Hv) * (1.0 - Hvm)
    tau_vm = (1.0 - Hvm) * p["tau_v1m"] + Hvm * p["tau_v2m"]
    tau_v = (1.0 - Hv) * tau_vm + Hv * p["tau_vp"]
    w_inf_m = (1.0 - Ho) * (1.0 - u / p["tau_winf"]) + Ho * p["winf_star"]
    w_inf = (1.0 - Hw) * w_inf_m
    tau_wm = p["tau_w1m"] + (p["tau_w2m"] - p["tau_w1m"]) * (1.0 + np.tanh(p["k_wm"] * (u - p["u_wm"]))) / 2.0
    tau_w = (1.0 - Hw) * tau_wm + Hw * p["tau_wp"]
    s_inf = (1.0 + np.tanh(p["k_s"] * (u - p["u_s"]))) / 2.0
    tau_s = (1.0 - Hw) * p["tau_s1"] + Hw * p["tau_s2"]
    return (v_inf, w_inf, s_inf), (tau_v, tau_w, tau_s)


def bo_iion(u, w, p=BO_EPI):
    v, ww, s = w[0], w[1], w[2]
    Hv = _H(u - p["theta_v"])
    Hw = _H(u - p["theta_w"])
    Ho = _H(u - p["theta_o"])
    J_fi = -v * Hv * (u - p["theta_v"]) * (p["u_u"] - u) / p["tau_fi"]
    tau_o = (1.0 - Ho) * p["tau_o1"] + Ho * p["tau_o2"]
    tau_so = p["tau_so1"] + (p["tau_so2"] - p["tau_so1"]) * (1.0 + np.tanh(p["k_so"] * (u - p["u_so"]))) / 2.0
    J_so = (u - p["u_o"]) * (1.0 - Hw) / tau_o + Hw / tau_so
    J_si = -Hw * ww * s / p["tau_si"]
    return J_fi + J_so + J_si


def bo_step(u_star, w, dt, p=BO_EPI):
    """All three variables are gates: Rush-Larsen at u*."""
    infs, taus = bo_gate_targets(u_star, p)
    return np.stack([infs[i] + (w[i] - infs[i]) * np.exp(-dt / taus[i]) for i in range(3)])


def bo_step_bdf(u_ext, w_bdf, w_ext, dt, alpha, p=BO_EPI):
    """All three variables are gates; targets depend on u only."""
    infs, taus = bo_gate_targets(u_ext, p)
    return np.stack([gate_bdf(w_bdf[i], infs[i], taus[i], dt, alpha) for i in range(3)])


def bo_initial(n):
    return np.zeros(n), np.vstack([np.ones(n), np.ones(n), np.zeros(n)])


# ---------------------------------------------------------------------------
# ten Tusscher-Panfilov 2006
# ---------------------------------------------------------------------------

TTP_CONST = dict(R=8314.472, T=310.0, F=96485.3415, Cm=0.185, Vc=0.016404, Vsr=0.001094,
                 Vss=0.00005468, Ko=5.4, Nao=140.0, Cao=2.0, pKNa=0.03,
                 KmK=1.0, KmNa=40.0, KmNai=87.5, KmCa=1.38, ksat=0.1, alpha=2.5, gamma=0.35,
                 KpCa=0.0005, Kup=0.00025, k1p=0.15, k2p=0.045, k3=0.060, k4=0.005, EC=1.5,
                 maxsr=2.5, minsr=1.0, Bufc=0.2, Kbufc=0.001, Bufsr=10.0, Kbufsr=0.3,
                 Bufss=0.4, Kbufss=0.00025)

# Conductances / maximal rates that the C-ABI exposes as overridable
# parameters, in this order.
TTP_PARAM_NAMES = ["GNa", "GK1", "Gto", "GKr", "GKs", "GCaL", "GbNa", "GbCa", "GpCa", "GpK",
                   "kNaCa", "PNaK", "Vrel", "Vleak", "Vmaxup", "Vxfer"]
_TTP_BASE = dict(GNa=14.838, GK1=5.405, Gto=0.294, GKr=0.153, GKs=0.392, GCaL=3.980e-5,
                 GbNa=0.00029, GbCa=0.000592, GpCa=0.1238, GpK=0.0146, kNaCa=1000.0,
                 PNaK=2.724, Vrel=0.102, Vleak=0.00036, Vmaxup=0.006375, Vxfer=0.0038)


def ttp06_params(variant="epi"):
    p = dict(_TTP_BASE)
    if variant == "endo":
        p["Gto"] = 0.073
    elif variant == "mid":
        p["GKs"] = 0.098
    elif variant != "epi":
        raise ValueError(variant)
    p["endo_s_gate"] = variant == "endo"
    return p


# Initial conditions printed in the paper (Section "Slab benchmark"),
# converted from V to mV; gate / concentration order is the state order.
TTP_IC = dict(V=-85.23, m=0.00172, h=0.7444, j=0.7045, xr1=0.00621, xr2=0.4712, xs=0.00095,
              s=0.999998, r=2.42e-8, d=3.373e-5, f=0.7888, f2=0.9755, fcass=0.9953,
              cai=0.000126, casr=3.64, cass=0.00036, nai=8.604, ki=136.89, rr=0.9073)
TTP_STATE = ["m", "h", "j", "xr1", "xr2", "xs", "s", "r", "d", "f", "f2", "fcass",
             "cai", "casr", "cass", "nai", "ki", "rr"]


def ttp06_initial(n):
    return np.full(n, TTP_IC["V"]), np.vstack([np.full(n, TTP_IC[k]) for k in TTP_STATE])


def ttp06_gate_targets(V, cass, p):
    """(y_inf, tau) for the 12 gates m h j xr1 xr2 xs s r d f f2 fcass."""
    V = np.asarray(V, np.float64)
    # fast sodium
    m_inf = 1.0 / (1.0 + np.exp((-56.86 - V) / 9.03)) ** 2
    a_m = 1.0 / (1.0 + np.exp((-60.0 - V) / 5.0))
    b_m = 0.1 / (1.0 + np.exp((V + 35.0) / 5.0)) + 0.10 / (1.0 + np.exp((V - 50.0) / 200.0))
    tau_m = a_m * b_m
    h_inf = 1.0 / (1.0 + np.exp((V + 71.55) / 7.43)) ** 2
    hi = V >= -40.0
    a_h = np.where(hi, 0.0, 0.057 * np.exp(-(V + 80.0) / 6.8))
    b_h = np.where(hi, 0.77 / (0.13 * (1.0 + np.exp(-(V + 10.66) / 11.1))),
                   2.7 * np.exp(0.079 * V) + 3.1e5 * np.exp(0.3485 * V))
    tau_h = 1.0 / (a_h + b_h)
    j_inf = h_inf
    a_j = np.where(hi, 0.0,
                   (-2.5428e4 * np.exp(0.2444 * V) - 6.948e-6 * np.exp(-0.04391 * V)) * (V + 37.78)
                   / (1.0 + np.exp(0.311 * (V + 79.23))))
    b_j = np.where(hi, 0.6 * np.exp(0.057 * V) / (1.0 + np.exp(-0.1 * (V + 32.0))),
                   0.02424 * np.exp(-0.01052 * V) / (1.0 + np.exp(-0.1378 * (V + 40.14))))
    tau_j = 1.0 / (a_j + b_j)
    # rapid delayed rectifier
    xr1_inf = 1.0 / (1.0 + np.exp((-26.0 - V) / 7.0))
    tau_xr1 = (450.0 / (1.0 + np.exp((-45.0 - V) / 10.0))) * (6.0 / (1.0 + np.exp((V + 30.0) / 11.5)))
    xr2_inf = 1.0 / (1.0 + np.exp((V + 88.0) / 24.0))
    tau_xr2 = (3.0 / (1.0 + np.exp((-60.0 - V) / 20.0))) * (1.12 / (1.0 + np.exp((V - 60.0) / 20.0)))
    # slow delayed rectifier
    xs_inf = 1.0 / (1.0 + np.exp((-5.0 - V) / 14.0))
    tau_xs = (1400.0 / np.sqrt(1.0 + np.exp((5.0 - V) / 6.0))) * (1.0 / (1.0 + np.exp((V - 35.0) / 15.0))) + 80.0
    # transient outward
    if p["endo_s_gate"]:
        s_inf = 1.0 / (1.0 + np.exp((V + 28.0) / 5.0))
        tau_s = 1000.0 * np.exp(-(V + 67.0) ** 2 / 1000.0) + 8.0
    else:
        s_inf = 1.0 / (1.0 + np.exp((V + 20.0) / 5.0))
        tau_s = 85.0 * np.exp(-(V + 45.0) ** 2 / 320.0) + 5.0 / (1.0 + np.exp((V - 20.0) / 5.0)) + 3.0
    r_inf = 1.0 / (1.0 + np.exp((20.0 - V) / 6.0))
    tau_r = 9.5 * np.exp(-(V + 40.0) ** 2 / 1800.0) + 0.8
    # L-type calcium
    d_inf = 1.0 / (1.0 + np.exp((-8.0 - V) / 7.5))
    tau_d = ((1.4 / (1.0 + np.exp((-35.0 - V) / 13.0)) + 0.25) * (1.4 / (1.0 + np.exp((V + 5.0) / 5.0)))
             + 1.0 / (1.0 + np.exp((50.0 - V) / 20.0)))
    f_inf = 1.0 / (1.0 + np.exp((V + 20.0) / 7.0))
    tau_f = (1102.5 * np.exp(-(V + 27.0) ** 2 / 225.0) + 200.0 / (1.0 + np.exp((13.0 - V) / 10.0))
             + 180.0 / (1.0 + np.exp((V + 30.0) / 10.0)) + 20.0)
    f2_inf = 0.67 / (1.0 + np.exp((V + 35.0) / 7.0)) + 0.33
    tau_f2 = (600.0 * np.exp(-(V + 25.0) ** 2 / 170.0) + 31.0 / (1.0 + np.exp((25.0 - V) / 10.0))
              + 16.0 / (1.0 + np.exp((V + 30.0) / 10.0)))
    cr = (np.asarray(cass) / 0.05) ** 2
    fcass_inf = 0.6 / (1.0 + cr) + 0.4
    tau_fcass = 80.0 / (1.0 + cr) + 2.0
    infs = [m_inf, h_inf, j_inf, xr1_inf, xr2_inf, xs_inf, s_inf, r_inf, d_inf, f_inf, f2_inf, fcass_inf]
    taus = [tau_m, tau_h, tau_j, tau_xr1, tau_xr2, tau_xs, tau_s, tau_r, tau_d, tau_f, tau_f2, tau_fcass]
    return infs, taus


def _z_over_expm1(z):
    """z / (e^z - 1), continuous at z = 0 (value 1)."""
    z = np.asarray(z, np.float64)
    small = np.abs(z) < 1e-12
    zs = np.where(small, 1.0, z)
    return np.where(small, 1.0 - 0.5 * z, zs / np.expm1(zs))


def ttp06_currents(V, g, c, p):
    """All TTP06 currents and intracellular fluxes at (V, gates g, concentrations c).

    g: the 12 gates in state order; c: cai, casr, cass, nai, ki, rr.
    Transmembrane currents in pA/pF (= mV/ms), fluxes in mM/ms.
    """
    K = TTP_CONST
    m, h, j, xr1, xr2, xs, s, r, d, f, f2, fcass = g
    cai, casr, cass, nai, ki, rr = c
    RTF = K["R"] * K["T"] / K["F"]
    E_Na = RTF * np.log(K["Nao"] / nai)
    E_K = RTF * np.log(K["Ko"] / ki)
    E_Ks = RTF * np.log((K["Ko"] + K["pKNa"] * K["Nao"]) / (ki + K["pKNa"] * nai))
    E_Ca = 0.5 * RTF * np.log(K["Cao"] / cai)
    sqKo = np.sqrt(K["Ko"] / 5.4)
    out = {}
    out["INa"] = p["GNa"] * m ** 3 * h * j * (V - E_Na)
    out["Ito"] = p["Gto"] * r * s * (V - E_K)
    out["IKr"] = p["GKr"] * sqKo * xr1 * xr2 * (V - E_K)
    out["IKs"] = p["GKs"] * xs ** 2 * (V - E_Ks)
    a_K1 = 0.1 / (1.0 + np.exp(0.06 * (V - E_K - 200.0)))
    b_K1 = ((3.0 * np.exp(0.0002 * (V - E_K + 100.0)) + np.exp(0.1 * (V - E_K - 10.0)))
            / (1.0 + np.exp(-0.5 * (V - E_K))))
    out["IK1"] = p["GK1"] * sqKo * (a_K1 / (a_K1 + b_K1)) * (V - E_K)
    z = 2.0 * (V - 15.0) / RTF
    out["ICaL"] = (p["GCaL"] * d * f * f2 * fcass * 2.0 * K["F"]
                   * (0.25 * cass * np.exp(z) - K["Cao"]) * _z_over_expm1(z))
    u1 = np.exp(K["gamma"] * V / RTF)
    u2 = np.exp((K["gamma"] - 1.0) * V / RTF)
    out["INaCa"] = (p["kNaCa"] * (u1 * nai ** 3 * K["Cao"] - u2 * K["Nao"] ** 3 * cai * K["alpha"])
                    / ((K["KmNai"] ** 3 + K["Nao"] ** 3) * (K["KmCa"] + K["Cao"]) * (1.0 + K["ksat"] * u2)))
    out["INaK"] = (p["PNaK"] * K["Ko"] * nai
                   / ((K["Ko"] + K["KmK"]) * (nai + K["KmNa"])
                      * (1.0 + 0.1245 * np.exp(-0.1 * V / RTF) + 0.0353 * np.exp(-V / RTF))))
    out["IpCa"] = p["GpCa"] * cai / (K["KpCa"] + cai)
    out["IpK"] = p["GpK"] * (V - E_K) / (1.0 + np.exp((25.0 - V) / 5.98))
    out["IbNa"] = p["GbNa"] * (V - E_Na)
    out["IbCa"] = p["GbCa"] * (V - E_Ca)
    # sarcoplasmic reticulum and subspace fluxes
    out["Iup"] = p["Vmaxup"] / (1.0 + K["Kup"] ** 2 / cai ** 2)
    out["Ileak"] = p["Vleak"] * (casr - cai)
    kcasr = K["maxsr"] - (K["maxsr"] - K["minsr"]) / (1.0 + (K["EC"] / casr) ** 2)
    k1 = K["k1p"] / kcasr
    k2 = K["k2p"] * kcasr
    O = k1 * cass ** 2 * rr / (K["k3"] + k1 * cass ** 2)
    out["Irel"] = p["Vrel"] * O * (casr - cass)
    out["Ixfer"] = p["Vxfer"] * (cass - cai)
    out["dRR"] = -k2 * cass * rr + K["k4"] * (1.0 - rr)
    return out


MEMBRANE = ["INa", "IK1", "Ito", "IKr", "IKs", "ICaL", "INaCa", "INaK", "IpCa", "IpK", "IbNa", "IbCa"]


def ttp06_iion(V, w, p):
    cur = ttp06_currents(V, w[:12], w[12:], p)
    return sum(cur[k] for k in MEMBRANE)


def _free_from_total(total, B, Kd):
    """Positive root c of c + B c/(c + Kd) = total (rapid buffering)."""
    b = B + Kd - total
    disc = np.sqrt(b * b + 4.0 * Kd * total)
    return np.where(b >= 0.0, 2.0 * Kd * total / (b + disc), 0.5 * (disc - b))


def ttp06_step(V_star, w, dt, p):
    K = TTP_CONST
    g_old = w[:12]
    c = w[12:]
    cai, casr, cass, nai, ki, rr = c
    infs, taus = ttp06_gate_targets(V_star, cass, p)
    g = np.stack([infs[i] + (g_old[i] - infs[i]) * np.exp(-dt / taus[i]) for i in range(12)])
    cur = ttp06_currents(V_star, g, c, p)
    cmF = K["Cm"] / K["F"]
    d_cai_tot = (-(cur["IbCa"] + cur["IpCa"] - 2.0 * cur["INaCa"]) * cmF / (2.0 * K["Vc"])
                 + (K["Vsr"] / K["Vc"]) * (cur["Ileak"] - cur["Iup"]) + cur["Ixfer"])
    d_casr_tot = cur["Iup"] - cur["Ileak"] - cur["Irel"]
    d_cass_tot = (-cur["ICaL"] * cmF / (2.0 * K["Vss"]) + (K["Vsr"] / K["Vss"]) * cur["Irel"]
                  - (K["Vc"] / K["Vss"]) * cur["Ixfer"])
    d_nai = -(cur["INa"] + cur["IbNa"] + 3.0 * cur["INaK"] + 3.0 * cur["INaCa"]) * cmF / K["Vc"]
    d_ki = -(cur["IK1"] + cur["Ito"] + cur["IKr"] + cur["IKs"] - 2.0 * cur["INaK"] + cur["IpK"]) * cmF / K["Vc"]
    cai_tot = cai + K["Bufc"] * cai / (cai + K["Kbufc"])
    casr_tot = casr + K["Bufsr"] * casr / (casr + K["Kbufsr"])
    cass_tot = cass + K["Bufss"] * cass / (cass + K["Kbufss"])
    cai_n = _free_from_total(cai_tot + dt * d_cai_tot, K["Bufc"], K["Kbufc"])
    casr_n = _free_from_total(casr_tot + dt * d_casr_tot, K["Bufsr"], K["Kbufsr"])
    cass_n = _free_from_total(cass_tot + dt * d_cass_tot, K["Bufss"], K["Kbufss"])
    nai_n = nai + dt * d_nai
    ki_n = ki + dt * d_ki
    rr_n = rr + dt * cur["dRR"]
    return np.vstack([g, cai_n, casr_n, cass_n, nai_n, ki_n, rr_n])


def _ttp_totals(c):
    """Buffered total calcium (cytosol, SR, subspace) of free concentrations."""
    K = TTP_CONST
    cai, casr, cass = c[0], c[1], c[2]
    return (cai + K["Bufc"] * cai / (cai + K["Kbufc"]),
            casr + K["Bufsr"] * casr / (casr + K["Kbufsr"]),
            cass + K["Bufss"] * cass / (cass + K["Kbufss"]))


def ttp06_step_bdf(V_ext, w_hist, cb, ce, dt, alpha, p):
    """Paper's scheme for TTP06.  w_hist = [w_n, w_{n-1}, ...]; cb, ce: the
    BDF and extrapolation coefficients over that history."""
    K = TTP_CONST
    w_bdf = sum(c * w for c, w in zip(cb, w_hist))
    w_ext = sum(c * w for c, w in zip(ce, w_hist))
    infs, taus = ttp06_gate_targets(V_ext, w_ext[14], p)          # fcass at cass_EXT
    g = np.stack([gate_bdf(w_bdf[i], infs[i], taus[i], dt, alpha) for i in range(12)])
    c_ext = w_ext[12:]
    cur = ttp06_currents(V_ext, g, c_ext, p)
    cmF = K["Cm"] / K["F"]
    d_cai_tot = (-(cur["IbCa"] + cur["IpCa"] - 2.0 * cur["INaCa"]) * cmF / (2.0 * K["Vc"])
                 + (K["Vsr"] / K["Vc"]) * (cur["Ileak"] - cur["Iup"]) + cur["Ixfer"])
    d_casr_tot = cur["Iup"] - cur["Ileak"] - cur["Irel"]
    d_cass_tot = (-cur["ICaL"] * cmF / (2.0 * K["Vss"]) + (K["Vsr"] / K["Vss"]) * cur["Irel"]
                  - (K["Vc"] / K["Vss"]) * cur["Ixfer"])
    d_nai = -(cur["INa"] + cur["IbNa"] + 3.0 * cur["INaK"] + 3.0 * cur["INaCa"]) * cmF / K["Vc"]
    d_ki = -(cur["IK1"] + cur["Ito"] + cur["IKr"] + cur["IKs"] - 2.0 * cur["INaK"] + cur["IpK"]) * cmF / K["Vc"]
    tot_bdf = [sum(c * t for c, t in zip(cb, ts)) for ts in zip(*[_ttp_totals(w[12:]) for w in w_hist])]
    cai_n = _free_from_total((tot_bdf[0] + dt * d_cai_tot) / alpha, K["Bufc"], K["Kbufc"])
    casr_n = _free_from_total((tot_bdf[1] + dt * d_casr_tot) / alpha, K["Bufsr"], K["Kbufsr"])
    cass_n = _free_from_total((tot_bdf[2] + dt * d_cass_tot) / alpha, K["Bufss"], K["Kbufss"])
    nai_n = (w_bdf[15] + dt * d_nai) / alpha
    ki_n = (w_bdf[16] + dt * d_ki) / alpha
    rr_n = (w_bdf[17] + dt * cur["dRR"]) / alpha
    return np.vstack([g, cai_n, casr_n, cass_n, nai_n, ki_n, rr_n])


# ---------------------------------------------------------------------------
# Uniform interface
# ---------------------------------------------------------------------------

class IonicModel:
    """Bundles one model's step / current / initial state."""

    def __init__(self, name: str, variant: str = ""):
        self.name = name
        self.variant = variant
        if name == "ttp06":
            self.p = ttp06_params(variant or "epi")
        elif name == "ap":
            self.p = dict(AP_DEFAULT)
        elif name == "bo":
            if variant not in ("", "epi"):
                raise ValueError("BO: only the EPI parameter set")
            self.p = dict(BO_EPI)
        elif name == "passive":
            self.p = {}
        else:
            raise ValueError(name)
        self.n_vars = N_VARS[name]
        self.threshold = ACT_THRESHOLD[name]
        self.mv_per_unit = MV_PER_UNIT[name]

    def initial(self, n):
        if self.name == "ap":
            return ap_initial(n)
        if self.name == "bo":
            return bo_initial(n)
        if self.name == "ttp06":
            return ttp06_initial(n)
        return np.zeros(n), np.zeros((0, n))

    def step(self, u_star, w, dt):
        if self.name == "ap":
            return ap_step(u_star, w, dt, self.p)
        if self.name == "bo":
            return bo_step(u_star, w, dt, self.p)
        if self.name == "ttp06":
            return ttp06_step(u_star, w, dt, self.p)
        return w

    def step_bdf(self, u_ext, w_hist, cb, ce, dt, alpha):
        """The paper's semi-implicit BDF step from w_hist = [w_n, w_{n-1}, ...]
        with BDF / extrapolation coefficients cb, ce and leading alpha."""
        if self.name == "ttp06":
            return ttp06_step_bdf(u_ext, w_hist, cb, ce, dt, alpha, self.p)
        w_bdf = sum(c * w for c, w in zip(cb, w_hist))
        w_ext = sum(c * w for c, w in zip(ce, w_hist))
        if self.name == "ap":
            return ap_step_bdf(u_ext, w_bdf, w_ext, dt, alpha, self.p)
        if self.name == "bo":
            return bo_step_bdf(u_ext, w_bdf, w_ext, dt, alpha, self.p)
        return w_hist[0]

    def iion(self, u, w):
        if self.name == "ap":
            return ap_iion(u, w, self.p)
        if self.name == "bo":
            return bo_iion(u, w, self.p)
        if self.name == "ttp06":
            return ttp06_iion(u, w, self.p)
        return np.zeros_like(np.asarray(u, np.float64))
