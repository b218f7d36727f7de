"""Pins of the oracle's second ionic integrator, the paper's semi-implicit
BDF step (eq. of the time-discrete ionic model): gates implicit, other
variables explicit or linearly implicit, BDF order of the potential.

- a gate at frozen potential follows the linear BDF recurrence, whose
  solution is known in closed form from its characteristic roots (fixes the
  BDF coefficients and the implicit treatment);
- at frozen potential, the error against a tight reference integration of
  the same ODEs shrinks as dt (BDF1) and dt^2 (BDF2) for Aliev-Panfilov and
  the full TTP06 state (fixes the extrapolated explicit terms, the history
  levels and the buffered-calcium totals);
- rest states are fixed points;
- a spatially uniform monodomain run with the BDF ionic scheme reproduces the
  single-cell update.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import workloads as W
from oracle import ionic as I
from oracle import monodomain as OM


def _run_frozen(model, u, w0, dt, steps, sigma):
    """Single cell at frozen potential u with the BDF ionic scheme of order
    sigma (lower orders at start-up)."""
    hist = [w0.copy()]
    for n in range(steps):
        s = min(sigma, n + 1)
        alpha, cb, ce = OM.BDF_COEFFS[s]
        w_new = model.step_bdf(np.array([u]), hist[:s], cb, ce, dt, alpha)
        hist = [w_new] + hist[:2]
    return hist[0]


def test_bo_gates_follow_bdf2_closed_form():
    m = I.IonicModel("bo", "epi")
    u, dt, steps = 0.2, 0.5, 60
    infs, taus = I.bo_gate_targets(np.array([u]), m.p)
    w0 = np.array([[0.9], [0.2], [0.7]])
    hist = [w0]
    seq = [w0[:, 0]]
    for n in range(steps):
        s = min(2, n + 1)
        alpha, cb, ce = OM.BDF_COEFFS[s]
        w = m.step_bdf(np.array([u]), hist[:s], cb, ce, dt, alpha)
        hist = [w] + hist[:1]
        seq.append(w[:, 0])
    seq = np.array(seq)
    for g in range(3):
        yinf, tau = float(infs[g][0]), float(taus[g][0])
        q = dt / tau
        e0 = seq[0, g] - yinf
        e1 = e0 / (1.0 + q)                         # BDF1 start-up step
        # (3/2 + q) e_{n+1} - 2 e_n + 1/2 e_{n-1} = 0 for n >= 1: e_n = A r1^n + B r2^n
        r = np.roots([1.5 + q, -2.0, 0.5]).astype(complex)
        coef = np.linalg.solve(np.array([[1.0, 1.0], [r[0], r[1]]], complex), np.array([e0, e1], complex))
        n = np.arange(1, steps + 1)
        closed = yinf + np.real(coef[0] * r[0] ** n + coef[1] * r[1] ** n)
        assert np.max(np.abs(seq[1:, g] - closed)) < 1e-13 * max(1.0, abs(yinf)), g


def _ap_reference(u, v0, T):
    p = I.AP_DEFAULT
    f = lambda t, y: [float(I.ap_dv(u, y[0], p))]
    return solve_ivp(f, (0.0, T), [v0], method="Radau", rtol=1e-12, atol=1e-14).y[0, -1]


def _ttp_reference(V, w0, T, p):
    K = I.TTP_CONST
    tot0 = I._ttp_totals(w0[12:15])

    def unpack(y):
        g = y[:12]
        cai = I._free_from_total(y[12], K["Bufc"], K["Kbufc"])
        casr = I._free_from_total(y[13], K["Bufsr"], K["Kbufsr"])
        cass = I._free_from_total(y[14], K["Bufss"], K["Kbufss"])
        return g, np.array([cai, casr, cass, y[15], y[16], y[17]])

    def rhs(t, y):
        g, c = unpack(y)
        infs, taus = I.ttp06_gate_targets(V, c[2], p)
        dg = [(infs[i] - g[i]) / taus[i] for i in range(12)]
        cur = I.ttp06_currents(V, g, c, p)
        cmF = K["Cm"] / K["F"]
        d_cai = (-(cur["IbCa"] + cur["IpCa"] - 2.0 * cur["INaCa"]) * cmF / (2.0 * K["Vc"])
                 + (K["Vsr"] / K["Vc"]) * (cur["Ileak"] - cur["Iup"]) + cur["Ixfer"])
        d_casr = cur["Iup"] - cur["Ileak"] - cur["Irel"]
        d_cass = (-cur["ICaL"] * cmF / (2.0 * K["Vss"]) + (K["Vsr"] / K["Vss"]) * cur["Irel"]
                  - (K["Vc"] / K["Vss"]) * cur["Ixfer"])
        d_nai = -(cur["INa"] + cur["IbNa"] + 3.0 * cur["INaK"] + 3.0 * cur["INaCa"]) * cmF / K["Vc"]
        d_ki = -(cur["IK1"] + cur["Ito"] + cur["IKr"] + cur["IKs"] - 2.0 * cur["INaK"] + cur["IpK"]) * cmF / K["Vc"]
        return np.array([float(x) for x in dg] + [d_cai, d_casr, d_cass, d_nai, d_ki, cur["dRR"]], float)

    y0 = np.concatenate([w0[:12], tot0, w0[15:]])
    yT = solve_ivp(rhs, (0.0, T), y0, method="Radau", rtol=1e-12, atol=1e-15).y[:, -1]
    g, c = unpack(yT)
    return np.concatenate([g, c])


@pytest.mark.parametrize("sigma,order", [(1, 1.0), (2, 2.0)])
def test_ap_bdf_order_at_frozen_potential(sigma, order):
    m = I.IonicModel("ap")
    u, v0, T = 0.6, 0.3, 20.0
    ref = _ap_reference(u, v0, T)
    errs = []
    for dt in (0.2, 0.1, 0.05):
        v = _run_frozen(m, u, np.array([[v0]]), dt, int(round(T / dt)), sigma)
        errs.append(abs(v[0, 0] - ref))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.25), (errs, rates)


@pytest.mark.parametrize("sigma,order", [(1, 1.0), (2, 2.0)])
def test_ttp06_bdf_order_at_frozen_potential(sigma, order):
    m = I.IonicModel("ttp06", "epi")
    V, T = -20.0, 2.0
    _, w0 = I.ttp06_initial(1)
    ref = _ttp_reference(V, w0[:, 0], T, m.p)
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        w = _run_frozen(m, V, w0, dt, int(round(T / dt)), sigma)[:, 0]
        errs.append(np.max(np.abs(w - ref) / np.maximum(np.abs(ref), 1e-3)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.3), (errs, rates)


def test_bdf_scheme_rest_fixed_points():
    ap = I.IonicModel("ap")
    w = _run_frozen(ap, 0.0, np.zeros((1, 1)), 0.05, 50, 2)
    assert np.all(w == 0.0)
    bo = I.IonicModel("bo", "epi")
    (vi, wi, si), _ = I.bo_gate_targets(np.array([0.0]), bo.p)
    w0 = np.array([vi, wi, si])
    w = _run_frozen(bo, 0.0, w0, 0.05, 50, 3)
    assert np.allclose(w, w0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("model,variant,bdf", [("ap", "", 2), ("bo", "epi", 3), ("ttp06", "endo", 2)])
def test_uniform_state_bdf_scheme_reduces_to_single_cell(model, variant, bdf):
    m = W.slab_q1(3.0, 2.0, 1.0, 0.5)
    big = W.Stimulus(W.CUBE, (1.5, 1.0, 0.5), 10.0, 50.0, 0.0, 1.0, 0.0)
    o = OM.Monodomain(m.xyz, m.conn, W.uniform_fibers(m.n_nodes), (0.17, 0.019, 0.019), 140.0, 0.01, model,
                      variant, [big], 0.05, bdf, "dense", ionic_scheme="bdf")
    u1, w1 = o.model.initial(1)
    hist = [u1.copy()] * 3
    whist = [w1.copy()] * 3
    scale = 50.0 / (140.0 * 0.01 * o.model.mv_per_unit)
    for step in range(60):
        s_n = min(bdf, step + 1)
        alpha, cb, ce = OM.BDF_COEFFS[s_n]
        ub = sum(c * h for c, h in zip(cb, hist))
        ue = sum(c * h for c, h in zip(ce, hist))
        w1 = o.model.step_bdf(ue, whist[:s_n], cb, ce, 0.05, alpha)
        whist = [w1] + whist[:2]
        iapp = scale if (step + 1) * 0.05 <= 1.0 + 1e-9 else 0.0
        unew = (ub + 0.05 * (iapp - o.model.iion(ue, w1))) / alpha
        hist = [unew] + hist[:2]
        o.step()
        assert np.max(np.abs(o.u - unew[0])) < 1e-10 * max(1.0, abs(unew[0])), step
        assert np.max(np.abs(o.w - w1)) < 1e-10 * max(1.0, np.max(np.abs(w1)))
