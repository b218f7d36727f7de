"""Pins of the oracle's ionic models and integrator.

What fixes them: exact rest-state fixed points (AP, BO), near-rest drift of
the TTP06 initial conditions the paper prints, Rush-Larsen = exact solution
of the frozen linear gate ODE (brute force), the rapid-buffer inversion
against bisection, and the removable singularity of I_CaL against the
unrewritten Goldman-Hodgkin-Katz form.
"""
import json
import os

import numpy as np
import pytest

from oracle import ionic as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "nversion_slab.json")


def test_ap_rest_is_exact_fixed_point():
    m = I.IonicModel("ap")
    u, w = m.initial(5)
    w1 = m.step(u, w, 0.05)
    assert np.array_equal(w1, w)
    assert np.array_equal(m.iion(u, w1), np.zeros(5))


def test_bo_rest_is_exact_fixed_point():
    m = I.IonicModel("bo")
    s_inf = (1 + np.tanh(I.BO_EPI["k_s"] * (0.0 - I.BO_EPI["u_s"]))) / 2
    w = np.array([[1.0], [1.0], [s_inf]])
    u = np.zeros(1)
    w1 = m.step(u, w, 0.05)
    assert np.max(np.abs(w1 - w)) < 1e-16
    assert m.iion(u, w1)[0] == 0.0


def test_ttp06_printed_ic_is_near_rest():
    """The paper's initial conditions are close to, not exactly at, rest: the
    unpaced cell drifts by well under a millivolt in 50 ms."""
    with open(GOLD) as fh:
        g = json.load(fh)
    ic = g["ttp06_initial_conditions"]
    assert ic["V_mV"] == I.TTP_IC["V"]
    for k in I.TTP_STATE:
        assert ic[k] == I.TTP_IC[k], k
    for variant in ("epi", "endo", "mid"):
        m = I.IonicModel("ttp06", variant)
        u, w = m.initial(1)
        dt = 0.05
        for _ in range(1000):
            w = m.step(u, w, dt)
            u = u - dt * m.iion(u, w)
        assert abs(u[0] - I.TTP_IC["V"]) < 1.0, (variant, u)


def test_rush_larsen_is_exact_for_frozen_gate():
    """Frozen V: dy/dt = (y_inf - y)/tau has the exact solution RL gives; check
    against 20000 explicit sub-steps for every TTP06 gate."""
    p = I.ttp06_params("endo")
    V = np.array([-80.0, -35.0, 10.0])
    cass = np.array([2e-4, 1e-3, 5e-3])
    rng = np.random.default_rng(0)
    g0 = rng.uniform(0, 1, (12, 3))
    w = np.vstack([g0, np.tile([[1.2e-4], [3.0], [cass[0]], [8.6], [136.9], [0.9]], (1, 3))])
    w[14] = cass
    dt = 0.05
    w1 = I.ttp06_step(V, w, dt, p)
    infs, taus = I.ttp06_gate_targets(V, cass, p)
    nsub = 20000
    for gi in range(12):
        y = g0[gi].copy()
        for _ in range(nsub):
            y = y + (dt / nsub) * (infs[gi] - y) / taus[gi]
        assert np.max(np.abs(w1[gi] - y)) < 1e-5 * max(1.0, np.max(np.abs(g0[gi] - infs[gi]))), gi


def test_rapid_buffer_inversion_matches_bisection():
    for B, Kd in ((0.2, 0.001), (10.0, 0.3), (0.4, 0.00025)):
        for c_true in (1e-5, 1e-4, 2e-3, 0.5, 4.0):
            total = c_true + B * c_true / (c_true + Kd)
            c = float(I._free_from_total(np.array(total), B, Kd))
            lo, hi = 0.0, total
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if mid + B * mid / (mid + Kd) > total:
                    hi = mid
                else:
                    lo = mid
            assert abs(c - lo) <= 1e-13 * c_true + 1e-300
            assert abs(c - c_true) <= 1e-12 * c_true


def test_ical_rewrite_matches_ghk_form_and_is_continuous():
    K = I.TTP_CONST
    p = I.ttp06_params("epi")
    RTF = K["R"] * K["T"] / K["F"]
    gates = [np.array([0.5])] * 12
    conc = [np.array(x) for x in ([1e-4], [3.0], [8e-4], [8.6], [136.0], [0.9])]
    for V in (-40.0, 5.0, 14.0, 16.5, 40.0):
        Varr = np.array([V])
        got = I.ttp06_currents(Varr, gates, conc, p)["ICaL"][0]
        e = np.exp(2 * (V - 15) / RTF)
        ref = (p["GCaL"] * 0.5 ** 4 * 4 * (V - 15) * K["F"] ** 2 / (K["R"] * K["T"])
               * (0.25 * 8e-4 * e - K["Cao"]) / (e - 1))
        assert abs(got - ref) < 1e-12 * abs(ref)
    at = I.ttp06_currents(np.array([15.0]), gates, conc, p)["ICaL"][0]
    near = I.ttp06_currents(np.array([15.0 + 1e-7]), gates, conc, p)["ICaL"][0]
    assert np.isfinite(at) and abs(at - near) < 1e-8 * abs(at)


def test_ttp06_membrane_current_balance_at_rest():
    """At the printed initial state all transmembrane currents are small
    (the cell is near rest): |I_ion| < 0.1 pA/pF."""
    for variant in ("epi", "endo", "mid"):
        m = I.IonicModel("ttp06", variant)
        u, w = m.initial(1)
        assert abs(m.iion(u, w)[0]) < 0.1


@pytest.mark.parametrize("model", ["ap", "bo", "ttp06"])
def test_action_potential_plausible(model):
    """Plausibility only (the paper prints no trace): a suprathreshold pulse
    gives one action potential that returns towards rest."""
    m = I.IonicModel(model, "epi" if model == "ttp06" else "")
    u, w = m.initial(1)
    amp = {"ap": 0.5, "bo": 0.5, "ttp06": 52.0}[model]
    dt = 0.02
    peak = -1e9
    for n in range(int(450 / dt)):
        t = (n + 1) * dt
        w = m.step(u, w, dt)
        u = u + dt * ((amp if t <= 1.0 else 0.0) - m.iion(u, w))
        peak = max(peak, u[0])
    lo, hi = {"ap": (0.9, 1.05), "bo": (1.3, 1.6), "ttp06": (25.0, 45.0)}[model]
    assert lo < peak < hi
    rest = {"ap": 0.0, "bo": 0.0, "ttp06": -85.23}[model]
    amp_ = peak - rest
    assert abs(u[0] - rest) < 0.15 * amp_
