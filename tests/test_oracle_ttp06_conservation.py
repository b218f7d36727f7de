"""Charge conservation of the oracle's TTP06 concentration bookkeeping.

The membrane currents of the ten Tusscher-Panfilov model carry the ions
whose concentrations the model tracks, so one explicit step must satisfy

  F [V_c (dNa_i + dK_i) + 2 (V_c dCa_i,tot + V_sr dCa_sr,tot + V_ss dCa_ss,tot)]
      = -C_m dt sum(membrane currents)

with the currents at the point where the step evaluates its rates (paper:
ionic model ODEs, eq. 1, and the time-discrete ionic model, eq. 4; the
transfer fluxes between the cytosol, the SR and the subspace cancel).  The
identity fixes every stoichiometric factor (3 INaK, 2 INaK, 3 INaCa, 2 INaCa)
and every volume ratio of the bookkeeping, whatever the current formulas.
For the paper's BDF scheme the same holds with alpha X_{n+1} - X_BDF in place
of X_{n+1} - X_n.  Planted mistakes in the bookkeeping break it.
"""
import inspect
import types

import numpy as np
import pytest

import workloads as W
from oracle import ionic as I

K = I.TTP_CONST


def _totals(mod, w):
    c = w[12:]
    cai_t, casr_t, cass_t = mod._ttp_totals(c)
    return np.asarray(c[3], np.longdouble), np.asarray(c[4], np.longdouble), \
        np.asarray(cai_t, np.longdouble), np.asarray(casr_t, np.longdouble), np.asarray(cass_t, np.longdouble)


def _charge(comb):
    """F [V_c (Na + K) + 2 (V_c Ca_i,tot + V_sr Ca_sr,tot + V_ss Ca_ss,tot)]
    of a (possibly combined) set of species amounts; also its magnitude for
    the rounding bound."""
    na, k, ci, csr, css = comb
    F, Vc, Vsr, Vss = (np.longdouble(K[x]) for x in ("F", "Vc", "Vsr", "Vss"))
    q = F * (Vc * (na + k) + 2 * (Vc * ci + Vsr * csr + Vss * css))
    return q


def _scale(w):
    na, k, ci, csr, css = _totals(I, w)
    F, Vc, Vsr, Vss = (np.longdouble(K[x]) for x in ("F", "Vc", "Vsr", "Vss"))
    return F * (Vc * (abs(na) + abs(k)) + 2 * (Vc * abs(ci) + Vsr * abs(csr) + Vss * abs(css)))


def _membrane_sum(mod, V, g, c, p):
    cur = mod.ttp06_currents(V, g, c, p)
    return sum(np.asarray(cur[k], np.longdouble) for k in mod.MEMBRANE)


def _rl_residual(mod, variant, dt, seed):
    n = 400
    V, w = W.random_state("ttp06", n, seed)
    p = mod.ttp06_params(variant)
    w1 = mod.ttp06_step(V, w, dt, p)
    before, after = _totals(mod, w), _totals(mod, w1)
    lhs = _charge([a - b for a, b in zip(after, before)])
    rhs = -np.longdouble(K["Cm"]) * np.longdouble(dt) * _membrane_sum(mod, V, w1[:12], w[12:], p)
    # rounding of the FP64 state (a few ulps of each stored amount)
    bound = 64 * np.finfo(np.float64).eps * (_scale(w) + _scale(w1))
    return np.abs(lhs - rhs), bound, np.abs(rhs)


def _bdf_residual(mod, variant, dt, order, seed):
    n = 300
    cb = {1: [1.0], 2: [2.0, -0.5], 3: [3.0, -1.5, 1.0 / 3.0]}[order]
    ce = {1: [1.0], 2: [2.0, -1.0], 3: [3.0, -3.0, 1.0]}[order]
    alpha = {1: 1.0, 2: 1.5, 3: 11.0 / 6.0}[order]
    V, w0 = W.random_state("ttp06", n, seed)
    rng = np.random.default_rng(seed + 1)
    hist = [w0]
    for _ in range(order - 1):     # earlier levels: small perturbations of w0
        wk = w0 * (1.0 + 0.01 * rng.uniform(-1, 1, w0.shape))
        hist.append(wk)
    p = mod.ttp06_params(variant)
    w1 = mod.ttp06_step_bdf(V, hist, cb, ce, dt, alpha, p)
    w_ext = sum(c * w for c, w in zip(ce, hist))
    new = _totals(mod, w1)
    bdf = [sum(np.longdouble(c) * t for c, t in zip(cb, ts)) for ts in zip(*[_totals(mod, w) for w in hist])]
    lhs = _charge([np.longdouble(alpha) * a - b for a, b in zip(new, bdf)])
    rhs = -np.longdouble(K["Cm"]) * np.longdouble(dt) * _membrane_sum(mod, V, w1[:12], w_ext[12:], p)
    bound = 64 * np.finfo(np.float64).eps * (sum(_scale(w) for w in hist) * 4 + _scale(w1) * 2)
    return np.abs(lhs - rhs), bound, np.abs(rhs)


@pytest.mark.parametrize("variant", ["endo", "mid", "epi"])
@pytest.mark.parametrize("dt", [0.05, 1.0])
def test_rush_larsen_step_conserves_charge(variant, dt):
    err, bound, rhs = _rl_residual(I, variant, dt, seed=101)
    assert np.all(err <= bound + 1e-12 * rhs), float(np.max(err / (bound + 1e-12 * rhs)))
    # the identity is not vacuous: the currents move real charge
    assert np.median(rhs) > 1e3 * np.median(bound)


@pytest.mark.parametrize("variant", ["endo", "epi"])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_bdf_step_conserves_charge(variant, order):
    err, bound, rhs = _bdf_residual(I, variant, 1.0, order, seed=202)
    assert np.all(err <= bound + 1e-12 * rhs), float(np.max(err / (bound + 1e-12 * rhs)))
    assert np.median(rhs) > 1e3 * np.median(bound)


# Mistakes planted in the oracle's bookkeeping (source text of both steps).
_MUTATIONS = [
    ('3.0 * cur["INaK"] + 3.0 * cur["INaCa"]', '2.0 * cur["INaK"] + 3.0 * cur["INaCa"]'),
    ('3.0 * cur["INaK"] + 3.0 * cur["INaCa"]', '3.0 * cur["INaK"] + 2.0 * cur["INaCa"]'),
    ('- 2.0 * cur["INaK"] + cur["IpK"]', '- 3.0 * cur["INaK"] + cur["IpK"]'),
    ('- 2.0 * cur["INaCa"]) * cmF / (2.0 * K["Vc"])', '- 3.0 * cur["INaCa"]) * cmF / (2.0 * K["Vc"])'),
    ('(K["Vsr"] / K["Vc"]) * (cur["Ileak"] - cur["Iup"])', '(K["Vss"] / K["Vc"]) * (cur["Ileak"] - cur["Iup"])'),
    ('(K["Vc"] / K["Vss"]) * cur["Ixfer"]', '(K["Vsr"] / K["Vss"]) * cur["Ixfer"]'),
    ('-cur["ICaL"] * cmF / (2.0 * K["Vss"])', '-cur["ICaL"] * cmF / K["Vss"]'),
    ('+ cur["IpK"]) * cmF / K["Vc"]', '+ cur["IpK"]) * cmF / K["Vss"]'),
]


def _mutant(old, new):
    src = inspect.getsource(I)
    assert old in src, old
    mod = types.ModuleType("ionic_mutant")
    exec(compile(src.replace(old, new), "ionic_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("k", range(len(_MUTATIONS)))
def test_planted_bookkeeping_mistake_breaks_conservation(k):
    mod = _mutant(*_MUTATIONS[k])
    err, bound, rhs = _rl_residual(mod, "endo", 1.0, seed=101)
    assert np.max(err / (bound + 1e-12 * rhs)) > 1e3
    err, bound, rhs = _bdf_residual(mod, "endo", 1.0, 2, seed=202)
    assert np.max(err / (bound + 1e-12 * rhs)) > 1e3
