"""Single-cell pacing (FP64, CPU).  Test infrastructure.

The paper initializes the ionic state of its ventricular cases by long
single-cell simulations paced at the cardiac period (Section "Ventricular
slab": 1000-cycle single-cell runs with a 0.8 s period, one per volume).  A
single cell is the monodomain step without diffusion: with K 1 = 0 and a
spatially uniform state the linear system reduces node by node to
  alpha u_{n+1} = u_BDF + dt (I_app(t_{n+1}) - I_ion(u_EXT, w_{n+1})),
with the ionic step of ionic.py at u_EXT (the same BDF order and start-up as
the tissue).  The stimulus of amplitude `amp` (mV/ms) is active on step n+1
when t_{n+1} lies in (k period, k period + dur] for some k >= 0.

Cells are vectorized: each column of the state is one cell, with its own
parameter set.
"""
from __future__ import annotations

import numpy as np

from .ionic import IonicModel
from .monodomain import BDF_COEFFS, stimulus_active


def pace(model, variant, n_cells, dt, period, amp, dur, n_beats, bdf=2, params=None, u0=None, w0=None,
         ionic_scheme="rl"):
    """Pace n_cells cells for n_beats periods.  params: list of per-cell
    parameter dicts overriding the model defaults (None: defaults).
    Returns (u, w) after the last step, u [n_cells], w [n_vars, n_cells]."""
    models = []
    for c in range(n_cells):
        m = IonicModel(model, variant)
        if params is not None:
            m.p.update(params[c])
        models.append(m)
    base = models[0]
    if u0 is None or w0 is None:
        u0, w0 = base.initial(n_cells)
    u = np.array(u0, np.float64)
    w = np.array(w0, np.float64).reshape(base.n_vars, n_cells)
    hist = [u.copy(), u.copy(), u.copy()]
    whist = [w.copy(), w.copy(), w.copy()]
    scale = 1.0 / base.mv_per_unit
    n_steps = int(round(n_beats * period / dt))
    for n in range(n_steps):
        s = min(bdf, n + 1)
        alpha, cb, ce = BDF_COEFFS[s]
        ub = sum(c * h for c, h in zip(cb, hist))
        ue = sum(c * h for c, h in zip(ce, hist))
        t1 = (n + 1) * dt
        iapp = amp * scale if stimulus_active(t1, 0.0, dur, period, dt) else 0.0
        wn = np.empty_like(w)
        iion = np.empty(n_cells)
        for c, m in enumerate(models):
            if ionic_scheme == "bdf":
                wc = m.step_bdf(ue[c:c + 1], [x[:, c:c + 1] for x in whist[:s]], cb, ce, dt, alpha)
            else:
                wc = m.step(ue[c:c + 1], whist[0][:, c:c + 1], dt)
            wn[:, c] = wc[:, 0]
            iion[c] = m.iion(ue[c:c + 1], wc)[0]
        un = (ub + dt * (iapp - iion)) / alpha
        hist = [un] + hist[:2]
        whist = [wn] + whist[:2]
    return hist[0], whist[0]
