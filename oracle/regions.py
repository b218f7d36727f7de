"""Monodomain on several subdomains (FP64).  Test infrastructure.

Follows the paper's multi-subdomain monodomain problem (eq. (2) with one
ionic model per subdomain Omega_i) and its ionic current interpolation over
subdomains (Section "Cardiac electrophysiology: numerical discretization"):

  - every subdomain Omega_i carries its own ionic model parameters (for
    TTP06 the cell type and conductance overrides) and its own
    conductivities; the stiffness matrix is the sum of the subdomain
    stiffness matrices K = sum_i K^i, each assembled over the elements of
    Omega_i with D^i;
  - the ionic state lives at the nodes of each subdomain separately, so a
    node on the interface of two subdomains carries two ionic states, each
    advanced by its own subdomain's model at the node's u_EXT;
  - the ionic load is s = sum_i M^i I_ion^i, M^i the mass matrix assembled
    over the elements of Omega_i;
  - a subdomain marked non-conductive (scar, "disable conduction") is taken
    out of the problem: its elements are dropped, and nodes no other element
    uses are removed from the unknowns (their outputs are NaN).

  - a subdomain may run an ionic model other than the simulation's (eq. (2)
    gives each Omega_i its own I_ion^i and H^i).  The potential u is one
    field, kept in the simulation model's units (mV for TTP06, the
    dimensionless variable of AP / BO, u_mV = a u + b); a subdomain whose
    model has units (a_i, b_i) sees u_i = (a u + b - b_i) / a_i, and since
    du_mV/dt = -a_i I_ion^i, its current enters the load in the field's
    units as (a_i / a) I_ion^i(u_i, w^i).  With one model this is the
    identity.

Elements are labelled by material ids 0..R-1 (one id per subdomain, the
paper's Material IDs).  Everything else (BDF start-up, u_BDF / u_EXT, the
ionic step - Rush-Larsen or the paper's semi-implicit BDF scheme, each
subdomain keeping its own state history -, applied current as M I_app in the
field's units, CG or direct solve, activation times) is the
single-subdomain oracle's, see monodomain.py.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fem
from .ionic import MV_OFFSET, IonicModel
from .monodomain import BDF_COEFFS, Monodomain, stimulus_profile, stimulus_active  # noqa: F401


@dataclass
class Region:
    """One subdomain: TTP06 cell type, parameter overrides (names of the
    model's parameter dict), conductivities (None: the global ones), whether
    it conducts, and its ionic model (None: the simulation's)."""
    variant: str = ""
    params: dict = field(default_factory=dict)
    sigma: tuple | None = None
    conductive: bool = True
    model: str | None = None


class MultiRegion:
    def __init__(self, xyz, conn, material, regions, fibers, sigma, chi, cm, model, stimuli=(),
                 dt=0.05, bdf=1, solver="auto", rtol=1e-13, max_it=5000, ionic_scheme="rl"):
        xyz = np.asarray(xyz, np.float64)
        conn = np.asarray(conn, np.int64)
        material = np.asarray(material, np.int64)
        if material.shape != (conn.shape[0],):
            raise ValueError("one material id per element")
        if material.min() < 0 or material.max() >= len(regions):
            raise ValueError("material id without a region")
        if ionic_scheme not in ("rl", "bdf"):
            raise ValueError(ionic_scheme)
        self.ionic_scheme = ionic_scheme
        self.n_full = xyz.shape[0]
        keep = np.array([regions[m].conductive for m in material], bool)
        live = np.unique(conn[keep])
        cidx = np.full(self.n_full, -1, np.int64)
        cidx[live] = np.arange(live.size)
        self.live = live
        self.n = live.size
        self.dt = float(dt)
        self.sigma = int(bdf)
        f0, s0, n0 = (np.asarray(a, np.float64)[live] for a in fibers)
        xyz_c = xyz[live]
        conn_c = cidx[conn[keep]]
        mat_c = material[keep]
        self.regions = []
        self.M = None
        self.K = None
        for r, reg in enumerate(regions):
            el = np.nonzero(mat_c == r)[0]
            if not reg.conductive or el.size == 0:
                continue
            s = reg.sigma if reg.sigma is not None else sigma
            Dn = fem.nodal_diffusion(f0, s0, n0, *s, chi, cm)
            Mr, Kr = fem.assemble(xyz_c, conn_c[el], Dn)
            nodes = np.unique(conn_c[el])
            m = IonicModel(reg.model or model, reg.variant)
            m.p.update(reg.params)
            self.regions.append(dict(nodes=nodes, M=Mr[:, nodes].tocsr(), model=m))
            self.M = Mr if self.M is None else self.M + Mr
            self.K = Kr if self.K is None else self.K + Kr
        # the solver, stimuli and activation bookkeeping of one subdomain on
        # the conductive nodes; its ionic model supplies units and threshold
        base = Monodomain.__new__(Monodomain)
        base.xyz = xyz_c
        base.n = self.n
        # the field's units, threshold and initial potential: the simulation's
        # model (the first conducting subdomain's when that one runs it)
        first = self.regions[0]["model"]
        base.model = first if first.name == model else IonicModel(model, "")
        a0, b0 = base.model.mv_per_unit, MV_OFFSET[model]
        for reg in self.regions:
            mr = reg["model"]
            ar, br = mr.mv_per_unit, MV_OFFSET[mr.name]
            # u_i = (a0 u + b0 - br) / ar;  I in the field's units = (ar / a0) I_i
            reg["u_scale"], reg["u_shift"], reg["i_scale"] = a0 / ar, (b0 - br) / ar, ar / a0
        base.chi, base.cm, base.dt, base.sigma = chi, cm, self.dt, self.sigma
        base.M, base.K = self.M.tocsr(), self.K.tocsr()
        base.A = {s: (BDF_COEFFS[s][0] / self.dt) * base.M + base.K for s in range(1, self.sigma + 1)}
        if solver == "auto":
            solver = "dense" if self.n <= 2000 else ("splu" if self.n <= 60000 else "cg")
        base.solver, base.rtol, base.max_it, base.block = solver, rtol, max_it, 1
        base.ionic_scheme = ionic_scheme
        base._lu, base._prec, base.cg_iters = {}, {}, []
        scale = 1.0 / (chi * cm * base.model.mv_per_unit)
        base.stims = []
        for st in stimuli:
            prof = stimulus_profile(st.shape, st.center, st.size, xyz_c)
            base.stims.append((prof * st.amp * scale, st.t0, st.dur, st.period))
        self.base = base
        u0, _ = base.model.initial(self.n)
        self.set_state(u0, None)

    def set_state(self, u, w, u_prev=None, step_index=0):
        """u on the conductive nodes (compact numbering); w: one state array
        [n_vars, n] per compact node, copied to every subdomain the node
        belongs to that runs the simulation's model (None, and subdomains of
        another model: that model's initial state).  Earlier ionic states
        of the BDF ionic scheme start as copies."""
        for reg in self.regions:
            nodes = reg["nodes"]
            if w is None or reg["model"].name != self.base.model.name:
                _, w0 = reg["model"].initial(nodes.size)
            else:
                w0 = np.asarray(w, np.float64)[:, nodes]
            reg["w"] = np.array(w0, np.float64)
            reg["w_hist"] = [reg["w"]] + [reg["w"].copy() for _ in range(1, self.sigma)]
        b = self.base
        u = np.array(u, np.float64)
        prev = list(u_prev) if u_prev is not None else []
        b.hist = [u] + [np.array(prev[k - 1], np.float64) if k - 1 < len(prev) else u.copy()
                        for k in range(1, self.sigma)]
        b.step_index = int(step_index)
        b.smax = np.full(self.n, -np.inf)
        b.at = np.full(self.n, np.nan)
        b.tcross = np.full(self.n, np.nan)

    def step(self):
        b = self.base
        n = b.step_index
        s = min(self.sigma, n + 1)
        alpha, cb, ce = BDF_COEFFS[s]
        u_bdf = sum(c * h for c, h in zip(cb, b.hist))
        u_ext = sum(c * h for c, h in zip(ce, b.hist))
        t_new = (n + 1) * self.dt
        load = np.zeros(self.n)
        for reg in self.regions:
            nodes = reg["nodes"]
            m = reg["model"]
            ui = reg["u_scale"] * u_ext[nodes] + reg["u_shift"]
            if self.ionic_scheme == "bdf":
                reg["w"] = m.step_bdf(ui, reg["w_hist"][:s], cb, ce, self.dt, alpha)
                reg["w_hist"] = [reg["w"]] + reg["w_hist"][:-1]
            else:
                reg["w"] = m.step(ui, reg["w"], self.dt)
            load += reg["M"] @ (reg["i_scale"] * m.iion(ui, reg["w"]))
        rhs = b.M @ (u_bdf / self.dt + b.applied(t_new)) - load
        u_new = b.solve(s, rhs, u_ext)
        slope = (u_new - b.hist[0]) / self.dt
        upd = slope > b.smax
        b.smax = np.where(upd, slope, b.smax)
        b.at = np.where(upd, t_new, b.at)
        cross = np.isnan(b.tcross) & (u_new > b.model.threshold)
        b.tcross = np.where(cross, t_new, b.tcross)
        b.hist = [u_new] + b.hist[:-1]
        b.step_index = n + 1
        return u_new

    def run(self, n_steps):
        for _ in range(n_steps):
            self.step()
        return self.base.u

    def _full(self, v):
        out = np.full(self.n_full, np.nan)
        out[self.live] = v
        return out

    @property
    def u(self):
        """Potential in model units on all nodes (NaN where removed)."""
        return self._full(self.base.u)

    def potential_mv(self):
        return self._full(self.base.potential_mv())

    def activation_times(self):
        return self._full(self.base.activation_times())

    def state(self, region):
        """(nodes in full numbering, state [n_vars, nodes]) of one conductive
        subdomain (index among the conductive ones)."""
        reg = self.regions[region]
        return self.live[reg["nodes"]], reg["w"]


def from_spec(spec, material, regions, solver="auto", rtol=1e-13, ionic_scheme="rl"):
    """Multi-subdomain oracle for a workloads.SimSpec and element labels."""
    p = spec.phys
    return MultiRegion(spec.mesh.xyz, spec.mesh.conn, material, regions, spec.fibers,
                       (p.sigma_l, p.sigma_t, p.sigma_n), p.chi, p.cm, spec.model, spec.stimuli,
                       spec.dt, spec.bdf, solver, rtol, ionic_scheme=ionic_scheme)
