"""BDF/IMEX monodomain time stepping with ionic current interpolation (FP64).

Test infrastructure.  Follows the paper's numerical discretization (Section
"Cardiac electrophysiology: numerical discretization"), step by step:

  1. BDF order sigma_n = min(sigma, n+1) (start-up with lower orders); the
     standard BDF coefficients alpha, u_BDF and the explicit extrapolation
     u_EXT of the same order (the paper cites but does not print them).
  2. Ionic step at every node with u* = u_EXT (eq. of the time-discrete ionic
     model): Rush-Larsen gates and explicit other variables, or the paper's
     semi-implicit BDF of the potential's order (ionic_scheme="bdf"; the
     ionic state then keeps sigma levels of history), see ionic.py.
  3. Ionic current interpolation: I_ion is evaluated at the nodes at
     (u_EXT, w_{n+1}) and the load vector is M I_ion (the ICI sum over
     subdomains, one subdomain here).  The applied current is treated the
     same way: M I_app with nodal I_app at t_{n+1}.
  4. Linear system (eq. of the algebraic linear system) with the BDF history
     term read as (1/dt) M u_BDF (the printed u_EXT there contradicts the
     time-discrete monodomain equation; identical for BDF1):
        (alpha/dt M + K) u_{n+1} = M (u_BDF/dt + I_app - I_ion).
  5. Activation time: the time at which du/dt (forward difference) is
     largest at a node (Section "Slab benchmark"); first strict maximum;
     reported only where u exceeded the model's activation threshold.

Solvers: dense LU for tiny meshes, sparse LU (factorized once per BDF order)
for small ones, textbook Jacobi-preconditioned CG for large ones.

Pins: cosine eigenmode decay (BDF1, BDF2 and BDF3 closed forms), charge
conservation, uniform-state reduction to the 0D ionic ODE, dense-solve
agreement, bistable-front speed, activation-time self-convergence; the
applied current's profiles (lattice counts, the Gaussian load against its
integral to the trapezoid rule's leading error term) and pulse windows.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem
from .ionic import IonicModel

# (alpha, coefficients of u_BDF over [u_n, u_{n-1}, ...], of u_EXT)
BDF_COEFFS = {
    1: (1.0, [1.0], [1.0]),
    2: (1.5, [2.0, -0.5], [2.0, -1.0]),
    3: (11.0 / 6.0, [3.0, -1.5, 1.0 / 3.0], [3.0, -3.0, 1.0]),
}

CUBE, SPHERE, GAUSS = 0, 1, 2


def stimulus_profile(shape, center, size, xyz):
    """Spatial factor of one impulse at the nodes.

    CUBE: 1 inside the closed cube of edge `size` (inclusive at nodes),
    SPHERE: 1 inside the closed ball of radius `size`,
    GAUSS: exp(-|x - c|^2 / (2 size^2)), untruncated.
    """
    d = np.asarray(xyz, np.float64) - np.asarray(center, np.float64)[None, :]
    if shape == CUBE:
        return (np.max(np.abs(d), axis=1) <= 0.5 * size + 1e-9).astype(np.float64)
    if shape == SPHERE:
        return (np.sqrt(np.sum(d * d, axis=1)) <= size + 1e-9).astype(np.float64)
    if shape == GAUSS:
        return np.exp(-np.sum(d * d, axis=1) / (2.0 * size * size))
    raise ValueError(shape)


def stimulus_active(t, t0, dur, period, dt):
    """True when t lies in (t0 + k period, t0 + k period + dur] for some k >= 0."""
    eps = 1e-6 * dt
    s = t - t0
    if s <= eps:
        return False
    if period > 0:
        s = s - period * np.floor((s - eps) / period)
    return eps < s <= dur + eps


class Monodomain:
    """One monodomain simulation on one subdomain."""

    def __init__(self, xyz, conn, fibers, sigma, chi, cm, model, variant="", stimuli=(),
                 dt=0.05, bdf=1, solver="auto", rtol=1e-13, max_it=5000, block=1, ionic_scheme="rl"):
        self.xyz = np.asarray(xyz, np.float64)
        self.n = self.xyz.shape[0]
        self.model = IonicModel(model, variant)
        self.chi, self.cm = chi, cm
        self.dt = float(dt)
        self.sigma = int(bdf)
        Dn = fem.nodal_diffusion(*fibers, *sigma, chi, cm)
        self.M, self.K = fem.assemble(self.xyz, conn, Dn)
        self.A = {}
        for s in range(1, self.sigma + 1):
            self.A[s] = (BDF_COEFFS[s][0] / self.dt) * self.M + self.K
        if solver == "auto":
            solver = "dense" if self.n <= 2000 else ("splu" if self.n <= 60000 else "cg")
        self.solver = solver
        self.rtol = rtol
        self.max_it = max_it
        self.block = int(block)
        if ionic_scheme not in ("rl", "bdf"):
            raise ValueError(ionic_scheme)
        self.ionic_scheme = ionic_scheme
        self._lu = {}
        self._prec = {}
        self.cg_iters = []
        # stimuli: (profile in model units per unit amplitude, t0, dur, period, amp)
        scale = 1.0 / (chi * cm * self.model.mv_per_unit)
        self.stims = []
        for st in stimuli:
            prof = stimulus_profile(st.shape, st.center, st.size, self.xyz)
            self.stims.append((prof * st.amp * scale, st.t0, st.dur, st.period))
        u0, w0 = self.model.initial(self.n)
        self.set_state(u0, w0)

    # -- state ------------------------------------------------------------
    def set_state(self, u, w, u_prev=None, step_index=0, w_prev=None):
        """u_n, ionic state and optional earlier potentials [u_{n-1}, ...]
        (and, for the BDF ionic scheme, earlier states [w_{n-1}, ...];
        copies of w when absent)."""
        u = np.array(u, np.float64)
        self.w = np.array(w, np.float64).reshape(self.model.n_vars, self.n)
        wp = list(w_prev) if w_prev is not None else []
        self.w_hist = [self.w] + [np.array(wp[k - 1], np.float64).reshape(self.model.n_vars, self.n)
                                  if k - 1 < len(wp) else self.w.copy() for k in range(1, self.sigma)]
        hist = [u]
        prev = list(u_prev) if u_prev is not None else []
        for k in range(1, self.sigma):
            hist.append(np.array(prev[k - 1], np.float64) if k - 1 < len(prev) else u.copy())
        self.hist = hist
        self.step_index = int(step_index)
        self.smax = np.full(self.n, -np.inf)
        self.at = np.full(self.n, np.nan)
        self.tcross = np.full(self.n, np.nan)

    @property
    def u(self):
        return self.hist[0]

    # -- pieces of one step --------------------------------------------------
    def applied(self, t):
        I = np.zeros(self.n)
        for prof, t0, dur, period in self.stims:
            if stimulus_active(t, t0, dur, period, self.dt):
                I += prof
        return I

    def solve(self, s, b, x0):
        A = self.A[s]
        if self.solver == "dense":
            return np.linalg.solve(A.toarray(), b)
        if self.solver == "splu":
            if s not in self._lu:
                self._lu[s] = spla.splu(A.tocsc())
            return self._lu[s].solve(b)
        return self.pcg(A, b, x0, s)

    def preconditioner(self, s):
        """Inverse of the preconditioner of A_s as a function r -> z.

        block == 1: Jacobi, z = r / diag(A).  block > 1: block Jacobi over
        consecutive runs of `block` rows (the last run may be shorter), each
        diagonal block of A inverted exactly.
        """
        if s in self._prec:
            return self._prec[s]
        A = self.A[s]
        b = self.block
        if b <= 1:
            dinv = 1.0 / A.diagonal()
            f = lambda r: dinv * r
        else:
            n = self.n
            nb = (n + b - 1) // b
            blocks = np.zeros((nb, b, b))
            idx = np.arange(nb * b)
            C = A.tocoo()
            same = (C.row // b) == (C.col // b)
            blocks[C.row[same] // b, C.row[same] % b, C.col[same] % b] = C.data[same]
            pad = idx[idx >= n]
            blocks[pad // b, pad % b, pad % b] = 1.0  # identity rows of the ragged last block
            inv = np.linalg.inv(blocks)

            def f(r):
                rp = np.zeros(nb * b)
                rp[:n] = r
                return np.einsum("kij,kj->ki", inv, rp.reshape(nb, b)).ravel()[:n]
        self._prec[s] = f
        return f

    def pcg(self, A, b, x0, s=None):
        """Preconditioned conjugate gradients (Hestenes-Stiefel form), Jacobi
        or block Jacobi; stops when ||b - A x||_2 <= rtol ||b||_2 for the
        recursively updated residual, confirmed by the true residual at exit
        (a solve whose true residual still misses the tolerance restarts
        from it, within the same iteration budget)."""
        if s is None:
            s = next(k for k, v in self.A.items() if v is A)
        P = self.preconditioner(s)
        x = x0.copy()
        bnorm = np.linalg.norm(b)
        it = 0
        while True:
            r = b - A @ x
            if np.linalg.norm(r) <= self.rtol * bnorm or it >= self.max_it:
                break
            z = P(r)
            p = z.copy()
            rz = r @ z
            while np.linalg.norm(r) > self.rtol * bnorm and it < self.max_it:
                q = A @ p
                alpha = rz / (p @ q)
                x += alpha * p
                r -= alpha * q
                z = P(r)
                rz_new = r @ z
                p = z + (rz_new / rz) * p
                rz = rz_new
                it += 1
        self.cg_iters.append(it)
        return x

    def step(self):
        n = self.step_index
        s = min(self.sigma, n + 1)
        alpha, cb, ce = BDF_COEFFS[s]
        u_bdf = sum(c * h for c, h in zip(cb, self.hist))
        u_ext = sum(c * h for c, h in zip(ce, self.hist))
        t_new = (n + 1) * self.dt
        if self.ionic_scheme == "bdf":
            self.w = self.model.step_bdf(u_ext, self.w_hist[:s], cb, ce, self.dt, alpha)
            self.w_hist = [self.w] + self.w_hist[:-1]
        else:
            self.w = self.model.step(u_ext, self.w, self.dt)
        i_ion = self.model.iion(u_ext, self.w)
        i_app = self.applied(t_new)
        g = u_bdf / self.dt + i_app - i_ion
        b = self.M @ g
        u_new = self.solve(s, b, u_ext)
        # activation
        slope = (u_new - self.hist[0]) / self.dt
        upd = slope > self.smax
        self.smax = np.where(upd, slope, self.smax)
        self.at = np.where(upd, t_new, self.at)
        cross = np.isnan(self.tcross) & (u_new > self.model.threshold)
        self.tcross = np.where(cross, t_new, self.tcross)
        self.hist = [u_new] + self.hist[:-1]
        self.step_index = n + 1
        return u_new

    def run(self, n_steps):
        for _ in range(n_steps):
            self.step()
        return self.u

    def activation_times(self):
        return np.where(np.isnan(self.tcross), np.nan, self.at)

    def potential_mv(self):
        return self.model.mv_per_unit * self.u + (
            -80.0 if self.model.name == "ap" else (-84.0 if self.model.name == "bo" else 0.0))


def from_spec(spec, solver="auto", rtol=1e-13, block=1, ionic_scheme="rl"):
    """Build an oracle simulation from a workloads.SimSpec."""
    p = spec.phys
    return Monodomain(spec.mesh.xyz, spec.mesh.conn, spec.fibers,
                      (p.sigma_l, p.sigma_t, p.sigma_n), p.chi, p.cm, spec.model,
                      spec.variant, spec.stimuli, spec.dt, spec.bdf, solver, rtol, block=block,
                      ionic_scheme=ionic_scheme)
