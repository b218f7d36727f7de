"""Pins of the oracle's time stepping against closed forms and invariants.

- cosine eigenmode of the slab with I_ion = 0 decays by the BDF1 / BDF2 / BDF3
  recurrences (fixes M, K, the RHS and the BDF coefficients; with the
  printed u_EXT history term BDF2 would follow another recurrence);
- charge conservation 1^T M u with I_ion = 0 (fixes the applied-current load);
- a spatially uniform state reproduces the single-cell (0D) update (fixes the
  ionic-current interpolation coupling, since K 1 = 0);
- CG agrees with a dense solve on tiny meshes, with Jacobi and with block
  Jacobi; block Jacobi is exact (one iteration) when its blocks hold the
  whole operator, including a ragged last block;
- Aliev-Panfilov plane front speed approaches the bistable-front closed form;
- activation times converge under mesh refinement.
"""
import numpy as np
import pytest

import workloads as W
from oracle import monodomain as OM


def _passive(mesh, D=(0.12, 0.013, 0.009), bdf=1, dt=0.05, stimuli=(), solver="splu"):
    f, s, n = W.uniform_fibers(mesh.n_nodes)
    return OM.Monodomain(mesh.xyz, mesh.conn, (f, s, n), D, 1.0, 1.0, "passive", "",
                         stimuli, dt, bdf, solver)


@pytest.mark.parametrize("k", [1, 4])
def test_cosine_mode_bdf1(k):
    D = (0.12, 0.013, 0.009)
    m = W.slab_q1(20.0, 7.0, 3.0, 0.5)
    o = _passive(m, D, 1)
    v = np.cos(k * np.pi * m.xyz[:, 0] / 20.0)
    o.set_state(v, np.zeros((0, m.n_nodes)))
    h = 0.5
    th = k * np.pi / (m.dims[0] - 1)
    lam = 6 / h ** 2 * (1 - np.cos(th)) / (2 + np.cos(th))
    a = 1.0
    for _ in range(20):
        o.step()
        a = a / (1 + 0.05 * D[0] * lam)
        assert np.max(np.abs(o.u - a * v)) < 1e-12


def test_cosine_mode_bdf2_recurrence():
    D = (0.12, 0.013, 0.009)
    m = W.slab_q1(20.0, 7.0, 3.0, 0.5)
    o = _passive(m, D, 2)
    # mode cos(2 pi x / Lx) * cos(pi y / Ly): eigenvalue D_l lam_x + D_t lam_y
    v = np.cos(2 * np.pi * m.xyz[:, 0] / 20.0) * np.cos(np.pi * m.xyz[:, 1] / 7.0)
    o.set_state(v, np.zeros((0, m.n_nodes)))
    h = 0.5

    def lam(kk, N):
        th = kk * np.pi / N
        return 6 / h ** 2 * (1 - np.cos(th)) / (2 + np.cos(th))

    mu = D[0] * lam(2, m.dims[0] - 1) + D[1] * lam(1, m.dims[1] - 1)
    dt = 0.05
    a_prev, a = 1.0, 1.0
    # first step: BDF1 start-up
    o.step()
    a_prev, a = a, a / (1 + dt * mu)
    assert np.max(np.abs(o.u - a * v)) < 1e-12
    for _ in range(30):
        o.step()
        a_prev, a = a, (2 * a - 0.5 * a_prev) / (1.5 + dt * mu)
        assert np.max(np.abs(o.u - a * v)) < 1e-12


def test_charge_conservation_bdf1():
    m = W.slab_q1(6.0, 3.0, 2.0, 0.5)
    st = W.Stimulus(W.GAUSS, (1.0, 1.2, 0.3), 0.8, 3.0, 0.0, 1.0, 0.0)
    o = _passive(m, stimuli=[st], solver="dense")
    one = np.ones(m.n_nodes)
    q = one @ (o.M @ o.u)
    for n in range(30):
        t = (n + 1) * o.dt
        iapp = o.applied(t)
        o.step()
        q_new = one @ (o.M @ o.u)
        assert abs(q_new - (q + o.dt * one @ (o.M @ iapp))) < 1e-12 * max(1.0, abs(q))
        q = q_new
    assert q > 0.5   # the pulse did inject charge


@pytest.mark.parametrize("model,variant,bdf", [("ap", "", 1), ("bo", "epi", 2), ("ttp06", "endo", 2)])
def test_uniform_state_reduces_to_single_cell(model, variant, bdf):
    m = W.slab_q1(3.0, 2.0, 1.0, 0.5)
    big = W.Stimulus(W.CUBE, (1.5, 1.0, 0.5), 10.0, 50.0, 0.0, 1.0, 0.0)
    f, s, n = W.uniform_fibers(m.n_nodes)
    o = OM.Monodomain(m.xyz, m.conn, (f, s, n), (0.17, 0.019, 0.019), 140.0, 0.01, model, variant,
                      [big], 0.05, bdf, "dense")
    # 0D reference: the same update with no diffusion, one cell
    u1, w1 = o.model.initial(1)
    hist = [u1.copy(), u1.copy()]
    scale = 50.0 / (140.0 * 0.01 * o.model.mv_per_unit)
    for step in range(60):
        s_n = min(bdf, step + 1)
        alpha, cb, ce = OM.BDF_COEFFS[s_n]
        ub = sum(c * h for c, h in zip(cb, hist))
        ue = sum(c * h for c, h in zip(ce, hist))
        w1 = o.model.step(ue, w1, 0.05)
        iapp = scale if (step + 1) * 0.05 <= 1.0 + 1e-9 else 0.0
        unew = (ub + 0.05 * (iapp - o.model.iion(ue, w1))) / alpha
        hist = [unew, hist[0]]
        o.step()
        tol = 1e-10 * max(1.0, abs(unew[0]))
        assert np.max(np.abs(o.u - unew[0])) < tol, (step, o.u[:3], unew)
        assert np.max(np.abs(o.w - w1)) < 1e-10 * max(1.0, np.max(np.abs(w1)))


def test_cg_matches_dense_solve():
    m = W.slab_q1(2.0, 2.0, 2.0, 0.5)
    st = W.corner_cube_stimulus(dims=(2.0, 2.0, 2.0))
    f, s, n = W.random_fibers(m.n_nodes, 7)
    args = (m.xyz, m.conn, (f, s, n), (0.17, 0.019, 0.019), 140.0, 0.01, "ap", "", [st], 0.05, 2)
    a = OM.Monodomain(*args, solver="dense")
    b = OM.Monodomain(*args, solver="cg", rtol=1e-14)
    for _ in range(40):
        a.step()
        b.step()
    assert np.max(np.abs(a.u - b.u)) < 1e-12


@pytest.mark.parametrize("block", [2, 8, 64])
def test_block_jacobi_cg_matches_dense_solve(block):
    m = W.slab_q1(2.0, 2.0, 2.0, 0.5)
    st = W.corner_cube_stimulus(dims=(2.0, 2.0, 2.0))
    f, s, n = W.random_fibers(m.n_nodes, 7)
    args = (m.xyz, m.conn, (f, s, n), (0.17, 0.019, 0.019), 140.0, 0.01, "ap", "", [st], 0.05, 2)
    a = OM.Monodomain(*args, solver="dense")
    b = OM.Monodomain(*args, solver="cg", rtol=1e-14, block=block)
    for _ in range(20):
        a.step()
        b.step()
    assert np.max(np.abs(a.u - b.u)) < 1e-12


def _block_diagonal_case(n, bs, seed):
    """SPD matrix whose couplings stay inside consecutive runs of bs rows."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    for lo in range(0, n, bs):
        hi = min(n, lo + bs)
        B = rng.standard_normal((hi - lo, hi - lo))
        A[lo:hi, lo:hi] = B @ B.T + (hi - lo) * np.eye(hi - lo)
    return sp.csr_matrix(A), rng.standard_normal(n)


@pytest.mark.parametrize("n,bs", [(64, 8), (61, 8), (50, 16), (7, 4)])
def test_block_jacobi_is_exact_on_block_diagonal_operator(n, bs):
    m = W.slab_q1(1.0, 1.0, 1.0, 0.5)  # any small instance; its operator is replaced
    o = OM.Monodomain(m.xyz, m.conn, W.uniform_fibers(m.n_nodes), (0.1, 0.1, 0.1), 1.0, 1.0,
                      "passive", "", (), 0.05, 1, "cg", 1e-12, block=bs)
    A, rhs = _block_diagonal_case(n, bs, seed=n)
    o.A = {1: A}
    o.n = n
    o._prec = {}
    o.cg_iters = []
    x = o.pcg(A, rhs, np.zeros(n), s=1)
    assert o.cg_iters == [1]
    assert np.allclose(A @ x, rhs, rtol=0, atol=1e-10 * np.linalg.norm(rhs))
    # half-size blocks miss couplings: more than one iteration
    o.block = max(1, bs // 2)
    o._prec = {}
    o.cg_iters = []
    o.pcg(A, rhs, np.zeros(n), s=1)
    assert o.cg_iters[0] > 1


def test_block_jacobi_single_block_is_exact():
    m = W.slab_q1(1.5, 1.0, 1.0, 0.5)
    o = OM.Monodomain(m.xyz, m.conn, W.random_fibers(m.n_nodes, 3), (0.17, 0.02, 0.02), 1.0, 1.0,
                      "passive", "", (), 0.05, 1, "cg", 1e-12, block=m.n_nodes + 5)
    rhs = np.random.default_rng(1).standard_normal(m.n_nodes)
    x = o.pcg(o.A[1], rhs, np.zeros(m.n_nodes), s=1)
    assert o.cg_iters == [1]
    assert np.allclose(o.A[1] @ x, rhs, rtol=0, atol=1e-10 * np.linalg.norm(rhs))


def test_aliev_panfilov_front_speed():
    """Thin cable, full-section stimulus.  With the recovery variable frozen
    ahead of the front, AP reduces to the bistable equation whose front speed
    is sqrt(D k / (2 T)) (1 - 2a)."""
    h = 0.1
    m = W.lattice_q1(121, 2, 2, h, h, h)
    f, s, n = W.uniform_fibers(m.n_nodes)
    stim = W.Stimulus(W.CUBE, (0.0, 0.05, 0.05), 2.0, 50.0, 0.0, 2.0, 0.0)
    o = OM.Monodomain(m.xyz, m.conn, (f, s, n), (0.17, 0.019, 0.019), 140.0, 0.01, "ap", "",
                      [stim], 0.01, 1, "splu")
    o.run(7000)
    tc = o.tcross
    x = m.xyz[:, 0]
    t4 = np.mean(tc[np.abs(x - 3.0) < 1e-9])
    t9 = np.mean(tc[np.abs(x - 9.0) < 1e-9])
    c = 6.0 / (t9 - t4)
    D = 0.17 / (140 * 0.01)
    c_ref = np.sqrt(D * 8.0 / (2 * 12.9)) * (1 - 2 * 0.15)
    assert abs(c - c_ref) / c_ref < 0.02, (c, c_ref)


def test_activation_time_converges_under_refinement():
    ats = []
    for h in (0.5, 0.25, 0.125):
        m = W.slab_q1(8.0, 1.0, 0.5, h)
        f, s, n = W.uniform_fibers(m.n_nodes)
        st = W.Stimulus(W.CUBE, (0.0, 0.0, 0.0), 2.0, 50.0, 0.0, 2.0, 0.0)
        o = OM.Monodomain(m.xyz, m.conn, (f, s, n), (0.17, 0.019, 0.019), 140.0, 0.01, "ap", "",
                          [st], 0.05, 2, "splu")
        o.run(1200)
        at = o.activation_times()
        far = np.argmin(np.sum((m.xyz - np.array([8.0, 1.0, 0.5])) ** 2, axis=1))
        assert np.isfinite(at[far])
        ats.append(at[far])
    d1 = abs(ats[0] - ats[1])
    d2 = abs(ats[1] - ats[2])
    assert d2 < 0.7 * d1, ats


def test_cosine_mode_bdf3_recurrence():
    """BDF3 (the paper's BDF of order up to 3): after the BDF1 and BDF2
    start-up steps the mode amplitude follows
    (11/6 a_{n+1} - 3 a_n + 3/2 a_{n-1} - 1/3 a_{n-2}) / dt = -mu a_{n+1}."""
    D = (0.12, 0.013, 0.009)
    m = W.slab_q1(20.0, 7.0, 3.0, 0.5)
    o = _passive(m, D, 3)
    v = np.cos(3 * np.pi * m.xyz[:, 0] / 20.0) * np.cos(2 * np.pi * m.xyz[:, 2] / 3.0)
    o.set_state(v, np.zeros((0, m.n_nodes)))
    h = 0.5

    def lam(kk, N):
        th = kk * np.pi / N
        return 6 / h ** 2 * (1 - np.cos(th)) / (2 + np.cos(th))

    mu = D[0] * lam(3, m.dims[0] - 1) + D[2] * lam(2, m.dims[2] - 1)
    dt = 0.05
    a = [1.0]
    o.step()                                        # BDF1
    a.append(a[-1] / (1 + dt * mu))
    assert np.max(np.abs(o.u - a[-1] * v)) < 1e-12
    o.step()                                        # BDF2
    a.append((2 * a[-1] - 0.5 * a[-2]) / (1.5 + dt * mu))
    assert np.max(np.abs(o.u - a[-1] * v)) < 1e-12
    for _ in range(30):
        o.step()
        a.append((3 * a[-1] - 1.5 * a[-2] + a[-3] / 3) / (11 / 6 + dt * mu))
        assert np.max(np.abs(o.u - a[-1] * v)) < 1e-12


@pytest.mark.parametrize("model,variant,bdf", [("ap", "", 1), ("bo", "epi", 2)])
def test_activation_time_is_the_steepest_step_of_the_trajectory(model, variant, bdf):
    """With the whole domain stimulated every node follows the single-cell
    trajectory u_0, u_1, ...; its activation time is then t_{k+1} for the
    first k maximizing (u_{k+1} - u_k) / dt (found here by argmax over the
    recorded trajectory), reported because u crossed the threshold."""
    m = W.slab_q1(3.0, 2.0, 1.0, 0.5)
    big = W.Stimulus(W.CUBE, (1.5, 1.0, 0.5), 10.0, 50.0, 0.0, 1.0, 0.0)
    f, s, n = W.uniform_fibers(m.n_nodes)
    o = OM.Monodomain(m.xyz, m.conn, (f, s, n), (0.17, 0.019, 0.019), 140.0, 0.01, model, variant,
                      [big], 0.05, bdf, "dense")
    traj = [o.u[0]]
    for _ in range(160):
        o.step()
        traj.append(o.u[0])
    traj = np.array(traj)
    assert np.max(traj) > o.model.threshold
    k = int(np.argmax(np.diff(traj)))
    at = o.activation_times()
    assert np.all(np.abs(at - (k + 1) * 0.05) < 1e-12), (at[:3], (k + 1) * 0.05)
