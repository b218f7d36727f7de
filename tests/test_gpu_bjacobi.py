"""GPU: block-Jacobi preconditioned CG (EP_BJACOBI) against the oracle.

The preconditioner does not change the solution a converged CG returns, so
single steps at rtol 1e-13 must agree with the oracle to 1e-10 relative (as
for Jacobi).  It does change the iteration count: the HIP path
(Chronopoulos-Gear) and the oracle (Hestenes-Stiefel, the same block
inverses) produce the same iterates in exact arithmetic, so their counts for
one step agree to within one iteration; a wrong block inverse would still
converge, but in a different number of iterations.
"""
import numpy as np
import pytest

import workloads as W
from oracle import monodomain as OM

pytestmark = pytest.mark.gpu


def _ep():
    import paper_2308_01651_amd as ep
    return ep


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _lv_spec(model="bo", variant="epi", n_t=8, n_phi=40, n_theta=18, n_steps=1):
    mesh, fib, endo = W.lv_shell(n_t, n_phi, n_theta)
    # a wide Gaussian: this coarse shell needs it for the front to start
    st = [W.Stimulus(W.GAUSS, tuple(mesh.xyz[endo[5]]), 4.0, 100.0, 0.0, 2.0, 0.0)]
    return W.SimSpec(mesh, fib, W.Physics(0.17, 0.0425, 0.0425), model, variant, st, 0.05, 2, n_steps, 1e-10)


def _slab_spec(model="ttp06", variant="endo"):
    mesh = W.slab_q1(5.0, 3.0, 2.0, 0.25)  # 2457 nodes: ragged last block for every block size > 1
    st = [W.corner_cube_stimulus(dims=(5.0, 3.0, 2.0))]
    return W.SimSpec(mesh, W.random_fibers(mesh.n_nodes, 3), W.Physics(), model, variant, st, 0.05, 2, 1, 1e-10)


def _one_step(spec, block, rtol, precision=None, fmt=None):
    ep = _ep()
    kw = {}
    if fmt is not None:
        kw["matrix_format"] = fmt
    sim = ep.Simulation.from_spec(spec, rtol=rtol, block=block,
                                  precision=ep.EP_FP64 if precision is None else precision, **kw)
    o = OM.from_spec(spec, solver="cg", rtol=rtol, block=block)
    u, w = W.random_state(spec.model, spec.mesh.n_nodes, seed=31)
    rng = np.random.default_rng(32)
    scale = 1.0 if spec.model == "ttp06" else 0.01
    u_prev = u + scale * rng.normal(size=u.size)
    o.set_state(u, w, [u_prev], 5)
    sim.set_state(u, w, u_prev[None, :], 5)
    o.step()
    sim.step(1)
    ug, wg, _ = sim.get_state()
    its = sim.get_stats()["cg_iters_last"]
    sim.close()
    return ug, o, its


@pytest.mark.parametrize("block", [2, 8, 32, 64])
def test_bjacobi_single_step_slab_dia(block):
    ep = _ep()
    spec = _slab_spec()
    ug, o, _ = _one_step(spec, block, 1e-13, fmt=ep.EP_FMT_DIA)
    assert _rel(ug, o.u) < 1e-10, _rel(ug, o.u)


@pytest.mark.parametrize("block", [4, 16])
def test_bjacobi_single_step_lv_sell(block):
    ep = _ep()
    spec = _lv_spec()
    ug, o, _ = _one_step(spec, block, 1e-13, fmt=ep.EP_FMT_SELL)
    assert _rel(ug, o.u) < 1e-10, _rel(ug, o.u)


@pytest.mark.parametrize("block", [1, 8, 16])
def test_bjacobi_iteration_count_matches_oracle(block):
    """Transmural lines of 8 nodes are contiguous rows: blocks of 8 and 16
    hold whole lines, and need fewer iterations than Jacobi."""
    spec = _lv_spec(n_t=8)
    ug, o, its = _one_step(spec, block, 1e-10)
    print(f"block {block}: HIP {its} its, oracle {o.cg_iters[-1]} its", flush=True)
    assert abs(its - o.cg_iters[-1]) <= 1, (its, o.cg_iters)
    assert _rel(ug, o.u) < 1e-8
    if block > 1:
        _, oj, its_j = _one_step(spec, 1, 1e-10)
        assert its < its_j, (its, its_j)


@pytest.mark.parametrize("model,variant", [("ttp06", "endo"), ("bo", "epi")])
def test_bjacobi_mixed_precision_trajectory(model, variant):
    """Mixed precision with FP32 block inverses against the FP64 Jacobi run,
    on a slab resolved well enough (h = 0.2 mm) for a robust front: on an
    under-resolved mesh where the front barely propagates, even the FP64
    runs with two preconditioners drift apart by 1e-2 mV at rtol 1e-10."""
    ep = _ep()
    mesh = W.slab_q1(10.0, 3.0, 2.0, 0.2)
    st = [W.corner_cube_stimulus(dims=(10.0, 3.0, 2.0))]
    spec = W.SimSpec(mesh, W.uniform_fibers(mesh.n_nodes), W.Physics(), model, variant, st, 0.05, 2, 600, 1e-10)
    ref = ep.Simulation.from_spec(spec)
    mix = ep.Simulation.from_spec(spec, precision=ep.EP_MIXED, block=16)
    ref.step(600)
    mix.step(600)
    du = mix.get_potential() - ref.get_potential()
    rms = float(np.sqrt(np.mean(du * du)))
    a, b = mix.get_activation_times(), ref.get_activation_times()
    print(f"{model}: rms {rms:.2e} mV, activated {np.sum(~np.isnan(b))}", flush=True)
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(b)
    assert ok.sum() > 1000
    assert rms <= 1e-3, rms
    assert np.max(np.abs(a[ok] - b[ok])) <= 0.1
    ref.close()
    mix.close()


@pytest.mark.parametrize("precond,block", [(0, 2), (1, 3), (1, 128), (1, 0), (7, 1)])
def test_bjacobi_rejects_bad_settings(precond, block):
    ep = _ep()
    sim = ep.Simulation(0)
    with pytest.raises(ep.EpError):
        sim.set_solver(0.05, 2, ep.EP_FP64, precond, block, 1e-10, 100)
    sim.close()
