"""GPU: the paper's semi-implicit BDF ionic integrator (EP_IONIC_BDF) against
the oracle's, FP64 (single step at rtol 1e-13: 1e-10 relative; trajectories
at rtol 1e-12: 1e-8 relative and activation times to the step); mixed
precision against FP64 at RMS 1e-3 mV and 0.1 ms; in a pool next to
Rush-Larsen instances, each result bitwise the same as alone.
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


def _slab(model, variant="", bdf=2, h=0.25, dims=(5.0, 3.0, 2.0), n_steps=1):
    mesh = W.slab_q1(*dims, h)
    st = [W.corner_cube_stimulus(dims=dims)]
    return W.SimSpec(mesh, W.random_fibers(mesh.n_nodes, 3), W.Physics(), model, variant, st, 0.05, bdf,
                     n_steps, 1e-10, "t")


@pytest.mark.parametrize("model,variant,bdf", [("ap", "", 2), ("bo", "epi", 3), ("ttp06", "endo", 2),
                                               ("ttp06", "epi", 3)])
def test_bdf_scheme_single_step(model, variant, bdf):
    ep = _ep()
    spec = _slab(model, variant, bdf)
    u, w = W.random_state(model, spec.mesh.n_nodes, seed=51)
    rng = np.random.default_rng(52)
    scale = 1.0 if model == "ttp06" else 0.01
    u_prev = np.stack([u + scale * rng.normal(size=u.size) for _ in range(bdf - 1)])
    sim = ep.Simulation.from_spec(spec, rtol=1e-13, ionic_scheme="bdf")
    o = OM.from_spec(spec, solver="cg", rtol=1e-13, ionic_scheme="bdf")
    sim.set_state(u, w, u_prev, 6)
    o.set_state(u, w, list(u_prev), 6)
    o.step()
    sim.step(1)
    ug, wg, _ = sim.get_state()
    sim.close()
    assert _rel(ug, o.u) < 1e-10, _rel(ug, o.u)
    for v in range(w.shape[0]):
        err = np.max(np.abs(wg[v] - o.w[v])) / max(np.max(np.abs(o.w[v])), 1e-30)
        assert err < 1e-11, (v, err)


@pytest.mark.parametrize("model,variant,bdf,steps", [("ap", "", 2, 300), ("ttp06", "endo", 2, 300),
                                                     ("bo", "epi", 3, 300)])
def test_bdf_scheme_trajectory(model, variant, bdf, steps):
    ep = _ep()
    spec = _slab(model, variant, bdf, h=0.5, dims=(10.0, 4.0, 2.0))
    # rtol 1e-12: at 1e-10 the BO/BDF3 front amplifies the solver tolerance to
    # ~2e-8 over 300 steps (the oracle solves exactly)
    sim = ep.Simulation.from_spec(spec, ionic_scheme="bdf", rtol=1e-12)
    o = OM.from_spec(spec, ionic_scheme="bdf")
    for chunk in range(3):
        o.run(steps // 3)
        sim.step(steps // 3)
        err = _rel(sim.get_potential(), o.potential_mv())
        assert err < 1e-8, (chunk, err)
    at_o, at_g = o.activation_times(), sim.get_activation_times()
    ok = ~np.isnan(at_o)
    assert ok.sum() > 50 and np.array_equal(ok, ~np.isnan(at_g))
    assert np.max(np.abs(at_o[ok] - at_g[ok])) <= spec.dt + 1e-9
    sim.close()


def test_bdf_scheme_mixed_precision_accuracy():
    ep = _ep()
    spec = _slab("ttp06", "endo", 2, h=0.5, dims=(20.0, 7.0, 3.0))
    ref = ep.Simulation.from_spec(spec, ionic_scheme="bdf")
    mix = ep.Simulation.from_spec(spec, precision=ep.EP_MIXED, ionic_scheme="bdf")
    ref.step(600)
    mix.step(600)
    du = mix.get_potential() - ref.get_potential()
    rms = float(np.sqrt(np.mean(du * du)))
    a, b = mix.get_activation_times(), ref.get_activation_times()
    ok = ~np.isnan(b)
    assert ok.sum() > 100 and np.array_equal(ok, ~np.isnan(a))
    assert rms <= 1e-3, rms
    assert np.max(np.abs(a[ok] - b[ok])) <= 0.1
    ref.close()
    mix.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_bdf_and_rush_larsen_instances_share_a_pool(prec):
    ep = _ep()
    specs = [(_slab("ttp06", "endo", 2), "bdf"), (_slab("ttp06", "endo", 2), "rl"), (_slab("bo", "epi", 3), "bdf")]
    steps = 60
    alone = []
    for sp, sch in specs:
        s = ep.Simulation.from_spec(sp, precision=prec, ionic_scheme=sch)
        s.step(steps)
        alone.append(s.get_state()[:2])
        s.close()
    pool = ep.Pool(8 << 30, 4, prec)
    sims = []
    for sp, sch in specs:
        s = ep.Simulation.from_spec(sp, precision=prec, ionic_scheme=sch, finalize=False)
        slot = pool.admit(s, steps)
        assert slot is not None
        sims.append((slot, s))
    pool.step(steps)
    for (slot, s), (u0, w0) in zip(sims, alone):
        u, w, _ = s.get_state()
        assert np.array_equal(u, u0) and np.array_equal(w, w0), slot
        pool.release(slot)
        s.close()
    pool.close()
