"""GPU: the batched and served forms against the FP64 oracle.

Uneven instances (Aliev-Panfilov slab, TTP06 slab, Bueno-Orovio ventricle
shell, and a block-Jacobi instance) run together in one pool, in FP64 and in
mixed precision; every pooled instance is compared with the oracle run of
its own specification at the single-simulation tolerances (FP64 trajectory:
relative L2 <= 1e-8, activation times to the time step; mixed precision:
RMS <= 1e-3 mV, activation times to 0.1 ms).  A short seeded request trace
goes through the continuous-batching loop and each finished request is
checked against the oracle the same way.  A sim destroyed while pooled
leaves its pool, whose other slots keep stepping.
"""
import numpy as np
import pytest

import workloads as W
from oracle import monodomain as OM

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _specs():
    a = W.SimSpec(W.slab_q1(6.0, 3.0, 2.0, 0.25), None, W.Physics(), "ap", "",
                  [W.corner_cube_stimulus(dims=(6.0, 3.0, 2.0))], 0.05, 2, 1, 1e-10, "ap-slab")
    b = W.SimSpec(W.slab_q1(8.0, 2.0, 1.5, 0.25), None, W.Physics(0.2, 0.02, 0.02), "ttp06", "endo",
                  [W.corner_cube_stimulus(dims=(8.0, 2.0, 1.5))], 0.05, 2, 1, 1e-10, "ttp-slab")
    m, fib, endo = W.lv_shell(4, 40, 16)
    c = W.SimSpec(m, fib, W.Physics(0.17, 0.0425, 0.0425), "bo", "epi",
                  [W.Stimulus(W.GAUSS, tuple(m.xyz[endo[5]]), 2.5, 36.0, 0.0, 2.0, 0.0)], 0.05, 2, 1, 1e-10, "bo-lv")
    d = W.SimSpec(W.slab_q1(5.0, 2.5, 1.5, 0.25), None, W.Physics(), "ttp06", "epi",
                  [W.corner_cube_stimulus(dims=(5.0, 2.5, 1.5))], 0.05, 1, 1, 1e-10, "ttp-slab-bj")
    for sp in (a, b, d):
        sp.fibers = W.uniform_fibers(sp.mesh.n_nodes)
    return [(a, 1), (b, 1), (c, 1), (d, 8)]


def _check(sim, spec, o, mixed):
    u = sim.get_potential()
    uo = o.potential_mv()
    at, ato = sim.get_activation_times(), o.activation_times()
    ok = ~np.isnan(ato)
    assert np.array_equal(ok, ~np.isnan(at)), spec.label
    if mixed:
        rms = np.sqrt(np.mean((u - uo) ** 2))
        assert rms <= 1e-3, (spec.label, rms)
        assert not ok.any() or np.max(np.abs(at[ok] - ato[ok])) <= 0.1, spec.label
    else:
        assert _rel(u, uo) < 1e-8, (spec.label, _rel(u, uo))
        assert not ok.any() or np.max(np.abs(at[ok] - ato[ok])) <= spec.dt + 1e-9, spec.label


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pooled_instances_match_the_oracle(precision):
    import paper_2308_01651_amd as ep
    mixed = precision == "mixed"
    prec = ep.EP_MIXED if mixed else ep.EP_FP64
    specs = _specs()
    steps = [120, 90, 100, 70]        # uneven lengths: slots finish at different steps
    pool = ep.Pool(8 << 30, 8, prec)
    sims = []
    for (sp, block), n in zip(specs, steps):
        s = ep.Simulation.from_spec(sp, precision=prec, finalize=False, block=block)
        slot = pool.admit(s, n)
        assert slot is not None
        sims.append((slot, s, sp, block, n))
    pool.step(max(steps))
    assert sorted(pool.poll()) == sorted(x[0] for x in sims)
    for slot, s, sp, block, n in sims:
        print(f"pool {precision}: {sp.label} ({sp.mesh.n_nodes} nodes, block {block}, {n} steps)", flush=True)
        assert s.get_stats()["steps"] == n
        o = OM.from_spec(sp, solver="splu", block=block)
        o.run(n)
        _check(s, sp, o, mixed)
        pool.release(slot)
        s.close()
    pool.close()


def test_served_requests_match_the_oracle():
    import paper_2308_01651_amd as ep
    from paper_2308_01651_amd import serve
    rng = np.random.default_rng(9)
    reqs = []
    t = 0.0
    for k, (sp, block) in enumerate(_specs()[:3] * 2):
        t += rng.exponential(0.05)
        sp = W.SimSpec(sp.mesh, sp.fibers, sp.phys, sp.model, sp.variant, sp.stimuli, sp.dt, sp.bdf,
                       int(rng.integers(40, 90)), sp.rtol, f"{sp.label}-{k}")
        reqs.append(W.Request(t, sp))
    got = {}

    def keep(rid, sim):
        got[rid] = (sim.get_potential(), sim.get_activation_times(), sim.get_stats()["steps"])

    out = serve.serve(reqs, 8 << 30, 3, ep.EP_FP64, steps_per_tick=10, on_done=keep)
    assert out["failed"] == 0 and len(got) == len(reqs)
    for rid, rq in enumerate(reqs):
        u, at, steps = got[rid]
        print(f"served request {rid}: {rq.spec.label}, {steps} steps", flush=True)
        assert steps == rq.spec.n_steps
        o = OM.from_spec(rq.spec, solver="splu")
        o.run(rq.spec.n_steps)
        assert _rel(u, o.potential_mv()) < 1e-8, (rid, _rel(u, o.potential_mv()))
        ato = o.activation_times()
        ok = ~np.isnan(ato)
        assert np.array_equal(ok, ~np.isnan(at))
        assert not ok.any() or np.max(np.abs(at[ok] - ato[ok])) <= rq.spec.dt + 1e-9


def test_destroying_a_pooled_sim_releases_its_slot():
    import paper_2308_01651_amd as ep
    (a, _), (b, _) = _specs()[:2]
    alone = ep.Simulation.from_spec(b)
    alone.step(30)
    u_alone = alone.get_state()[0]
    alone.close()
    pool = ep.Pool(8 << 30, 4, ep.EP_FP64)
    sa = ep.Simulation.from_spec(a, finalize=False)
    sb = ep.Simulation.from_spec(b, finalize=False)
    pool.admit(sa, 100)
    slot_b = pool.admit(sb, 30)
    pool.step(10)
    sa.close()                                   # destroyed while pooled
    assert pool.info()["active"] == 1
    pool.step(20)
    assert pool.poll() == [slot_b]
    assert np.array_equal(sb.get_state()[0], u_alone)
    pool.release(slot_b)
    sb.close()
    pool.close()
