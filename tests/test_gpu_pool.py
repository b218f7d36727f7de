"""GPU: batched / serving pool.

Each simulation's result is bitwise the same alone and in a mix of uneven
simulations (per-instance reductions in a fixed order, tiles per instance),
for FP64 and mixed precision; admission respects the slot count and the HBM
budget (EP_EAGAIN); simulations finish at their own step counts.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _specs():
    a = W.SimSpec(W.slab_q1(6.0, 3.0, 2.0, 0.25), None, W.Physics(), "ap", "",
                  [W.corner_cube_stimulus(dims=(6.0, 3.0, 2.0))], 0.05, 2, 1, 1e-10, "ap-slab")
    b = W.SimSpec(W.slab_q1(8.0, 2.0, 1.5, 0.25), None, W.Physics(0.2, 0.02, 0.02), "ttp06", "endo",
                  [W.corner_cube_stimulus(dims=(8.0, 2.0, 1.5))], 0.05, 2, 1, 1e-10, "ttp-slab")
    m, fib, endo = W.lv_shell(4, 40, 16)
    c = W.SimSpec(m, fib, W.Physics(0.17, 0.0425, 0.0425), "bo", "epi",
                  [W.Stimulus(W.GAUSS, tuple(m.xyz[endo[5]]), 2.5, 36.0, 0.0, 2.0, 0.0)], 0.05, 2, 1, 1e-10, "bo-lv")
    for sp in (a, b):
        sp.fibers = W.uniform_fibers(sp.mesh.n_nodes)
    return [a, b, c]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pool_matches_alone_bitwise(precision):
    import paper_2308_01651_amd as ep
    prec = ep.EP_FP64 if precision == "fp64" else ep.EP_MIXED
    specs = _specs()
    steps = 80
    alone = []
    for sp in specs:
        s = ep.Simulation.from_spec(sp, precision=prec)
        s.step(steps)
        alone.append((s.get_state()[0], s.get_activation_times(), s.get_stats()["cg_iters_total"]))
        s.close()
    pool = ep.Pool(8 << 30, 8, prec)
    sims = []
    for sp in specs:
        s = ep.Simulation.from_spec(sp, precision=prec, finalize=False)
        slot = pool.admit(s, steps)
        assert slot is not None
        sims.append((slot, s))
    pool.step(steps)
    assert sorted(pool.poll()) == sorted(sl for sl, _ in sims)
    for (slot, s), (u0, at0, it0) in zip(sims, alone):
        u, _, _ = s.get_state()
        assert np.array_equal(u, u0), (slot, np.max(np.abs(u - u0)))
        assert np.array_equal(np.isnan(s.get_activation_times()), np.isnan(at0))
        assert s.get_stats()["cg_iters_total"] == it0
        pool.release(slot)
        s.close()
    pool.close()


def test_pool_admission_and_uneven_targets():
    import paper_2308_01651_amd as ep
    specs = _specs()
    pool = ep.Pool(8 << 30, 2, ep.EP_FP64)
    s0 = ep.Simulation.from_spec(specs[0], finalize=False)
    s1 = ep.Simulation.from_spec(specs[1], finalize=False)
    s2 = ep.Simulation.from_spec(specs[2], finalize=False)
    assert pool.admit(s0, 10) is not None
    assert pool.admit(s1, 25) is not None
    assert pool.admit(s2, 5) is None            # no free slot
    pool.step(10)
    done = pool.poll()
    assert len(done) == 1
    sim, st = pool.release(done[0])
    assert sim is s0 and sim.get_stats()["steps"] == 10
    assert pool.admit(s2, 5) is not None        # the freed slot is reused
    pool.step(20)
    assert sorted(pool.poll()) == [0, 1]
    for slot in list(pool.sims):
        sim, _ = pool.release(slot)
    assert s1.get_stats()["steps"] == 25 and s2.get_stats()["steps"] == 5
    # an HBM budget smaller than the simulation's footprint rejects it
    small = ep.Pool(1 << 20, 4, ep.EP_FP64)
    s3 = ep.Simulation.from_spec(specs[0], finalize=False)
    assert small.admit(s3, 10) is None
    small.close()
    for s in (s0, s1, s2, s3):
        s.close()
    pool.close()
