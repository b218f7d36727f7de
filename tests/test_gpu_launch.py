"""GPU: launch shapes, graph replay and the launch-shape tuner.

The ionic nodes-per-thread setting, the tile map, HIP-graph replay of the
step and the tuner choose which thread / workgroup computes a node and how
launches are issued, never the arithmetic: every result must be bitwise the
same as with the default launches, for single simulations and in the pool.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _ep():
    import paper_2308_01651_amd as ep
    return ep


def _spec(model="ttp06", variant="endo"):
    mesh = W.slab_q1(10.0, 3.5, 1.5, 0.125)       # 81 x 29 x 13 = 30,537 nodes, 60 tiles
    return W.SimSpec(mesh, W.uniform_fibers(mesh.n_nodes), W.Physics(), model, variant,
                     [W.corner_cube_stimulus(dims=(10.0, 3.5, 1.5))], 0.05, 2, 1, 1e-10, "t")


def _run(spec, prec, steps, opts=(), tune=0):
    ep = _ep()
    s = ep.Simulation.from_spec(spec, precision=prec)
    for k, v in opts:
        s.set_option(k, v)
    done = 0
    chosen = None
    if tune:
        chosen = s.autotune(tune)
        done = 5 * tune
    s.step(steps - done)
    u, w, _ = s.get_state()
    at = s.get_activation_times()
    it = s.get_stats()["cg_iters_total"]
    s.close()
    return u, w, at, it, chosen


@pytest.mark.parametrize("model,variant,prec", [("ttp06", "endo", 0), ("ttp06", "endo", 1), ("bo", "epi", 0),
                                                ("ap", "", 1)])
def test_launch_shapes_and_graphs_are_bitwise_neutral(model, variant, prec):
    ep = _ep()
    spec = _spec(model, variant)
    ref = _run(spec, prec, 60)
    variants = [
        [(ep.EP_OPT_IONIC_NPT, 2)],
        [(ep.EP_OPT_IONIC_NPT, 4), (ep.EP_OPT_TILE_MAP, 1)],
        [(ep.EP_OPT_GRAPH, 1)],
        [(ep.EP_OPT_GRAPH, 1), (ep.EP_OPT_IONIC_NPT, 2), (ep.EP_OPT_TILE_MAP, 1)],
        [(ep.EP_OPT_TILE_MAP, 2)],
        [(ep.EP_OPT_GRAPH, 1), (ep.EP_OPT_TILE_MAP, 2)],
    ]
    for opts in variants:
        got = _run(spec, prec, 60, opts)
        assert np.array_equal(got[0], ref[0]), opts
        assert np.array_equal(got[1], ref[1]), opts
        assert np.array_equal(got[2], ref[2], equal_nan=True), opts
        assert got[3] == ref[3], opts


def test_graph_toggled_mid_run_and_with_timers():
    ep = _ep()
    spec = _spec()
    ref = _run(spec, 0, 90)
    s = ep.Simulation.from_spec(spec)
    s.set_option(ep.EP_OPT_GRAPH, 1)
    s.step(30)
    s.set_option(ep.EP_OPT_KERNEL_TIMERS, 1)     # graphs are bypassed while timing
    s.step(30)
    s.set_option(ep.EP_OPT_KERNEL_TIMERS, 0)
    s.set_option(ep.EP_OPT_IONIC_NPT, 2)         # drops and re-captures the graphs
    s.step(30)
    u, w, _ = s.get_state()
    s.close()
    assert np.array_equal(u, ref[0]) and np.array_equal(w, ref[1])


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_is_bitwise_neutral(prec):
    spec = _spec()
    ref = _run(spec, prec, 80)
    got = _run(spec, prec, 80, tune=6)
    npt, tmap = got[4]
    assert npt in (1, 2, 4) and tmap in (0, 1, 2)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    assert got[3] == ref[3]


def test_launch_options_rejected():
    ep = _ep()
    s = ep.Simulation.from_spec(_spec())
    for k, v in [(ep.EP_OPT_IONIC_NPT, 3), (ep.EP_OPT_TILE_MAP, 3), (ep.EP_OPT_GRAPH, 0.5), (99, 1)]:
        with pytest.raises(ep.EpError):
            s.set_option(k, v)
    with pytest.raises(ep.EpError):
        s.autotune(0)
    s.close()


@pytest.mark.parametrize("case", ["c1", "q2", "p1"])
def test_lattice_band_tile_map(case):
    """Tile map 2 on the C1 lattice (865 tiles; every tile taken by exactly
    one workgroup or results would differ) and on operators that are not the
    Q1 lattice DIA (sliced-ELL Q2, the Kuhn P1 DIA), where it runs map 0:
    bitwise equal to the default launches."""
    ep = _ep()
    if case == "c1":
        spec = W.config_c1(h=0.1, n_steps=1)
        steps = 20
    else:
        dims = (4.0, 2.0, 1.0)
        mesh = W.slab_q2(*dims, 0.5) if case == "q2" else W.slab_p1(*dims, 0.25)
        spec = W.SimSpec(mesh, W.uniform_fibers(mesh.n_nodes), W.Physics(), "ttp06", "endo",
                         [W.corner_cube_stimulus(dims=dims)], 0.05, 2, 1, 1e-10, "t")
        steps = 60
    for prec in (0, 1):
        ref = _run(spec, prec, steps)
        got = _run(spec, prec, steps, [(ep.EP_OPT_TILE_MAP, 2)])
        print(f"{case} prec {prec}: {steps} steps, {ref[3]} CG iterations", flush=True)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (case, prec)
        assert got[3] == ref[3]


@pytest.mark.parametrize("prec", [0, 1])
def test_pool_graph_and_autotune_match_alone(prec):
    ep = _ep()
    specs = [_spec("ttp06", "endo"), _spec("bo", "epi"), _spec("ap", "")]
    specs[1].mesh = W.slab_q1(6.0, 2.0, 1.0, 0.125)
    specs[1].fibers = W.uniform_fibers(specs[1].mesh.n_nodes)
    steps = 70
    alone = [_run(sp, prec, steps) for sp in specs]
    pool = ep.Pool(8 << 30, 4, prec)
    sims = []
    for sp in specs:
        s = ep.Simulation.from_spec(sp, precision=prec, finalize=False)
        slot = pool.admit(s, steps)
        assert slot is not None
        sims.append((slot, s))
    pool.set_option(ep.EP_OPT_GRAPH, 1)
    pool.step(10)
    npt, tmap = pool.autotune(4)                 # 20 more steps, graphs bypassed
    assert npt in (1, 2, 4) and tmap in (0, 1)
    pool.step(steps)                             # graphs again, with the tuned shapes
    assert sorted(pool.poll()) == sorted(sl for sl, _ in sims)
    for (slot, s), ref in zip(sims, alone):
        u, w, _ = s.get_state()
        assert np.array_equal(u, ref[0]), slot
        assert np.array_equal(w, ref[1]), slot
        assert s.get_stats()["cg_iters_total"] == ref[3]
        pool.release(slot)
        s.close()
    pool.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_repeated_kernel_timing_leaves_results_unchanged(prec):
    """ep_sim_time_kernel between steps (SpMV, rhs) must not change the run."""
    ep = _ep()
    spec = _spec()
    ref = _run(spec, prec, 40)
    s = ep.Simulation.from_spec(spec, precision=prec)
    s.step(20)
    t1 = s.time_kernel_us("cg_spmv", 50)
    t2 = s.time_kernel_us("rhs", 20)
    assert t1 > 0 and t2 > 0
    with pytest.raises(ep.EpError):
        s.time_kernel_us("cg_update", 5)
    s.step(20)
    u, w, _ = s.get_state()
    assert np.array_equal(u, ref[0]) and np.array_equal(w, ref[1])
    assert s.get_stats()["cg_iters_total"] == ref[3]
    s.close()
