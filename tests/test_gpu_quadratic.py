"""GPU: hexahedra of degree 2 to 6 ((p + 1)^3 nodes) and quadratic (10-node)
tetrahedra against the oracle.

The operators of these lattices ((2p + 1)^3 entries in a row of an element
vertex: 125 for Q2 up to 2,197 for Q6) are stored in the sliced-ELL format; everything else (ionic step at every node, ICI load,
PCG, activation) is the path of the other elements.  Tolerances as for Q1:
a single step at rtol 1e-13 to 1e-10 relative, trajectories at rtol 1e-10 to
1e-8 with activation times to the time step, mixed precision against FP64
at RMS 1e-3 mV and 0.1 ms.
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


def _spec(dims=(4.0, 2.0, 1.0), h=0.5, model="ttp06", variant="endo", bdf=2, curved=False, kind="q2"):
    if kind in ("q4", "q5", "q6"):
        mesh = W.slab_qp(*dims, h, int(kind[1]))
    else:
        mesh = {"q2": W.slab_q2, "q3": W.slab_q3, "p2": W.slab_p2}[kind](*dims, h)
    if curved:
        rng = np.random.default_rng(8)
        mesh.xyz = mesh.xyz + rng.uniform(-0.02, 0.02, mesh.xyz.shape)
    st = [W.corner_cube_stimulus(dims=dims)]
    # the Lagrange basis of degree >= 2 has negative lobes, so a nodal D that
    # jumps from node to node (random fibers) interpolates to an indefinite
    # tensor at some quadrature points, which finalize rejects; these
    # elements get a smooth fiber field that turns in all three directions
    fib = W.smooth_fibers(mesh.xyz, 9)
    return W.SimSpec(mesh, fib, W.Physics(), model, variant, st, 0.05, bdf, 1, 1e-10, "t")


@pytest.mark.parametrize("kind,model,variant,bdf,curved", [("q2", "ttp06", "endo", 2, False),
                                                           ("q2", "bo", "epi", 3, True), ("q2", "ap", "", 1, False),
                                                           ("q3", "ttp06", "endo", 2, False),
                                                           ("q3", "bo", "epi", 3, True),
                                                           ("q4", "ttp06", "endo", 2, False),
                                                           ("q5", "bo", "epi", 3, False),
                                                           ("q6", "ttp06", "endo", 2, False),
                                                           ("p2", "ttp06", "epi", 2, False),
                                                           ("p2", "ttp06", "endo", 2, True),
                                                           ("p2", "bo", "epi", 2, False)])
def test_quadratic_single_step(kind, model, variant, bdf, curved):
    ep = _ep()
    spec = _spec(model=model, variant=variant, bdf=bdf, curved=curved, kind=kind)
    n = spec.mesh.n_nodes
    u, w = W.random_state(model, n, seed=71)
    rng = np.random.default_rng(72)
    scale = 1.0 if model == "ttp06" else 0.01
    u_prev = np.stack([u + scale * rng.normal(size=n) for _ in range(bdf - 1)]) if bdf > 1 else None
    o = OM.from_spec(spec, solver="splu", rtol=1e-13)
    o.set_state(u, w, list(u_prev) if u_prev is not None else None, 5)
    o.step()
    sim = ep.Simulation.from_spec(spec, rtol=1e-13)
    assert sim.get_stats()["matrix_format"] == ep.EP_FMT_SELL
    sim.set_state(u, w, u_prev, 5)
    sim.step(1)
    ug, wg, _ = sim.get_state()
    sim.close()
    assert _rel(ug, o.u) < 1e-10, _rel(ug, o.u)
    for v in range(w.shape[0]):
        err = np.max(np.abs(wg[v] - o.w[v])) / max(np.max(np.abs(o.w[v])), 1e-30)
        assert err < 1e-11, (v, err)


@pytest.mark.parametrize("kind,prec", [("q2", 0), ("q2", 1), ("q3", 0), ("q3", 1), ("q4", 0), ("q4", 1), ("q5", 0),
                                       ("p2", 0)])
def test_quadratic_trajectory(kind, prec):
    ep = _ep()
    spec = _spec(dims=(6.0, 3.0, 1.0), h=0.5 if kind != "q5" else 1.0, kind=kind)
    o = OM.from_spec(spec, solver="splu")
    ref = ep.Simulation.from_spec(spec)
    sim = ep.Simulation.from_spec(spec, precision=prec)
    steps = 300
    for chunk in range(3):
        o.run(steps // 3)
        ref.step(steps // 3)
        sim.step(steps // 3)
        print(f"{kind} trajectory prec={prec}: {(chunk + 1) * steps // 3} steps", flush=True)
        err = _rel(ref.get_potential(), o.potential_mv())
        assert err < 1e-8, (chunk, err)
    at_o, at_r, at_s = o.activation_times(), ref.get_activation_times(), sim.get_activation_times()
    ok = ~np.isnan(at_o)
    assert ok.sum() > 100 and np.array_equal(ok, ~np.isnan(at_r))
    assert np.max(np.abs(at_o[ok] - at_r[ok])) <= spec.dt + 1e-9
    if prec == 1:
        du = sim.get_potential() - ref.get_potential()
        assert np.sqrt(np.mean(du * du)) <= 1e-3
        assert np.array_equal(ok, ~np.isnan(at_s)) and np.max(np.abs(at_s[ok] - at_r[ok])) <= 0.1
    ref.close()
    sim.close()


# ---- matrix-free operator (sum factorization) -------------------------------

@pytest.mark.parametrize("kind,model,variant,bdf,curved", [("q2", "ttp06", "endo", 2, False),
                                                           ("q2", "bo", "epi", 3, True),
                                                           ("q3", "ttp06", "endo", 2, False),
                                                           ("q3", "ap", "", 1, True)])
def test_matrix_free_single_step(kind, model, variant, bdf, curved):
    """One step with the operator applied element by element (no assembled
    matrix on the device) against the oracle's assembled step, from the same
    random state, at rtol 1e-13: 1e-10 relative."""
    ep = _ep()
    spec = _spec(model=model, variant=variant, bdf=bdf, curved=curved, kind=kind)
    n = spec.mesh.n_nodes
    u, w = W.random_state(model, n, seed=73)
    rng = np.random.default_rng(74)
    scale = 1.0 if model == "ttp06" else 0.01
    u_prev = np.stack([u + scale * rng.normal(size=n) for _ in range(bdf - 1)]) if bdf > 1 else None
    o = OM.from_spec(spec, solver="splu", rtol=1e-13)
    o.set_state(u, w, list(u_prev) if u_prev is not None else None, 5)
    o.step()
    sim = ep.Simulation.from_spec(spec, rtol=1e-13, matrix_format=ep.EP_FMT_MF)
    assert sim.get_stats()["matrix_format"] == ep.EP_FMT_MF
    sim.set_state(u, w, u_prev, 5)
    sim.step(1)
    ug, wg, _ = sim.get_state()
    sim.close()
    assert _rel(ug, o.u) < 1e-10, _rel(ug, o.u)
    for v in range(w.shape[0]):
        err = np.max(np.abs(wg[v] - o.w[v])) / max(np.max(np.abs(o.w[v])), 1e-30)
        assert err < 1e-11, (v, err)


@pytest.mark.parametrize("kind", ["q2", "q3"])
def test_matrix_free_trajectory_matches_oracle_and_assembled(kind):
    """300 steps with the matrix-free operator: against the oracle (1e-8
    relative, activation times to the step) and against the assembled
    (sliced ELL) run of the same workload."""
    ep = _ep()
    spec = _spec(dims=(6.0, 3.0, 1.0), h=0.5, kind=kind)
    o = OM.from_spec(spec, solver="splu")
    mf = ep.Simulation.from_spec(spec, matrix_format=ep.EP_FMT_MF)
    sell = ep.Simulation.from_spec(spec)
    for chunk in range(3):
        o.run(100)
        mf.step(100)
        sell.step(100)
        err = _rel(mf.get_potential(), o.potential_mv())
        print(f"{kind} matrix-free: {(chunk + 1) * 100} steps, rel {err:.2e}", flush=True)
        assert err < 1e-8, (chunk, err)
    assert _rel(mf.get_potential(), sell.get_potential()) < 1e-8
    at_o, at_m = o.activation_times(), mf.get_activation_times()
    ok = ~np.isnan(at_o)
    assert ok.sum() > 100 and np.array_equal(ok, ~np.isnan(at_m))
    assert np.max(np.abs(at_o[ok] - at_m[ok])) <= spec.dt + 1e-9
    mf.close()
    sell.close()


def test_matrix_free_rejections():
    ep = _ep()
    spec = _spec(kind="q2")
    for kw in (dict(precision=ep.EP_MIXED), dict(block=4)):
        with pytest.raises(ep.EpError):
            ep.Simulation.from_spec(spec, matrix_format=ep.EP_FMT_MF, **kw)
    q1 = W.SimSpec(W.slab_q1(2.0, 1.0, 1.0, 0.25), None, W.Physics(), "ap", "", [], 0.05, 1, 1, 1e-10, "t")
    q1.fibers = W.uniform_fibers(q1.mesh.n_nodes)
    with pytest.raises(ep.EpError):
        ep.Simulation.from_spec(q1, matrix_format=ep.EP_FMT_MF)
    pool = ep.Pool(1 << 30, 2, ep.EP_FP64)
    s = ep.Simulation.from_spec(spec, matrix_format=ep.EP_FMT_MF, finalize=False)
    with pytest.raises(ep.EpError):
        pool.admit(s, 10)
    s.close()
    pool.close()


@pytest.mark.parametrize("kind", ["q2", "q3"])
def test_matrix_free_compressed_geometry(kind):
    """Straight (affine) elements with uniform fibers: every element's
    quadrature-point factors are an element constant times the Gauss weight,
    so the operator keeps 7 numbers per element.  Single step against the
    oracle at rtol 1e-13 (1e-10), 200 steps against the sliced-ELL run, and
    the geometry storage is the compressed one (device bytes)."""
    ep = _ep()
    dims = (4.0, 2.0, 1.0)
    mesh = {"q2": W.slab_q2, "q3": W.slab_q3}[kind](*dims, 0.5)
    spec = W.SimSpec(mesh, W.uniform_fibers(mesh.n_nodes), W.Physics(), "ttp06", "endo",
                     [W.corner_cube_stimulus(dims=dims)], 0.05, 2, 1, 1e-10, "t")
    n = mesh.n_nodes
    u, w = W.random_state("ttp06", n, seed=75)
    u_prev = (u + np.random.default_rng(76).normal(size=n))[None, :]
    o = OM.from_spec(spec, solver="splu", rtol=1e-13)
    o.set_state(u, w, [u_prev[0]], 5)
    o.step()
    sim = ep.Simulation.from_spec(spec, rtol=1e-13, matrix_format=ep.EP_FMT_MF)
    sim.set_state(u, w, u_prev, 5)
    sim.step(1)
    assert _rel(sim.get_state()[0], o.u) < 1e-10
    sim.close()
    mf = ep.Simulation.from_spec(spec, matrix_format=ep.EP_FMT_MF)
    sell = ep.Simulation.from_spec(spec)
    mf.step(200)
    sell.step(200)
    assert _rel(mf.get_potential(), sell.get_potential()) < 200 * spec.rtol
    # the same mesh with fibers that vary from node to node keeps the full factors
    spec_s = W.SimSpec(mesh, W.smooth_fibers(mesh.xyz, 9), W.Physics(), "ttp06", "endo",
                       [W.corner_cube_stimulus(dims=dims)], 0.05, 2, 1, 1e-10, "t")
    full = ep.Simulation.from_spec(spec_s, matrix_format=ep.EP_FMT_MF)
    q = {"q2": 27, "q3": 64}[kind]
    n_el = mesh.conn.shape[0]
    saved = full.get_stats()["device_bytes"] - mf.get_stats()["device_bytes"]
    assert saved >= 0.9 * n_el * 7 * (q - 1) * 8, (saved, n_el)
    assert mf.get_stats()["mf_compressed"] == 1 and full.get_stats()["mf_compressed"] == 0
    assert sell.get_stats()["mf_compressed"] == 0
    for s in (mf, sell, full):
        s.close()
