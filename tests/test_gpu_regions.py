"""GPU: several subdomains (per-subdomain cell type, parameters and
conductivities; interface nodes with one ionic state per subdomain and the
ionic load sum_i M^i I_ion^i; non-conductive subdomains removed) against the
multi-subdomain oracle.

Tolerances as for one subdomain: a single step from the same state at rtol
1e-13 agrees to 1e-10 relative; trajectories at rtol 1e-10 to 1e-8 relative
with activation times to the time step; mixed precision against FP64 at RMS
1e-3 mV and 0.1 ms.  Removed nodes report NaN on both sides.  One subdomain,
or several identical ones, through the subdomain path give bitwise the
one-subdomain result (the interface correction is then exactly zero).
"""
import numpy as np
import pytest

import workloads as W
from oracle import regions as R
from oracle.ionic import TTP_PARAM_NAMES

pytestmark = pytest.mark.gpu


def _ep():
    import paper_2308_01651_amd as ep
    return ep


def _rel(a, b):
    ok = np.isfinite(b)
    return np.linalg.norm(a[ok] - b[ok]) / max(np.linalg.norm(b[ok]), 1e-300)


def _slab(kind="q1", dims=(4.0, 2.0, 1.0), h=0.25, model="ttp06", variant="endo", bdf=2):
    mesh = (W.slab_q1 if kind == "q1" else W.slab_p1)(*dims, h)
    st = [W.corner_cube_stimulus(dims=dims)]
    return W.SimSpec(mesh, W.random_fibers(mesh.n_nodes, 7), W.Physics(), model, variant, st, 0.05, bdf, 1,
                     1e-10, "t")


def _layers(spec, scar=False):
    """Three TTP06 layers along x (endo / mid / epi, the epi layer with GKr
    x1.5 and higher conductivity), optionally a non-conductive box."""
    m = spec.mesh
    L = m.xyz[:, 0].max()
    mat = W.material_layers(m, 0, [L / 3, 2 * L / 3])
    gkr = 0.153 * 1.5
    oregs = [R.Region("endo"), R.Region("mid"),
             R.Region("epi", params={"GKr": gkr}, sigma=(0.25, 0.03, 0.03))]
    gregs = {0: dict(variant="endo"), 1: dict(variant="mid"),
             2: dict(variant="epi", params=_ttp_params({"GKr": gkr}), sigma=(0.25, 0.03, 0.03))}
    if scar:
        mat = W.material_box(m, (0.4 * L, 0.0, 0.0), (0.6 * L, 0.6 * m.xyz[:, 1].max(), 1e9), 3, mat)
        oregs.append(R.Region(conductive=False))
        gregs[3] = dict(conductive=False)
    return mat, oregs, gregs


def _ttp_params(over):
    """Positional TTP06 overrides up to the last named one (epi defaults)."""
    from oracle.ionic import ttp06_params
    p = ttp06_params("epi")
    last = max(TTP_PARAM_NAMES.index(k) for k in over)
    return [float(over.get(k, p[k])) for k in TTP_PARAM_NAMES[: last + 1]]


@pytest.mark.parametrize("kind,scar", [("q1", False), ("q1", True), ("p1", False)])
def test_regions_single_step(kind, scar):
    ep = _ep()
    spec = _slab(kind)
    mat, oregs, gregs = _layers(spec, scar)
    n = spec.mesh.n_nodes
    u, w = W.random_state("ttp06", n, seed=61)
    rng = np.random.default_rng(62)
    u_prev = u + rng.normal(size=n)
    o = R.from_spec(spec, mat, oregs, solver="splu", rtol=1e-13)
    live = o.live
    o.set_state(u[live], w[:, live], [u_prev[live]], 4)
    o.step()
    sim = ep.Simulation.from_spec(spec, rtol=1e-13, material=mat, regions=gregs)
    sim.set_state(u, w, u_prev[None], 4)
    sim.step(1)
    ug, wg, _ = sim.get_state()
    sim.close()
    assert np.array_equal(np.isnan(ug), np.isnan(o.u))
    assert _rel(ug, o.u) < 1e-10, _rel(ug, o.u)
    # a node's state (get_state) is that of its lowest conducting subdomain
    seen = np.zeros(n, bool)
    for r in range(len(o.regions)):
        nodes, wr = o.state(r)
        prim = ~seen[nodes]
        seen[nodes] = True
        if prim.any():
            idx = nodes[prim]
            err = np.max(np.abs(wg[:, idx] - wr[:, prim]) / np.maximum(np.abs(wr[:, prim]), 1e-30))
            assert err < 1e-9, (r, err)


@pytest.mark.parametrize("kind,scar,prec", [("q1", True, 0), ("p1", False, 0), ("q1", True, 1)])
def test_regions_trajectory(kind, scar, prec):
    ep = _ep()
    spec = _slab(kind, dims=(6.0, 3.0, 1.0), h=0.25)
    mat, oregs, gregs = _layers(spec, scar)
    steps = 300
    o = R.from_spec(spec, mat, oregs, solver="splu")
    ref = ep.Simulation.from_spec(spec, material=mat, regions=gregs)
    sim = ep.Simulation.from_spec(spec, precision=prec, material=mat, regions=gregs)
    for chunk in range(3):
        o.run(steps // 3)
        ref.step(steps // 3)
        sim.step(steps // 3)
        print(f"regions {kind} scar={scar} prec={prec}: {(chunk + 1) * steps // 3} steps", flush=True)
        err = _rel(ref.get_potential(), o.potential_mv())
        assert err < 1e-8, (chunk, err)
    at_o, at_r, at_s = o.activation_times(), ref.get_activation_times(), sim.get_activation_times()
    ok = ~np.isnan(at_o)
    assert ok.sum() > 50 and np.array_equal(ok, ~np.isnan(at_r))
    assert np.max(np.abs(at_o[ok] - at_r[ok])) <= spec.dt + 1e-9
    if prec == 1:
        du = sim.get_potential() - ref.get_potential()
        fin = np.isfinite(du)
        assert np.array_equal(fin, np.isfinite(ref.get_potential()))
        assert np.sqrt(np.mean(du[fin] ** 2)) <= 1e-3
        assert np.array_equal(ok, ~np.isnan(at_s)) and np.max(np.abs(at_s[ok] - at_r[ok])) <= 0.1
    if scar:
        removed = np.setdiff1d(np.arange(spec.mesh.n_nodes), o.live)
        assert removed.size > 0 and np.all(np.isnan(ref.get_potential()[removed]))
    ref.close()
    sim.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_identical_subdomains_are_bitwise_one_subdomain(prec):
    ep = _ep()
    spec = _slab(dims=(4.0, 2.0, 1.0))
    mat = W.material_layers(spec.mesh, 0, [1.3, 2.6])
    one = ep.Simulation.from_spec(spec, precision=prec)
    three = ep.Simulation.from_spec(spec, precision=prec, material=mat)
    one.step(80)
    three.step(80)
    a, b = one.get_state(), three.get_state()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(one.get_activation_times(), three.get_activation_times(), equal_nan=True)
    one.close()
    three.close()


def test_region_errors():
    ep = _ep()
    spec = _slab()
    mat = W.material_layers(spec.mesh, 0, [2.0])
    # a subdomain model without material ids, and an unknown model
    with pytest.raises(ep.EpError):
        ep.Simulation.from_spec(spec, regions={1: dict(model="bo")})
    s = ep.Simulation.from_spec(spec, material=mat, finalize=False)
    with pytest.raises(ep.EpError):
        ep.check(ep.lib.ep_sim_set_region_model(s._h, 0, 17), "ep_sim_set_region_model")
    s.close()
    bad = mat.copy()
    bad[0] = ep.EP_MAX_REGIONS
    with pytest.raises(ep.EpError):
        ep.Simulation.from_spec(spec, material=bad)
    s = ep.Simulation.from_spec(spec, material=mat, finalize=False)
    with pytest.raises(ep.EpError):
        s.set_region(ep.EP_MAX_REGIONS)
    with pytest.raises(ep.EpError):
        s.set_region(0, variant=7)
    s.close()


def test_ventricle_shell_with_scar_and_border_zone():
    """Tetrahedral LV shell (BO model): a non-conductive scar through the
    wall, a border zone around it with slower conduction and a shorter
    tau_so1, healthy tissue elsewhere (the paper's pathological-ventricle
    setup in miniature, on a generated shell).  Trajectory parity with the
    multi-subdomain oracle; removed nodes NaN on both sides."""
    ep = _ep()
    mesh, fib, endo = W.lv_shell(5, 48, 20)
    # a wide, strong Gaussian: this coarse shell (about 2.6 mm elements
    # around the circumference) needs it to start a front
    st = [W.Stimulus(W.GAUSS, tuple(mesh.xyz[endo[7]]), 5.0, 200.0, 0.0, 2.0, 0.0)]
    spec = W.SimSpec(mesh, fib, W.Physics(0.17, 0.0425, 0.0425), "bo", "epi", st, 0.05, 2, 1, 1e-10, "t")
    c = W.element_centroids(mesh)
    ang = np.arctan2(c[:, 1], c[:, 0])
    zc = c[:, 2]
    mat = np.zeros(mesh.n_elems, np.int32)
    mat[(np.abs(ang - 1.0) < 0.45) & (zc < -12.0) & (zc > -28.0)] = 1      # border zone
    mat[(np.abs(ang - 1.0) < 0.25) & (zc < -15.0) & (zc > -25.0)] = 2      # scar
    assert (mat == 1).sum() > 50 and (mat == 2).sum() > 20
    bz_params = [0.0, 1.55, 0.3, 0.13, 0.006, 0.006, 60.0, 1150.0, 1.4506, 60.0, 15.0, 65.0, 0.03, 200.0,
                 0.11, 400.0, 6.0, 20.0]              # BO EPI with tau_so1 30.0181 -> 20
    o = R.from_spec(spec, mat, [R.Region(), R.Region(params={"tau_so1": 20.0}, sigma=(0.08, 0.02, 0.02)),
                                R.Region(conductive=False)], solver="splu")
    sim = ep.Simulation.from_spec(spec, material=mat, regions={
        1: dict(params=bz_params, sigma=(0.08, 0.02, 0.02)), 2: dict(conductive=False)})
    for chunk in range(2):
        o.run(150)
        sim.step(150)
        err = _rel(sim.get_potential(), o.potential_mv())
        print(f"ventricle scar: {(chunk + 1) * 150} steps, rel {err:.2e}", flush=True)
        assert err < 1e-8, (chunk, err)
    u = sim.get_potential()
    assert np.array_equal(np.isnan(u), np.isnan(o.potential_mv()))
    assert np.isnan(u).sum() > 0
    at_o, at_g = o.activation_times(), sim.get_activation_times()
    ok = ~np.isnan(at_o)
    assert ok.sum() > 100 and np.array_equal(ok, ~np.isnan(at_g))
    assert np.max(np.abs(at_o[ok] - at_g[ok])) <= spec.dt + 1e-9
    sim.close()


# ---- a subdomain with its own ionic model; the BDF ionic scheme -------------

def _two_models(spec):
    """TTP06 endocardial tissue (the field in mV) with a Bueno-Orovio border
    band across the slab and an Aliev-Panfilov patch (each in its own units,
    converted to the field's)."""
    m = spec.mesh
    L = m.xyz[:, 0].max()
    mat = W.material_box(m, (0.45 * L, 0.0, 0.0), (0.75 * L, 1e9, 1e9), 1)
    mat = W.material_box(m, (0.8 * L, 0.0, 0.0), (L + 1.0, 0.5 * m.xyz[:, 1].max(), 1e9), 2, mat)
    oregs = [R.Region("endo"), R.Region(model="bo"), R.Region(model="ap")]
    gregs = {0: dict(variant="endo"), 1: dict(model="bo"), 2: dict(model="ap")}
    return mat, oregs, gregs


@pytest.mark.parametrize("kind", ["q1", "p1"])
def test_two_ionic_models_single_step(kind):
    ep = _ep()
    spec = _slab(kind)
    mat, oregs, gregs = _two_models(spec)
    n = spec.mesh.n_nodes
    u, w = W.random_state("ttp06", n, seed=71)
    u_prev = u + np.random.default_rng(72).normal(size=n)
    o = R.from_spec(spec, mat, oregs, solver="splu", rtol=1e-13)
    o.set_state(u, w, [u_prev], 4)
    sim = ep.Simulation.from_spec(spec, rtol=1e-13, material=mat, regions=gregs)
    sim.set_state(u, w, u_prev[None], 4)
    # both start the BO and AP points from their models' initial conditions
    for _ in range(3):
        o.step()
    sim.step(3)
    ug, wg, _ = sim.get_state()
    sim.close()
    assert _rel(ug, o.u) < 1e-10, _rel(ug, o.u)
    # BO state of the nodes whose lowest subdomain is the BO band
    seen = np.zeros(n, bool)
    nodes0, _ = o.state(0)
    seen[nodes0] = True
    nodes1, w1 = o.state(1)
    prim = ~seen[nodes1]
    err = np.max(np.abs(wg[:3, nodes1[prim]] - w1[:, prim]) / np.maximum(np.abs(w1[:, prim]), 1e-30))
    assert err < 1e-9, err


@pytest.mark.parametrize("prec", [0, 1])
def test_two_ionic_models_trajectory(prec):
    """The front leaves the TTP06 corner, crosses the BO band and reaches the
    AP patch; FP64 against the oracle (trajectory bar), mixed precision
    against FP64 (1e-3 mV RMS, threshold times 0.1 ms)."""
    ep = _ep()
    spec = _slab("q1", dims=(6.0, 2.0, 1.0), h=0.25)
    mat, oregs, gregs = _two_models(spec)
    o = R.from_spec(spec, mat, oregs, solver="splu")
    ref = ep.Simulation.from_spec(spec, rtol=1e-12, material=mat, regions=gregs)
    sim = ep.Simulation.from_spec(spec, precision=prec, rtol=1e-12, material=mat, regions=gregs)
    for chunk in range(4):
        o.run(100)
        ref.step(100)
        sim.step(100)
        err = _rel(ref.get_potential(), o.potential_mv())
        print(f"two models prec={prec}: {(chunk + 1) * 100} steps, rel {err:.2e}", flush=True)
        assert err < 1e-8, (chunk, err)
    at_o, at_r = o.activation_times(), ref.get_activation_times()
    ok = ~np.isnan(at_o)
    far = spec.mesh.xyz[:, 0] > 5.0
    assert np.all(ok[far])                        # the front reached the AP patch
    assert np.array_equal(ok, ~np.isnan(at_r))
    assert np.max(np.abs(at_o[ok] - at_r[ok])) <= spec.dt + 1e-9
    if prec == 1:
        du = sim.get_potential() - ref.get_potential()
        assert np.sqrt(np.mean(du * du)) <= 1e-3
        tm, tr = sim.get_threshold_times(), ref.get_threshold_times()
        both = ~np.isnan(tm) & ~np.isnan(tr)
        assert np.array_equal(np.isnan(tm), np.isnan(tr))
        assert np.max(np.abs(tm[both] - tr[both])) <= 0.1
    for s in (ref, sim):
        s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_regions_with_bdf_ionic_scheme(prec):
    """The paper's semi-implicit BDF ionic scheme (BDF3) on three TTP06
    layers with a scar: FP64 against the multi-subdomain oracle's BDF scheme,
    mixed precision against FP64."""
    ep = _ep()
    spec = _slab("q1", dims=(4.0, 2.0, 1.0), h=0.25, bdf=3)
    mat, oregs, gregs = _layers(spec, scar=True)
    o = R.from_spec(spec, mat, oregs, solver="splu", ionic_scheme="bdf")
    ref = ep.Simulation.from_spec(spec, rtol=1e-12, material=mat, regions=gregs, ionic_scheme="bdf")
    sim = ep.Simulation.from_spec(spec, precision=prec, rtol=1e-12, material=mat, regions=gregs,
                                  ionic_scheme="bdf")
    for chunk in range(2):
        o.run(100)
        ref.step(100)
        sim.step(100)
        err = _rel(ref.get_potential(), o.potential_mv())
        assert err < 1e-8, (chunk, err)
    if prec == 1:
        du = sim.get_potential() - ref.get_potential()
        fin = np.isfinite(du)
        assert np.sqrt(np.mean(du[fin] ** 2)) <= 1e-3
    for s in (ref, sim):
        s.close()
