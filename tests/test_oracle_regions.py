"""Pins of the multi-subdomain oracle (oracle/regions.py).

- Subdomains with identical settings reproduce the one-subdomain oracle (a
  separately written code path): this fixes the duplicated ionic states on
  interfaces and the ionic load sum_i M^i I^i (counting an interface twice,
  or using M for every subdomain, fails it).
- sum_i M^i is the full mass matrix.
- With no diffusion and a uniform initial state, nodes far from the
  interface follow their own subdomain's single-cell dynamics, stepped here
  by a separate loop (fixes which parameters each subdomain uses).
- Conduction speed scales with the square root of the subdomain's
  conductivity (reaction-diffusion scaling), measured in each half of a cable.
- A non-conductive subdomain is removed: the result equals the one-subdomain
  oracle on the mesh without those elements (nodes re-numbered), the removed
  nodes report NaN, and a scar band across the slab blocks conduction.
"""
import numpy as np
import pytest

import workloads as W
from oracle import monodomain as OM
from oracle import regions as R
from oracle.ionic import IonicModel


def _spec(mesh, model="ttp06", variant="endo", dims=None, bdf=2, phys=None, stim=None):
    dims = dims or tuple(mesh.xyz.max(axis=0))
    st = stim if stim is not None else [W.corner_cube_stimulus(dims=dims)]
    return W.SimSpec(mesh, W.uniform_fibers(mesh.n_nodes), phys or W.Physics(), model, variant, st, 0.05, bdf,
                     1, 1e-10, "t")


@pytest.mark.parametrize("kind", ["q1", "p1"])
def test_identical_subdomains_reproduce_one_subdomain(kind):
    mesh = (W.slab_q1 if kind == "q1" else W.slab_p1)(4.0, 2.0, 1.0, 0.25)
    spec = _spec(mesh)
    mat = W.material_layers(mesh, 0, [1.3, 2.6])
    one = OM.from_spec(spec, solver="splu")
    three = R.from_spec(spec, mat, [R.Region("endo")] * 3, solver="splu")
    for _ in range(60):
        one.step()
        three.step()
    scale = np.max(np.abs(one.u))
    assert np.max(np.abs(one.u - three.u)) < 1e-10 * scale
    assert np.array_equal(np.isnan(one.activation_times()), np.isnan(three.activation_times()))


def test_subdomain_masses_sum_to_the_mass_matrix():
    mesh = W.slab_p1(3.0, 2.0, 1.0, 0.5)
    spec = _spec(mesh)
    mat = W.material_box(mesh, (1.0, 0.0, 0.0), (2.0, 2.0, 1.0), 1)
    o = R.from_spec(spec, mat, [R.Region("endo"), R.Region("epi", sigma=(0.3, 0.05, 0.05))])
    M1 = OM.from_spec(spec).M.toarray()
    total = sum(reg["M"] @ np.eye(mesh.n_nodes)[reg["nodes"]] for reg in o.regions)
    assert np.allclose(total, M1, rtol=0, atol=1e-15)
    # the two subdomains share exactly the nodes on the planes x = 1 and x = 2
    a, b = (set(reg["nodes"].tolist()) for reg in o.regions)
    shared = np.array(sorted(a & b))
    on_planes = np.isclose(mesh.xyz[:, 0], 1.0) | np.isclose(mesh.xyz[:, 0], 2.0)
    assert np.array_equal(shared, np.nonzero(on_planes)[0])


def _single_cell(model, variant, params, u0, w0, dt, steps, iapp_until, iapp, bdf):
    """Rush-Larsen / BDF steps of one cell with a constant applied current."""
    m = IonicModel(model, variant)
    m.p.update(params)
    hist = [np.array([u0])] * 3
    w = w0.copy()
    for n in range(steps):
        s = min(bdf, n + 1)
        alpha, cb, ce = OM.BDF_COEFFS[s]
        ub = sum(c * h for c, h in zip(cb, hist))
        ue = sum(c * h for c, h in zip(ce, hist))
        w = m.step(ue, w, dt)
        ia = iapp if (n + 1) * dt <= iapp_until + 1e-9 else 0.0
        hist = [(ub + dt * (ia - m.iion(ue, w))) / alpha] + hist[:2]
    return hist[0][0]


def test_uncoupled_subdomains_follow_their_own_cell_models():
    # no diffusion; the whole slab stimulated; left half endo, right half
    # epi with GKr doubled.  The mass coupling across the interface decays by
    # about 0.27 per element, so nodes 16 elements away see ~1e-9 of it.
    mesh = W.slab_q1(40.0, 1.0, 1.0, 1.0)
    phys = W.Physics(0.0, 0.0, 0.0)
    big = W.Stimulus(W.CUBE, (20.0, 0.5, 0.5), 90.0, 50.0, 0.0, 1.0, 0.0)
    spec = _spec(mesh, phys=phys, stim=[big])
    mat = W.material_layers(mesh, 0, [20.0])
    regs = [R.Region("endo"), R.Region("epi", params={"GKr": 0.306})]
    o = R.from_spec(spec, mat, regs, solver="splu")
    steps = 200
    o.run(steps)
    u0, w0 = IonicModel("ttp06", "endo").initial(1)
    scale = 50.0 / (140.0 * 0.01)
    left = _single_cell("ttp06", "endo", {}, u0[0], w0, 0.05, steps, 1.0, scale, 2)
    right = _single_cell("ttp06", "epi", {"GKr": 0.306}, u0[0], w0, 0.05, steps, 1.0, scale, 2)
    assert abs(left - right) > 0.5               # the two cell models differ
    x = mesh.xyz[:, 0]
    far_l, far_r = x <= 4.0, x >= 36.0
    assert np.max(np.abs(o.u[far_l] - left)) < 1e-8 * abs(left)
    assert np.max(np.abs(o.u[far_r] - right)) < 1e-8 * abs(right)


def test_conduction_speed_scales_with_sqrt_conductivity():
    # two disconnected cables in one mesh, one subdomain each (sigma and
    # 4 sigma), both paced at x = 0: their speeds differ by sqrt(4)
    c = W.slab_q1(10.0, 0.2, 0.2, 0.1)
    xyz = np.vstack([c.xyz, c.xyz + np.array([0.0, 1.0, 0.0])])
    conn = np.vstack([c.conn, c.conn + c.n_nodes]).astype(np.int32)
    mesh = W.Mesh(xyz, conn, None, "two cables")
    phys = W.Physics(0.17, 0.17, 0.17)
    st = [W.Stimulus(W.CUBE, (0.0, y, 0.1), 1.0, 50.0, 0.0, 2.0, 0.0) for y in (0.1, 1.1)]
    spec = _spec(mesh, phys=phys, stim=st)
    mat = np.repeat(np.array([0, 1], np.int32), c.n_elems)
    o = R.from_spec(spec, mat, [R.Region("endo"), R.Region("endo", sigma=(0.68, 0.68, 0.68))], solver="splu")
    o.run(int(30.0 / 0.05))
    at = o.activation_times()
    x = mesh.xyz[:, 0]

    def speed(cable):
        sel = (x >= 2.0) & (x <= 7.0) & (np.arange(mesh.n_nodes) // c.n_nodes == cable)
        assert np.all(np.isfinite(at[sel]))
        return 1.0 / np.polyfit(x[sel], at[sel], 1)[0]

    v1, v2 = speed(0), speed(1)
    assert 1.8 < v2 / v1 < 2.2, (v1, v2)


def test_scar_equals_mesh_without_its_elements():
    mesh = W.slab_q1(4.0, 2.0, 1.0, 0.25)
    spec = _spec(mesh)
    mat = W.material_box(mesh, (1.5, 0.0, 0.0), (2.5, 1.2, 1.0), 1)
    o = R.from_spec(spec, mat, [R.Region("endo"), R.Region(conductive=False)], solver="splu")
    keep = mat == 0
    live = np.unique(mesh.conn[keep])
    cidx = np.full(mesh.n_nodes, -1)
    cidx[live] = np.arange(live.size)
    sub = W.Mesh(mesh.xyz[live], cidx[mesh.conn[keep]].astype(np.int32), None, "sub")
    ref = OM.from_spec(_spec(sub, dims=(4.0, 2.0, 1.0)), solver="splu")
    for _ in range(60):
        o.step()
        ref.step()
    u = o.u
    removed = np.setdiff1d(np.arange(mesh.n_nodes), live)
    assert removed.size > 0 and np.all(np.isnan(u[removed]))
    assert np.max(np.abs(u[live] - ref.u)) < 1e-10 * np.max(np.abs(ref.u))


def test_scar_band_blocks_conduction():
    mesh = W.slab_q1(6.0, 1.0, 0.5, 0.25)
    spec = _spec(mesh, stim=[W.Stimulus(W.CUBE, (0.0, 0.5, 0.25), 1.0, 50.0, 0.0, 2.0, 0.0)])
    mat = W.material_box(mesh, (2.9, -1.0, -1.0), (3.6, 2.0, 2.0), 1)
    o = R.from_spec(spec, mat, [R.Region("endo"), R.Region(conductive=False)], solver="splu")
    o.run(int(25.0 / 0.05))
    at = o.activation_times()
    x = mesh.xyz[:, 0]
    assert np.all(np.isfinite(at[x <= 2.75]))
    assert np.all(np.isnan(at[x >= 3.75]))
    # without the scar the whole slab activates
    o2 = R.from_spec(spec, mat, [R.Region("endo"), R.Region("endo")], solver="splu")
    o2.run(int(25.0 / 0.05))
    assert np.all(np.isfinite(o2.activation_times()))


# ---- a subdomain with its own ionic model; the BDF ionic scheme -------------

def test_whole_slab_in_another_model_is_the_affine_image_of_that_model():
    """The field keeps the simulation model's units (TTP06: mV).  When every
    element belongs to a Bueno-Orovio subdomain, the run must be the plain
    Bueno-Orovio simulation (a separate code path, its own dimensionless
    units) mapped by u_mV = 85.7 u - 84: the semi-discrete problem and the
    BDF / extrapolation weights (which sum to alpha and 1) commute with an
    affine change of the potential because K 1 = 0.  A wrong scale, shift
    or direction of the conversion, or a current not rescaled, fails it."""
    mesh = W.slab_q1(3.0, 1.5, 1.0, 0.25)
    dims = tuple(mesh.xyz.max(axis=0))
    stim = [W.Stimulus(W.CUBE, (0.0, 0.0, 0.0), 1.5, 50.0, 0.0, 2.0, 0.0)]
    spec_bo = _spec(mesh, "bo", "epi", dims=dims, stim=stim)
    plain = OM.from_spec(spec_bo, solver="splu")
    spec_t = _spec(mesh, "ttp06", "endo", dims=dims, stim=stim)
    mat = np.zeros(mesh.n_elems, np.int32)
    mixed = R.from_spec(spec_t, mat, [R.Region(model="bo")], solver="splu")
    # same initial potential: the BO rest state in mV
    u0, w0 = IonicModel("bo").initial(mesh.n_nodes)
    mixed.set_state(85.7 * u0 - 84.0, None)
    for _ in range(120):
        plain.step()
        mixed.step()
    ref = 85.7 * plain.u - 84.0
    assert np.max(np.abs(ref)) > 10.0                 # an action potential is under way
    assert np.max(np.abs(mixed.u - ref)) < 1e-9 * np.max(np.abs(ref)), np.max(np.abs(mixed.u - ref))


def test_aliev_panfilov_subdomain_in_a_bueno_orovio_field():
    """Same identity between two dimensionless models: an AP subdomain
    covering the slab in a BO-unit field equals the plain AP run mapped by
    u_BO = (100 u_AP - 80 + 84) / 85.7."""
    mesh = W.slab_q1(3.0, 1.5, 1.0, 0.25)
    dims = tuple(mesh.xyz.max(axis=0))
    stim = [W.Stimulus(W.CUBE, (0.0, 0.0, 0.0), 1.5, 50.0, 0.0, 2.0, 0.0)]
    plain = OM.from_spec(_spec(mesh, "ap", "", dims=dims, stim=stim), solver="splu")
    mixed = R.from_spec(_spec(mesh, "bo", "epi", dims=dims, stim=stim), np.zeros(mesh.n_elems, np.int32),
                        [R.Region(model="ap")], solver="splu")
    mixed.set_state((100.0 * plain.u - 80.0 + 84.0) / 85.7, None)
    for _ in range(120):
        plain.step()
        mixed.step()
    ref = (100.0 * plain.u + 4.0) / 85.7
    assert np.max(ref) > 0.5
    assert np.max(np.abs(mixed.u - ref)) < 1e-9 * np.max(np.abs(ref))


def test_two_models_across_an_interface():
    """TTP06 (endo) and a BO border zone in one slab: interface nodes carry
    both states, the load adds both currents in the field's units, and the
    front crosses the interface into the BO half."""
    mesh = W.slab_q1(6.0, 1.0, 0.5, 0.25)
    spec = _spec(mesh, "ttp06", "endo", dims=tuple(mesh.xyz.max(axis=0)))
    mat = W.material_box(mesh, (3.0, 0.0, 0.0), (6.0, 1.0, 0.5), 1)
    o = R.from_spec(spec, mat, [R.Region("endo"), R.Region(model="bo")], solver="splu")
    names = [reg["model"].name for reg in o.regions]
    assert names == ["ttp06", "bo"] and o.regions[1]["w"].shape[0] == 3
    o.run(400)
    at = o.activation_times()
    far = mesh.xyz[:, 0] > 5.5
    assert np.all(np.isfinite(at[far])) and np.all(at[far] < 20.0)
    # the BO half uses its own units: at rest its potential is BO rest in mV
    assert np.all(np.isfinite(o.u))


def test_identical_subdomains_reproduce_one_subdomain_bdf_ionic_scheme():
    """The paper's semi-implicit BDF ionic scheme on three identical
    subdomains reproduces the one-subdomain oracle's BDF scheme."""
    mesh = W.slab_q1(4.0, 2.0, 1.0, 0.25)
    spec = _spec(mesh, bdf=3)
    mat = W.material_layers(mesh, 0, [1.3, 2.6])
    one = OM.from_spec(spec, solver="splu", ionic_scheme="bdf")
    three = R.from_spec(spec, mat, [R.Region("endo")] * 3, solver="splu", ionic_scheme="bdf")
    for _ in range(60):
        one.step()
        three.step()
    assert np.max(np.abs(one.u - three.u)) < 1e-10 * np.max(np.abs(one.u))
    # and differs from the Rush-Larsen run (the scheme is really used)
    rl = R.from_spec(spec, mat, [R.Region("endo")] * 3, solver="splu")
    rl.run(60)
    assert np.max(np.abs(rl.u - three.u)) > 1e-6
