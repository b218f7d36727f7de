"""GPU: the N-version slab benchmark (Section "Slab benchmark").

TTP06 epicardium with the printed initial conditions and conductivities, the
1.5 mm corner-cube stimulus of 35.714 mV/ms for 2 ms, BDF2, hexahedra.  This
is the one pin of the TTP06 transcription together with the whole pipeline
(assembly, ICI right-hand side, CG, activation times) at real size.

What the paper fixes and what is checked here:
- the convergence study reports a latest activation time of 42.0 ms (hex) at
  its finest discretization, and the activation time at the far corner P8
  converging to 42-43 ms;
- the latest activation time sits at P8 (the corner opposite the stimulus);
- activation times grow monotonically as the mesh is refined (the coarse
  consistent-mass ICI discretization propagates too fast).
The P8 activation time at dx = 0.1 mm, dt = 0.005 ms and dx = 0.05 mm,
dt = 0.005 ms is extrapolated to dx -> 0 assuming second-order spatial
convergence and compared with the printed 42.0 ms within 0.5 ms.  The
dx = 0.1 mm value on its own is about 1.1 ms below the 42-43 ms band the paper
quotes for that resolution; the design notes record that deviation.

Tetrahedra (printed: 41.8 ms at the finest level): the paper's tetrahedral
slabs are unstructured; here the lattice is split with the mirrored Kuhn
pattern, so that no body diagonal is preferred (with every cell split the
same way, all long edges point from the stimulus towards P8 and the front
arrives about 1 ms early at every level).  At the paper's finest time step,
dt = 0.001 ms, dx = 0.1 mm and 0.05 mm are extrapolated to dx -> 0 at second
order and compared with 41.8 ms within 0.5 ms.
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "nversion_slab.json")


def _run_slab(dx, dt, t_end, scheme="rl", kind="hex"):
    import paper_2308_01651_amd as ep
    g = json.load(open(GOLD))
    D = g["conductivity_m2_per_s"]
    # printed conductivities are already divided by chi*C_m; 1 m^2/s = 1e3 mm^2/ms
    phys = W.Physics(D["longitudinal"] * 1e3, D["transversal"] * 1e3, D["normal"] * 1e3, 1.0, 1.0)
    Lx, Ly, Lz = g["domain_mm"]
    if kind == "hex":
        mesh = W.slab_q1(Lx, Ly, Lz, dx)
    else:
        mesh = W.slab_p1(Lx, Ly, Lz, dx, split=kind)
    st = g["stimulus"]
    stim = [W.Stimulus(W.CUBE, tuple(st["center_mm"]), st["edge_mm"], st["amplitude_mV_per_ms"],
                       st["t0_ms"], st["duration_ms"], 0.0)]
    n = int(round(t_end / dt))
    spec = W.SimSpec(mesh, W.uniform_fibers(mesh.n_nodes), phys, "ttp06", "epi", stim, dt, 2, n,
                     1e-10, f"nversion-{kind}-{dx}-{dt}")
    sim = ep.Simulation.from_spec(spec, ionic_scheme=scheme)
    done = 0
    while done < n:
        k = min(n // 4 + 1, n - done)
        sim.step(k)
        done += k
        print(f"nversion {kind} {scheme} dx={dx} dt={dt}: {done * dt:.1f} ms", flush=True)
    at = sim.get_activation_times()
    sim.close()
    p8 = int(np.argmin(np.sum((mesh.xyz - np.array([Lx, Ly, Lz])) ** 2, axis=1)))
    return at, p8


@pytest.mark.parametrize("scheme", ["rl", "bdf"])
def test_nversion_hex_p8_converges_to_printed_value(scheme):
    """Both ionic integrators: Rush-Larsen and the paper's semi-implicit BDF."""
    g = json.load(open(GOLD))
    target = g["latest_activation_converged_ms"]["hex"]
    res = {}
    for dx in (0.1, 0.05):
        at, p8 = _run_slab(dx, 0.005, 46.0, scheme)
        assert np.all(np.isfinite(at)), "some node never activated"
        assert at[p8] == np.nanmax(at), "latest activation is not at the far corner P8"
        res[dx] = float(at[p8])
        print(f"nversion {scheme} hex dx={dx} dt=0.005: AT(P8) = {res[dx]:.3f} ms", flush=True)
    assert res[0.05] > res[0.1], res
    extrapolated = res[0.05] + (res[0.05] - res[0.1]) / 3.0
    print(f"nversion {scheme} hex: extrapolated AT(P8) = {extrapolated:.3f} ms (printed {target} ms)", flush=True)
    assert abs(extrapolated - target) <= 0.5, (res, extrapolated)


def test_nversion_tet_p8_converges_to_printed_value():
    g = json.load(open(GOLD))
    target = g["latest_activation_converged_ms"]["tet"]
    res = {}
    for dx in (0.1, 0.05):
        at, p8 = _run_slab(dx, 0.001, 46.0, "rl", "mirrored")
        assert np.all(np.isfinite(at)), "some node never activated"
        assert at[p8] == np.nanmax(at), "latest activation is not at the far corner P8"
        res[dx] = float(at[p8])
        print(f"nversion tet dx={dx} dt=0.001: AT(P8) = {res[dx]:.3f} ms", flush=True)
    assert res[0.05] > res[0.1], res
    extrapolated = res[0.05] + (res[0.05] - res[0.1]) / 3.0
    print(f"nversion tet: extrapolated AT(P8) = {extrapolated:.3f} ms (printed {target} ms)", flush=True)
    assert abs(extrapolated - target) <= 0.5, (res, extrapolated)
