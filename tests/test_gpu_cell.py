"""GPU: single-cell pacing (ep_cell_pace) against the oracle's pacing loop,
cells with their own parameter overrides, FP64, two beats (the per-step
arithmetic of both sides agrees to rounding; over 2400 steps the states
must agree to 1e-9 relative); the paced state seeds a tissue run."""
import numpy as np
import pytest

from oracle import cell as OC
from oracle import ionic as I

pytestmark = pytest.mark.gpu

CASES = {
    "ap": ("", ["k", "a", "eps0", "mu1", "mu2", "T"], 0, [8.0, 7.5, 8.5, 9.0, 7.0]),
    "bo": ("epi", list(I.BO_EPI.keys()), 14, [0.11, 0.10, 0.12, 0.115, 0.105]),
    "ttp06": ("endo", I.TTP_PARAM_NAMES, 0, [14.838, 12.0, 16.0, 10.0, 15.0]),
}


@pytest.mark.parametrize("model", ["ap", "bo", "ttp06"])
def test_cell_pace_matches_oracle(model):
    import paper_2308_01651_amd as ep
    variant, names, slot, values = CASES[model]
    n = len(values)
    m = I.IonicModel(model, variant)
    base = [m.p[k] for k in names[: slot + 1]]
    params = np.array([base[:slot] + [v] for v in values])
    dt, period, amp, dur, beats = 0.05, 60.0, 40.0, 1.0, 2
    got = ep.cell_pace(model, variant, n, params=params, dt=dt, bdf=2, period=period, stim_mV_per_ms=amp,
                       stim_dur=dur, n_beats=beats)
    u, w = OC.pace(model, variant, n, dt, period, amp, dur, beats, 2,
                   params=[{names[slot]: v} for v in values])
    ref = np.vstack([u[None, :], w]).T
    scale = np.maximum(np.abs(ref), 1e-6)
    assert np.max(np.abs(got - ref) / scale) < 1e-9, np.max(np.abs(got - ref) / scale)


def test_cell_pace_seeds_a_tissue_run():
    import paper_2308_01651_amd as ep
    import workloads as W
    st = ep.cell_pace("ttp06", "endo", 1, dt=0.05, period=400.0, stim_mV_per_ms=40.0, stim_dur=1.0, n_beats=1)
    assert np.all(np.isfinite(st))
    mesh = W.slab_q1(2.0, 1.0, 1.0, 0.25)
    sim = ep.Simulation()
    sim.upload_mesh(mesh.elem, mesh.xyz, mesh.conn)
    sim.set_conductivity(0.17, 0.019, 0.019, 140.0, 0.01)
    sim.set_ionic_model(ep.EP_TTP06, ep.EP_CELL_ENDO, init_state=st[0])
    sim.set_solver(0.05, 2)
    sim.finalize()
    u, w, _ = sim.get_state()
    assert np.allclose(u, st[0, 0]) and np.allclose(w[:, 0], st[0, 1:])
    sim.step(10)
    assert np.all(np.isfinite(sim.get_potential()))
    sim.close()


def test_cell_pace_rejects_bad_arguments():
    import paper_2308_01651_amd as ep
    with pytest.raises(ep.EpError):
        ep.cell_pace("ap", "", 0)
    with pytest.raises(ep.EpError):
        ep.cell_pace("ap", "", 1, dt=-1.0)
    with pytest.raises(ep.EpError):
        ep.cell_pace("ap", "", 1, params=np.zeros((1, 7)))
