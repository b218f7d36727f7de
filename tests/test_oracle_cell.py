"""Pins of the single-cell pacing oracle.

- it equals the monodomain oracle run on a small mesh with a spatially
  uniform state and a stimulus covering the whole mesh (K 1 = 0), beat by
  beat, for both ionic integrators (fixes the reduction, the BDF start-up
  and the periodic stimulus timing);
- cells with different parameter sets evolve independently (vectorization);
- a paced Aliev-Panfilov cell reaches a periodic state: the state at the end
  of consecutive beats converges.
"""
import numpy as np
import pytest

import workloads as W
from oracle import cell as OC
from oracle import monodomain as OM


@pytest.mark.parametrize("model,variant,bdf,scheme", [("ap", "", 2, "rl"), ("bo", "epi", 1, "rl"),
                                                      ("ttp06", "endo", 2, "rl"), ("ttp06", "epi", 2, "bdf")])
def test_pacing_equals_uniform_tissue(model, variant, bdf, scheme):
    period, dur, dt = 20.0, 1.0, 0.05
    amp = 40.0                                          # mV/ms
    m = W.slab_q1(1.0, 1.0, 1.0, 0.5)
    # chi = C_m = 1: the tissue amplitude in uA/mm^3 equals mV/ms
    st = W.Stimulus(W.CUBE, (0.5, 0.5, 0.5), 10.0, amp, 0.0, dur, period)
    o = OM.Monodomain(m.xyz, m.conn, W.uniform_fibers(m.n_nodes), (0.1, 0.01, 0.01), 1.0, 1.0, model, variant,
                      [st], dt, bdf, "dense", ionic_scheme=scheme)
    o.run(int(round(2 * period / dt)))
    u, w = OC.pace(model, variant, 1, dt, period, amp, dur, 2, bdf, ionic_scheme=scheme)
    assert np.allclose(o.u, u[0], rtol=1e-11, atol=1e-12)
    assert np.allclose(o.w, w[:, :1], rtol=1e-10, atol=1e-14)


def test_cells_are_independent():
    params = [{"k": 8.0}, {"k": 7.0}, {"k": 9.0}]
    u3, w3 = OC.pace("ap", "", 3, 0.05, 30.0, 40.0, 1.0, 1, 2, params=params)
    for c in range(3):
        u1, w1 = OC.pace("ap", "", 1, 0.05, 30.0, 40.0, 1.0, 1, 2, params=[params[c]])
        assert u1[0] == u3[c] and np.array_equal(w1[:, 0], w3[:, c])


def test_aliev_panfilov_pacing_reaches_a_periodic_state():
    """At a 1 s period the cell recovers fully between beats; the end-of-beat
    state converges geometrically."""
    u, w = OC.pace("ap", "", 1, 0.1, 1000.0, 40.0, 1.0, 1, 2)
    ends = []
    for _ in range(4):
        u, w = OC.pace("ap", "", 1, 0.1, 1000.0, 40.0, 1.0, 1, 2, u0=u, w0=w)
        ends.append(np.concatenate([u, w[:, 0]]))
    d = [np.max(np.abs(ends[k + 1] - ends[k])) for k in range(3)]
    assert d[0] > d[1] > d[2] and d[2] < 1e-4, d
