"""Pins of the oracle's applied current (its spatial profiles and its pulse
timing) against counts and integrals that follow from the definitions.

- a cube at a lattice corner covers (edge / h + 1)^3 nodes; a ball's nodes
  are the integer triples within r / h, counted exactly in integers;
- the mass-weighted load of a Gaussian profile, 1^T M p, is the trilinear
  interpolant's integral, i.e. the product trapezoid rule, whose difference
  from the exact integral over the box is its Euler-Maclaurin leading term
  (fixes the profile's normalization and width and the mass matrix's
  scaling together: a std off by a factor sqrt(2) moves the load by 65 %);
- a pulse train is on exactly in the windows (t0 + k T, t0 + k T + dur],
  listed pulse by pulse.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fem
from oracle import monodomain as OM


def test_corner_cube_covers_the_lattice_block():
    for h, edge in ((0.25, 1.5), (0.5, 1.5), (0.1, 1.0)):
        m = W.slab_q1(4.0, 3.0, 2.0, h)
        st = W.corner_cube_stimulus(edge=edge, dims=(4.0, 3.0, 2.0))
        p = OM.stimulus_profile(st.shape, st.center, st.size, m.xyz)
        k = int(round(edge / h)) + 1
        assert set(np.unique(p)) <= {0.0, 1.0}
        assert int(p.sum()) == k ** 3, (h, edge, int(p.sum()))
        inside = np.all(m.xyz <= edge + 1e-9, axis=1)
        assert np.array_equal(p > 0, inside)


def test_sphere_nodes_are_the_integer_triples_in_the_ball():
    h, r = 0.25, 1.1
    m = W.slab_q1(4.0, 4.0, 4.0, h)
    c = (2.0, 2.0, 2.0)
    p = OM.stimulus_profile(W.SPHERE, c, r, m.xyz)
    R = int(r / h) + 1
    lim = (r / h) ** 2
    count = sum(1 for i in range(-R, R + 1) for j in range(-R, R + 1) for k in range(-R, R + 1)
                if i * i + j * j + k * k <= lim + 1e-9)
    assert int(p.sum()) == count


def _gauss_load(h, s=1.0, L=10.0, amp=3.0):
    m = W.slab_q1(L, L, L, h)
    f, sv, n = W.uniform_fibers(m.n_nodes)
    M, _ = fem.assemble(m.xyz, m.conn, fem.nodal_diffusion(f, sv, n, 0.1, 0.1, 0.1, 1.0, 1.0))
    p = amp * OM.stimulus_profile(W.GAUSS, (L / 2, L / 2, L / 2), s, m.xyz)
    return float(np.ones(m.n_nodes) @ (M @ p))


def test_gaussian_load_matches_its_integral_to_the_trapezoid_error():
    """Q1 on a uniform lattice integrates the interpolant by the product
    trapezoid rule; for the Gaussian on the box [0, L]^3 its error is, to
    leading order (Euler-Maclaurin), h^2 / 12 (f'(b) - f'(a)) per axis
    relative to that axis's integral, three times over."""
    from math import erf, exp, pi, sqrt
    s, amp, L = 1.0, 3.0, 10.0
    b = L / 2
    axis = s * sqrt(2.0 * pi) * erf(b / (sqrt(2.0) * s))      # integral over [-b, b]
    exact = amp * axis ** 3
    dfa = -2.0 * (b / (s * s)) * exp(-b * b / (2.0 * s * s))   # f'(b) - f'(a), f(x) = exp(-x^2 / 2 s^2)
    for h in (0.5, 0.25):
        err = (_gauss_load(h, s, L, amp) - exact) / exact
        pred = 3.0 * (h * h / 12.0) * dfa / axis
        assert abs(err - pred) < 0.15 * abs(pred), (h, err, pred)


def _on_by_listing(t, t0, dur, period):
    """Pulse k covers (t0 + k period, t0 + k period + dur]; list them up to t."""
    k = 0
    while True:
        a = t0 + k * period
        if a >= t or (period <= 0 and k > 0):
            return False
        if t <= a + dur + 1e-12:
            return True
        k += 1


@pytest.mark.parametrize("t0,dur,period", [(0.0, 2.0, 0.0), (1.0, 0.5, 0.0), (0.0, 2.0, 10.0), (3.0, 1.0, 4.5)])
def test_pulse_windows_match_the_listing(t0, dur, period):
    dt = 0.05
    for n in range(1, 1200):
        t = n * dt
        want = _on_by_listing(t, t0, dur, period)
        assert OM.stimulus_active(t, t0, dur, period, dt) == want, (t, t0, dur, period)
