"""GPU: the tetrahedral left-ventricle workload at full size (1,512,000 P1
nodes, 8.7M tetrahedra, Bueno-Orovio EPI, BDF2, five Gaussian endocardial
stimuli; the paper's idealized-ventricle setup, Section "Idealized left
ventricle", on a generated prolate-spheroid shell).

- one step from a near-rest random state, in the launch configuration the
  workload runs in (the operator format the library picks; block-Jacobi 32
  and Jacobi), compared in
  full with the oracle's step (CG to 1e-13);
- 600 steps (30 ms) in mixed precision against FP64: RMS over nodes (held
  against the FP64 run's own sensitivity to its solver tolerance) and the
  threshold-crossing times.  The max-slope activation time is compared too,
  within five steps: where the slope has a nearly flat top (inside the
  stimulated regions the slope is set by the constant applied current for
  2 ms) its argmax is ill-conditioned, and two FP64 runs with different
  preconditioners at rtol 1e-10 already differ by up to five steps.
"""
import numpy as np
import pytest

import workloads as W
from oracle import monodomain as OM

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_c2_full_size_single_step():
    import paper_2308_01651_amd as ep
    spec = W.config_c2(n_steps=1)
    n = spec.mesh.n_nodes
    u, w = W.random_state("bo", n, seed=41)
    u = 0.05 * u                                # mostly near rest, some sub-threshold
    rng = np.random.default_rng(42)
    u_prev = u + 1e-3 * rng.normal(size=n)
    res = {}
    for block in (1, 32):
        sim = ep.Simulation.from_spec(spec, rtol=1e-13, block=block)
        fmt = {ep.EP_FMT_SELL: "SELL", ep.EP_FMT_DIA: "DIA"}[sim.get_stats()["matrix_format"]]
        sim.set_state(u, w, u_prev[None], 3)
        sim.step(1)
        res[block] = sim.get_state()[:2]
        print(f"C2 single step, {fmt}, block {block}: {sim.get_stats()['cg_iters_last']} CG iterations", flush=True)
        sim.close()
    o = OM.from_spec(spec, solver="cg", rtol=1e-13)
    o.set_state(u, w, [u_prev], 3)
    o.step()
    for block, (ug, wg) in res.items():
        assert _rel(ug, o.u) < 1e-10, (block, _rel(ug, o.u))
        for v in range(w.shape[0]):
            assert np.max(np.abs(wg[v] - o.w[v])) <= 1e-11 * max(np.max(np.abs(o.w[v])), 1e-30), (block, v)


def test_c2_full_size_mixed_precision_trajectory():
    """Mixed precision against FP64 over 30 ms.  While the five fronts sweep
    the shell, the potential on a steep BO upstroke turns tiny timing shifts
    into mV: two FP64 runs at rtol 1e-10 and 1e-12 already differ by about
    7e-3 mV RMS at 30 ms, above the 1e-3 mV mixed-precision budget.  The
    potential is therefore held to the larger of 1e-3 mV and ten times that
    FP64-to-FP64 difference, measured in the same run; threshold-crossing
    times to 0.1 ms."""
    import paper_2308_01651_amd as ep
    spec = W.config_c2(n_steps=600)
    ref = ep.Simulation.from_spec(spec)
    tight = ep.Simulation.from_spec(spec, rtol=1e-12)
    mix = ep.Simulation.from_spec(spec, precision=ep.EP_MIXED)
    for k in range(3):
        for s in (ref, tight, mix):
            s.step(200)
        print(f"C2 mixed vs FP64: {(k + 1) * 10} ms", flush=True)
    u_ref = ref.get_potential()
    du = mix.get_potential() - u_ref
    dt_ = tight.get_potential() - u_ref
    rms = float(np.sqrt(np.mean(du * du)))
    rms_fp64 = float(np.sqrt(np.mean(dt_ * dt_)))
    tc_m, tc_r = mix.get_threshold_times(), ref.get_threshold_times()
    at_m, at_r = mix.get_activation_times(), ref.get_activation_times()
    ok = ~np.isnan(tc_r)
    print(f"C2 mixed: rms {rms:.2e} mV (FP64 rtol 1e-12 vs 1e-10: {rms_fp64:.2e} mV), "
          f"{ok.sum()} nodes crossed threshold", flush=True)
    t_end = 600 * spec.dt
    assert ok.sum() > 100000
    assert rms <= max(1e-3, 10.0 * rms_fp64), (rms, rms_fp64)

    def same_times(a, b, tol):
        # nodes activated in one run only must have activated within tol of the end
        both = ~np.isnan(a) & ~np.isnan(b)
        only = np.isnan(a) ^ np.isnan(b)
        late = np.where(np.isnan(a), b, a)[only]
        assert np.all(late >= t_end - tol - 1e-9), np.min(late)
        return np.max(np.abs(a[both] - b[both]))

    assert same_times(tc_m, tc_r, 0.1) <= 0.1
    assert same_times(at_m, at_r, 5 * spec.dt) <= 5 * spec.dt + 1e-9
    for s in (ref, tight, mix):
        s.close()
