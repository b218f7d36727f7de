#!/usr/bin/env python3
"""Benchmark: monodomain node-steps/s on one MI355X.

Workload (default): TTP06 endocardial monodomain on the 20 x 7 x 3 mm slab
at h = 0.1 mm (201 x 71 x 31 = 442,401 Q1 nodes), corner-cube stimulus,
BDF2 IMEX, dt = 0.05 ms, Jacobi-PCG to rtol 1e-10.  A step is one full
time step (ionic update, ICI right-hand side, linear solve, activation).
Inputs are synthetic (generated mesh, model initial conditions) and resident
in HBM before timing starts.

Timed: `--warmup` untimed steps, then exactly `--steps` steps bracketed by
device synchronization.  `value` is FP64 plain node-steps/s; the mixed
precision (FP32 ionic + inner CG, FP64 refinement) run of the same workload
is reported beside it.  A second, instrumented pass over the same window
brackets every kernel launch with HIP events for the roofline of the
dominant kernel.  The oracle (FP64 CPU) is timed on a bounded sample of the
same workload in a one-thread subprocess.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _workload(name):
    import workloads as W
    if name == "c1":
        return W.config_c1(h=0.1, n_steps=2000), "ttp06-slab-20x7x3mm-h0.1-442401nodes-bdf2-dt0.05"
    if name == "c1big":
        return W.config_c1(h=0.05, n_steps=200), "ttp06-slab-20x7x3mm-h0.05-3449001nodes-bdf2-dt0.05"
    if name == "c0":
        return W.config_c0(), "ap-slab-20x7x3mm-h0.5-4305nodes-bdf1-dt0.05"
    if name in ("c1q2", "c1q3"):
        # the C1 slab with triquadratic elements of 0.2 mm (the same 442,401
        # nodes) or tricubic elements of 0.3 mm (438,340 nodes)
        c1 = W.config_c1(h=0.1, n_steps=2000)
        mesh = W.slab_q2(20.0, 7.0, 3.0, 0.2) if name == "c1q2" else W.slab_q3(20.0, 7.0, 3.0, 0.3)
        fib = c1.fibers if mesh.n_nodes == c1.mesh.n_nodes else W.uniform_fibers(mesh.n_nodes)
        spec = W.SimSpec(mesh, fib, c1.phys, c1.model, c1.variant, c1.stimuli, c1.dt, c1.bdf, c1.n_steps,
                         c1.rtol, name)
        return spec, f"ttp06-slab-20x7x3mm-{name[2:]}-{mesh.n_nodes}nodes-bdf2-dt0.05"
    raise SystemExit(f"unknown workload {name}")


def kernel_bytes(kind, n, nnz, mixed, nvars_model, fmt="DIA", n_diag=0, pipe=False, ent=0, n_elems=0,
                 mf_cmp=False):
    """Algorithmic HBM bytes per launch of each kernel: every array the kernel
    must touch, read or written once.  The operator counts as stored: the
    symmetric DIA format keeps n_diag diagonals (offsets >= 0) of n values
    and no column indices; SELL keeps a value and a 4-byte column index per
    nonzero.  Gathers of the input vector count once.  pipe: the FP64
    pipelined CG, whose "cg_spmv" is its start kernel (w_0 = A u_0 and
    m_0 = P^-1 w_0: reads z, dinv, writes w, m_0) and whose iteration kernel
    "cg_pipe" reads m (gathered), dinv, z, w, p, s, x, r and writes z, s, p,
    x, r, w, m'.  MF (matrix-free, ent = element-node entries over n_elems
    elements): an operator application reads per entry the gathered x and
    the node index and writes the element result (20 B), plus 7 geometry
    factors per entry (56 B) or, compressed (mf_cmp), 7 constants per
    element; the node sums read each result with its 4-byte entry index
    (12 B); the mass-only application of the rhs reads 1 geometry factor per
    entry, or 1 constant per element compressed."""
    if fmt == "MF":
        geo7 = 56 * (n_elems if mf_cmp else ent)
        geo1 = 8 * (n_elems if mf_cmp else ent)
        if kind in ("cg_spmv", "cg_pipe"):
            return 32 * ent + geo7 + n * (24 if kind == "cg_spmv" else 112)
        if kind == "rhs":
            return (20 + 20 + 24) * ent + geo1 + geo7 + n * 48
    def mat(vb):
        return n_diag * n * vb if fmt == "DIA" else nnz * (vb + 4)
    if kind == "cg_pipe":
        # FP32 inner form: FP32 operator and vectors, the solution in FP64
        return mat(4) + n * 68 if mixed else mat(8) + n * 120
    if kind == "cg_spmv" and pipe:
        return mat(4) + n * 16 if mixed else mat(8) + n * 32
    if kind == "cg_spmv":
        return mat(4 if mixed else 8) + n * (8 if mixed else 16)
    if kind == "cg_update":
        return n * (56 if mixed else 96)
    if kind == "rhs":
        return 2 * mat(8) + n * (36 if mixed else 48)
    if kind == "ir_residual":
        return mat(8) + n * 28
    if kind == "ionic":
        if nvars_model == 18:
            return n * (192 if mixed else 320)
        return n * (16 + 2 * nvars_model * (4 if mixed else 8) + 16)
    if kind == "activation":
        return n * 32
    return 0  # cg_finalize: one workgroup, partial sums only


# the device code compiled into the time-step kernels (single-cell pacing and
# the host-side library are not part of what the counter runs measured)
STEP_KERNEL_SOURCES = ("ep_device.h", "ionic_models.h", "kernels.hip")


def _src_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2308_01651_amd", "csrc")
    for f in STEP_KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def _shape_key(kernel_kind, launch):
    """Launch-shape suffix of a counter entry: the tile map of the CG and rhs
    kernels, the nodes per thread of the ionic kernel."""
    if kernel_kind in ("cg_spmv", "cg_update", "rhs", "ir_residual", "cg_pipe", "cg_spmv_pipe_start"):
        return f"@xmap{launch.get('tile_map', 0)}"
    if kernel_kind == "ionic":
        return f"@npt{launch.get('ionic_npt', 1)}"
    return ""


def _counters(name, kernel_kind, precision, workload, launch):
    """Entry of a committed counter summary (profiles/<name>) for this kernel,
    precision, workload and launch shape, or None when there is none for the
    current kernel sources."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None, None
    try:
        d = json.load(open(p))
    except Exception:
        return None, None
    key = f"{workload}:{precision}:{kernel_kind}{_shape_key(kernel_kind, launch)}"
    e = d.get("entries", {}).get(key)
    h = _src_hash()
    if not e or e.get("src_hash", d.get("src_hash")) != h:
        return None, d
    return e, d


def _traffic(kernel_kind, precision, workload, launch):
    """HBM bytes per launch from committed rocprofv3 counter runs (FETCH_SIZE,
    WRITE_SIZE, scaled by the copy-kernel calibration), or None when no run
    exists for the current kernel sources and this launch shape."""
    e, d = _counters("traffic.json", kernel_kind, precision, workload, launch)
    if e is None:
        return None
    f = d.get("copy_calibration", {})
    ff, fw = f.get("fetch_factor"), f.get("write_factor")
    if not ff or not fw:
        return None
    return (e["fetch_kib_per_dispatch"] * ff + e["write_kib_per_dispatch"] * fw) * 1024.0


FP64_VECTOR_TFLOPS, FP32_VECTOR_TFLOPS = 78.6, 157.3


def _alu(kernel_kind, precision, workload, launch, avg_s):
    """ALU roofline of a kernel from committed counter runs: its FP64 and FP32
    flops per launch (SQ_INSTS_VALU_FLOPS_* x 64 lanes) over the live average
    launch duration, against the vector peaks, and the VALU busy share the
    counter run measured; None without a run for the current sources."""
    e, _ = _counters("valu.json", kernel_kind, precision, workload, launch)
    if e is None:
        return None
    r64 = e["fp64_flops_per_dispatch"] / avg_s / 1e12
    r32 = e["fp32_flops_per_dispatch"] / avg_s / 1e12
    return {"bound": "alu", "fp64_TFLOPs": r64, "fp32_TFLOPs": r32,
            "peak": {"fp64": FP64_VECTOR_TFLOPS, "fp32": FP32_VECTOR_TFLOPS}, "unit": "TFLOP/s",
            "frac": r64 / FP64_VECTOR_TFLOPS + r32 / FP32_VECTOR_TFLOPS,
            "valu_busy_counters": e["valu_busy_pct"] / 100.0,
            "flops_per_launch": e["fp64_flops_per_dispatch"] + e["fp32_flops_per_dispatch"]}


TUNE_TRIAL = 3   # steps per candidate launch shape (the tuner runs 5 candidates)
TUNE_TRIAL_POOL = 8   # the same for the batched pool, whose step times vary more between candidates


def _warm(sim, ep, warmup, graph, autotune, make_scratch):
    """Untimed: the launch-shape tuner on a scratch copy of the simulation
    (make_scratch() builds it; the tuner steps it 5 x TUNE_TRIAL times), then
    the tuned shapes and graph capture on `sim` and `warmup` steps (at least
    two with graphs, so that capture does not fall in the timed region).  The
    timed steps of `sim` are then steps warmup + 1 onwards.  Returns the
    launch settings and the steps taken."""
    launch = {"ionic_npt": 1, "tile_map": 0, "graph": bool(graph), "tuned": False}
    if autotune:
        scratch = make_scratch()
        npt, tmap = scratch.autotune(TUNE_TRIAL)
        scratch.close()
        sim.set_option(ep.EP_OPT_IONIC_NPT, npt)
        sim.set_option(ep.EP_OPT_TILE_MAP, tmap)
        launch.update(ionic_npt=npt, tile_map=tmap, tuned=True, tuning_steps=5 * TUNE_TRIAL,
                      tuned_on="scratch copy")
    if graph:
        sim.set_option(ep.EP_OPT_GRAPH, 1)
    w = max(2, warmup) if graph else max(0, warmup)
    if w:
        sim.step(w)
    sim.sync()
    return launch, w


def run_gpu(spec, precision, steps, warmup, instrument_steps, graph=True, autotune=True, ionic_scheme="rl",
            material=None, regions=None, matrix_format=0, cg_variant=0, initial_guess=0):
    import paper_2308_01651_amd as ep
    import torch

    def make():
        return ep.Simulation.from_spec(spec, precision=precision, ionic_scheme=ionic_scheme, material=material,
                                       regions=regions, matrix_format=matrix_format, cg_variant=cg_variant,
                                       initial_guess=initial_guess)
    sim = make()
    st0 = sim.get_stats()
    launch, pre_steps = _warm(sim, ep, warmup, graph, autotune, make)
    torch.cuda.synchronize()
    it0 = sim.get_stats()["cg_iters_total"]
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        sim.step(1)
        lat.append(time.perf_counter() - a)
    sim.sync()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    st = sim.get_stats()
    u_end = sim.get_potential()
    at_end = sim.get_activation_times()
    res = {
        "seconds": T,
        "node_steps_per_s": spec.mesh.n_nodes * steps / T,
        "ms_per_step": 1e3 * T / steps,
        "step_latency_ms_p50": 1e3 * float(np.percentile(lat, 50)),
        "step_latency_ms_p99": 1e3 * float(np.percentile(lat, 99)),
        "cg_iters_per_step": (st["cg_iters_total"] - it0) / steps,
        "ir_sweeps_total": st["ir_sweeps_total"],
        "rel_residual_last": st["rel_residual_last"],
        "matrix_format": {1: "SELL", 2: "DIA", 3: "MF"}[st["matrix_format"]],
        "n_diag": st["n_diag"],
        "mf_compressed": bool(st["mf_compressed"]),
        "nnz": st["nnz"],
        "device_bytes": st["device_bytes"],
        "setup_ms": st0["ms_setup"],
        "launch": launch,
    }
    # kernel durations on the state the timed region ended with: HIP events
    # around back-to-back launches on the sim's stream (SpMV and rhs only:
    # the kernels whose outputs the next step recomputes)
    try:
        res["loop_us"] = {"cg_pipe": sim.time_kernel_us("cg_pipe", 200)}   # pipelined FP64 CG
    except ep.EpError:
        res["loop_us"] = {"cg_spmv": sim.time_kernel_us("cg_spmv", 200)}
    res["loop_us"]["rhs"] = sim.time_kernel_us("rhs", 50)
    sim.close()
    # instrumented pass: a fresh simulation over the same window (same warmup,
    # same steps) with HIP events around every launch, so the per-kernel
    # breakdown describes the timed steps and not a later phase of the beat
    if instrument_steps > 0:
        sim = make()
        sim.set_option(ep.EP_OPT_IONIC_NPT, launch["ionic_npt"])
        sim.set_option(ep.EP_OPT_TILE_MAP, launch["tile_map"])
        sim.step(pre_steps)
        sim.sync()
        sim.set_option(ep.EP_OPT_KERNEL_TIMERS, 1)
        st1 = sim.get_stats()
        it1, prev_it, prev_sw = st1["cg_iters_total"], st1["cg_iters_total"], st1["ir_sweeps_total"]
        per_step_its, per_step_sweeps = [], []
        for _ in range(instrument_steps):
            sim.step(1)
            st1 = sim.get_stats()
            per_step_its.append(st1["cg_iters_total"] - prev_it)
            per_step_sweeps.append(st1["ir_sweeps_total"] - prev_sw)
            prev_it, prev_sw = st1["cg_iters_total"], st1["ir_sweeps_total"]
        sim.sync()
        kt = sim.get_kernel_times()
        # CG iterations per step (mixed: inner FP32 iterations summed over the
        # step's refinement sweeps) and refinement sweeps per step
        res["cg_iters_histogram"] = {str(k): int(v) for k, v in zip(*np.unique(per_step_its, return_counts=True))}
        if precision == ep.EP_MIXED:
            res["ir_sweeps_histogram"] = {str(k): int(v)
                                          for k, v in zip(*np.unique(per_step_sweeps, return_counts=True))}
        res["event_pair_overhead_us"] = sim.timer_overhead_us(500)
        res["instrumented_steps"] = instrument_steps
        res["instrumented_cg_iters"] = sim.get_stats()["cg_iters_total"] - it1
        res["kernel_ms"] = {k: v[0] for k, v in kt.items()}
        res["kernel_launches"] = {k: v[1] for k, v in kt.items()}
        sim.close()
    return res, u_end, at_end


def roofline(res, spec, precision_name, workload_key):
    """Roofline of the dominant kernel (most time in the instrumented pass).

    Per-launch duration: for the SpMV and rhs kernels, HIP events around 200
    (50) back-to-back launches on the state the timed region ended with;
    otherwise the instrumented pass's per-launch events divided by the
    launches that did work (FP64: SpMV = CG iterations + one per step, update
    = CG iterations; launches after convergence return at once and their time
    is charged to the working ones).  The per-launch event durations carry
    the events' own cost (an empty pair is measured and reported beside)."""
    launch = res.get("launch", {})
    n = spec.mesh.n_nodes
    nnz = res["nnz"]
    mixed = precision_name == "mixed"
    nv = {"ttp06": 18, "bo": 3, "ap": 1, "passive": 0}[spec.model]
    ms = res["kernel_ms"]
    cnt = res["kernel_launches"]
    ovh = res.get("event_pair_overhead_us", 0.0)
    work = dict(cnt)
    pipe = cnt.get("cg_pipe", 0) > 0
    if not mixed:
        its, steps = res["instrumented_cg_iters"], res["instrumented_steps"]
        if pipe:
            work["cg_pipe"] = min(cnt["cg_pipe"], its)
            work["cg_spmv"] = min(cnt["cg_spmv"], steps)
        else:
            work["cg_spmv"] = min(cnt["cg_spmv"], its + steps)
            work["cg_update"] = min(cnt["cg_update"], its)
    kinds = [k for k in ms if cnt[k] > 0]
    dom = max((k for k in kinds if k != "cg_finalize"), key=lambda k: ms[k])
    # n_diag counts the operator's diagonals; the symmetric DIA stores the (n_diag + 1) / 2 with offset >= 0
    fmt, nd = res["matrix_format"], (int(res["n_diag"]) + 1) // 2
    ent, n_el, cmp = int(spec.mesh.conn.size), int(spec.mesh.conn.shape[0]), bool(res.get("mf_compressed"))
    bytes_per = kernel_bytes(dom, n, nnz, mixed, nv, fmt, nd, pipe, ent, n_el, cmp)
    raw_s = ms[dom] / 1e3 / work[dom]
    loop = res.get("loop_us", {})
    avg_s = 1e-6 * loop[dom] if dom in loop else raw_s
    achieved = bytes_per / avg_s / 1e9
    per_kernel = {}
    for k in kinds:
        b = kernel_bytes(k, n, nnz, mixed, nv, fmt, nd, pipe, ent, n_el, cmp)
        a = ms[k] / 1e3 / work[k]
        per_kernel[k] = {"avg_us_events": 1e6 * a, "launches": cnt[k], "launches_with_work": work[k],
                         "share": ms[k] / sum(ms.values()), "GBps_events": b / a / 1e9 if b else None,
                         "algo_bytes": b}
        if k in loop:
            per_kernel[k]["avg_us_loop"] = loop[k]
            per_kernel[k]["GBps_loop"] = b / (1e-6 * loop[k]) / 1e9
        # the pipelined solve's "cg_spmv" launches are its start kernel
        ck = "cg_spmv_pipe_start" if (pipe and k == "cg_spmv") else k
        t = _traffic(ck, precision_name, workload_key, launch)
        if t is not None:
            per_kernel[k]["traffic"] = t
        al = _alu(ck, precision_name, workload_key, launch, 1e-6 * per_kernel[k].get("avg_us_loop", 1e6 * a))
        if al is not None:
            per_kernel[k]["alu"] = al
    tr = _traffic(dom, precision_name, workload_key, launch)
    return {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": tr, "algo_bytes_per_launch": bytes_per,
            "avg_launch_us": 1e6 * avg_s, "avg_launch_us_events": 1e6 * raw_s, "event_pair_overhead_us": ovh,
            "duration_source": "back-to-back launches" if dom in loop else "per-launch events",
            "launches": cnt[dom], "launches_with_work": work[dom]}, per_kernel


def run_batched(specs, precision, steps, warmup, graph=True, autotune=True):
    """All instances resident in one pool, stepped together (one launch per phase)."""
    import paper_2308_01651_amd as ep
    import torch
    pool = ep.Pool(200 << 30, len(specs), precision)
    sims = []
    t0 = time.perf_counter()
    for sp in specs:
        s = ep.Simulation.from_spec(sp, precision=precision, finalize=False)
        if pool.admit(s, 5 * TUNE_TRIAL_POOL + max(2, warmup) + steps + 1) is None:
            raise RuntimeError("batched instance did not fit the pool")
        sims.append(s)
    setup = time.perf_counter() - t0
    launch = {"ionic_npt": 1, "tile_map": 0, "graph": bool(graph), "tuned": False}
    if autotune:
        npt, tmap = pool.autotune(TUNE_TRIAL_POOL)
        launch.update(ionic_npt=npt, tile_map=tmap, tuned=True, tuning_steps=5 * TUNE_TRIAL_POOL)
    if graph:
        pool.set_option(ep.EP_OPT_GRAPH, 1)
    pool.step(max(2, warmup))
    torch.cuda.synchronize()
    it0 = sum(s.get_stats()["cg_iters_total"] for s in sims)
    t0 = time.perf_counter()
    pool.step(steps)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    n_tot = sum(sp.mesh.n_nodes for sp in specs)
    its = (sum(s.get_stats()["cg_iters_total"] for s in sims) - it0) / (steps * len(sims))
    fields = [(s.get_state()[0], s.get_activation_times()) for s in sims]
    for slot in list(pool.sims):
        pool.release(slot)
    for s in sims:
        s.close()
    pool.close()
    return {"instances": len(specs), "total_nodes": n_tot, "steps": steps, "warmup": warmup, "seconds": T,
            "node_steps_per_s": n_tot * steps / T, "ms_per_step": 1e3 * T / steps,
            "cg_iters_per_instance_step": its, "setup_s": setup, "launch": launch}, fields


def run_sequential(specs, precision, steps, warmup):
    """The same instances as plain single simulations, one after another
    (each: setup, warmup, then `steps` timed steps); node-steps/s over the
    timed steps of all of them."""
    import paper_2308_01651_amd as ep
    T = 0.0
    work = 0
    for sp in specs:
        s = ep.Simulation.from_spec(sp, precision=precision)
        s.step(max(2, warmup))
        s.sync()
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        T += time.perf_counter() - t0
        work += sp.mesh.n_nodes * steps
        s.close()
    return {"instances": len(specs), "steps_each": steps, "seconds": T, "node_steps_per_s": work / T}


def run_serving(precision, max_slots, trace, budget):
    import paper_2308_01651_amd as ep
    from paper_2308_01651_amd import serve
    # mixed precision: Bueno-Orovio requests keep their ionic step in FP64
    # (its FP32 step misses the 1e-3 mV bar on the ventricle, measured)
    out = serve.serve(trace, budget, max_slots, precision, steps_per_tick=20,
                      progress=lambda m: print("[bench] " + m, file=sys.stderr, flush=True),
                      ionic_fp64=lambda spec: spec.model == "bo")
    out.pop("records")
    return out


CPU_SAMPLE = r"""
import json, os, sys, time
sys.path.insert(0, {root!r})
import workloads as W
from oracle import monodomain as OM
spec = W.config_c1(h={h}, n_steps=1)
o = OM.from_spec(spec, solver="cg", rtol=spec.rtol)
o.step()                      # untimed first step
budget = {budget}
t0 = time.perf_counter(); k = 0
while True:
    o.step(); k += 1
    if time.perf_counter() - t0 > budget and k >= 3:
        break
T = time.perf_counter() - t0
import numpy as np
np.save({out!r}, np.stack([o.potential_mv(), o.activation_times()]))
print(json.dumps({{"steps": k, "seconds": T, "n": spec.mesh.n_nodes}}))
"""


def cpu_baseline(h, budget_s):
    """Time the oracle on a bounded sample (one thread); also returns its
    potential and activation times after the sample for the parity check."""
    import tempfile
    env = dict(os.environ)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[v] = "1"
    fd, out = tempfile.mkstemp(suffix=".npy")
    os.close(fd)
    code = CPU_SAMPLE.format(root=ROOT, h=h, budget=budget_s, out=out)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=900)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}, None, 0
    d = json.loads(r.stdout.strip().splitlines()[-1])
    fields = np.load(out)
    os.unlink(out)
    return ({"value": d["n"] * d["steps"] / d["seconds"], "unit": "node-steps/s", "cores": 1, "kind": "oracle",
             "sample": f"steps 2..{d['steps'] + 1} of the same {d['n']}-node TTP06 slab from rest "
                       f"(FP64 NumPy/SciPy, Jacobi-PCG to rtol 1e-10, one thread), {d['seconds']:.1f} s"},
            fields, d["steps"] + 1)


def oracle_check(spec, fields, steps):
    """The GPU path over the oracle sample's steps from rest, both precisions:
    error of the potential and of the activation times against the oracle."""
    import paper_2308_01651_amd as ep
    out = {"steps": steps}
    u_o, at_o = fields
    for name, prec in (("fp64", ep.EP_FP64), ("mixed", ep.EP_MIXED)):
        sim = ep.Simulation.from_spec(spec, precision=prec)
        sim.step(steps)
        u, at = sim.get_potential(), sim.get_activation_times()
        sim.close()
        du = u - u_o
        ok = ~np.isnan(at_o) & ~np.isnan(at)
        out[name] = {"rel_l2": float(np.linalg.norm(du) / np.linalg.norm(u_o)),
                     "rms_mV": float(np.sqrt(np.mean(du * du))), "max_abs_mV": float(np.max(np.abs(du))),
                     "activated_equal": bool(np.array_equal(np.isnan(at_o), np.isnan(at))),
                     "max_abs_dAT_ms": float(np.max(np.abs(at[ok] - at_o[ok]))) if ok.any() else None}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--instrument-steps", type=int, default=-1,
                    help="length of the event-instrumented region (default: same as --steps)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2000)
    ap.add_argument("--sequential-steps", type=int, default=200,
                    help="timed steps per instance of the sequential plain-FP64 run of the batched workload")
    ap.add_argument("--serve-budget-gib", type=float, default=1.0,
                    help="HBM budget of the serving pool (binds: the trace's concurrent requests need more)")
    ap.add_argument("--graph", type=int, default=0, choices=[0, 1],
                    help="replay the step from captured HIP graphs (measured slower than eager "
                         "launches on ROCm 7.2; the graph variant is reported beside the main run)")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="pick launch shapes with the library's tuner during warmup")
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-full", action="store_true",
                    help="the configured trace: 128 requests, 1e4-1e6 nodes, 50-500 ms (long)")
    ap.add_argument("--matrix-format", default="auto", choices=["auto", "sell", "dia", "mf"],
                    help="operator storage of the main runs (mf: matrix-free, hexahedra of degree 2 or 3)")
    ap.add_argument("--no-variants", action="store_true",
                    help="only the main runs (no launch, solver, scheme or subdomain variants)")
    ap.add_argument("--no-element-variants", action="store_true",
                    help="skip the quadratic-element variants (their SELL SpMV launches share the kernel "
                         "instantiation of the C1 SpMV and would mix into its profile)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 512 MiB five times (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 8, "copies": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the time step runs on one GPU per simulation; sharding a mesh over several "
                                   "GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import paper_2308_01651_amd as ep
    spec, wname = _workload(args.workload)
    instr = args.steps if args.instrument_steps < 0 else args.instrument_steps
    out = {}
    fields = {}
    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    for pn in precs:
        print(f"[bench] {wname} {pn}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
        fmt = {"auto": 0, "sell": ep.EP_FMT_SELL, "dia": ep.EP_FMT_DIA, "mf": ep.EP_FMT_MF}[args.matrix_format]
        res, u, at = run_gpu(spec, ep.EP_FP64 if pn == "fp64" else ep.EP_MIXED, args.steps, args.warmup, instr,
                             bool(args.graph), bool(args.autotune), matrix_format=fmt)
        if instr > 0:
            rl, pk = roofline(res, spec, pn, args.workload)
            res["roofline"] = rl
            res["per_kernel"] = pk
        else:
            rl = {"kernel": None, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": None, "traffic": None}
            res["roofline"] = rl
        out[pn] = res
        fields[pn] = (u, at)
        print(f"[bench] {pn}: {res['node_steps_per_s']:.4g} node-steps/s, {res['ms_per_step']:.3f} ms/step, "
              f"dominant {rl['kernel']} {rl['achieved']} GB/s", file=sys.stderr, flush=True)
    if "fp64" in out and not args.no_variants:
        # the same run with the default launches (eager, untuned) and with graph replay, for comparison
        import workloads as W
        # three transmural TTP06 layers (endocardial, mid-myocardial,
        # epicardial thirds of the slab thickness), one subdomain each
        zmax = float(spec.mesh.xyz[:, 2].max())
        layers = W.material_layers(spec.mesh, 2, [zmax / 3, 2 * zmax / 3])
        layer_regions = {0: dict(variant="endo"), 1: dict(variant="mid"), 2: dict(variant="epi")}
        for name, g, t, sch, mat, regs, cgv, x0 in (
                ("fp64_default_launches", False, False, "rl", None, None, 0, 0),
                ("fp64_graph_replay", True, bool(args.autotune), "rl", None, None, 0, 0),
                ("fp64_chronopoulos_gear_cg", bool(args.graph), bool(args.autotune), "rl", None, None, 2, 0),
                ("fp64_extrapolated_initial_guess", bool(args.graph), bool(args.autotune), "rl", None, None, 0, 1),
                ("fp64_paper_bdf_ionic_scheme", bool(args.graph), bool(args.autotune), "bdf", None, None, 0, 0),
                ("fp64_three_cell_layers", bool(args.graph), bool(args.autotune), "rl", layers, layer_regions, 0, 0)):
            if g == bool(args.graph) and t == bool(args.autotune) and sch == "rl" and mat is None and cgv == 0 \
                    and x0 == 0:
                continue
            r0, _, _ = run_gpu(spec, ep.EP_FP64, args.steps, args.warmup, 0, g, t, sch, mat, regs, cg_variant=cgv,
                               initial_guess=x0)
            out[name] = {k: r0[k] for k in ("node_steps_per_s", "ms_per_step", "cg_iters_per_step", "step_latency_ms_p50",
                                            "step_latency_ms_p99", "launch")}
            print(f"[bench] {name}: {r0['node_steps_per_s']:.4g} node-steps/s", file=sys.stderr, flush=True)
        if args.workload == "c1" and not args.no_element_variants:
            # triquadratic elements on the same node lattice (element size 0.2 mm:
            # 100 x 35 x 15 elements, 201 x 71 x 31 nodes), operator in sliced ELL,
            # quadratic tetrahedra (each cell Kuhn-split) on the same lattice, and
            # tricubic elements of 0.3 mm (67 x 23 x 10 elements, 202 x 70 x 31
            # nodes: the C1 node count within 1 %)
            for name, gen, h, fmt in (("fp64_q2_elements_same_nodes", W.slab_q2, 0.2, 0),
                                      ("fp64_q2_matrix_free_same_nodes", W.slab_q2, 0.2, ep.EP_FMT_MF),
                                      ("fp64_p2_elements_same_nodes", W.slab_p2, 0.2, 0),
                                      ("fp64_q3_elements_438k_nodes", W.slab_q3, 0.3, 0),
                                      ("fp64_q3_matrix_free_438k_nodes", W.slab_q3, 0.3, ep.EP_FMT_MF)):
                mesh = gen(20.0, 7.0, 3.0, h)
                fib = spec.fibers if mesh.n_nodes == spec.mesh.n_nodes else W.uniform_fibers(mesh.n_nodes)
                hi = W.SimSpec(mesh, fib, spec.phys, spec.model, spec.variant,
                               spec.stimuli, spec.dt, spec.bdf, spec.n_steps, spec.rtol, name)
                r0, _, _ = run_gpu(hi, ep.EP_FP64, args.steps, args.warmup, 0, bool(args.graph), bool(args.autotune),
                                   matrix_format=fmt)
                out[name] = {k: r0[k] for k in (
                    "node_steps_per_s", "ms_per_step", "step_latency_ms_p50", "step_latency_ms_p99", "launch",
                    "cg_iters_per_step", "matrix_format", "nnz", "device_bytes")}
                print(f"[bench] {name}: {r0['node_steps_per_s']:.4g} node-steps/s, "
                      f"{r0['cg_iters_per_step']:.1f} CG its/step, nnz {r0['nnz']}", file=sys.stderr, flush=True)
    if "fp64" in fields and "mixed" in fields:
        du = fields["mixed"][0] - fields["fp64"][0]
        a64, a32 = fields["fp64"][1], fields["mixed"][1]
        ok = ~np.isnan(a64) & ~np.isnan(a32)
        out["mixed"]["vs_fp64"] = {
            "rms_mV": float(np.sqrt(np.mean(du ** 2))), "max_abs_mV": float(np.max(np.abs(du))),
            "max_abs_dAT_ms": float(np.max(np.abs(a64[ok] - a32[ok]))) if ok.any() else None,
            "activated_nodes_equal": bool(np.array_equal(np.isnan(a64), np.isnan(a32)))}
    import workloads as W
    batched = None
    if not args.no_batched and args.workload == "c1":
        specs = W.config_c3()
        batched = {}
        bf = {}
        for pn in ("fp64", "mixed"):
            print(f"[bench] batched: 64 slab instances, {pn}", file=sys.stderr, flush=True)
            r, f = run_batched(specs, ep.EP_FP64 if pn == "fp64" else ep.EP_MIXED, args.batched_steps, 20,
                               bool(args.graph), bool(args.autotune))
            batched[pn] = r
            bf[pn] = f
            print(f"[bench] batched {pn}: {r['node_steps_per_s']:.4g} node-steps/s", file=sys.stderr, flush=True)
        d2 = [float(np.mean((a[0] - b[0]) ** 2)) for a, b in zip(bf["fp64"], bf["mixed"])]
        mv = [100.0 if sp.model == "ap" else 1.0 for sp in specs]   # mV per model unit
        rms = float(np.sqrt(np.mean([d * m * m for d, m in zip(d2, mv)])))
        dat = []
        for a, b in zip(bf["fp64"], bf["mixed"]):
            ok = ~np.isnan(a[1]) & ~np.isnan(b[1])
            if ok.any():
                dat.append(float(np.max(np.abs(a[1][ok] - b[1][ok]))))
        batched["mixed"]["vs_fp64"] = {"rms_mV": rms, "max_abs_dAT_ms": max(dat) if dat else None}
        # the same 64 instances as plain FP64 single simulations, one after
        # another: the batched forms against the plain form on one workload
        print("[bench] batched: the same instances as sequential plain FP64 sims", file=sys.stderr, flush=True)
        batched["sequential_fp64"] = run_sequential(specs, ep.EP_FP64, args.sequential_steps, 5)
        print(f"[bench] sequential fp64: {batched['sequential_fp64']['node_steps_per_s']:.4g} node-steps/s",
              file=sys.stderr, flush=True)
    serving = None
    if not args.no_serve and args.workload == "c1":
        nreq, nmax, tmin, tmax = ((128, 1e6, 50.0, 500.0) if args.serve_full
                                  else (args.serve_requests, 3e5, 50.0, 200.0))
        trace = W.serving_trace(seed=5, n_req=nreq, rate_per_s=4.0, n_min=1e4, n_max=nmax,
                                t_min=tmin, t_max=tmax)
        offered = sum(r.spec.mesh.n_nodes * r.spec.n_steps for r in trace) / max(r.arrival_s for r in trace)
        serving = {"trace": {"requests": nreq, "rate_per_s": 4.0, "nodes": [1e4, nmax],
                             "simulated_ms": [tmin, tmax], "models": "ttp06|bo", "geometry": "slab|lv",
                             "seed": 5, "offered_node_steps_per_s": offered}}
        print("[bench] serving: continuous batching, mixed precision", file=sys.stderr, flush=True)
        budget = int(args.serve_budget_gib * (1 << 30))
        serving["batched_mixed"] = run_serving(ep.EP_MIXED, 32, trace, budget)
        print("[bench] serving: sequential plain FP64", file=sys.stderr, flush=True)
        serving["sequential_fp64"] = run_serving(ep.EP_FP64, 1, trace, budget)
    cpu = None
    oracle_cmp = None
    if not args.no_cpu_baseline and args.workload in ("c1", "c1big"):
        print("[bench] cpu baseline (oracle, 1 thread)", file=sys.stderr, flush=True)
        cpu, ofields, osteps = cpu_baseline(spec.mesh.xyz[1, 0] - spec.mesh.xyz[0, 0], args.cpu_budget)
        if ofields is not None:
            oracle_cmp = oracle_check(spec, ofields, osteps)
            print(f"[bench] oracle check over {osteps} steps: fp64 rel L2 {oracle_cmp['fp64']['rel_l2']:.2e}, "
                  f"mixed RMS {oracle_cmp['mixed']['rms_mV']:.2e} mV", file=sys.stderr, flush=True)
    main_res = out["fp64"] if "fp64" in out else out["mixed"]
    line = {
        "metric": "monodomain node-steps/s (TTP06, 442k nodes) plain vs batched/FP32; p99 latency",
        "value": main_res["node_steps_per_s"],
        "unit": "node-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if "fp64" in out else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wname, "n_nodes": spec.mesh.n_nodes, "model": spec.model,
                   "variant": spec.variant, "bdf": spec.bdf, "dt_ms": spec.dt, "rtol": spec.rtol,
                   "precision": "fp64" if "fp64" in out else "mixed", "parallelism": "single-gpu"},
        "p50_step_latency_ms": main_res["step_latency_ms_p50"],
        "p99_step_latency_ms": main_res["step_latency_ms_p99"],
        "roofline": {k: main_res["roofline"][k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernel": main_res["roofline"]["kernel"],
        "roofline_detail": {k: main_res["roofline"].get(k) for k in ("algo_bytes_per_launch", "avg_launch_us",
                                                                      "duration_source",
                                                                      "avg_launch_us_events", "event_pair_overhead_us",
                                                                      "launches", "launches_with_work")},
        "cpu_baseline": cpu,
        "oracle_check": oracle_cmp,
        "variants": out,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
