"""Continuous-batching request loop over the simulation pool.

Requests (arrival time, simulation spec) are taken in arrival order.  An
arrived request is set up (FE assembly, operator and state upload:
ep_sim_finalize on the simulation's own stream) by a host worker thread while
the resident simulations keep stepping, once its estimated device footprint
(ep_sim_device_bytes_estimate) fits the HBM budget next to the resident and
in-preparation ones; a request that does not fit waits, and so do all later
ones.  A prepared simulation joins the pool (ep_pool_admit of a finalized
sim: the descriptor is linked into the pool's table, no assembly) as soon as
a slot is free.  Resident simulations advance together `steps_per_tick`
steps at a time (ep_pool_step: one launch per phase over all of them);
finished ones are harvested (ep_pool_poll / ep_pool_release) and their
slots and memory reused.  All time stepping runs in the HIP library; this
loop only schedules.

Time-to-solution of a request = completion time - arrival time (queueing,
setup and stepping included).  `gpu_busy_fraction` is the share of the
loop's wall time spent inside ep_pool_step (the device has work queued from
the call until its last state read), i.e. one minus the time the GPU waits
for the loop.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time
from typing import List

import numpy as np

from . import EP_FP64, Pool, Simulation


@dataclasses.dataclass
class Record:
    rid: int
    n_nodes: int
    n_steps: int
    arrival_s: float
    admit_s: float = float("nan")
    done_s: float = float("nan")
    status: int = 0

    @property
    def tts_s(self):
        return self.done_s - self.arrival_s


def serve(requests, hbm_budget_bytes: int, max_slots: int, precision: int = EP_FP64,
          steps_per_tick: int = 20, device: int = 0, progress=None, on_done=None, prepare_workers: int = 2,
          ionic_fp64=None) -> dict:
    """Run a trace of workloads.Request to completion; returns records and
    aggregates.  on_done(request index, Simulation), if given, is called for
    each finished request before its simulation is freed (to read results).
    ionic_fp64(spec) -> bool, if given, selects the FP64 ionic step per
    request in mixed precision."""
    reqs = sorted(enumerate(requests), key=lambda t: t[1].arrival_s)
    recs: List[Record] = [Record(i, r.spec.mesh.n_nodes, r.spec.n_steps, r.arrival_s) for i, r in reqs]
    by_id = {r.rid: r for r in recs}
    pool = Pool(hbm_budget_bytes, max_slots, precision, device)
    workers = cf.ThreadPoolExecutor(max_workers=max(1, prepare_workers))
    preparing = collections.deque()     # (rid, future, reserved bytes), arrival order
    slot_of = {}
    nxt = 0
    reserved = 0
    busy = 0.0
    peak_bytes = 0
    t0 = time.perf_counter()
    pending = len(reqs)
    last_print = 0.0

    def configure(spec):
        sim = Simulation.from_spec(spec, precision=precision, device=device, finalize=False,
                                   ionic_fp64=bool(ionic_fp64(spec)) if ionic_fp64 else False)
        return sim

    def prepare(sim):
        sim.finalize()
        return sim

    try:
        while pending > 0:
            now = time.perf_counter() - t0
            in_use = pool.info()["bytes_in_use"]
            # start the set-up of arrived requests, in arrival order, while the
            # budget holds them (in-preparation footprints are reserved)
            while nxt < len(reqs) and reqs[nxt][1].arrival_s <= now and len(preparing) < 2 * max(1, prepare_workers):
                rid, rq = reqs[nxt]
                sim = configure(rq.spec)
                need = sim.device_bytes_estimate()
                if in_use + reserved + need > hbm_budget_bytes:
                    sim.close()
                    if in_use == 0 and reserved == 0:
                        raise RuntimeError(f"request {rid} does not fit an empty pool (HBM budget too small)")
                    break
                reserved += need
                preparing.append((rid, workers.submit(prepare, sim), need))
                nxt += 1
            # prepared simulations join the pool in arrival order
            while preparing and preparing[0][1].done():
                rid, fut, need = preparing[0]
                sim = fut.result()
                slot = pool.admit(sim, by_id[rid].n_steps)
                if slot is None:
                    if pool.info()["active"] == 0:
                        raise RuntimeError(f"request {rid} does not fit an empty pool (HBM budget too small)")
                    break                     # no free slot (or its real footprint does not fit yet)
                preparing.popleft()
                reserved -= need
                slot_of[slot] = rid
                by_id[rid].admit_s = time.perf_counter() - t0
                peak_bytes = max(peak_bytes, pool.info()["bytes_in_use"])
            if pool.info()["active"] > 0:
                ts = time.perf_counter()
                pool.step(steps_per_tick)
                busy += time.perf_counter() - ts
            elif preparing:
                cf.wait([preparing[0][1]], timeout=0.05)
            elif nxt < len(reqs):
                time.sleep(max(0.0, min(0.05, reqs[nxt][1].arrival_s - (time.perf_counter() - t0))))
            for slot in pool.poll():
                sim, st = pool.release(slot, allow_error=True)
                rid = slot_of.pop(slot)
                by_id[rid].done_s = time.perf_counter() - t0
                by_id[rid].status = int(st)
                if on_done is not None:
                    on_done(rid, sim)
                sim.close()
                pending -= 1
            if progress and time.perf_counter() - t0 - last_print > 5.0:
                last_print = time.perf_counter() - t0
                progress(f"serve: {len(recs) - pending}/{len(recs)} done at {last_print:.1f} s")
    finally:
        workers.shutdown(wait=True)
        for _, fut, _ in preparing:
            if fut.done() and fut.exception() is None:
                fut.result().close()
        pool.close()
    wall = time.perf_counter() - t0
    makespan = max(r.done_s for r in recs) - min(r.arrival_s for r in recs)
    work = float(sum(r.n_nodes * r.n_steps for r in recs))
    tts = np.array([r.tts_s for r in recs])
    return {
        "records": recs,
        "n_requests": len(recs),
        "node_steps": work,
        "makespan_s": makespan,
        "node_steps_per_s": work / makespan,
        "tts_p50_s": float(np.percentile(tts, 50)),
        "tts_p99_s": float(np.percentile(tts, 99)),
        "tts_mean_s": float(tts.mean()),
        "queue_p50_s": float(np.percentile([r.admit_s - r.arrival_s for r in recs], 50)),
        "gpu_busy_fraction": busy / wall if wall > 0 else None,
        "hbm_budget_bytes": int(hbm_budget_bytes),
        "peak_bytes_in_use": int(peak_bytes),
        "failed": int(sum(1 for r in recs if r.status != 0)),
    }
