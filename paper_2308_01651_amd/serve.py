"""Continuous-batching request loop over the simulation pool.

Requests (arrival time, simulation spec) are admitted in arrival order as
soon as they have arrived and the pool has a free slot and HBM budget
(ep_pool_admit; a request that does not fit waits, and so do all later
ones).  Resident simulations advance together `steps_per_tick` steps at a
time (ep_pool_step: one launch per phase over all of them); finished ones are
harvested (ep_pool_poll / ep_pool_release) and their slots reused.  All time
stepping runs in the HIP library; this loop only schedules.

Time-to-solution of a request = completion time - arrival time (queueing,
setup on admission and stepping included).
"""
from __future__ import annotations

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
          steps_per_tick: int = 20, device: int = 0, progress=None, on_done=None) -> dict:
    """Run a trace of workloads.Request to completion; returns records and
    aggregates.  on_done(request index, Simulation), if given, is called for
    each finished request before its simulation is freed (to read results)."""
    reqs = sorted(enumerate(requests), key=lambda t: t[1].arrival_s)
    recs: List[Record] = [Record(i, r.spec.mesh.n_nodes, r.spec.n_steps, r.arrival_s) for i, r in reqs]
    by_id = {r.rid: r for r in recs}
    pool = Pool(hbm_budget_bytes, max_slots, precision, device)
    slot_of = {}
    nxt = 0
    t0 = time.perf_counter()
    pending = len(reqs)
    last_print = 0.0
    while pending > 0:
        now = time.perf_counter() - t0
        # admit in arrival order while requests fit
        while nxt < len(reqs) and reqs[nxt][1].arrival_s <= now:
            rid, rq = reqs[nxt]
            sim = Simulation.from_spec(rq.spec, precision=precision, device=device, finalize=False)
            slot = pool.admit(sim, rq.spec.n_steps)
            if slot is None:
                sim.close()
                if pool.info()["active"] == 0:
                    pool.close()
                    raise RuntimeError(f"request {rid} does not fit an empty pool (HBM budget too small)")
                break
            slot_of[slot] = rid
            by_id[rid].admit_s = time.perf_counter() - t0
            nxt += 1
        if pool.info()["active"] > 0:
            pool.step(steps_per_tick)
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
    pool.close()
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
        "failed": int(sum(1 for r in recs if r.status != 0)),
    }
