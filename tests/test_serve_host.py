"""Host logic of the continuous-batching loop (`serve.serve`) with the pool
and the simulations replaced by bookkeeping stand-ins (CPU only): every
request finishes, in-use device bytes never exceed the budget, requests join
the pool in arrival order, time-to-solution accounts for queueing, and a
request larger than an empty pool's budget is refused with an error."""
import types

import pytest

from paper_2308_01651_amd import serve

BYTES_PER_NODE = 100


class FakeSim:
    def __init__(self, spec):
        self.n = spec.mesh.n_nodes
        self.finalized = False
        self.closed = False

    @classmethod
    def from_spec(cls, spec, **kw):
        return cls(spec)

    def device_bytes_estimate(self):
        return self.n * BYTES_PER_NODE

    def finalize(self):
        self.finalized = True

    def close(self):
        self.closed = True


class FakePool:
    log = None

    def __init__(self, budget, max_slots, precision, device=0):
        self.budget, self.max_slots = budget, max_slots
        self.slots = {}              # slot -> [sim, steps left]
        self.peak = 0
        self.admitted = []
        FakePool.log = self

    def info(self):
        return {"bytes_in_use": sum(s.device_bytes_estimate() for s, _ in self.slots.values()),
                "active": sum(1 for _, left in self.slots.values() if left > 0)}

    def admit(self, sim, n_steps):
        assert sim.finalized
        if len(self.slots) >= self.max_slots:
            return None
        if self.info()["bytes_in_use"] + sim.device_bytes_estimate() > self.budget:
            return None
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = [sim, n_steps]
        self.admitted.append(sim)
        self.peak = max(self.peak, self.info()["bytes_in_use"])
        return slot

    def step(self, k):
        for v in self.slots.values():
            v[1] = max(0, v[1] - k)

    def poll(self):
        return [s for s, (_, left) in self.slots.items() if left == 0]

    def release(self, slot, allow_error=False):
        sim, _ = self.slots.pop(slot)
        return sim, 0

    def close(self):
        pass


def _req(t, n, steps):
    mesh = types.SimpleNamespace(n_nodes=n)
    return types.SimpleNamespace(arrival_s=t, spec=types.SimpleNamespace(mesh=mesh, n_steps=steps))


@pytest.fixture
def fakes(monkeypatch):
    monkeypatch.setattr(serve, "Pool", FakePool)
    monkeypatch.setattr(serve, "Simulation", FakeSim)


def test_every_request_finishes_within_the_budget(fakes):
    sizes = [300, 1200, 500, 800, 100, 900, 700, 400, 600, 200]
    reqs = [_req(0.002 * i, n, 40 + 20 * (i % 3)) for i, n in enumerate(sizes)]
    budget = 1500 * BYTES_PER_NODE
    done = []
    out = serve.serve(reqs, budget, 3, steps_per_tick=20, on_done=lambda rid, sim: done.append(rid))
    pool = FakePool.log
    assert out["n_requests"] == len(reqs) and out["failed"] == 0
    assert sorted(done) == list(range(len(reqs)))
    assert pool.peak <= budget and out["peak_bytes_in_use"] <= budget
    # joined in arrival order (the loop never lets a later request pass one that waits)
    assert [s.n for s in pool.admitted] == sizes
    assert all(r.tts_s >= r.admit_s - r.arrival_s >= 0 for r in out["records"])
    assert out["node_steps"] == sum(r.n_nodes * r.n_steps for r in out["records"])


def test_request_larger_than_an_empty_pool_is_refused(fakes):
    reqs = [_req(0.0, 50, 20), _req(0.001, 10_000, 20)]
    with pytest.raises(RuntimeError):
        serve.serve(reqs, 1000 * BYTES_PER_NODE, 2, steps_per_tick=20)
