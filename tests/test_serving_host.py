"""Scheduling of the continuous-batching loop, on the CPU with a fake backend
and a simulated clock (no GPU)."""
import dataclasses

from paper_2404_17057_amd import serving as S
from paper_2404_17057_amd import workloads as W


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


@dataclasses.dataclass
class FakePb:
    n_particles: int
    nbytes: int


class FakeSim:
    def __init__(self, pb):
        self.pb = pb
        self.steps = 0


class FakeBackend:
    """Steps cost `cost` seconds per particle-step of the whole batch."""

    def __init__(self, clock, cost=1e-10):
        self.clock = clock
        self.cost = cost
        self.batches = []
        self.live_bytes = 0
        self.max_live = 0
        self.max_slots_seen = 0

    def footprint(self, pb):
        return pb.nbytes

    def create(self, pb):
        self.live_bytes += pb.nbytes
        self.max_live = max(self.max_live, self.live_bytes)
        return FakeSim(pb)

    def step_batch(self, sims, counts):
        self.batches.append([(id(s), c) for s, c in zip(sims, counts)])
        self.max_slots_seen = max(self.max_slots_seen, len(sims))
        for s, c in zip(sims, counts):
            s.steps += c
        self.clock.t += self.cost * sum(s.pb.n_particles * c for s, c in zip(sims, counts))

    def sync(self):
        pass

    def finish(self, sim):
        self.live_bytes -= sim.pb.nbytes
        return f"steps={sim.steps}", 0


def _run(n=60, rate=200.0, budget=64 << 20, slots=8, k=16):
    clock = Clock()
    be = FakeBackend(clock)
    specs = W.request_stream(n=n, rate=rate, seed=7)
    sizes = {}

    def build(spec):
        npart = spec.nx * spec.ny * 4
        sizes[spec.req_id] = npart
        return FakePb(npart, npart * 10)

    srv = S.Server(be, build, hbm_budget=budget, max_slots=slots, steps_per_launch=k,
                   clock=clock, sleep=clock.sleep)
    done = srv.run(specs)
    return specs, done, be, sizes


def test_every_request_completes_with_its_step_count():
    specs, done, be, _ = _run()
    assert sorted(d.req_id for d in done) == [s.req_id for s in specs]
    by = {s.req_id: s for s in specs}
    for d in done:
        assert d.digest == f"steps={by[d.req_id].steps}"
        assert d.finished >= d.admitted >= d.arrival


def test_admission_respects_memory_and_slots():
    _, _, be, _ = _run(budget=48 << 20, slots=5)
    assert be.max_live <= 48 << 20
    assert be.max_slots_seen <= 5


def test_requests_join_while_others_run():
    """Continuous batching: a request admitted while others are mid-run shares
    their later launches."""
    _, done, be, _ = _run(n=40, slots=16)
    ids_per_batch = [set(i for i, _ in b) for b in be.batches]
    grew = any(len(b2 - b1) > 0 and len(b1 & b2) > 0 for b1, b2 in zip(ids_per_batch, ids_per_batch[1:]))
    assert grew
    summ = S.summarize(done)
    assert summ["requests"] == 40
    assert summ["p99_time_to_solution_s"] >= summ["p50_time_to_solution_s"] > 0


def test_oversized_request_is_rejected():
    clock = Clock()
    be = FakeBackend(clock)
    specs = W.request_stream(n=1, seed=3)
    srv = S.Server(be, lambda s: FakePb(10, 1 << 40), hbm_budget=1 << 20, clock=clock, sleep=clock.sleep)
    try:
        srv.run(specs)
    except ValueError:
        return
    raise AssertionError("an oversized request must be rejected")
