"""Continuous-batching request loop for independent MPM problems.

Requests arrive over time (a Poisson stream), each an independent 2D problem
of its own grid and particle count.  The loop keeps the admitted problems
resident in device memory and advances all of them together: every sweep of
a step is one launch whose workgroups cover the tiles of every resident
problem (`mpm_step_batch`, replays of captured step graphs),
`steps_per_launch` steps per call.  A request is admitted as soon as a slot
and enough device memory (its `mpm_footprint`) are free.  As soon as a batch
completes the next one is launched; the host work between batches (reading
back the problems that just finished, building and initialising new ones on
a side stream) then overlaps with it, and new problems join the batch after
it.  Finished problems are read back and their memory returned.
Time-to-solution is completion time minus arrival time.

The loop talks to a backend with five calls (footprint, create, step_batch,
finish, sync), so its scheduling can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import hashlib
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Completed:
    req_id: int
    arrival: float
    admitted: float
    finished: float
    particles: int
    steps: int
    digest: str            # sha256 of the final density (id order), for comparisons
    status: int = 0

    @property
    def time_to_solution(self) -> float:
        return self.finished - self.arrival


class GPUBackend:
    """Backend over libmpm.so: device workspaces from a torch allocator, one
    main stream for the batched steps and one side stream for admissions."""

    def __init__(self, precision: int, device: str = "cuda:0"):
        import torch
        from . import mpm as G
        self.G = G
        self.torch = torch
        self.precision = precision
        self.device = torch.device(device)
        self.main = torch.cuda.Stream(device=self.device)
        self.side = torch.cuda.Stream(device=self.device)
        self._ev = None

    def footprint(self, pb) -> int:
        return self.G.footprint(pb, self.precision)

    def create(self, pb):
        # init on the side stream: overlaps with the batch in flight
        return self.G.Simulation(pb, self.precision, device=str(self.device), stream=self.side)

    def step_batch(self, sims, counts):
        for s in sims:
            s.stream = self.main
        self.G.step_batch(sims, counts, stream=self.main)
        self._ev = self.torch.cuda.Event()
        self._ev.record(self.main)

    def sync(self):
        if self._ev is not None:
            self._ev.synchronize()

    def finish(self, sim):
        # on the side stream: overlaps with the batch in flight on the main one
        sim.stream = self.side
        rho = sim.read([self.G.F_RHO], check=False)[self.G.F_RHO]
        st = sim.status()
        sim.close()
        sim.workspace = None
        return hashlib.sha256(rho.tobytes()).hexdigest(), st["rc"]


class Server:
    def __init__(self, backend, build: Callable, hbm_budget: int = 64 << 30, max_slots: int = 64,
                 steps_per_launch: int = 16, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep,
                 progress: Optional[Callable[[int], None]] = None, progress_every: int = 100):
        self.backend = backend
        self.build = build
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.k = steps_per_launch
        self.clock = clock
        self.sleep = sleep
        self.progress = progress
        self.progress_every = progress_every
        self.log: List[str] = []

    def run(self, specs: Sequence) -> List[Completed]:
        pending = collections.deque(sorted(specs, key=lambda s: s.arrival))
        queue = collections.deque()
        active = []                         # dicts: sim, spec, left, bytes, admitted
        used = 0
        done: List[Completed] = []
        t0 = self.clock()
        in_flight = False
        # what ran concurrently: problems per batched launch, and admissions
        # made while a batch was on the device
        self.batch_sizes: List[int] = []
        self.overlapped_admissions = 0
        while pending or queue or active:
            finished = []
            if in_flight:
                self.backend.sync()
                in_flight = False
                keep = []
                for a in active:
                    if a.get("ran"):
                        a["left"] -= a.pop("ran")
                    (finished if a["left"] <= 0 and "launched" in a else keep).append(a)
                active = keep
            # the next batch goes out first; the host work below overlaps it
            if active:
                counts = [min(self.k, a["left"]) for a in active]
                for a, c in zip(active, counts):
                    a["ran"] = c
                    a["launched"] = True
                self.backend.step_batch([a["sim"] for a in active], counts)
                self.batch_sizes.append(len(active))
                in_flight = True
            now = self.clock() - t0
            for a in finished:
                digest, rc = self.backend.finish(a["sim"])
                used -= a["bytes"]
                done.append(Completed(a["spec"].req_id, a["spec"].arrival, a["admitted"], now,
                                      a["particles"], a["spec"].steps, digest, rc))
                if self.progress and len(done) % self.progress_every == 0:
                    self.progress(len(done))
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # admissions: the new problems join the batch after the one in flight
            while queue and len(active) < self.max_slots:
                spec = queue[0]
                pb = self.build(spec)
                need = self.backend.footprint(pb)
                if need > self.budget:
                    raise ValueError(f"request {spec.req_id} needs {need} bytes, budget {self.budget}")
                if used + need > self.budget:
                    break
                queue.popleft()
                sim = self.backend.create(pb)
                used += need
                self.overlapped_admissions += int(in_flight)
                active.append(dict(sim=sim, spec=spec, left=spec.steps, bytes=need,
                                   admitted=self.clock() - t0, particles=pb.n_particles))
            if not in_flight and not active and pending:
                self.sleep(max(0.0, min(0.01, pending[0].arrival - (self.clock() - t0))))
        return done


def summarize(done: Sequence[Completed]) -> Dict[str, float]:
    tts = np.array([d.time_to_solution for d in done])
    work = float(sum(d.particles * d.steps for d in done))
    span = max(d.finished for d in done) - min(d.arrival for d in done)
    rate = work / span
    # the requests behind the tail: their size, queueing and the time their
    # own work would take at the stream's aggregate rate
    slowest = sorted(done, key=lambda d: d.time_to_solution, reverse=True)[:3]
    return {
        "requests": len(done),
        "p50_time_to_solution_s": float(np.percentile(tts, 50)),
        "p99_time_to_solution_s": float(np.percentile(tts, 99)),
        "mean_queue_s": float(np.mean([d.admitted - d.arrival for d in done])),
        "aggregate_particle_steps_per_s": rate,
        "makespan_s": span,
        "errors": int(sum(1 for d in done if d.status != 0)),
        "slowest": [{"req_id": d.req_id, "particle_steps": d.particles * d.steps,
                     "queue_s": round(d.admitted - d.arrival, 4),
                     "time_to_solution_s": round(d.time_to_solution, 4),
                     "own_work_at_aggregate_rate_s": round(d.particles * d.steps / rate, 4)}
                    for d in slowest],
    }
