"""Serving loop: continuous batching of simulation requests on one GPU.

Requests arrive over time.  The scheduler admits them first-come first-served
whenever their device footprint fits the HBM budget next to the requests
already resident; admitted requests keep their whole state resident in
device memory and advance together, chunk by chunk, in batched launches (one
launch per time step covers every resident request of the same kernel kind).
Between chunks finished requests retire (results copied out, memory released)
and newly arrived ones are admitted, so work from requests that arrived at
different times overlaps on the device.  Batched results are bit-identical
to running each request alone (the kernels' arithmetic per cell does not
depend on the batch).

The scheduling core (Scheduler) is independent of the GPU; the GPU executor
(GpuExecutor) drives the library through its C ABI.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, Iterable, List, Optional

import numpy as np


@dataclass
class Job:
    """One simulation request."""
    id: int
    arrival: float               # seconds after the stream starts
    footprint: int               # device bytes while resident
    nsteps: int
    cells: int
    payload: object = None       # executor-specific problem description (or a
                                 # callable returning it at admission)
    # filled in by the scheduler
    admitted: Optional[float] = None
    finished: Optional[float] = None
    done_steps: int = 0
    result: object = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


@dataclass
class Stats:
    latencies: List[float] = field(default_factory=list)
    queueing: List[float] = field(default_factory=list)    # arrival -> admitted
    service: List[float] = field(default_factory=list)     # admitted -> finished
    cell_steps: int = 0
    wall: float = 0.0
    peak_bytes: int = 0
    chunks: int = 0
    max_resident: int = 0
    rejected: int = 0

    def summary(self) -> dict:
        def arr(v):
            return np.asarray(v) if v else np.zeros(1)
        lat, q, sv = arr(self.latencies), arr(self.queueing), arr(self.service)
        return {
            "completed": len(self.latencies),
            "rejected": self.rejected,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "p50_queueing_s": float(np.percentile(q, 50)),
            "p99_queueing_s": float(np.percentile(q, 99)),
            "p50_service_s": float(np.percentile(sv, 50)),
            "p99_service_s": float(np.percentile(sv, 99)),
            "aggregate_glups": self.cell_steps / self.wall / 1e9 if self.wall else 0.0,
            "wall_s": self.wall,
            "peak_resident_bytes": self.peak_bytes,
            "max_resident_requests": self.max_resident,
            "chunks": self.chunks,
        }


class Scheduler:
    """FCFS admission by footprint, continuous batching by chunks of steps.

    executor must provide:
      admit(job)                  upload the job's state (overlaps a running
                                  chunk; returns when the upload is done)
      launch(jobs, steps_each)    start advancing resident jobs (async)
      wait()                      block until the launched chunk is done
      retire(job) -> result       copy results out and release memory
                                  (GpuExecutor: (fields, energy, comps))
    clock() returns seconds since the stream started; idle(dt) waits for
    the next arrival when nothing is resident.
    """

    def __init__(self, executor, budget_bytes: int, chunk_steps: int,
                 clock: Callable[[], float], idle: Callable[[float], None],
                 on_retire: Optional[Callable[[Job], None]] = None):
        if budget_bytes <= 0 or chunk_steps <= 0:
            raise ValueError("budget and chunk must be positive")
        self.ex = executor
        self.budget = budget_bytes
        self.chunk = chunk_steps
        self.clock = clock
        self.idle = idle
        self.on_retire = on_retire
        self.done: List[Job] = []

    def run(self, jobs: Iterable[Job]) -> Stats:
        pending = sorted(jobs, key=lambda j: (j.arrival, j.id))
        queue: List[Job] = []          # arrived, not yet admitted
        resident: List[Job] = []
        st = Stats()
        in_use = 0
        start = self.clock()
        while pending or queue or resident:
            now = self.clock()
            while pending and pending[0].arrival <= now:
                j = pending.pop(0)
                if j.footprint > self.budget:
                    st.rejected += 1          # can never fit
                    continue
                queue.append(j)
            steps = [min(self.chunk, j.nsteps - j.done_steps) for j in resident]
            if resident:
                self.ex.launch(resident, steps)
            # admit (upload) arrivals while the chunk runs, in arrival order,
            # as long as the head of the queue fits next to everything resident
            joining = []
            while queue and in_use + queue[0].footprint <= self.budget:
                j = queue.pop(0)
                self.ex.admit(j)
                j.admitted = self.clock()
                in_use += j.footprint
                joining.append(j)
            st.peak_bytes = max(st.peak_bytes, in_use)
            if resident:
                self.ex.wait()
                st.chunks += 1
                for j, s in zip(resident, steps):
                    j.done_steps += s
                    st.cell_steps += j.cells * s
                for j in [j for j in resident if j.done_steps >= j.nsteps]:
                    j.result = self.ex.retire(j)
                    j.finished = self.clock()
                    in_use -= j.footprint
                    resident.remove(j)
                    self.done.append(j)
                    st.latencies.append(j.latency)
                    st.queueing.append(j.admitted - j.arrival)
                    st.service.append(j.finished - j.admitted)
                    if self.on_retire:
                        self.on_retire(j)
            resident.extend(joining)
            st.max_resident = max(st.max_resident, len(resident))
            if not resident and not queue and pending:
                self.idle(max(0.0, pending[0].arrival - self.clock()))
        st.wall = self.clock() - start
        return st


class GpuExecutor:
    """Runs jobs through libhalfwave: one plan (and arena) per resident job;
    uploads on a copy stream; each chunk advances every group of resident
    jobs that share a kernel (physics, storage format, compensation) in one
    batched call on that group's own stream, so the groups' launches
    overlap on the device (all streams at the default priority)."""

    max_streams = 4

    def __init__(self, device="cuda:0", energy_every: int = 0):
        import torch
        import paper_2310_00236_amd as hw
        self.hw = hw
        self.torch = torch
        self.device = torch.device(device)
        self.copy = torch.cuda.Stream(self.device)
        self.streams = {}           # kernel group -> stream
        self.busy = []              # streams with work in the current chunk
        self.energy_every = energy_every
        self.plans = {}

    @staticmethod
    def group(pb):
        return (pb.physics, pb.order, pb.storage, pb.comp)

    def _stream(self, key):
        if key not in self.streams:
            if len(self.streams) < self.max_streams:
                self.streams[key] = self.torch.cuda.Stream(self.device)
            else:                   # more groups than streams: share round-robin
                pool = list(dict.fromkeys(self.streams.values()))
                self.streams[key] = pool[len(self.streams) % len(pool)]
        return self.streams[key]

    def admit(self, job: Job):
        # the payload is (problem, material, fields), or a callable that
        # draws them when the request is admitted
        payload = job.payload() if callable(job.payload) else job.payload
        pb, material, fields = payload
        plan = self.hw.Plan(pb, device=self.device)
        plan.set_tuned_tile()
        plan.set_material(material, stream=self.copy)
        plan.set_fields(fields, stream=self.copy)
        self.plans[job.id] = plan

    def launch(self, jobs, steps):
        groups = {}
        for j, s in zip(jobs, steps):
            plan = self.plans[j.id]
            groups.setdefault(self.group(plan.pb), []).append((plan, s))
        self.busy = []
        for key, members in groups.items():
            stream = self._stream(key)
            self.hw.batch_advance([m[0] for m in members], [m[1] for m in members],
                                  self.energy_every, stream=stream)
            self.busy.append(stream)

    def wait(self):
        for stream in self.busy:
            stream.synchronize()
        self.busy = []

    def retire(self, job: Job):
        plan = self.plans.pop(job.id)
        stream = self._stream(self.group(plan.pb))
        out, comps = plan.get_fields(comps=True, stream=stream)
        energy = plan.energy_trace(stream=stream)[0] if self.energy_every else None
        plan.close()
        return out, energy, comps


def job_for(req, problem, material, fields, trace_cap=0) -> Job:
    import paper_2310_00236_amd as hw
    return Job(id=req.index, arrival=req.arrival, footprint=hw.footprint(problem),
               nsteps=req.nsteps, cells=problem.cells,
               payload=(problem, material, fields))


def serve(jobs: List[Job], budget_bytes: int, chunk_steps: int = 200,
          device="cuda:0", energy_every: int = 0, realtime: bool = True,
          on_retire: Optional[Callable[[Job], None]] = None):
    """Run a request stream on the GPU; returns (stats summary, jobs done).

    realtime=False treats every request as arrived at time 0; on_retire is
    called with each finished job."""
    ex = GpuExecutor(device, energy_every)
    if not realtime:
        for j in jobs:
            j.arrival = 0.0
    t0 = time.perf_counter()
    sched = Scheduler(ex, budget_bytes, chunk_steps,
                      lambda: time.perf_counter() - t0, time.sleep, on_retire)
    st = sched.run(jobs)
    return st.summary(), sched.done
