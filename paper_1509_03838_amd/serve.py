"""Continuous-batching server for entangled integer-convolution jobs.

Jobs (M streams of n int32 samples and a kernel of K taps each, optionally
with one stream whose computation is lost) arrive over time. The server

* releases each job at its arrival time (wall clock since the start),
* admits waiting jobs first-come-first-served while their HBM footprint
  (inputs, outputs, kernel, plan tables) fits in a budget,
* launches every batch of admitted jobs as one fused plan (entangle ->
  convolve -> recover, ne_plan_create_in: no device allocation, tables
  uploaded on the lane's stream) on the first free lane (a HIP stream), so
  batches on different lanes overlap on the device and jobs that arrive
  while others run join the next batch,
* retires a batch when its completion event has fired, records each job's
  latency (arrival -> recovered outputs in HBM) and frees its memory.

All arithmetic runs in libne; this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import ne
from .workloads import Job


@dataclass
class JobRecord:
    index: int
    arrival: float
    M: int
    n: int
    K: int
    lost: int
    admitted: float = 0.0
    done: float = 0.0
    batch: int = -1
    outputs: list | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Batch:
    jobs: list
    lane: int
    event: object
    plan: object
    tensors: list
    nbytes: int


@dataclass
class ServeReport:
    jobs: int
    makespan_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    max_ms: float
    jobs_per_s: float
    gout_per_s: float
    batches: int
    mean_batch: float
    peak_bytes: int
    lost_jobs: int
    records: list = field(repr=False, default_factory=list)

    def as_dict(self) -> dict:
        return {k: v for k, v in self.__dict__.items() if k != "records"}


class Server:
    def __init__(self, hbm_budget: int = 2 << 30, lanes: int = 4, max_batch: int = 64,
                 in_bits: int = 11, keep_outputs: bool = False, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.budget, self.max_batch, self.in_bits = hbm_budget, max_batch, in_bits
        self.keep = keep_outputs
        self.dev = torch.device(device)
        self.lanes = [torch.cuda.Stream(device=self.dev) for _ in range(lanes)]
        self._nbatch = 0

    @staticmethod
    def footprint(job: Job) -> int:
        g = job.group
        K = g.operand.size
        return g.M * g.n * 4 + K * 4 + g.M * (g.n + K - 1) * 8 + 4096

    def _stage(self, jobs: list[Job]):
        """Client-side buffers: each job's inputs in pinned host memory."""
        torch = self.torch
        return [([torch.from_numpy(np.ascontiguousarray(row)).pin_memory() for row in j.group.c],
                 torch.from_numpy(j.group.operand).pin_memory()) for j in jobs]

    def run(self, jobs: list[Job], start_delay: float = 0.05) -> ServeReport:
        torch = self.torch
        staged = self._stage(jobs)
        recs = [JobRecord(i, j.arrival_s, j.group.M, j.group.n, j.group.operand.size, j.group.fail)
                for i, j in enumerate(jobs)]
        for j in jobs:
            if self.footprint(j) > self.budget:
                raise ValueError("a job's footprint exceeds the HBM budget")
        order = sorted(range(len(jobs)), key=lambda i: jobs[i].arrival_s)
        nxt = 0
        waiting: deque[int] = deque()
        busy: dict[int, _Batch] = {}
        free = list(range(len(self.lanes)))
        in_use = peak = 0
        nbatches = nbatch_jobs = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter() + start_delay
        done = 0
        while done < len(jobs):
            now = time.perf_counter() - t0
            while nxt < len(order) and jobs[order[nxt]].arrival_s <= now:
                waiting.append(order[nxt])
                nxt += 1
            # retire finished batches
            for lane, b in list(busy.items()):
                if b.event.query():
                    t = time.perf_counter() - t0
                    for i in b.jobs:
                        recs[i].done = t
                    in_use -= b.nbytes
                    b.plan.close()
                    del busy[lane]
                    free.append(lane)
                    done += len(b.jobs)
            # admit and launch
            while free and waiting:
                take, nbytes = [], 0
                while waiting and len(take) < self.max_batch:
                    f = self.footprint(jobs[waiting[0]])
                    if in_use + nbytes + f > self.budget:
                        break
                    take.append(waiting.popleft())
                    nbytes += f
                if not take:
                    break
                lane = free.pop()
                self._launch(lane, take, jobs, staged, recs, busy, nbytes, t0)
                in_use += nbytes
                peak = max(peak, in_use)
                nbatches += 1
                nbatch_jobs += len(take)
        makespan = max(r.done for r in recs) - min(r.arrival for r in recs)
        lat = np.array([r.latency for r in recs]) * 1e3
        samples = sum(r.M * (r.n + r.K - 1) for r in recs)
        return ServeReport(
            jobs=len(recs), makespan_s=makespan, p50_ms=float(np.percentile(lat, 50)),
            p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
            max_ms=float(lat.max()), jobs_per_s=len(recs) / makespan,
            gout_per_s=samples / makespan / 1e9, batches=nbatches,
            mean_batch=nbatch_jobs / max(1, nbatches), peak_bytes=peak,
            lost_jobs=sum(r.lost >= 0 for r in recs), records=recs)

    def _launch(self, lane, take, jobs, staged, recs, busy, nbytes, t0):
        torch = self.torch
        s = self.lanes[lane]
        tensors, specs = [], []
        with torch.cuda.stream(s):
            for i in take:
                g = jobs[i].group
                hc, hk = staged[i]
                c = [t.to(self.dev, non_blocking=True) for t in hc]
                k = hk.to(self.dev, non_blocking=True)
                n_out = g.n + g.operand.size - 1
                out = [torch.empty(n_out, dtype=torch.int64, device=self.dev) for _ in range(g.M)]
                specs.append(ne.GroupSpec("conv", c, k, out, 0, g.fail, self.in_bits))
                tensors.append((c, k, out))
                recs[i].admitted = time.perf_counter() - t0
                recs[i].batch = self._nbatch
                if self.keep:
                    recs[i].outputs = out
            ws = torch.empty(ne.workspace_size(specs) + 256, dtype=torch.uint8, device=self.dev)
            ws_al = ws[(-ws.data_ptr()) % 256:]  # the plan tables want 256-byte alignment
            plan = ne.Plan(specs, "entangled", workspace=ws_al, stream=s)
            plan.run(s)
            ev = torch.cuda.Event()
            ev.record(s)
        busy[lane] = _Batch(take, lane, ev, plan, tensors + [ws], nbytes)
        self._nbatch += 1
