"""Continuous-batching server for entangled integer-convolution jobs.

Jobs (M streams of n int32 samples and a kernel of K taps each, optionally
with one stream whose computation is lost) arrive over time. The server

* releases each job at its arrival time (wall clock since the start),
* admits waiting jobs first-come-first-served while their HBM footprint
  (inputs, outputs, kernel, plan tables) fits in a budget,
* places a batch's buffers (inputs, kernels, outputs, plan tables) in one
  device pool of the budget's size, allocated once: nothing is allocated on
  the device while serving (an allocation could stall every lane),
* launches every batch of admitted jobs as one fused plan (entangle ->
  convolve -> recover, ne_plan_create_in: tables uploaded on the lane's
  stream) on the first free lane (a HIP stream), so batches on different
  lanes overlap on the device and jobs that arrive while others run join the
  next batch,
* retires a batch when its completion event has fired, records each job's
  latency (arrival -> recovered outputs in HBM) and returns its memory to
  the pool.

All arithmetic runs in libne; this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import ne
from .workloads import Job


_ALIGN = 256


def _up(x: int) -> int:
    return (x + _ALIGN - 1) & ~(_ALIGN - 1)


class _Pool:
    """First-fit allocator of byte ranges of one device buffer (host-side
    bookkeeping only), with neighbouring free ranges merged."""

    def __init__(self, nbytes: int):
        self.free = [(0, nbytes)]  # sorted (offset, size)

    def alloc(self, nbytes: int):
        nbytes = _up(max(nbytes, 1))
        for i, (off, size) in enumerate(self.free):
            if size >= nbytes:
                if size == nbytes:
                    del self.free[i]
                else:
                    self.free[i] = (off + nbytes, size - nbytes)
                return off, nbytes
        return None

    def release(self, off: int, nbytes: int):
        fr = self.free
        lo, hi = 0, len(fr)
        while lo < hi:
            mid = (lo + hi) // 2
            if fr[mid][0] < off:
                lo = mid + 1
            else:
                hi = mid
        fr.insert(lo, (off, nbytes))
        if lo + 1 < len(fr) and fr[lo][0] + fr[lo][1] == fr[lo + 1][0]:
            fr[lo] = (fr[lo][0], fr[lo][1] + fr[lo + 1][1])
            del fr[lo + 1]
        if lo > 0 and fr[lo - 1][0] + fr[lo - 1][1] == fr[lo][0]:
            fr[lo - 1] = (fr[lo - 1][0], fr[lo - 1][1] + fr[lo][1])
            del fr[lo]


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
    ranges: list


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
    deferred_jobs: int   # jobs that waited for HBM footprint while a lane was free
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
        self.arena = torch.empty(hbm_budget + _ALIGN, dtype=torch.uint8, device=self.dev)
        self.base = (-self.arena.data_ptr()) % _ALIGN
        self.pool = _Pool(hbm_budget)
        self._nbatch = 0
        self._warm: set[int] = set()

    @staticmethod
    def footprint(job: Job) -> int:
        """Pool bytes of a job: its aligned buffers and a share of the plan
        tables (one descriptor, work items)."""
        g = job.group
        K = g.operand.size
        return (g.M * _up(g.n * 4) + _up(K * 4) + g.M * _up((g.n + K - 1) * 8) +
                _up(1024 + 8 * (g.n + K) // 1024))

    def _view(self, off: int, nbytes: int, dtype, count: int):
        t = self.arena[self.base + off:self.base + off + nbytes]
        return t.view(dtype)[:count]

    def _stage(self, jobs: list[Job]):
        """Client-side buffers: each job's inputs in pinned host memory."""
        torch = self.torch
        return [([torch.from_numpy(np.ascontiguousarray(row)).pin_memory() for row in j.group.c],
                 torch.from_numpy(j.group.operand).pin_memory()) for j in jobs]

    def warmup(self, ms) -> None:
        """Runs one tiny job per stream count and ring layout the server may
        use, so that the first real jobs do not pay for loading the kernel
        variants (each is loaded on its first launch)."""
        torch = self.torch
        for M in sorted(set(ms) - self._warm):
            c = [torch.zeros(256, dtype=torch.int32, device=self.dev) for _ in range(M)]
            k = torch.ones(16, dtype=torch.int32, device=self.dev)
            out = [torch.empty(271, dtype=torch.int64, device=self.dev) for _ in range(M)]
            for rw in (1, 4):
                spec = ne.GroupSpec("conv", c, k, out, 0, -1, self.in_bits, ring_waves=rw)
                plan = ne.Plan([spec], "entangled")
                plan.run()
                plan.close()
            self._warm.add(M)
        torch.cuda.synchronize()

    def run(self, jobs: list[Job], start_delay: float = 0.05) -> ServeReport:
        torch = self.torch
        self.warmup({j.group.M for j in jobs})
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
        deferred_jobs: set[int] = set()
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
                        if self.keep:  # the pool reuses the buffers: keep copies
                            recs[i].outputs = [o.clone() for o in recs[i].outputs]
                    if self.keep:
                        torch.cuda.current_stream().synchronize()
                    in_use -= b.nbytes
                    b.plan.close()
                    for r in b.ranges:
                        self.pool.release(*r)
                    del busy[lane]
                    free.append(lane)
                    done += len(b.jobs)
            # admit and launch
            while free and waiting:
                take, nbytes = [], 0
                while waiting and len(take) < self.max_batch:
                    f = self.footprint(jobs[waiting[0]])
                    if in_use + nbytes + f > self.budget:
                        deferred_jobs.add(waiting[0])
                        break
                    take.append(waiting.popleft())
                    nbytes += f
                if not take:
                    break
                lane = free[-1]
                if not self._launch(lane, take, jobs, staged, recs, busy, nbytes, t0):
                    if not busy and len(take) == 1:
                        raise MemoryError("a job does not fit the device pool")
                    waiting.extendleft(reversed(take))  # fragmented pool: retry later
                    break
                free.pop()
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
            lost_jobs=sum(r.lost >= 0 for r in recs), deferred_jobs=len(deferred_jobs),
            records=recs)

    def _launch(self, lane, take, jobs, staged, recs, busy, nbytes, t0) -> bool:
        torch = self.torch
        s = self.lanes[lane]
        ranges = []

        def alloc(nb, dtype, count):
            r = self.pool.alloc(nb)
            if r is None:
                raise MemoryError
            ranges.append(r)
            return self._view(r[0], nb, dtype, count)

        tensors, specs = [], []
        try:
            for i in take:
                g = jobs[i].group
                n_out = g.n + g.operand.size - 1
                c = [alloc(g.n * 4, torch.int32, g.n) for _ in range(g.M)]
                k = alloc(g.operand.size * 4, torch.int32, g.operand.size)
                out = [alloc(n_out * 8, torch.int64, n_out) for _ in range(g.M)]
                specs.append(ne.GroupSpec("conv", c, k, out, 0, g.fail, self.in_bits))
                tensors.append((c, k, out))
            wsb = ne.workspace_size(specs)
            ws = alloc(wsb, torch.uint8, wsb)
        except MemoryError:
            for r in ranges:
                self.pool.release(*r)
            return False
        with torch.cuda.stream(s):
            for i, (c, k, out) in zip(take, tensors):
                hc, hk = staged[i]
                for d, h in zip(c, hc):
                    d.copy_(h, non_blocking=True)
                k.copy_(hk, non_blocking=True)
                recs[i].admitted = time.perf_counter() - t0
                recs[i].batch = self._nbatch
                if self.keep:
                    recs[i].outputs = out
            plan = ne.Plan(specs, "entangled", workspace=ws, stream=s)
            plan.run(s)
            ev = torch.cuda.Event()
            ev.record(s)
        busy[lane] = _Batch(take, lane, ev, plan, tensors, nbytes, ranges)
        self._nbatch += 1
        return True
