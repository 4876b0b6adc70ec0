"""Autotuner for the fused executor's tile steps.

The fused kernels process a strip of `steps` tiles per block (convolution:
1024 outputs per step; element-wise: 256 lanes x 4 or 2 positions per
step). Longer strips amortise the per-block set-up (the Toeplitz operand, the
first window with its halo) but leave fewer blocks to balance the load; the
best length depends on the operation, M, the digit counts and the sizes.
Convolutions also choose how many waves share one staging ring (4: one ring
per block, barriers in the step loop; 1: a ring per wave, none, but a halo
per wave). The tuner groups a batch into workload classes, times every
candidate on a few representative groups of each class with HIP events, and
keeps the fastest per class in a JSON cache on disk, so later plans (and
later processes) reuse the choice without timing.

Class key: convolution (mode, M, in_bits, 32-bit words or not, K bucket, n bucket); element-wise
(mode, op, M <= 4 or not, n bucket); K buckets are powers of two, n buckets
powers of four.

A batch of several classes is then checked whole: classes timed alone do
not share the device, and a batch's launches do (on parallel graph
branches), so the tuned choices are kept only if the whole plan runs faster
with them than with the planner's defaults; the verdict is cached under the
batch's set of classes.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Sequence

from . import ne

CONV_LIKE = ("conv", "circ", "xcorr")  # operations that run on the convolution kernel
CONV_CANDIDATES = tuple((st, rw) for st in (1, 2, 4, 8, 16) for rw in (4, 1))
STREAM_CANDIDATES = tuple((st, 0) for st in (1, 2, 4, 8))
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ne_tune.json")


def _bucket(x: int) -> int:
    return max(0, int(x).bit_length() - 1)


def class_key(spec: ne.GroupSpec, mode: str) -> str:
    n = spec.c[0].numel() if spec.c else 0
    nb = _bucket(n) // 2
    if spec.op in CONV_LIKE:
        K = spec.operand.numel() if spec.operand is not None else 0
        w = "|w32" if getattr(spec, "word_bits", 0) == 32 else ""
        return f"{mode}|conv|M{len(spec.c)}|b{spec.in_bits}{w}|K{_bucket(K)}|n{nb}"
    return f"{mode}|{spec.op}|M{'<=4' if len(spec.c) <= 4 else '>4'}|n{nb}"


def _fits(spec, mode: str) -> bool:
    """Whether the planner accepts a spec as set. A per-wave ring's LDS
    window grows with the exact tap count, so a choice timed on one member
    of a power-of-two K bucket may not fit a longer one (sizing only: no
    device is touched)."""
    if not isinstance(spec, ne.GroupSpec):
        return True
    try:
        ne.workspace_size([spec], mode)
        return True
    except ne.NeError:
        return False


def plan_key(classes, mode: str) -> str:
    """Cache key of a batch's whole-plan verdict: its set of class keys."""
    h = hashlib.sha256("\n".join(sorted(classes)).encode()).hexdigest()[:16]
    return f"{mode}|plan|{h}"


def _choice(v):
    """A cached choice: [steps, ring_waves] (a bare int: steps)."""
    if isinstance(v, int):
        return (v, 0)
    return (int(v[0]), int(v[1]))


class Tuner:
    def __init__(self, cache_path: str | None = DEFAULT_CACHE, repeats: int = 5,
                 max_groups: int = 256, min_work: int = 1 << 26, rounds: int = 2):
        """min_work: input samples the representatives of a class should
        hold (at least one group; at most max_groups)."""
        self.path, self.repeats, self.rounds = cache_path, repeats, rounds
        self.max_groups, self.min_work = max_groups, min_work
        self.cache: dict[str, tuple[int, int]] = {}
        if cache_path and os.path.exists(cache_path):
            try:
                with open(cache_path) as f:
                    data = json.load(f)
                self.cache = {k: _choice(v) for k, v in data.get("steps", {}).items()}
            except (OSError, ValueError, TypeError, IndexError):
                self.cache = {}

    def save(self):
        """Writes the cache; an unwritable location only loses the reuse."""
        if not self.path:
            return
        try:
            os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
            tmp = self.path + f".tmp{os.getpid()}"
            with open(tmp, "w") as f:
                json.dump({"steps": {k: list(v) for k, v in self.cache.items()}}, f, indent=1,
                          sort_keys=True)
            os.replace(tmp, self.path)
        except OSError:
            pass

    @staticmethod
    def _apply(specs, choice):
        for sp in specs:
            sp.steps, sp.ring_waves = choice

    def _time(self, specs: Sequence[ne.GroupSpec], mode: str, choice=None) -> float:
        """Milliseconds per run of a plan over specs, with choice applied to
        all of them first (None: as they are set)."""
        import torch
        if choice is not None:
            self._apply(specs, choice)
        try:
            plan = ne.Plan(specs, mode)
        except ne.NeError:
            return float("inf")  # e.g. per-wave windows that do not fit in LDS
        try:
            plan.run()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(self.repeats):
                plan.run()
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) / self.repeats
        finally:
            plan.close()

    def tune(self, specs: Sequence[ne.GroupSpec], mode: str = "entangled") -> dict:
        """Sets `steps` (and, for convolutions, `ring_waves`) on every spec,
        timing the classes not cached yet, and returns the class -> choice
        table used (with several classes, also the whole-plan verdict under
        plan_key: "tuned" or "planner defaults")."""
        classes: dict[str, list[ne.GroupSpec]] = {}
        for sp in specs:
            classes.setdefault(class_key(sp, mode), []).append(sp)
        changed = False
        for key, members in classes.items():
            if key in self.cache:
                continue
            # representatives: the largest groups of the class, enough of
            # them to fill the device the way the whole batch does
            reps, work = [], 0
            for sp in sorted(members, key=lambda s: -s.c[0].numel()):
                if len(reps) >= self.max_groups or work >= self.min_work:
                    break
                reps.append(sp)
                work += len(sp.c) * sp.c[0].numel()
            saved = [(s.steps, s.ring_waves) for s in reps]
            cands = CONV_CANDIDATES if reps[0].op in CONV_LIKE else STREAM_CANDIDATES
            # every candidate timed in `rounds` interleaved passes; the best
            # pass counts (a slow pass is noise, a fast one is not)
            times = {c: float("inf") for c in cands}
            for _ in range(self.rounds):
                for c in cands:
                    times[c] = min(times[c], self._time(reps, mode, c))
            for s, v in zip(reps, saved):
                s.steps, s.ring_waves = v
            self.cache[key] = min(times, key=times.get)
            changed = True
        for key, members in classes.items():
            self._apply(members, self.cache[key])
            for s in members:
                if s.ring_waves == 1 and not _fits(s, mode):
                    s.ring_waves = 0  # the planner takes the layout that fits
        if len(classes) > 1:
            # the whole batch: tuned choices against the planner's defaults
            pkey = plan_key(classes, mode)
            if pkey not in self.cache:
                tuned = [(s.steps, s.ring_waves) for s in specs]
                t_tuned = min(self._time(specs, mode) for _ in range(self.rounds))
                t_default = min(self._time(specs, mode, (0, 0)) for _ in range(self.rounds))
                for s, v in zip(specs, tuned):
                    s.steps, s.ring_waves = v
                self.cache[pkey] = (1 if t_default < 0.99 * t_tuned else 0, 0)
                changed = True
            if self.cache[pkey][0] == 1:
                self._apply(specs, (0, 0))
        if changed:
            self.save()
        table = {k: self.cache[k] for k in classes}
        if len(classes) > 1:
            table[pkey] = "planner defaults" if self.cache[pkey][0] == 1 else "tuned"
        return table
