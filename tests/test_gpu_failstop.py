"""Fail-stop identification by deadline: each entangled stream's operation
runs as its own task on its own HIP stream; a stream delayed past the
deadline (a slow core) is named lost by ne_wait_streams and recovery from
the other M - 1 streams equals the CPU oracle. Every delay is bounded, and
each test synchronizes before it ends."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
SLOW_US = 250_000      # a slow core: its work completes this much later
DEADLINE_US = 40_000   # the others finish within a few milliseconds


def run_tasks(c, g, slow=(), skip=(), deadline_us=DEADLINE_US):
    """Entangle, run the convolution of every stream as its own task (stream
    m on its own HIP stream, delayed if m in `slow`, never launched if m in
    `skip`), identify the late stream by the deadline, recover from the
    others. Returns (lost index, recovered outputs or None)."""
    M, n = c.shape
    K = g.size
    l = ne.params(M)[0]
    cd = [torch.from_numpy(np.ascontiguousarray(r)).to(DEV) for r in c]
    gd = torch.from_numpy(g).to(DEV)
    eps = [torch.empty(n, dtype=torch.int64, device=DEV) for _ in range(M)]
    delta = [torch.empty(n + K - 1, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.entangle(cd, eps, l)
    ready = torch.cuda.Event()
    ready.record()
    streams = [torch.cuda.Stream() for _ in range(M)]
    events = []
    try:
        for m, s in enumerate(streams):
            if m in skip:
                events.append(None)
                continue
            s.wait_event(ready)
            if m in slow:
                ne.stream_delay(SLOW_US, stream=s)
            ne.lsb_apply("conv", eps, gd, delta, mask=1 << m, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
            events.append(ev)
        try:
            lost = ne.wait_streams(events, deadline_us)
        except ne.NeError as e:
            return e.status, None
        main = torch.cuda.current_stream()
        for m, ev in enumerate(events):
            if m != lost and ev is not None:
                main.wait_event(ev)
        dhat = [torch.empty(n + K - 1, dtype=torch.int64, device=DEV) for _ in range(M)]
        ne.extract_recover([None if m == lost else t for m, t in enumerate(delta)], lost, dhat, l)
        main.synchronize()
        return lost, np.stack([t.cpu().numpy() for t in dhat])
    finally:
        torch.cuda.synchronize()  # the slow streams end within SLOW_US


# Each stream's task needs a hardware queue of its own: with more HIP
# streams than the process's hardware queues (4 by default), streams share a
# queue and a slow one holds up its queue-mates, which are then late too.
@pytest.mark.parametrize("M", [3, 4])
def test_late_stream_is_identified_and_recovered(M):
    g = wl.rng(8100 + M)
    c = wl.uniform_i32(g, -(1 << 9), 1 << 9, (M, 30_011))
    k = wl.uniform_i32(g, -(1 << 9), 1 << 9, 33)
    ref = oracle.apply("conv", c, k)
    for slow in range(M):
        lost, got = run_tasks(c, k, slow=(slow,))
        assert lost == slow
        assert np.array_equal(got, ref), (M, slow)


def test_no_late_stream_and_a_stream_never_launched():
    g = wl.rng(8200)
    c = wl.uniform_i32(g, -(1 << 9), 1 << 9, (4, 10_007))
    k = wl.uniform_i32(g, -(1 << 9), 1 << 9, 17)
    ref = oracle.apply("conv", c, k)
    lost, got = run_tasks(c, k)
    assert lost == -1 and np.array_equal(got, ref)
    lost, got = run_tasks(c, k, skip=(2,))
    assert lost == 2 and np.array_equal(got, ref)


def test_two_late_streams_exceed_what_one_redundant_stream_covers():
    g = wl.rng(8300)
    c = wl.uniform_i32(g, -(1 << 9), 1 << 9, (4, 5_003))
    k = wl.uniform_i32(g, -(1 << 9), 1 << 9, 9)
    status, got = run_tasks(c, k, slow=(0, 3))
    assert status == -8 and got is None


# A child process whose runtime has one hardware queue per stream
# (GPU_MAX_HW_QUEUES is read when the runtime starts): then a slow stream
# delays no other, and the late one is named for M = 6 and 8 too.
@pytest.mark.parametrize("M", [6, 8])
def test_late_stream_is_identified_with_a_queue_per_stream(M):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, GPU_MAX_HW_QUEUES=str(M),
               PYTHONPATH=os.pathsep.join(p for p in (root, os.environ.get("PYTHONPATH")) if p))
    r = subprocess.run([sys.executable, os.path.abspath(__file__), str(M)], env=env, cwd=root,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert f"M={M} ok" in r.stdout


if __name__ == "__main__":
    # the child of the test above: every stream slow in turn, and none
    M = int(sys.argv[1])
    g = wl.rng(8400 + M)
    c = wl.uniform_i32(g, -(1 << 9), 1 << 9, (M, 20_011))
    k = wl.uniform_i32(g, -(1 << 9), 1 << 9, 29)
    ref = oracle.apply("conv", c, k)
    for slow in list(range(M)) + [None]:
        lost, got = run_tasks(c, k, slow=() if slow is None else (slow,))
        expect = -1 if slow is None else slow
        if lost != expect or not np.array_equal(got, ref):
            print(f"M={M} slow={slow}: named {lost}", flush=True)
            sys.exit(1)
    print(f"M={M} ok", flush=True)
