"""Parity at the benchmark sizes, in the launch configuration bench.py times
(one captured plan over the whole batch): sampled outputs against the CPU
oracle, computed one by one (convolution) or by definition (element-wise
operations, inner products in full)."""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def build(groups, in_bits, lost=-1, steps=8):
    c = [[torch.from_numpy(np.ascontiguousarray(r)).to(DEV) for r in g.c] for g in groups]
    k = [None if g.op == "scale" else torch.from_numpy(g.operand).to(DEV) for g in groups]
    outs, specs = [], []
    for g, cc, kk in zip(groups, c, k):
        no = ne.n_out(g.op, g.n, 0 if g.operand is None else g.operand.size)
        o = [torch.empty(max(no, 1), dtype=torch.int64, device=DEV)[:no] for _ in range(g.M)]
        outs.append(o)
        specs.append(ne.GroupSpec(g.op, cc, kk, o, g.scalar, lost, in_bits, steps=steps))
    return specs, outs, (c, k)


def launch(specs):
    plan = ne.Plan(specs)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(s)
        plan.launch(s)
        plan.launch(s)  # a second replay over the same buffers
        s.synchronize()
    assert plan.flags() == 0
    return plan


def positions(n_out, rng, count):
    edge = np.concatenate([np.arange(min(n_out, 80)), np.arange(max(0, n_out - 80), n_out)])
    return np.unique(np.concatenate([edge, rng.integers(0, n_out, count)]))


def check_conv(g, out, rng, count):
    pos = positions(g.n + g.operand.size - 1, rng, count)
    for m in range(g.M):
        got = out[m][torch.from_numpy(pos).to(DEV)].cpu().numpy()
        assert np.array_equal(got, oracle.conv_at(g.c[m], g.operand, pos)), (g.M, g.n, m)


def test_batched_benchmark_configuration():
    """All 64 stream-triples of 2^20 samples, 64 taps, one lost stream per
    group (rotating), 8-step strips."""
    groups = wl.config_batched()
    for lost in (-1, 1):
        specs, outs, keep = build(groups, 12, lost)
        launch(specs)
        rng = wl.rng(11)
        for g, o in zip(groups, outs):
            check_conv(g, o, rng, 600)


def test_long_kernel_benchmark_configuration():
    """All 256 stream-triples of 262,144 int16-range samples, 1024 taps."""
    groups = wl.config_long_kernel()
    specs, outs, keep = build(groups, 16)
    launch(specs)
    rng = wl.rng(12)
    for g, o in zip(groups, outs):
        check_conv(g, o, rng, 150)


def test_uneven_benchmark_configuration():
    """All 512 groups of the uneven batch (M 3..8, up to 2^22 samples, five
    operations) in one captured plan with its parallel branches."""
    groups = wl.config_uneven()
    specs, outs, keep = build(groups, 10, steps=0)
    launch(specs)
    rng = wl.rng(13)
    for g, o in zip(groups, outs):
        if g.op == "conv":
            check_conv(g, o, rng, 200)
            continue
        if g.op == "inner":
            ref = oracle.apply("inner", g.c, g.operand)
            got = np.stack([t.cpu().numpy() for t in o])
            assert np.array_equal(got, ref), (g.op, g.M, g.n)
            continue
        pos = positions(g.n, rng, 2000)
        idx = torch.from_numpy(pos).to(DEV)
        for m in range(g.M):
            x = g.c[m]
            if g.op == "scale":
                ref = oracle.apply("scale", x[pos], None, g.scalar)
            elif g.op == "add":
                ref = oracle.apply("add", x[pos], g.operand[pos])
            else:
                ref = oracle.apply("perm", x, g.operand)[pos]
            assert np.array_equal(o[m][idx].cpu().numpy(), ref), (g.op, g.M, g.n, m)


@pytest.mark.parametrize("M", [3, 8])
def test_paper_experiment_longest_kernel(M):
    """The longest point of the paper's experiment (Sec. V, Fig. 2): M
    streams of 10^6 samples, 4500 taps, every mode and one lost stream, each
    replayed twice from one captured plan."""
    g = wl.config_fig2(M, 4500)
    c = [torch.from_numpy(np.ascontiguousarray(r)).to(DEV) for r in g.c]
    k = torch.from_numpy(g.operand).to(DEV)
    n_out = g.n + g.operand.size - 1
    rng = wl.rng(14)
    pos = positions(n_out, rng, 300)
    idx = torch.from_numpy(pos).to(DEV)
    ref = [oracle.conv_at(g.c[m], g.operand, pos) for m in range(M)]
    for mode, lost in (("entangled", -1), ("entangled", M - 1), ("plain", -1),
                       ("plain_same", -1), ("checksum", -1), ("checksum", 0)):
        out = [torch.full((n_out,), -1, dtype=torch.int64, device=DEV) for _ in range(M)]
        spec = ne.GroupSpec("conv", c, k, out, 0, lost, wl.FIG2_BITS)
        plan = ne.Plan([spec], mode)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            plan.capture(s)
            plan.launch(s)
            plan.launch(s)
            s.synchronize()
        assert plan.flags() == 0
        for m in range(M):
            assert np.array_equal(out[m][idx].cpu().numpy(), ref[m]), (mode, lost, m)
        plan.close()
