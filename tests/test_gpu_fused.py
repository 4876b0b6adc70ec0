"""GPU parity of the batched, fused executor (ne_plan_*): every mode, every
operation, uneven batches, every single-stream loss, graph replay -- all
against the CPU oracle, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
POISON = 0x3C3C3C3C3C3C3C3C


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def host(ts):
    torch.cuda.synchronize()
    return np.stack([t.cpu().numpy() for t in ts]) if ts else np.zeros((0, 0), np.int64)


class DevGroup:
    """A workloads.Group on the device with output buffers."""

    def __init__(self, grp: wl.Group, in_bits: int, lost: int = -1, mode: str = "entangled",
                 ring_waves: int = 0, tap_copies: int = 0):
        self.grp = grp
        self.c = [dev32(row) for row in grp.c]
        self.operand = None if grp.op == "scale" else dev32(grp.operand)
        self.n_out = ne.n_out(grp.op, grp.n, 0 if grp.operand is None else grp.operand.size)
        self.out = [torch.full((max(self.n_out, 1),), POISON, dtype=torch.int64, device=DEV)[:self.n_out]
                    for _ in range(grp.M)]
        self.spec = ne.GroupSpec(grp.op, self.c, self.operand, self.out, grp.scalar, lost, in_bits,
                                 ring_waves=ring_waves, tap_copies=tap_copies)

    def result(self):
        return host(self.out)

    def reference(self):
        g = self.grp
        return oracle.apply(g.op, g.c, g.operand if g.op != "scale" else None, g.scalar)


def run(groups, mode="entangled", **kw):
    plan = ne.Plan([g.spec for g in groups], mode, **kw)
    plan.run()
    torch.cuda.synchronize()
    flags = plan.flags()
    return plan, flags


def make(op, M, n, K, bits, seed):
    g = wl.rng(seed)
    lo, hi = -(1 << (bits - 1)), 1 << (bits - 1)
    c = wl.uniform_i32(g, lo, hi, (M, n))
    s = 0
    if op == "conv":
        operand = wl.uniform_i32(g, lo, hi, K)
    elif op in ("add", "inner"):
        operand = wl.uniform_i32(g, lo, hi, n)
    elif op == "perm":
        operand = wl.permutation(g, n)
    else:
        operand, s = np.zeros(0, np.int32), int(g.integers(lo, hi))
    return wl.Group(op, c, operand, s)


# ------------------------------------------------------------ small config

def test_small_config_every_loss_fused():
    grp = wl.config_small()
    ref = oracle.apply("conv", grp.c, grp.operand)
    for lost in (-1, 0, 1, 2):
        dg = DevGroup(grp, 8, lost)
        _, flags = run([dg])
        assert flags == 0
        assert np.array_equal(dg.result(), ref), lost


@pytest.mark.parametrize("mode", ["entangled", "plain", "plain_same", "checksum", "checksum_same"])
@pytest.mark.parametrize("M", [3, 4, 5, 8])
@pytest.mark.parametrize("n,K,bits", [(1, 1, 8), (5, 3, 12), (3001, 37, 12), (4096, 64, 12),
                                      (5000, 300, 10), (2049, 1024, 16), (1, 1024, 11)])
def test_conv_modes(mode, M, n, K, bits):
    grp = make("conv", M, n, K, bits, seed=M * 1000 + n + K)
    ref = oracle.apply("conv", grp.c, grp.operand)
    losses = [-1] + list(range(M)) if mode in ("entangled", "checksum", "checksum_same") else [-1]
    for lost in losses:
        for rw in (4, 1):  # one staging ring per block / per wave
            dg = DevGroup(grp, bits, lost, mode, ring_waves=rw)
            try:
                _, flags = run([dg], mode, conv_steps=3)
            except ne.NeError as e:
                assert e.status == -4 and rw == 1, (mode, M, K, rw, e)  # windows too large for LDS
                continue
            assert flags == 0, (mode, lost, flags, rw)
            assert np.array_equal(dg.result(), ref), (mode, M, n, K, lost, rw)


@pytest.mark.parametrize("mode", ["entangled", "plain", "plain_same", "checksum", "checksum_same"])
@pytest.mark.parametrize("op", ["scale", "add", "inner", "perm"])
@pytest.mark.parametrize("M", [3, 5, 8])
def test_streaming_ops_modes(mode, op, M):
    for n in (1, 255, 4097, 70001):
        grp = make(op, M, n, 0, 10, seed=n * 13 + M + len(op))
        ref = oracle.apply(op, grp.c, grp.operand if op != "scale" else None, grp.scalar)
        losses = [-1, 0, M - 1] if mode in ("entangled", "checksum", "checksum_same") else [-1]
        for lost in losses:
            dg = DevGroup(grp, 10, lost, mode)
            _, flags = run([dg], mode)
            assert flags == 0
            assert np.array_equal(dg.result(), ref), (mode, op, M, n, lost)


def test_uneven_batch_matches_standalone_and_oracle():
    """Uneven groups (M 3..8, lengths 2^12..2^15, taps 8..512, all five ops)
    in one plan: each result equals the oracle and its standalone run."""
    groups = wl.config_uneven(seed=5, groups=40, n_hi=1 << 15)
    rng = wl.rng(99)
    devs = [DevGroup(g, 10, int(rng.integers(-1, g.M))) for g in groups]
    plan, flags = run(devs)
    assert flags == 0
    assert plan.stats()["groups"] == 40
    for dg in devs:
        ref = dg.reference()
        assert np.array_equal(dg.result(), ref), (dg.grp.op, dg.grp.M, dg.grp.n)
    for dg in devs[:6]:
        alone = DevGroup(dg.grp, 10, dg.spec.lost)
        run([alone])
        assert np.array_equal(alone.result(), dg.result())


def test_uneven_graph_branches_replay():
    """A captured uneven plan (dozens of launches on parallel graph branches,
    permutation layout passes first, inner-product recovery last), replayed
    several times with eager work in between: every replay equals the oracle."""
    groups = wl.config_uneven(seed=8, groups=60, n_hi=1 << 14)
    devs = [DevGroup(g, 10) for g in groups]
    plan = ne.Plan([d.spec for d in devs])
    assert plan.stats()["launches"] > 8
    s = torch.cuda.Stream()
    refs = [d.reference() for d in devs]
    with torch.cuda.stream(s):
        plan.capture(s)
        for rep in range(3):
            for d in devs:
                for t in d.out:
                    t.fill_(POISON)
            plan.launch(s)
            s.synchronize()
            y = torch.ones(4096, device=DEV).cumsum(0)  # unrelated eager work
            assert float(y[-1]) == 4096.0
            for d, ref in zip(devs, refs):
                assert np.array_equal(d.result(), ref), (rep, d.grp.op, d.grp.M)
    assert plan.flags() == 0


def test_graph_replay_matches_eager():
    groups = [make("conv", 3, 20000, 64, 12, 1), make("scale", 4, 9000, 0, 12, 2),
              make("inner", 5, 7777, 0, 12, 3), make("perm", 3, 5000, 0, 12, 4)]
    devs = [DevGroup(g, 12) for g in groups]
    plan = ne.Plan([d.spec for d in devs])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(s)
        for rep in range(4):
            for d in devs:
                for t in d.out:
                    t.fill_(POISON)
            x = torch.arange(1000, device=DEV).sum()  # unrelated eager work
            plan.launch(s)
            s.synchronize()
            assert int(x) == 499500
            for d in devs:
                assert np.array_equal(d.result(), d.reference()), (rep, d.grp.op)
    assert plan.flags() == 0


def test_declared_range_violation_is_flagged():
    grp = make("conv", 3, 5000, 16, 12, 7)
    grp.c[1, 100] = 1 << 12   # outside the declared 12 bits
    dg = DevGroup(grp, 12)
    _, flags = run([dg])
    assert flags & ne.FLAG_INPUT_RANGE


def test_batched_config_full_length_sampled():
    """Two stream-triples at the batched size (2^20 samples, 64 taps): every
    loss gives the same outputs, equal to the oracle at sampled positions and
    to the plain mode everywhere."""
    groups = wl.config_batched(groups=2)
    pos = np.unique(np.concatenate([np.arange(0, 300), np.arange((1 << 20) - 300, (1 << 20) + 63),
                                    wl.rng(1).integers(0, (1 << 20) + 63, 4000)]))
    for grp in groups:
        outs = []
        for lost in (-1, 0, 1, 2):
            dg = DevGroup(grp, 12, lost)
            _, flags = run([dg])
            assert flags == 0
            outs.append(dg.result())
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])
        plain = DevGroup(grp, 12, -1, "plain")
        run([plain], "plain")
        assert np.array_equal(plain.result(), outs[0])
        for m in range(3):
            assert np.array_equal(outs[0][m][pos], oracle.conv_at(grp.c[m], grp.operand, pos))


def test_long_kernel_config_shape():
    """The long-kernel shape: 16-bit samples, 1024 taps (more digits)."""
    grp = wl.config_long_kernel(groups=1, n=9000)[0]
    ref = oracle.apply("conv", grp.c, grp.operand)
    for lost in (-1, 2):
        dg = DevGroup(grp, 16, lost)
        _, flags = run([dg])
        assert flags == 0
        assert np.array_equal(dg.result(), ref)


@pytest.mark.parametrize("steps", [1, 2, 7])
@pytest.mark.parametrize("ring_waves", [1, 4])
def test_tuning_steps(steps, ring_waves):
    grp = make("conv", 4, 30001, 129, 12, 8)
    ref = oracle.apply("conv", grp.c, grp.operand)
    dg = DevGroup(grp, 12, 1, ring_waves=ring_waves)
    run([dg], conv_steps=steps, stream_steps=steps)
    assert np.array_equal(dg.result(), ref)


@pytest.mark.parametrize("mode,m_lo", [("entangled", 3), ("plain", 1), ("plain_same", 1),
                                       ("checksum", 2), ("checksum_same", 2)])
def test_every_convolution_variant(mode, m_lo):
    """Every (M, digit-count) kernel variant the planner can pick for this
    mode, in each LDS layout (block ring with 4 or 1 tap copies, per-wave
    rings), on a short convolution with a ragged tail, with and without a
    lost stream: inputs of 1, 2, 8, 9, 12, 15, 16, 17, 24, 25 and 31 bits
    (words split into two fields at 1-15 bits for M = 3, at 1-8 for M = 4)."""
    ran = 0
    for M in range(m_lo, 9):
        for bits in (1, 2, 8, 9, 12, 15, 16, 17, 24, 25, 31):
            grp = make("conv", M, 1500, 7, bits, seed=7000 + 100 * M + bits)
            ref = oracle.apply("conv", grp.c, grp.operand)
            for lost, rw, tc in ([(-1, 4, 4), (M - 1, 1, 0), (M - 1, 4, 1)]
                                 if mode in ("entangled", "checksum", "checksum_same")
                                 else [(-1, 4, 4), (-1, 1, 0), (-1, 4, 1)]):
                dg = DevGroup(grp, bits, lost, mode, ring_waves=rw, tap_copies=tc)
                try:
                    _, flags = run([dg], mode)
                except ne.NeError as e:
                    assert e.status == -2, (mode, M, bits, e)  # only the range check may refuse
                    continue
                assert flags == 0, (mode, M, bits, lost, flags)
                assert np.array_equal(dg.result(), ref), (mode, M, bits, lost)
                ran += 1
    assert ran > 0


@pytest.mark.parametrize("ring_waves,tap_copies", [(1, 0), (4, 4), (4, 1)])
def test_sparse_top_tap_digit_windows(ring_waves, tap_copies):
    """16-bit taps need a third balanced digit only above 127 * 257; the
    kernel runs that digit plane just for the 64-wide chunks whose operand
    fragments touch such a tap. One large tap at chunk edges, every loss."""
    g = wl.rng(99)
    M, n, K = 3, 3000, 200
    c = wl.uniform_i32(g, -(1 << 15), 1 << 15, (M, n))
    for pos in (0, 14, 15, 63, 64, 78, 79, 127, 128, 142, 143, 199):
        k = wl.uniform_i32(g, -30000, 30000, K)
        k[pos] = 32767 - pos % 7
        grp = wl.Group("conv", c, k)
        ref = oracle.apply("conv", grp.c, grp.operand)
        for lost in (-1, 0, 2):
            dg = DevGroup(grp, 16, lost, ring_waves=ring_waves, tap_copies=tap_copies)
            _, flags = run([dg], conv_steps=2)
            assert flags == 0
            assert np.array_equal(dg.result(), ref), (pos, lost)


# ------------------------------------- the other operators in the fused path

def make_more(op, M, n, K, bits, seed):
    """Subtraction and product take a vector of n values, circular
    convolution and cross-correlation K taps, the outer product K values."""
    g = wl.rng(seed)
    lo, hi = -(1 << (bits - 1)), 1 << (bits - 1)
    c = wl.uniform_i32(g, lo, hi, (M, n))
    operand = wl.uniform_i32(g, lo, hi, K if op in ("circ", "xcorr", "outer") else n)
    return wl.Group(op, c, operand, 0)


@pytest.mark.parametrize("mode", ["entangled", "plain", "plain_same", "checksum", "checksum_same"])
@pytest.mark.parametrize("op", ["sub", "mul"])
@pytest.mark.parametrize("M", [3, 5, 8])
def test_more_streaming_ops_fused(mode, op, M):
    """Subtraction (operand entangled on the fly, footnote 3; M g for the
    checksum stream) and element-by-element product in the element-wise
    fused kernel, ragged lengths, every mode and loss position."""
    for n in (1, 255, 4097, 70001):
        grp = make_more(op, M, n, 0, 10, seed=n * 17 + M + len(op))
        ref = oracle.apply(op, grp.c, grp.operand)
        losses = [-1, 0, M - 1] if mode in ("entangled", "checksum", "checksum_same") else [-1]
        for lost in losses:
            dg = DevGroup(grp, 10, lost, mode)
            _, flags = run([dg], mode)
            assert flags == 0
            assert np.array_equal(dg.result(), ref), (mode, op, M, n, lost)


@pytest.mark.parametrize("mode", ["entangled", "plain", "plain_same", "checksum", "checksum_same"])
@pytest.mark.parametrize("M", [3, 5, 8])
@pytest.mark.parametrize("n,K", [(1, 1), (5, 3), (1001, 1), (777, 13), (4097, 64), (3, 1500)])
def test_outer_product_fused(mode, M, n, K):
    """The outer product in the element-wise fused kernel: lanes over the
    n K outputs (input o / K, operand value o mod K), ragged in both, every
    mode and loss position; outputs equal the oracle's row-major product."""
    grp = make_more("outer", M, n, K, 10, seed=n * 7 + K + M)
    ref = oracle.apply("outer", grp.c, grp.operand)
    losses = [-1, 0, M - 1] if mode in ("entangled", "checksum", "checksum_same") else [-1]
    for lost in losses:
        dg = DevGroup(grp, 10, lost, mode)
        _, flags = run([dg], mode)
        assert flags == 0
        assert np.array_equal(dg.result(), ref), (mode, M, n, K, lost)


@pytest.mark.parametrize("mode", ["entangled", "plain", "plain_same", "checksum", "checksum_same"])
@pytest.mark.parametrize("op", ["circ", "xcorr"])
@pytest.mark.parametrize("M", [3, 8])
@pytest.mark.parametrize("n,K,bits", [(1, 1, 8), (5, 3, 12), (3001, 37, 12), (700, 1500, 10),
                                      (2049, 1024, 16)])
def test_circular_and_cross_correlation_fused(mode, op, M, n, K, bits):
    """The convolution kernel with the window wrapped modulo n (taps longer
    than the stream wrap more than once) or with the taps reversed, in every
    LDS layout, every mode and loss position."""
    grp = make_more(op, M, n, K, bits, seed=M * 1000 + n + K + len(op))
    ref = oracle.apply(op, grp.c, grp.operand)
    losses = [-1, 0, M - 1] if mode in ("entangled", "checksum", "checksum_same") else [-1]
    for lost in losses:
        for rw, tc in ((4, 4), (1, 0), (4, 1)):
            dg = DevGroup(grp, bits, lost, mode, ring_waves=rw, tap_copies=tc)
            try:
                _, flags = run([dg], mode, conv_steps=3)
            except ne.NeError as e:
                assert e.status == -4 and rw == 1, (mode, M, K, rw, e)  # windows too large for LDS
                continue
            assert flags == 0, (mode, op, lost, flags, rw, tc)
            assert np.array_equal(dg.result(), ref), (mode, op, M, n, K, lost, rw, tc)


def test_all_operators_in_one_captured_plan():
    """Groups of all ten operators with uneven M, lengths and losses in one
    plan, captured as a graph and replayed twice with eager work in between:
    every replay matches the oracle."""
    rng = wl.rng(4242)
    specs = []
    for i, op in enumerate(["conv", "scale", "add", "inner", "perm", "sub", "mul", "circ",
                            "xcorr", "outer"] * 3):
        M = int(rng.integers(3, 9))
        n = int(rng.integers(1, 20000))
        if op == "outer":
            grp = make_more(op, M, n // 16 + 1, int(rng.integers(1, 40)), 10, seed=5000 + i)
        elif op in ("conv", "circ", "xcorr"):
            grp = make_more("circ", M, n, int(rng.integers(1, 300)), 10, seed=5000 + i)
            grp = wl.Group(op, grp.c, grp.operand, 0)
        elif op in ("sub", "mul"):
            grp = make_more(op, M, n, 0, 10, seed=5000 + i)
        else:
            grp = make(op, M, n, 0, 10, seed=5000 + i)
        specs.append((grp, DevGroup(grp, 10, int(rng.integers(-1, M)))))
    plan = ne.Plan([d.spec for _, d in specs], "entangled")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(s)
        for rep in range(2):
            for _, d in specs:
                for o in d.out:
                    o.fill_(POISON)
            plan.launch(s)
            s.synchronize()
            assert plan.flags() == 0
            for grp, d in specs:
                assert np.array_equal(d.result(), d.reference()), (grp.op, grp.M, grp.n, rep)
    plan.close()


def test_split_words_take_fewer_digit_planes():
    """12-bit samples at M = 3 (the batched workload's range): entangled
    words run on 2 + 2 digit planes (split at bit l) instead of 5, so the
    matrix-core work issued is twice the plain convolution's (2 planes), not
    2.5 times; plain-same issues what the entangled run does, the checksum
    method on that datapath 4/3 of it (one more stream). Bit-exact in every
    mode."""
    grp = make("conv", 3, 20000, 64, 12, seed=4321)
    ref = oracle.apply("conv", grp.c, grp.operand)
    macs = {}
    for mode in ("entangled", "plain", "plain_same", "checksum_same"):
        dg = DevGroup(grp, 12, -1, mode)
        plan, flags = run([dg], mode)
        assert flags == 0 and np.array_equal(dg.result(), ref), mode
        macs[mode] = plan.stats()["mfma_macs"]
        plan.close()
    assert macs["entangled"] == 2 * macs["plain"]
    assert macs["plain_same"] == macs["entangled"]
    assert 3 * macs["checksum_same"] == 4 * macs["entangled"]
