"""GPU parity of the 32-bit word path (ne_*32): entangle, every LSB
operation and extraction in int32 words, through the C-ABI, against the CPU
oracle run at w = 32 on the same seeded inputs, bit for bit. Input ranges
keep every output within D of ne_params(M, 32)."""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
POISON = -0x5A5A5A5B


def dev32(a, offset=0):
    """An int32 device copy of a; with offset > 0 it starts `offset` words
    into a larger buffer (not 16-byte aligned: the one-position kernels)."""
    a = np.ascontiguousarray(a, dtype=np.int32)
    buf = torch.zeros(a.size + offset + 1, dtype=torch.int32, device=DEV)
    t = buf[offset:offset + a.size]
    if a.size:
        t.copy_(torch.from_numpy(a))
    return t


def empty32(M, n, offset=0, fill=None):
    out = []
    for _ in range(M):
        buf = torch.empty(n + offset + 1, dtype=torch.int32, device=DEV)
        if fill is not None:
            buf.fill_(fill)
        out.append(buf[offset:offset + n])
    return out


def host(ts):
    torch.cuda.synchronize()
    return np.stack([t.cpu().numpy().astype(np.int64) for t in ts])


# op -> (sample half-range, operand half-range, operand length or None for
# a length-n operand); all within D(M = 3, w = 32) = 1,046,528 at n <= 4099
RANGES = {"conv": (128, 128, 16), "circ": (128, 128, 16), "xcorr": (128, 128, 16),
          "scale": (1 << 12, None, 0), "add": (1 << 18, 1 << 18, None),
          "sub": (1 << 18, 1 << 18, None), "mul": (1 << 9, 1 << 9, None),
          "inner": (15, 15, None), "perm": (1 << 19, None, None), "outer": (1 << 9, 1 << 9, 8)}


def make_case(op, M, n, seed):
    rng = wl.rng(seed)
    a, b, K = RANGES[op]
    c = wl.uniform_i32(rng, -a, a, (M, n))
    g, s = None, 0
    if op == "scale":
        s = -201
    elif op == "perm":
        g = rng.permutation(n).astype(np.int32)
    else:
        g = wl.uniform_i32(rng, -b, b, n if K is None else K)
    return c, g, s


def run32(c, op, g, s, lost, offset=0):
    """entangle32 -> lsb_apply32 on every stream but `lost` -> extract32.
    Returns (eps, delta, dhat) on the host."""
    M, n = c.shape
    l = ne.params(M, 32)[0]
    cd = [dev32(row, offset) for row in c]
    eps = empty32(M, n, offset)
    ne.entangle32(cd, eps, l, n=n)
    operand = None
    if g is not None:
        operand = dev32(g, offset)
        if op in ("add", "sub"):
            ge = empty32(1, n, offset)[0]
            ne.entangle_operand32(operand, ge, l)
            operand = ge
    no = ne.n_out(op, n, 0 if g is None else g.size)
    delta = empty32(M, no, offset, fill=POISON)
    mask = (1 << M) - 1 & ~(1 << lost if lost >= 0 else 0)
    ne.lsb_apply32(op, eps, operand, delta, scalar=s, mask=mask, n_in=n)
    dhat = empty32(M, no, offset, fill=POISON)
    ne.extract_recover32([None if m == lost else delta[m] for m in range(M)], lost, dhat, l, n=no)
    return host(eps), host(delta), host(dhat)


@pytest.mark.parametrize("op", list(RANGES))
@pytest.mark.parametrize("M", [3, 4, 5, 8])
def test_word32_pipeline_matches_oracle(op, M):
    """Every step at w = 32 equals the oracle at w = 32, and the recovered
    outputs equal the plain operation, for no loss and each of three lost
    streams; the lost stream's words are never written."""
    n = 4099
    c, g, s = make_case(op, M, n, 9100 + 17 * M + list(RANGES).index(op))
    want = oracle.apply(op, c, g, s)
    for lost in (-1, 0, M // 2, M - 1):
        d_or, eps_or, delta_or = oracle.pipeline(c, op, g, s, r=max(lost, 0), w=32)
        assert np.array_equal(d_or, want), (op, M, lost)
        eps, delta, dhat = run32(c, op, g, s, lost)
        assert np.array_equal(eps, eps_or), (op, M, lost)
        live = [m for m in range(M) if m != lost]
        assert np.array_equal(delta[live], delta_or[live]), (op, M, lost)
        if lost >= 0:
            assert (delta[lost] == POISON).all()
        assert np.array_equal(dhat, want), (op, M, lost)


@pytest.mark.parametrize("op", ["conv", "scale", "add", "perm", "xcorr"])
def test_word32_unaligned_buffers(op):
    """Buffers one word past a 16-byte boundary take the one-position
    kernels; results are the same."""
    M, n = 3, 1001
    c, g, s = make_case(op, M, n, 9300)
    _, _, dhat = run32(c, op, g, s, 1, offset=1)
    assert np.array_equal(dhat, oracle.apply(op, c, g, s))


@pytest.mark.parametrize("M", [3, 6, 9, 12, 16, 17])
def test_word32_every_group_size(M):
    """Entanglement and recovery for group sizes up to the largest that
    w = 32 admits (M = 17: l = 2, k = 0), at the edge of the range
    (samples of magnitude D and -D), every lost stream."""
    l, _, D = ne.params(M, 32)
    n = 1031
    rng = wl.rng(9400 + M)
    c = rng.integers(-D, D + 1, size=(M, n)).astype(np.int64)
    c[:, 0], c[:, 1] = D, -D
    c32 = c.astype(np.int32)
    assert np.array_equal(c32, c)
    for lost in range(-1, M):
        d_or, eps_or, _ = oracle.pipeline(c, "scale", None, 1, r=max(lost, 0), w=32)
        eps, _, dhat = run32(c32, "scale", None, 1, lost)
        assert np.array_equal(eps, eps_or), (M, lost)
        assert np.array_equal(dhat, c), (M, lost)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5])
def test_word32_tiny_streams(n):
    """Empty streams and streams shorter than one 4-position group; the
    circular convolution with more taps than samples wraps them."""
    M = 4
    for op in ("conv", "circ", "inner", "outer", "mul"):
        c, g, s = make_case(op, M, n, 9500 + n)
        if op == "circ" and n:
            g = wl.uniform_i32(wl.rng(9501), -128, 128, 37)
        _, _, dhat = run32(c, op, g, s, 2)
        assert np.array_equal(dhat, oracle.apply(op, c, g, s).reshape(dhat.shape)), (op, n)


def test_word32_small_configuration_full_size():
    """The small configuration (3 streams of 65,536 int32 samples in
    [-2^7, 2^7), 16-tap convolution, worst case 2^18 within D = 1,046,528 at
    w = 32) compared in full, each stream lost in turn."""
    M, n, K = 3, 1 << 16, 16
    rng = wl.rng(wl.SEED_BASE + 1)
    c = wl.uniform_i32(rng, -128, 128, (M, n))
    g = wl.uniform_i32(rng, -128, 128, K)
    want = oracle.apply("conv", c, g)
    for lost in (-1, 0, 1, 2):
        _, _, dhat = run32(c, "conv", g, 0, lost)
        assert np.array_equal(dhat, want), lost


def test_word32_benchmark_size():
    """The size the benchmark times (3 streams of 2^22 samples in
    [-2^7, 2^7), 16 taps) with stream 1 lost: sampled outputs against the
    oracle's convolution at those positions, and every output against the
    64-bit path's result."""
    M, n, K = 3, 1 << 22, 16
    rng = wl.rng(wl.SEED_BASE + 11)
    c = wl.uniform_i32(rng, -128, 128, (M, n))
    g = wl.uniform_i32(rng, -128, 128, K)
    _, _, dhat = run32(c, "conv", g, 0, 1)
    pos = np.unique(np.concatenate([np.arange(64), np.arange(n - 64, n + K - 1),
                                    wl.rng(7).integers(0, n + K - 1, 4000)]))
    for m in range(M):
        assert np.array_equal(dhat[m, pos], oracle.conv_at(c[m], g, pos)), m
    # the 64-bit path on the same inputs: every output
    l64 = ne.params(M)[0]
    cd = [dev32(row) for row in c]
    eps = [torch.empty(n, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.entangle(cd, eps, l64)
    no = n + K - 1
    delta = [torch.empty(no, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.lsb_apply("conv", eps, dev32(g), delta, mask=0b101)
    out = [torch.empty(no, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.extract_recover([delta[0], None, delta[2]], 1, out, l64)
    torch.cuda.synchronize()
    for m in range(M):
        assert np.array_equal(dhat[m], out[m].cpu().numpy()), m


# ------------------------------------------------ fused executor, w = 32

MODES = ["entangled", "plain", "plain_same", "checksum"]


def fused32(c, op, g, s, mode, lost, bits, K=None, **spec_kw):
    """One group with word_bits = 32 in a plan: int32 outputs (poisoned
    first); returns (outputs, flags)."""
    M, n = c.shape
    cd = [dev32(row) for row in c]
    gd = None if g is None else dev32(g)
    no = ne.n_out(op, n, 0 if g is None else g.size)
    out = empty32(M, no, fill=POISON)
    spec = ne.GroupSpec(op, cd, gd, out, s, lost, bits, word_bits=32, **spec_kw)
    plan = ne.Plan([spec], mode)
    plan.run()
    torch.cuda.synchronize()
    flags = plan.flags()
    plan.close()
    return host(out), flags


def fused_case(op, M, n, seed, bits):
    rng = wl.rng(seed)
    lo, hi = -(1 << (bits - 1)), 1 << (bits - 1)
    c = wl.uniform_i32(rng, lo, hi, (M, n))
    g, s = None, 0
    if op in ("conv", "circ", "xcorr", "outer"):
        g = wl.uniform_i32(rng, lo, hi, 16)
    elif op == "perm":
        g = rng.permutation(n).astype(np.int32)
    elif op == "scale":
        s = int(rng.integers(lo, hi))
    else:
        g = wl.uniform_i32(rng, lo, hi, n)
    return c, g, s


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("op", ["conv", "circ", "xcorr", "scale", "add", "sub", "mul", "inner",
                                "perm", "outer"])
@pytest.mark.parametrize("M", [3, 5, 8])
def test_fused_word32_matches_oracle(mode, op, M):
    """Every fused operation in every mode with 32-bit words (l and D of
    w = 32, int32 outputs): bit-exact against the oracle, every output
    written, no flag raised; entangled and checksum groups also with a lost
    stream."""
    bits = 7 if op != "inner" else 5
    for n in (1, 5, 3001):
        c, g, s = fused_case(op, M, n, 9600 + 31 * M + n + len(op), bits)
        want = oracle.apply(op, c, g, s)
        if mode == "entangled":
            # the same values through the oracle's w = 32 pipeline
            assert np.array_equal(oracle.pipeline(c, op, g, s, r=1, w=32)[0], want)
        losses = [-1, 1, M - 1] if mode in ("entangled", "checksum") else [-1]
        for lost in losses:
            got, flags = fused32(c, op, g, s, mode, lost, bits)
            assert flags == 0, (mode, op, M, n, lost, flags)
            assert np.array_equal(got, want), (mode, op, M, n, lost)


@pytest.mark.parametrize("mode,m_lo", [("entangled", 3), ("plain_same", 1)])
def test_fused_word32_every_convolution_variant(mode, m_lo):
    """Every input width that 32-bit words admit for a convolution (the
    digit counts follow the shorter shift l of w = 32), each LDS layout,
    against the oracle; the range check refuses the rest."""
    ran = 0
    for M in range(m_lo, 9):
        for bits in range(1, 17):
            rng = wl.rng(9700 + 100 * M + bits)
            lo, hi = -(1 << (bits - 1)), 1 << (bits - 1)
            c = wl.uniform_i32(rng, lo, hi, (M, 1500))
            g = wl.uniform_i32(rng, lo, hi, 1)
            want = oracle.apply("conv", c, g)
            for rw, tc in ((4, 4), (1, 0), (4, 1)):
                lost = M - 1 if mode == "entangled" else -1
                try:
                    got, flags = fused32(c, "conv", g, 0, mode, lost, bits, ring_waves=rw,
                                         tap_copies=tc)
                except ne.NeError as e:
                    assert e.status == -2, (mode, M, bits, e)
                    continue
                assert flags == 0, (mode, M, bits, rw, tc)
                assert np.array_equal(got, want), (mode, M, bits, rw, tc)
                ran += 1
    assert ran > 0


def test_fused_word32_and_word64_groups_in_one_captured_plan():
    """Groups of both word widths share the plan's launches; the captured
    graph is replayed three times with eager work in between, each replay
    against the oracle."""
    M, n = 3, 5000
    rng = wl.rng(9800)
    specs, wants, outs = [], [], []
    for wb, op, K in ((32, "conv", 16), (0, "conv", 16), (32, "scale", 0), (0, "add", 0),
                      (32, "perm", 0), (32, "inner", 0)):
        bits = 4 if op == "inner" else 8
        c, g, s = fused_case(op, M, n, int(rng.integers(1 << 30)), bits)
        cd = [dev32(row) for row in c]
        no = ne.n_out(op, n, 0 if g is None else g.size)
        if wb == 32:
            out = empty32(M, no, fill=POISON)
        else:
            out = [torch.full((no,), POISON, dtype=torch.int64, device=DEV) for _ in range(M)]
        specs.append(ne.GroupSpec(op, cd, None if g is None else dev32(g), out, s, 1, bits,
                                  word_bits=wb))
        wants.append(oracle.apply(op, c, g, s))
        outs.append(out)
    plan = ne.Plan(specs, "entangled")
    stream = torch.cuda.Stream()
    plan.capture(stream)
    for rep in range(3):
        for out in outs:
            for t in out:
                t.fill_(POISON if t.dtype == torch.int32 else -7)
        torch.cuda.synchronize()
        plan.launch(stream)
        stream.synchronize()
        assert plan.flags() == 0
        for out, want in zip(outs, wants):
            assert np.array_equal(host(out), want), rep
    plan.close()


def test_fused_word32_benchmark_size():
    """The w = 32 benchmark workload in the fused executor (3 streams of 2^22
    samples in [-2^7, 2^7), 16 taps, stream 1 lost): sampled outputs against
    the oracle's convolution at those positions."""
    M, n, K = 3, 1 << 22, 16
    rng = wl.rng(wl.SEED_BASE + 11)
    c = wl.uniform_i32(rng, -128, 128, (M, n))
    g = wl.uniform_i32(rng, -128, 128, K)
    got, flags = fused32(c, "conv", g, 0, "entangled", 1, 8)
    assert flags == 0
    pos = np.unique(np.concatenate([np.arange(64), np.arange(n - 64, n + K - 1),
                                    wl.rng(8).integers(0, n + K - 1, 4000)]))
    for m in range(M):
        assert np.array_equal(got[m, pos], oracle.conv_at(c[m], g, pos)), m


# ------------------------------------------------- series, w = 32

SERIES = [wl.CHAIN_RECIPE, ("conv", "conv"), ("scale", "perm", "inner", "scale"),
          ("perm", "add", "conv", "inner"), ("sub", "mul", "circ", "xcorr"),
          ("outer", "sub", "perm"),
          # a convolution before a permutation-led run writes interleaved rows
          ("conv", "perm", "conv", "perm", "add"), ("circ", "perm", "scale"), ("xcorr", "perm")]


def device_ops32(ops, l, bits):
    """ChainOps with int32 device operands; an added or subtracted vector
    entangled with itself in 32-bit words."""
    dops = []
    for op, g, s in ops:
        if op == "scale":
            dops.append(ne.ChainOp(op, None, s))
            continue
        dg = dev32(g)
        if op in ("add", "sub"):
            ge = empty32(1, g.size)[0]
            ne.entangle_operand32(dg, ge, l)
            dg = ge
        dops.append(ne.ChainOp(op, dg, s, operand_bits=bits))
    return dops


def series32(c, ops, lost, bits):
    """entangle32 -> the series on every stream but `lost` (ne_chain_apply32)
    -> extract32; returns (recovered outputs, last-stage words)."""
    M, n = c.shape
    l = ne.params(M, 32)[0]
    dops = device_ops32(ops, l, bits)
    no, _ = ne.chain_check(M, bits, n, dops, w=32)
    cd = [dev32(r) for r in c]
    eps = empty32(M, n)
    ne.entangle32(cd, eps, l, n=n)
    delta = empty32(M, no, fill=POISON)
    mask = ((1 << M) - 1) & ~(1 << lost if lost >= 0 else 0)
    ne.chain_apply(eps, dops, delta, mask=mask, n_in=n, w=32)
    dhat = empty32(M, no, fill=POISON)
    ne.extract_recover32([None if m == lost else delta[m] for m in range(M)], lost, dhat, l, n=no)
    return host(dhat), host(delta)


@pytest.mark.parametrize("recipe", SERIES)
@pytest.mark.parametrize("M", [3, 5, 8])
def test_word32_series_matches_oracle(recipe, M):
    """A series between one entanglement and one extraction in 32-bit words
    (2-bit samples and operands keep every stage within D of w = 32):
    the recovered outputs equal the plain series, the live streams' last
    stage equals the oracle's w = 32 pipeline, for no loss and two losses."""
    n = 3001
    rng = wl.rng(9900 + M + len(recipe))
    c = wl.uniform_i32(rng, -2, 2, (M, n))
    ops = wl.chain_series(rng, n, recipe, bits=2, K=9)
    want = oracle.chain(c, ops)
    _, last = oracle.chain_pipeline(c, ops, r=0, w=32)
    for lost in (-1, 0, M - 1):
        dhat, delta = series32(c, ops, lost, 2)
        assert np.array_equal(dhat, want), (recipe, M, lost)
        live = [m for m in range(M) if m != lost]
        assert np.array_equal(delta[live], last[live]), (recipe, M, lost)


WHOLE32 = SERIES + [("scale", "add", "sub"), ("perm",), ("perm", "mul"), ("conv", "scale", "perm"),
                    ("add", "conv")]


@pytest.mark.parametrize("recipe", WHOLE32)
@pytest.mark.parametrize("M", [3, 5, 8, 17])
def test_word32_series_in_one_call(recipe, M):
    """ne_chain_run32: int32 samples in, recovered int32 outputs out, the
    entanglement and recovery folded into the series' first and last runs of
    element-wise operations (one pass for a single run); every recipe against
    the oracle and the three-call path, with and without a lost stream, up to
    the widest group of 32-bit words (M = 17)."""
    n = 3001
    rng = wl.rng(9950 + M + len(recipe))
    c = wl.uniform_i32(rng, -2, 2, (M, n))
    ops = wl.chain_series(rng, n, recipe, bits=2, K=9)
    want = oracle.chain(c, ops)
    l = ne.params(M, 32)[0]
    dops = device_ops32(ops, l, 2)
    no, _ = ne.chain_check(M, 2, n, dops, w=32)
    cd = [dev32(r) for r in c]
    for lost in (-1, 0, M - 1):
        dhat = empty32(M, no, fill=POISON)
        ne.chain_run(cd, dops, dhat, lost, w=32)
        assert np.array_equal(host(dhat), want), (recipe, M, lost)
        three, _ = series32(c, ops, lost, 2)
        assert np.array_equal(three, want), (recipe, M, lost)


@pytest.mark.parametrize("recipe,n", [(("conv", "scale"), 0), (("scale",), 1), (("perm",), 1),
                                      (("conv",), 5), (("add", "perm"), 2),
                                      (("conv", "perm"), 3)])
def test_word32_series_in_one_call_edge_cases(recipe, n):
    """ne_chain_run32 on empty and one- to five-sample streams, one-operation
    series (no workspace), rows after a tiny convolution."""
    M = 4
    c = wl.uniform_i32(wl.rng(9980 + n), -2, 2, (M, n))
    ops = wl.chain_series(wl.rng(9990 + n), n, recipe, bits=2, K=3)
    want = oracle.chain(c, ops)
    l = ne.params(M, 32)[0]
    dops = device_ops32(ops, l, 2)
    no, _ = ne.chain_check(M, 2, n, dops, w=32)
    cd = [dev32(r) for r in c]
    for lost in (-1, 2):
        dhat = empty32(M, no, fill=POISON)
        ne.chain_run(cd, dops, dhat, lost, w=32)
        assert np.array_equal(host(dhat), want), (recipe, n, lost)


def _conv_mod32(x, g, kind):
    """The convolution kinds modulo 2^32 by definition (uint64 products and
    sums wrap modulo 2^64, a multiple of 2^32)."""
    xu = x.astype(np.int64).astype(np.uint64)
    gu = g.astype(np.int64).astype(np.uint64)
    n, K = x.size, g.size
    if kind == "xcorr":
        gu = gu[::-1].copy()
    if kind == "circ":
        y = np.zeros(n, dtype=np.uint64)
        for j in range(K):
            y += gu[j] * np.roll(xu, j)
    else:
        y = np.zeros(n + K - 1, dtype=np.uint64)
        for j in range(K):
            y[j:j + n] += gu[j] * xu
    return (y & np.uint64(0xFFFFFFFF)).astype(np.int64)


@pytest.mark.parametrize("case", ["one_wide", "all_wide", "second_chunk", "narrow"])
@pytest.mark.parametrize("kind", ["conv", "circ", "xcorr"])
def test_word32_convolution_tap_width(case, kind):
    """The 32-bit convolution kinds on arbitrary 32-bit words (the whole
    int32 range) against their definition modulo 2^32: one wide tap among
    narrow ones, all taps wide, a wide tap in the second 1024-tap chunk only,
    taps at the edges of 24 signed bits."""
    rng = wl.rng(9970 + len(case) + len(kind))
    n = 3000
    x = wl.uniform_i32(rng, -(1 << 31), 1 << 31, (2, n))
    if case == "one_wide":
        g = wl.uniform_i32(rng, -100, 100, 8)
        g[3] = (1 << 24) + 3
    elif case == "all_wide":
        g = wl.uniform_i32(rng, 1 << 23, 1 << 30, 5) * np.int32(-1)
    elif case == "second_chunk":
        g = wl.uniform_i32(rng, -(1 << 23), 1 << 23, 1100)
        g[1050] = -(1 << 23) - 1
    else:
        g = np.array([-(1 << 23), (1 << 23) - 1, -1, 0, 1], dtype=np.int32)
    eps = [dev32(r) for r in x]
    no = ne.n_out(kind, n, g.size)
    out = empty32(2, no, fill=POISON)
    ne.lsb_apply32(kind, eps, dev32(g), out)
    got = host(out) & 0xFFFFFFFF
    for m in range(2):
        assert np.array_equal(got[m], _conv_mod32(x[m], g, kind)), (case, kind, m)
