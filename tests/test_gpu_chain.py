"""Series of LSB operations on entangled streams (ne_chain_*): one
entanglement, the whole series on every stream, one extraction; bit-exact
against the CPU oracle, with and without a lost stream."""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
POISON = -0x5A5A5A5A5A5A5A5A

SERIES = [wl.CHAIN_RECIPE, ("conv", "conv"), ("scale", "perm", "inner", "scale"),
          ("perm", "add", "conv", "inner"), ("add",), ("inner", "conv", "add"),
          ("sub", "mul", "circ", "xcorr"), ("outer", "sub", "perm"),
          # a convolution before a permutation-led run writes interleaved rows
          ("conv", "perm", "conv", "perm", "add"), ("circ", "perm", "scale"), ("xcorr", "perm")]


def dev32(a):
    """An int32 device copy; empty arrays get a zero-length view of a
    one-element buffer (a device address the library accepts)."""
    a = np.ascontiguousarray(a, dtype=np.int32)
    if a.size == 0:
        return torch.zeros(1, dtype=torch.int32, device=DEV)[:0]
    return torch.from_numpy(a).to(DEV)


def device_ops(ops, l, bits, entangled=True):
    """ChainOps with device operands; an added vector is entangled with
    itself for entangled streams (footnote 3), widened to int64 otherwise."""
    out = []
    for op, g, s in ops:
        if op == "scale":
            out.append(ne.ChainOp(op, None, s))
            continue
        dg = dev32(g)
        if op in ("add", "sub"):
            if entangled:
                ge = torch.empty(max(g.size, 1), dtype=torch.int64, device=DEV)[:g.size]
                ne.entangle_operand(dg, ge, l)
                dg = ge
            else:
                dg = dg.to(torch.int64)
        out.append(ne.ChainOp(op, dg, s, operand_bits=bits))
    return out


def run_series(c, ops, lost, in_bits, bits):
    """Entangle, the series on the streams other than `lost`, extract.
    Returns (recovered outputs, last-stage entangled outputs) on the host."""
    M, n = c.shape
    l = ne.params(M)[0]
    dops = device_ops(ops, l, bits)
    no, _ = ne.chain_check(M, in_bits, n, dops)
    cd = [dev32(r) for r in c]
    eps = [torch.empty(max(n, 1), dtype=torch.int64, device=DEV)[:n] for _ in range(M)]
    ne.entangle(cd, eps, l)
    delta = [torch.full((max(no, 1),), POISON, dtype=torch.int64, device=DEV)[:no]
             for _ in range(M)]
    mask = ((1 << M) - 1) & ~(1 << lost if lost >= 0 else 0)
    ne.chain_apply(eps, dops, delta, mask=mask)
    dhat = [torch.full((max(no, 1),), POISON, dtype=torch.int64, device=DEV)[:no]
            for _ in range(M)]
    ne.extract_recover([None if m == lost else delta[m] for m in range(M)], lost, dhat, l, n=no)
    torch.cuda.synchronize()
    return (np.stack([t.cpu().numpy() for t in dhat]),
            np.stack([t.cpu().numpy() for t in delta]))


@pytest.mark.parametrize("recipe", SERIES)
@pytest.mark.parametrize("M", [3, 5, 8])
def test_series_recovers_plain_result(recipe, M):
    """Every recipe within D(M = 3): 6-bit samples and operands."""
    n = 3001
    c = wl.uniform_i32(wl.rng(300 + M), -32, 32, (M, n))
    ops = wl.chain_series(wl.rng(400 + M), n, recipe, bits=6, K=37)
    want = oracle.chain(c, ops)
    _, last = oracle.chain_pipeline(c, ops, r=0)
    for lost in (-1, 0, M - 1):
        dhat, delta = run_series(c, ops, lost, 6, 6)
        assert np.array_equal(dhat, want), (recipe, M, lost)
        live = [m for m in range(M) if m != lost]
        assert np.array_equal(delta[live], last[live]), (recipe, M, lost)


@pytest.mark.parametrize("recipe,n", [(("conv", "scale"), 0), (("inner", "conv"), 0),
                                      (("scale",), 1), (("perm", "inner"), 1), (("conv",), 5)])
def test_series_edge_cases(recipe, n):
    """Empty and one-sample streams, a single operation (no workspace)."""
    M = 4
    c = wl.uniform_i32(wl.rng(500 + n), -100, 100, (M, n))
    ops = wl.chain_series(wl.rng(600 + n), n, recipe, bits=8, K=3)
    want = oracle.chain(c, ops)
    for lost in (-1, 2):
        dhat, _ = run_series(c, ops, lost, 8, 8)
        assert np.array_equal(dhat, want), (recipe, n, lost)


def test_series_on_plain_streams():
    """The failure-intolerant baseline of a series: the same launches on raw
    (not entangled) int64 words."""
    M, n = 3, 2000
    c = wl.uniform_i32(wl.rng(700), -512, 512, (M, n))
    ops = wl.chain_series(wl.rng(701), n, wl.CHAIN_RECIPE, bits=10, K=21)
    dops = device_ops(ops, 0, 10, entangled=False)
    x = [dev32(r).to(torch.int64) for r in c]
    no = n + 20
    out = [torch.empty(no, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.chain_apply(x, dops, out)
    got = np.stack([t.cpu().numpy() for t in out])
    assert np.array_equal(got, oracle.chain(c, ops))


def test_series_benchmark_size():
    """The series the benchmark times, at its size (3 streams of 2^22
    samples, 64-tap convolution), one stream lost, compared in full."""
    M, n = 3, 1 << 22
    c = wl.uniform_i32(wl.rng(wl.SEED_BASE + 6), -512, 512, (M, n))
    ops = wl.chain_series(wl.rng(wl.SEED_BASE + 7), n, wl.CHAIN_RECIPE, bits=10, K=64)
    dhat, _ = run_series(c, ops, 1, 10, 10)
    assert np.array_equal(dhat, oracle.chain(c, ops))


# ------------------------------------------------ the whole method in one call

def run_whole(c, ops, lost, bits):
    """ne_chain_run: int32 streams in, recovered outputs out."""
    M, n = c.shape
    l = ne.params(M)[0]
    dops = device_ops(ops, l, bits)
    no = n
    for o in dops:
        no = ne.n_out(o.op, no, o.n_operand)
    cd = [dev32(r) for r in c]
    dhat = [torch.full((max(no, 1),), POISON, dtype=torch.int64, device=DEV)[:no]
            for _ in range(M)]
    ne.chain_run(cd, dops, dhat, lost)
    torch.cuda.synchronize()
    return np.stack([t.cpu().numpy() for t in dhat])


WHOLE = SERIES + [("scale", "add", "sub"), ("perm",), ("perm", "mul"), ("conv", "scale", "perm"),
                  ("add", "conv")]


@pytest.mark.parametrize("recipe", WHOLE)
@pytest.mark.parametrize("M", [3, 5, 8])
def test_series_in_one_call_recovers_plain_result(recipe, M):
    """ne_chain_run: entanglement folded into a leading element-wise run,
    recovery into a trailing one (one pass for a series that is one such
    run), separate passes otherwise; every recipe against the oracle, with
    and without a lost stream, ragged lengths."""
    n = 3001
    c = wl.uniform_i32(wl.rng(310 + M), -32, 32, (M, n))
    ops = wl.chain_series(wl.rng(410 + M), n, recipe, bits=6, K=37)
    want = oracle.chain(c, ops)
    for lost in (-1, 0, M - 1):
        assert np.array_equal(run_whole(c, ops, lost, 6), want), (recipe, M, lost)


@pytest.mark.parametrize("recipe,n", [(("conv", "scale"), 0), (("scale",), 1), (("perm",), 1),
                                      (("conv",), 5), (("add", "perm"), 2)])
def test_series_in_one_call_edge_cases(recipe, n):
    """Empty and one- or two-sample streams, one-operation series (no
    workspace), a permutation that follows a fused run."""
    M = 4
    c = wl.uniform_i32(wl.rng(520 + n), -100, 100, (M, n))
    ops = wl.chain_series(wl.rng(620 + n), n, recipe, bits=8, K=3)
    want = oracle.chain(c, ops)
    for lost in (-1, 2):
        assert np.array_equal(run_whole(c, ops, lost, 8), want), (recipe, n, lost)


def test_series_in_one_call_benchmark_size():
    """The benchmark's series at its size through ne_chain_run, one stream
    lost, compared in full."""
    M, n = 3, 1 << 22
    c = wl.uniform_i32(wl.rng(wl.SEED_BASE + 6), -512, 512, (M, n))
    ops = wl.chain_series(wl.rng(wl.SEED_BASE + 7), n, wl.CHAIN_RECIPE, bits=10, K=64)
    got = run_whole(c, ops, 1, 10)
    assert np.array_equal(got, oracle.chain(c, ops))


@pytest.mark.parametrize("M", [8, 9])
def test_series_rows_at_the_row_limit(M):
    """Rows hold at most 8 streams: M = 8 gathers from rows with and without a
    lost stream; M = 9 gathers from planes with all 9 streams computed and
    from rows once one is lost (8 computed), through both calls."""
    n = 2001
    c = wl.uniform_i32(wl.rng(800 + M), -8, 8, (M, n))
    ops = wl.chain_series(wl.rng(810 + M), n, ("conv", "perm", "add"), bits=4, K=9)
    want = oracle.chain(c, ops)
    for lost in (-1, 0, M - 1):
        dhat, _ = run_series(c, ops, lost, 4, 4)
        assert np.array_equal(dhat, want), (M, lost)
        assert np.array_equal(run_whole(c, ops, lost, 4), want), (M, lost)


@pytest.mark.parametrize("M", [16, 32])
@pytest.mark.parametrize("recipe", [("add", "scale"), ("conv", "perm", "add"),
                                    ("scale", "conv", "add", "perm")])
def test_series_many_streams(M, recipe):
    """Groups of 16 and 32 streams (l = 4 and 2): the one-pass series (its
    entanglement and recovery in one kernel), a permutation after a
    convolution gathering from planes (past the 8-stream row limit), a
    permutation leading the last run; through both calls, with and without a
    lost stream."""
    n = 1001
    c = wl.uniform_i32(wl.rng(950 + M), -8, 8, (M, n))
    ops = wl.chain_series(wl.rng(900 + M), n, recipe, bits=4, K=5)
    want = oracle.chain(c, ops)
    for lost in (-1, 0, M - 1):
        dhat, _ = run_series(c, ops, lost, 4, 4)
        assert np.array_equal(dhat, want), (M, recipe, lost)
        assert np.array_equal(run_whole(c, ops, lost, 4), want), (M, recipe, lost)


@pytest.mark.parametrize("stream", [0, 2])
def test_series_one_computed_stream(stream):
    """ne_chain_apply with one stream in the mask: rows of one word between
    a convolution and the permutation after it; the stream's last-stage
    words equal the oracle's pipeline, the other outputs stay untouched."""
    M, n = 3, 2001
    c = wl.uniform_i32(wl.rng(840 + stream), -32, 32, (M, n))
    ops = wl.chain_series(wl.rng(850 + stream), n, ("conv", "perm", "add"), bits=6, K=21)
    _, last = oracle.chain_pipeline(c, ops, r=0)
    l = ne.params(M)[0]
    dops = device_ops(ops, l, 6)
    no, _ = ne.chain_check(M, 6, n, dops)
    cd = [dev32(r) for r in c]
    eps = [torch.empty(n, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.entangle(cd, eps, l)
    delta = [torch.full((no,), POISON, dtype=torch.int64, device=DEV) for _ in range(M)]
    ws = torch.empty(ne.chain_workspace_size(M, n, dops) + 256, dtype=torch.uint8, device=DEV)
    ws = ws[(-ws.data_ptr()) % 256:]
    ne.chain_apply(eps, dops, delta, mask=1 << stream, workspace=ws)
    torch.cuda.synchronize()
    got = np.stack([t.cpu().numpy() for t in delta])
    assert np.array_equal(got[stream], last[stream])
    for m in range(M):
        if m != stream:
            assert (got[m] == POISON).all()
