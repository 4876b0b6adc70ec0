"""GPU parity: every step of the HIP path, called through the C-ABI, against
the CPU oracle on the same seeded inputs, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
POISON = 0x5DEECE66D5DEECE6


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def streams(a, dtype):
    return [dev(row, dtype) for row in a]


def empty64(M, n, fill=None):
    out = [torch.empty(max(n, 1), dtype=torch.int64, device=DEV)[:n] for _ in range(M)]
    if fill is not None:
        for t in out:
            t.fill_(fill)
    return out


def gpu_pipeline(grp, r=-1, poison=True, inplace=False):
    """Entangle -> op on every stream except r -> extract without r."""
    M, n = grp.c.shape
    l, _, _ = ne.params(M)
    c = streams(grp.c, torch.int32)
    eps = empty64(M, n)
    ne.entangle(c, eps, l)
    operand = None
    if grp.op in ("conv", "inner", "perm", "mul", "circ", "xcorr", "outer"):
        operand = dev(grp.operand, torch.int32)
    elif grp.op in ("add", "sub"):
        g32 = dev(grp.operand, torch.int32)
        operand = torch.empty(n, dtype=torch.int64, device=DEV)
        ne.entangle_operand(g32, operand, l)
    no = ne.n_out(grp.op, n, 0 if grp.operand is None else grp.operand.size)
    delta = empty64(M, no, fill=POISON if poison else None)
    mask = (1 << M) - 1
    if r >= 0:
        mask &= ~(1 << r)
    ne.lsb_apply(grp.op, eps, operand, delta, scalar=grp.scalar, mask=mask, n_in=n)
    if r >= 0:
        # the lost stream was never written
        assert bool((delta[r] == POISON).all()) or no == 0
    dhat = delta if inplace else empty64(M, no)
    ne.extract_recover([None if j == r else t for j, t in enumerate(delta)], r, dhat, l, n=no)
    return np.stack([host(t) for t in dhat]) if no else np.zeros((M, 0), np.int64), eps


# --------------------------------------------------------------- entangle

@pytest.mark.parametrize("M", [3, 4, 5, 8, 11, 16, 32])
@pytest.mark.parametrize("n", [1, 3, 4, 5, 1023, 4099])
def test_entangle_matches_oracle(M, n):
    l, _, _ = ne.params(M)
    c = wl.uniform_i32(wl.rng(M * 1000 + n), -(1 << 11), 1 << 11, (M, n))
    eps = empty64(M, n)
    ne.entangle(streams(c, torch.int32), eps, l)
    assert np.array_equal(np.stack([host(t) for t in eps]), oracle.entangle(c, l))


def test_entangle_unaligned_views():
    M, n = 3, 1001
    l, _, _ = ne.params(M)
    c = wl.uniform_i32(wl.rng(5), -100, 100, (M, n + 1))
    base = [dev(row, torch.int32) for row in c]
    views = [t[1:] for t in base]           # 4-byte offset: scalar path
    eps_base = empty64(M, n + 1)
    eps = [t[1:] for t in eps_base]
    ne.entangle(views, eps, l)
    assert np.array_equal(np.stack([host(t) for t in eps]), oracle.entangle(c[:, 1:], l))


@pytest.mark.parametrize("M", [3, 6])
def test_entangle_inplace_and_operand(M):
    l, _, _ = ne.params(M)
    c = wl.uniform_i32(wl.rng(77), -(1 << 15), 1 << 15, (M, 3001))
    x = streams(c.astype(np.int64), torch.int64)
    ne.entangle_inplace(x, l)
    assert np.array_equal(np.stack([host(t) for t in x]), oracle.entangle(c, l))
    g = dev(c[0], torch.int32)
    ge = torch.empty(3001, dtype=torch.int64, device=DEV)
    ne.entangle_operand(g, ge, l)
    assert np.array_equal(host(ge), oracle.entangle_operand(c[0], l))


# ------------------------------------------------------------------ ops

CONV_SHAPES = [(1, 1), (7, 1), (1, 5), (3, 16), (65536, 16), (5000, 64), (1025, 1024),
               (3000, 1025), (2049, 2100)]


@pytest.mark.parametrize("n,K", CONV_SHAPES)
def test_conv_matches_oracle(n, K):
    M = 3
    l, _, _ = ne.params(M)
    g = wl.rng(n * 7 + K)
    c = wl.uniform_i32(g, -(1 << 11), 1 << 11, (M, n))
    k = wl.uniform_i32(g, -(1 << 11), 1 << 11, K)
    eps_h = oracle.entangle(c, l)
    delta = empty64(M, n + K - 1)
    ne.lsb_apply("conv", streams(eps_h, torch.int64), dev(k, torch.int32), delta)
    assert np.array_equal(np.stack([host(t) for t in delta]), oracle.apply("conv", eps_h, k))
    d = empty64(M, n + K - 1)
    ne.plain_apply("conv", streams(c, torch.int32), dev(k, torch.int32), d)
    assert np.array_equal(np.stack([host(t) for t in d]), oracle.apply("conv", c, k))


def test_conv_full_64bit_words():
    """Arbitrary 64-bit words and 32-bit taps: the product is exact modulo 2^64."""
    g = np.random.default_rng(3)
    x = g.integers(-(1 << 63), (1 << 63) - 1, size=(2, 777), dtype=np.int64)
    k = g.integers(-(1 << 31), (1 << 31) - 1, size=33, dtype=np.int64).astype(np.int32)
    y = empty64(2, 777 + 32)
    ne.lsb_apply("conv", streams(x, torch.int64), dev(k, torch.int32), y)
    ref = [[sum(int(k[j]) * int(row[t - j]) for j in range(33) if 0 <= t - j < 777) % (1 << 64)
            for t in range(0, 809, 37)] for row in x]
    got = [[int(v) % (1 << 64) for v in host(t)[::37]] for t in y]
    assert got == ref


@pytest.mark.parametrize("op", ["scale", "add", "inner", "perm"])
@pytest.mark.parametrize("n", [1, 2, 3, 1000, 4097, 70001])
def test_streaming_ops_match_oracle(op, n):
    M = 4
    l, _, _ = ne.params(M)
    g = wl.rng(n + len(op))
    c = wl.uniform_i32(g, -(1 << 9), 1 << 9, (M, n))
    s = 0
    if op == "perm":
        operand = wl.permutation(g, n)
    elif op == "scale":
        operand, s = None, int(g.integers(-(1 << 9), 1 << 9))
    else:
        operand = wl.uniform_i32(g, -(1 << 9), 1 << 9, n)
    eps_h = oracle.entangle(c, l)
    gop = oracle.entangle_operand(operand, l) if op == "add" else operand
    no = ne.n_out(op, n, n)
    delta = empty64(M, no)
    dop = None if gop is None else dev(gop, torch.int64 if op == "add" else torch.int32)
    ne.lsb_apply(op, streams(eps_h, torch.int64), dop, delta, scalar=s, n_in=n)
    assert np.array_equal(np.stack([host(t) for t in delta]), oracle.apply(op, eps_h, gop, s))
    d = empty64(M, no)
    ne.plain_apply(op, streams(c, torch.int32), None if operand is None else dev(operand, torch.int32),
                   d, scalar=s)
    assert np.array_equal(np.stack([host(t) for t in d]), oracle.apply(op, c, operand, s))


# ---------------------------------------------------------------- extract

def entangled_outputs(d, l):
    """delta_m = d_m + 2^l d_(m-1 mod M): the entangled outputs that belong
    to outputs d (linearity of the operation, eq. (9) with eq. (15))."""
    d = d.astype(object)
    return (d + np.roll(d, 1, axis=0) * (1 << l)).astype(np.int64)


@pytest.mark.parametrize("M", list(range(3, 13)) + [16, 21, 32])
def test_extract_matches_oracle_at_boundary(M):
    """Outputs spread over [-D, D] including +-D; every loss r, delta_r
    poisoned; the GPU's 64-bit-only recovery equals the oracle's 2w-bit one."""
    l, _, D = ne.params(M)
    g = np.random.default_rng(M)
    n = 2051
    d = g.integers(-D, D + 1, size=(M, n), dtype=np.int64)
    d[:, :5] = np.array([D, -D, 0, 1, -1])[None, :]
    delta_h = entangled_outputs(d, l)
    for r in [-1] + list(range(M)):
        dl = streams(delta_h, torch.int64)
        if r >= 0:
            dl[r].fill_(POISON)
        out = empty64(M, n)
        ne.extract_recover(dl, r, out, l)
        got = np.stack([host(t) for t in out])
        assert np.array_equal(got, d), (M, r)
        assert np.array_equal(got, oracle.extract(delta_h, max(r, 0), l))


def test_extract_null_lost_stream_and_inplace():
    M = 5
    l, _, D = ne.params(M)
    d = np.random.default_rng(1).integers(-D, D, size=(M, 999), dtype=np.int64)
    delta_h = entangled_outputs(d, l)
    dl = streams(delta_h, torch.int64)
    dl[2] = None
    out = empty64(M, 999)
    ne.extract_recover(dl, 2, out, l, n=999)
    assert np.array_equal(np.stack([host(t) for t in out]), d)
    # in place: dhat aliases delta stream by stream
    dl = streams(delta_h, torch.int64)
    dl[4].fill_(POISON)
    ne.extract_recover(dl, 4, dl, l)
    assert np.array_equal(np.stack([host(t) for t in dl]), d)


# --------------------------------------------------------- whole pipeline

def test_small_config_every_loss():
    """M = 3 streams of 65,536 8-bit samples, 16 taps: the whole method under
    no loss and under the loss of each stream in turn."""
    grp = wl.config_small()
    plain = oracle.apply("conv", grp.c, grp.operand)
    eps_ref = oracle.entangle(grp.c, ne.params(3)[0])
    for r in (-1, 0, 1, 2):
        dhat, eps = gpu_pipeline(grp, r)
        assert np.array_equal(dhat, plain), r
        assert np.array_equal(np.stack([host(t) for t in eps]), eps_ref)


@pytest.mark.parametrize("op", wl.OP_KINDS)
@pytest.mark.parametrize("M", [3, 4, 5, 6, 7, 8])
def test_pipeline_all_ops(op, M):
    g = wl.rng(M * 31 + len(op))
    n = 3001 + M
    c = wl.uniform_i32(g, -(1 << 9), 1 << 9, (M, n))
    s = 0
    if op == "conv":
        operand = wl.uniform_i32(g, -(1 << 9), 1 << 9, 37 * M)
    elif op in ("add", "inner"):
        operand = wl.uniform_i32(g, -(1 << 9), 1 << 9, n)
    elif op == "perm":
        operand = wl.permutation(g, n)
    else:
        operand, s = np.zeros(0, np.int32), int(g.integers(-(1 << 9), 1 << 9))
    grp = wl.Group(op, c, operand, s)
    plain = oracle.apply(op, c, operand, s)
    for r in range(-1, M):
        dhat, _ = gpu_pipeline(grp, r, inplace=(r % 2 == 1))
        assert np.array_equal(dhat, plain), (op, M, r)


def test_dynamic_range_edge_scale():
    """Outputs exactly at +-D (M = 3): c = +-(2^19 - 1), s = 2^22 gives
    |d| = 2^41 - 2^22 = D of eq. (11), the largest the method admits."""
    l, _, D = ne.params(3)
    v = (1 << 19) - 1
    c = np.array([[v, -v, v, 0], [-v, v, v, 1], [v, v, -v, -1]], np.int32)
    grp = wl.Group("scale", c, np.zeros(0, np.int32), 1 << 22)
    plain = oracle.apply("scale", c, None, 1 << 22)
    assert np.abs(plain).max() == D
    for r in range(-1, 3):
        dhat, _ = gpu_pipeline(grp, r)
        assert np.array_equal(dhat, plain)


def test_batched_config_two_full_groups_sampled():
    """Two stream-triples at the full batched size (2^20 samples, 64 taps):
    sampled outputs against the oracle's convolution by definition, and the
    all-subsets invariant at every position."""
    groups = wl.config_batched(groups=2)
    pos = np.unique(np.concatenate([np.arange(0, 200), np.arange((1 << 20) - 100, (1 << 20) + 63),
                                    wl.rng(9).integers(0, (1 << 20) + 63, 3000)]))
    for grp in groups:
        outs = []
        for r in (0, 1, 2):
            dhat, _ = gpu_pipeline(grp, r)
            outs.append(dhat)
        assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
        for m in range(3):
            assert np.array_equal(outs[0][m][pos], oracle.conv_at(grp.c[m], grp.operand, pos))


def test_checksum_method_matches_oracle():
    M, n, K = 3, 5003, 64
    g = wl.rng(11)
    c = wl.uniform_i32(g, -(1 << 11), 1 << 11, (M, n))
    k = wl.uniform_i32(g, -(1 << 11), 1 << 11, K)
    cs = streams(c, torch.int32)
    rsum = torch.empty(n, dtype=torch.int64, device=DEV)
    ne.checksum(cs, rsum)
    assert np.array_equal(host(rsum), oracle.checksum(c))
    kd = dev(k, torch.int32)
    d = empty64(M, n + K - 1)
    ne.plain_apply("conv", cs, kd, d)
    e = empty64(1, n + K - 1)
    ne.lsb_apply("conv", [rsum], kd, e)
    plain = oracle.apply("conv", c, k)
    for r in range(M):
        dr = torch.empty(n + K - 1, dtype=torch.int64, device=DEV)
        ne.checksum_recover([None if j == r else t for j, t in enumerate(d)], e[0], r, dr)
        assert np.array_equal(host(dr), plain[r])


# ------------------------------------------- the other operators of eq. (2)

@pytest.mark.parametrize("op", ["sub", "mul", "circ", "xcorr", "outer"])
@pytest.mark.parametrize("M", [3, 5, 8])
def test_pipeline_more_ops(op, M):
    """Subtraction (operand entangled like addition), element-by-element
    product, circular convolution (taps longer than the stream: they wrap),
    cross-correlation and outer product through entangle -> op -> extract,
    every loss, bit-exact against the oracle."""
    g = wl.rng(M * 57 + len(op))
    n = 301 + M if op == "outer" else 3001 + M
    c = wl.uniform_i32(g, -(1 << 9), 1 << 9, (M, n))
    if op in ("sub", "mul"):
        operand = wl.uniform_i32(g, -(1 << 9), 1 << 9, n)
    elif op == "circ":
        operand = wl.uniform_i32(g, -(1 << 9), 1 << 9, n + 77)
    else:
        operand = wl.uniform_i32(g, -(1 << 9), 1 << 9, 37)
    grp = wl.Group(op, c, operand, 0)
    plain = oracle.apply(op, c, operand)
    for r in range(-1, M):
        dhat, _ = gpu_pipeline(grp, r, inplace=(r % 2 == 1))
        assert np.array_equal(dhat, plain), (op, M, r)


@pytest.mark.parametrize("op", ["sub", "mul", "circ", "xcorr", "outer"])
@pytest.mark.parametrize("n", [1, 5, 1000, 4097])
def test_plain_more_ops(op, n):
    """The failure-intolerant per-step calls of the same operators on raw
    int32 streams (int32 operands throughout)."""
    g = wl.rng(n + 13 * len(op))
    M = 3
    c = wl.uniform_i32(g, -(1 << 20), 1 << 20, (M, n))
    K = 1 if n == 1 else 19
    operand = wl.uniform_i32(g, -(1 << 10), 1 << 10, n if op in ("sub", "mul") else K)
    no = ne.n_out(op, n, operand.size)
    d = empty64(M, no, fill=POISON)
    ne.plain_apply(op, streams(c, torch.int32), dev(operand, torch.int32), d)
    got = np.stack([host(t) for t in d])
    assert np.array_equal(got, oracle.apply(op, c, operand)), (op, n)


@pytest.mark.parametrize("n", [1, 3, 4, 5, 4099, 1 << 20, (1 << 22) + 7])
def test_stream_widen_copies_exactly(n):
    """The bandwidth reference: every int32 widened to int64, ragged tails
    included, nothing written past n."""
    g = wl.rng(60 + n % 97)
    src = torch.from_numpy(wl.uniform_i32(g, -(1 << 31), (1 << 31) - 1, n)).to(DEV)
    dst = torch.full((n + 8,), POISON, dtype=torch.int64, device=DEV)
    ne.stream_widen(src, dst)
    torch.cuda.synchronize()
    got = dst.cpu().numpy()
    assert np.array_equal(got[:n], src.cpu().numpy().astype(np.int64))
    assert (got[n:] == POISON).all()


def test_mfma_i8_peak_runs_and_reports_its_work():
    """The matrix-core rate reference launches and reports 2 x 16 x 16 x 64 x
    8 operations per wave and iteration; every wave writes its folded word."""
    blocks, iters = 16, 8
    for varied in (False, True):
        sink = torch.full((4 * blocks + 4,), -7, dtype=torch.int32, device=DEV)
        ops = ne.mfma_i8_peak(sink, blocks, iters, varied)
        torch.cuda.synchronize()
        assert ops == 2 * 16 * 16 * 64 * 8 * iters * 4 * blocks
        s = sink.cpu().numpy()
        assert (s[4 * blocks:] == -7).all()
    with pytest.raises(ne.NeError):
        ne.mfma_i8_peak(sink, blocks, 12, True)  # varied rounds come in sets of 8


def _conv_mod64(x, g, kind):
    """The convolution kinds modulo 2^64 by definition (uint64 products and
    sums wrap modulo 2^64)."""
    xu = x.astype(np.uint64)
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
    return y.astype(np.int64)


@pytest.mark.parametrize("kind", ["conv", "circ", "xcorr"])
def test_word64_convolution_full_range(kind):
    """The 64-bit vector-ALU convolution (each word's low half staged as a
    signed int32, its borrow moved into the high half) on words over the
    whole int64 range -- low halves of exactly 2^31 and 2^31 - 1, the words
    -2^63 and 2^63 - 1 among them -- with taps at the int32 extremes, against
    its definition modulo 2^64; more than one 1024-tap chunk."""
    rng = wl.rng(9960 + len(kind))
    n, K = 3000, 1100
    x = rng.integers(-(1 << 63), (1 << 63) - 1, (2, n), dtype=np.int64, endpoint=True)
    special = np.array([-(1 << 63), (1 << 63) - 1, 0x80000000, 0x7FFFFFFF, -0x80000000,
                        -0x7FFFFFFF, 0xFFFFFFFF, -1, 0, 1, (1 << 32) | 0x80000000], dtype=np.int64)
    x[:, :special.size] = special
    x[:, n - special.size:] = special[::-1]
    g = wl.uniform_i32(rng, -(1 << 31), 1 << 31, K)
    g[:4] = [-(1 << 31), (1 << 31) - 1, -1, 1]
    g[1030:1033] = [-(1 << 31), (1 << 31) - 1, -(1 << 31)]
    eps = [torch.from_numpy(r.copy()).to(DEV) for r in x]
    no = ne.n_out(kind, n, K)
    out = [torch.full((no,), 0x5A5A, dtype=torch.int64, device=DEV) for _ in range(2)]
    ne.lsb_apply(kind, eps, torch.from_numpy(g).to(DEV), out)
    torch.cuda.synchronize()
    for m in range(2):
        assert np.array_equal(out[m].cpu().numpy(), _conv_mod64(x[m], g, kind)), (kind, m)
