"""Entangled integer matrix product (ne_gemm): D_m = C_m G for M blocks,
bit-exact against the CPU oracle in every mode, with and without a lost
block, for every kernel variant, ragged tiles and the benchmark size."""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
POISON = -0x5A5A5A5A5A5A5A5A


SPLIT = [False, True]  # one fused launch / the two-phase form through workspace


def run(c, g, mode="entangled", lost=-1, in_bits=12, split=False):
    """c: (M, N, P) int32, g: (P, Q) int32 -> (outputs (M, N, Q), flags)."""
    M, N, P = c.shape
    Q = g.shape[1]
    cd = [torch.from_numpy(np.ascontiguousarray(b)).to(DEV) for b in c]
    gd = torch.from_numpy(np.ascontiguousarray(g)).to(DEV)
    out = [torch.full((N, Q), POISON, dtype=torch.int64, device=DEV) for _ in range(M)]
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = None
    if split:
        nb = ne.gemm_workspace_size(mode, M, N, P, Q, in_bits)
        ws = torch.full((nb + 256,), 0x5A, dtype=torch.uint8, device=DEV)  # stale bytes
        ws = ws[(-ws.data_ptr()) % 256:][:nb]
    ne.gemm(cd, gd, out, mode, lost, in_bits, flags=flags, workspace=ws)
    torch.cuda.synchronize()
    return np.stack([o.cpu().numpy() for o in out]), int(flags.item())


def draw(seed, M, N, P, Q, bits):
    g = wl.rng(seed)
    lo, hi = -(1 << (bits - 1)), 1 << (bits - 1)
    return wl.uniform_i32(g, lo, hi, (M, N, P)), wl.uniform_i32(g, lo, hi, (P, Q))


MODES = [("entangled", 3), ("plain", 1), ("plain_same", 1), ("checksum", 2)]


@pytest.mark.parametrize("split", SPLIT)
@pytest.mark.parametrize("mode,m_lo", MODES)
@pytest.mark.parametrize("M", [3, 4, 8])
def test_gemm_modes_and_losses(mode, m_lo, M, split):
    """Ragged tiles in every dimension (N, Q not multiples of 32, P not a
    multiple of 64 nor of 4), every loss position."""
    c, g = draw(1000 + M, M, 37, 70, 45, 12)
    want = oracle.gemm(c, g)
    for lost in (-1, 0, M - 1):
        got, flags = run(c, g, mode, lost, split=split)
        assert flags == 0, (mode, M, lost, flags)
        if mode in ("plain", "plain_same") and lost >= 0:
            keep = [m for m in range(M) if m != lost]
            assert np.array_equal(got[keep], want[keep]), (mode, M, lost)
            assert (got[lost] == POISON).all()  # a lost plain block is not written
        else:
            assert np.array_equal(got, want), (mode, M, lost)


@pytest.mark.parametrize("split", SPLIT)
@pytest.mark.parametrize("mode,m_lo", MODES)
def test_gemm_every_variant(mode, m_lo, split):
    """Every (M, digit counts) variant the call can pick: inputs of 1 to 16
    bits at a small shape, one lost block where the mode recovers it."""
    ran = 0
    for M in range(m_lo, 9):
        for bits in (1, 2, 7, 8, 9, 12, 15, 16):
            c, g = draw(2000 + 17 * M + bits, M, 19, 67, 21, bits)
            want = oracle.gemm(c, g)
            lost = M - 1 if mode in ("entangled", "checksum") else -1
            try:
                got, flags = run(c, g, mode, lost, bits, split=split)
            except ne.NeError as e:
                assert e.status == -2, (mode, M, bits, e)  # only the range check may refuse
                continue
            assert flags == 0
            assert np.array_equal(got, want), (mode, M, bits)
            ran += 1
    assert ran > 0


@pytest.mark.parametrize("split", SPLIT)
@pytest.mark.parametrize("mode,m_lo", MODES)
def test_gemm_128_row_blocks(mode, m_lo, split):
    """Padded rows a multiple of 128, where the two-phase product runs
    128-row blocks: N = 250 (a ragged last block), every M and digit-count
    variant, one lost block where the mode recovers it."""
    ran = 0
    for M in range(m_lo, 9):
        for bits in (1, 7, 9, 12, 16):
            c, g = draw(3000 + 17 * M + bits, M, 250, 131, 70, bits)
            want = oracle.gemm(c, g)
            lost = M - 1 if mode in ("entangled", "checksum") else -1
            try:
                got, flags = run(c, g, mode, lost, bits, split=split)
            except ne.NeError as e:
                assert e.status == -2, (mode, M, bits, e)  # only the range check may refuse
                continue
            assert flags == 0
            assert np.array_equal(got, want), (mode, M, bits)
            ran += 1
    assert ran > 0


@pytest.mark.parametrize("split", SPLIT)
@pytest.mark.parametrize("N", [64, 256])
def test_gemm_vector_loads_and_extremes(split, N):
    """P a multiple of 4 (16-byte row loads), values at both ends of the
    declared 16-bit range, several chunks of the inner dimension; 64 and
    256 rows (64- and 128-row blocks of the two-phase product)."""
    M, P, Q = 3, 256, 64
    c = np.full((M, N, P), -(1 << 15), np.int32)
    c[1] = (1 << 15) - 1
    g = np.full((P, Q), -(1 << 15), np.int32)
    g[::3] = (1 << 15) - 1
    for lost in (-1, 1):
        got, flags = run(c, g, "entangled", lost, 16, split=split)
        assert flags == 0
        assert np.array_equal(got, oracle.gemm(c, g))


@pytest.mark.parametrize("split", SPLIT)
def test_gemm_empty_inner_dimension_gives_zeros(split):
    c = np.zeros((3, 5, 0), np.int32)
    g = np.zeros((0, 7), np.int32)
    got, flags = run(c, g, "entangled", 1, split=split)
    assert flags == 0 and (got == 0).all()


@pytest.mark.parametrize("split", SPLIT)
def test_gemm_declared_range_violation_is_flagged(split):
    c, g = draw(5, 3, 16, 64, 16, 8)
    c[2, 3, 5] = 200  # outside 8 bits
    _, flags = run(c, g, "entangled", -1, 8, split=split)
    assert flags & ne.FLAG_INPUT_RANGE


@pytest.mark.parametrize("split", SPLIT)
def test_gemm_benchmark_size(split):
    """The product the benchmark times (3 blocks of 4096 x 1024 times
    1024 x 4096, 12-bit values), one block lost, sampled against the oracle
    entry by entry, edges included."""
    M, N, P, Q = 3, 4096, 1024, 4096
    c, g = wl.config_gemm()
    got, flags = run(c, g, "entangled", 1, wl.GEMM_BITS, split=split)
    assert flags == 0
    rng = wl.rng(77)
    rows = np.concatenate([[0, N - 1, 31, 32], rng.integers(0, N, 400)])
    cols = np.concatenate([[Q - 1, 0, 32, 31], rng.integers(0, Q, 400)])
    for m in range(M):
        assert np.array_equal(got[m][rows, cols], oracle.gemm_at(c[m], g, rows, cols)), m
