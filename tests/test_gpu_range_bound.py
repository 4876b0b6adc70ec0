"""Worst-case magnitudes on the fused path (the benchmarked hot path), bit for
bit against the CPU oracle.

Random inputs reach about sqrt(K) of a convolution's worst case, so they
never drive the kernel's int32 digit accumulators, their 32-bit merge
(acc16) or the recovery epilogue near their limits. Here every sample and
every tap sits at -2^(b-1) or 2^(b-1)-1 (constant, alternating and random
sign patterns), so full-overlap outputs reach +-K 2^(2b-2): at the largest b
and K the range condition admits (|d| <= D of eq. (11)/(13) for the method,
the word's signed range otherwise, M times the value for the checksum
stream), with K on both sides of the acc16 merge, under every single-stream
loss and in every LDS layout. The element-wise operators run at their own
bounds the same way, so the fused recovery sees values next to D.
"""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
POISON = 0x3C3C3C3C3C3C3C3C
LAYOUTS = [(4, 4), (1, 0), (4, 1)]  # (ring_waves, tap_copies)


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def limit(mode: str, M: int, w: int = 64) -> int:
    """Largest admissible |d| of one output: D of eq. (11)/(13) for the
    method; the signed word range otherwise (M times the value for the
    checksum stream)."""
    if mode == "entangled":
        return oracle.params(M, w)[2]
    lim = (1 << (w - 1)) - 1
    return lim // M if mode in ("checksum", "checksum_same") else lim


def extremes(pattern: int, n: int, b: int, g: np.random.Generator) -> np.ndarray:
    """n values at the ends of [-2^(b-1), 2^(b-1)): all low, all high,
    alternating, or random ends."""
    lo, hi = -(1 << (b - 1)), (1 << (b - 1)) - 1
    if pattern == 0:
        v = np.full(n, lo, np.int64)
    elif pattern == 1:
        v = np.full(n, hi, np.int64)
    elif pattern == 2:
        v = np.where(np.arange(n) % 2 == 0, lo, hi)
    else:
        v = np.where(g.integers(0, 2, n) == 0, lo, hi)
    return v.astype(np.int32)


def conv_cases(mode: str, M: int, w: int = 64):
    """(b, K) pairs at the range bound: the widest inputs admitted with 64
    taps, with 7 and with the most taps at that width, and the widest inputs
    admitted at all."""
    lim = limit(mode, M, w)
    top = 31 if w == 64 else 16
    b1 = max(b for b in range(1, top + 1) if (1 << (2 * b - 2)) * 64 <= lim)
    k1 = min(lim >> (2 * b1 - 2), 700)
    bmax = max(b for b in range(1, top + 1) if (1 << (2 * b - 2)) <= lim)
    kmax = min(lim >> (2 * bmax - 2), 700)
    return sorted({(b1, 7), (b1, 64), (b1, k1), (bmax, kmax)})


def losses(mode: str, M: int):
    if mode not in ("entangled", "checksum", "checksum_same"):
        return [-1]
    return [-1] + (list(range(M)) if M <= 5 else [0, M // 2, M - 1])


def run_group(op, c, operand, scalar, lost, bits, mode, n_out, rw=0, tc=0, word_bits=0,
              steps=2):
    dt = torch.int32 if word_bits == 32 else torch.int64
    out = [torch.full((max(n_out, 1),), POISON, dtype=torch.int64, device=DEV)[:n_out].to(dt)
           for _ in range(c.shape[0])]
    spec = ne.GroupSpec(op, [dev32(r) for r in c], None if operand is None else dev32(operand),
                        out, scalar, lost, bits, ring_waves=rw, tap_copies=tc,
                        word_bits=word_bits)
    plan = ne.Plan([spec], mode, conv_steps=steps, stream_steps=steps)
    plan.run()
    torch.cuda.synchronize()
    flags = plan.flags()
    plan.close()
    return np.stack([t.cpu().numpy().astype(np.int64) for t in out]), flags


@pytest.mark.parametrize("word_bits", [0, 32])
@pytest.mark.parametrize("mode,m_lo", [("entangled", 3), ("plain", 1), ("plain_same", 1),
                                       ("checksum", 2), ("checksum_same", 2)])
def test_convolution_at_the_range_bound(mode, m_lo, word_bits):
    w = 32 if word_bits == 32 else 64
    g = wl.rng(4242 + m_lo + w)
    n = 2500
    ran = 0
    for M in range(m_lo, 9):
        for b, K in conv_cases(mode, M, w):
            lim = limit(mode, M, w)
            assert (1 << (2 * b - 2)) * K <= lim
            for tp in (0, 2, 3):
                c = np.stack([extremes((m + tp) % 4, n, b, g) for m in range(M)])
                k = extremes(tp, K, b, g)
                ref = oracle.apply("conv", c, k, w=w)
                if tp == 0:  # the all-low stream meets the all-low taps
                    assert np.abs(ref).max() == K << (2 * b - 2)
                for lost in losses(mode, M):
                    for rw, tc in LAYOUTS:
                        if tp != 3 and (rw, tc) != LAYOUTS[0]:
                            continue  # the other layouts see the random-ends pattern
                        try:
                            got, flags = run_group("conv", c, k, 0, lost, b, mode, n + K - 1,
                                                   rw, tc, word_bits)
                        except ne.NeError as e:
                            # only a per-wave ring too large for LDS may refuse
                            assert e.status == -4 and rw == 1, (mode, M, b, K, rw, e)
                            continue
                        assert flags == 0, (mode, M, b, K, tp, lost, rw, tc, flags)
                        assert np.array_equal(got, ref), (mode, M, b, K, tp, lost, rw, tc)
                        ran += 1
    assert ran > 0


@pytest.mark.parametrize("mode", ["entangled", "checksum", "checksum_same", "plain"])
@pytest.mark.parametrize("M", [3, 8])
def test_convolution_one_past_the_bound_is_refused(mode, M):
    """The plan refuses the next tap count past the bound (NE_ERANGE)."""
    lim = limit(mode, M)
    b = max(b for b in range(1, 32) if (1 << (2 * b - 2)) * 64 <= lim)
    K = (lim >> (2 * b - 2)) + 1
    c = np.zeros((M, 16), np.int32)
    with pytest.raises(ne.NeError) as e:
        run_group("conv", c, np.zeros(K, np.int32), 0, -1, b, mode, 16 + K - 1)
    assert e.value.status == -2


def elementwise_cases(op: str, mode: str, M: int, n: int):
    """(bits, scalar) of op at its bound: the worst case is B|s| (scale),
    2B (add, sub), B^2 (mul, outer), n B^2 (inner), B (perm), B = 2^(b-1)."""
    lim = limit(mode, M)
    if op == "scale":
        return [(32, lim >> 31), (32, -(lim >> 31)), (31, -(lim >> 30))]
    if op in ("add", "sub", "perm"):
        return [(32, 0)]
    reach = n if op == "inner" else 1
    b = max(b for b in range(1, 33) if (1 << (2 * b - 2)) * reach <= lim)
    return [(b, 0)]


@pytest.mark.parametrize("mode", ["entangled", "plain", "plain_same", "checksum", "checksum_same"])
@pytest.mark.parametrize("op", ["scale", "add", "sub", "mul", "inner", "outer", "perm"])
@pytest.mark.parametrize("M", [3, 5, 8])
def test_elementwise_at_the_range_bound(mode, op, M):
    g = wl.rng(777 + M + len(op))
    n = 4097
    for b, s in elementwise_cases(op, mode, M, n):
        for tp in (0, 1, 3):
            c = np.stack([extremes((m + tp) % 4, n, b, g) for m in range(M)])
            if op == "perm":
                operand = wl.permutation(g, n)
            elif op == "outer":
                operand = extremes(tp, 8, b, g)
            elif op == "scale":
                operand = None
            else:
                operand = extremes(3 - tp, n, b, g)
            ref = oracle.apply(op, c, operand, s)
            n_out = ref.shape[1]
            for lost in losses(mode, M):
                got, flags = run_group(op, c, operand, s, lost, b, mode, n_out)
                assert flags == 0, (op, mode, M, b, s, lost, flags)
                assert np.array_equal(got, ref), (op, mode, M, b, s, tp, lost)


def split_acc16_limit(mode: str, M: int, b: int) -> int:
    """Most taps for which every field's whole digit sum of a split word fits
    in int32: |field| K 2^(b-1) < 2^31, |field| = 2^(b-1) (M 2^(b-1) for the
    checksum stream)."""
    field = (1 << (b - 1)) * (M if mode == "checksum_same" else 1)
    return ((1 << 31) - 1) // (field << (b - 1))


@pytest.mark.parametrize("mode", ["entangled", "plain_same", "checksum_same"])
@pytest.mark.parametrize("M,b", [(3, 12), (3, 15), (3, 8), (4, 8)])
def test_split_words_at_their_limits(mode, M, b):
    """Words split into two fields (12- and 15-bit samples at M = 3, 8-bit
    at M = 3 and 4): every sample and tap at the ends of its range, with the
    tap count on both sides of the 32-bit field sums (their largest K, and
    one more), and the longest kernel of the paper's experiment at 15 bits,
    under every loss and in every LDS layout."""
    g = wl.rng(9100 + M * 31 + b)
    k32 = split_acc16_limit(mode, M, b)
    Ks = sorted({k for k in (k32, k32 + 1, 64, 4500 if b == 15 else 0) if 0 < k <= 4500})
    n = 3000
    ran = 0
    for K in Ks:
        assert (1 << (2 * b - 2)) * K <= limit(mode, M)
        for tp in (0, 2, 3):
            c = np.stack([extremes((m + tp) % 4, n, b, g) for m in range(M)])
            k = extremes(tp, K, b, g)
            ref = oracle.apply("conv", c, k)
            for lost in losses(mode, M):
                for rw, tc in LAYOUTS:
                    if tp != 3 and (rw, tc) != LAYOUTS[0]:
                        continue
                    try:
                        got, flags = run_group("conv", c, k, 0, lost, b, mode, n + K - 1, rw, tc)
                    except ne.NeError as e:
                        assert e.status == -4 and rw == 1, (mode, M, b, K, rw, e)
                        continue
                    assert flags == 0, (mode, M, b, K, tp, lost, rw, tc, flags)
                    assert np.array_equal(got, ref), (mode, M, b, K, tp, lost, rw, tc)
                    ran += 1
    assert ran > 0
