"""Pins for the CPU oracle: each check ties it to something other than its
own code -- the paper's Table I and printed instantiation, textbook
definitions evaluated by numpy, exhaustive enumeration of the admissible
output range at tiny word widths, closed forms, and the invariant that
every single-stream loss recovers the plain result. Runs on the CPU."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import bigint
from paper_1509_03838_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_w32.txt")


def table1():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(tuple(int(v) for v in line.split()))
    return rows


# ----------------------------------------------------------------- params

@pytest.mark.parametrize("row", table1())
def test_params_reproduce_table1(row):
    M, l, k, bits_prop, bits_cs = row
    gl, gk, _ = oracle.params(M, 32)
    assert (gl, gk) == (l, k)
    assert (M - 2) * gl + gk == bits_prop
    # eq. (12): (M-1)l + k <= w
    assert (M - 1) * gl + gk <= 32
    # the checksum column is w - ceil(log2 M)
    assert 32 - math.ceil(math.log2(M)) == bits_cs
    assert bigint.params(M, 32)[:2] == (l, k)


def test_params_practical_instantiation():
    # Sec. III-A: w = 32, l = 11, k = 10 for M = 3
    assert oracle.params(3, 32)[:2] == (11, 10)


@pytest.mark.parametrize("w", [32, 64])
@pytest.mark.parametrize("M", list(range(3, 32)))
def test_dynamic_range_is_sufficient(M, w):
    """Whatever D eq. (11)/(13) give must make the method exact: an
    entangled output d_m + 2^l d_(m-1) fits in w bits, and an output fits the
    (M-1)l-bit window that eq. (17) sign-extends."""
    l, k, D = oracle.params(M, w)
    if l == 1:
        assert D == 0  # eq. (13) degenerates: 2^(l-1) - 1 = 0
        return
    assert D >= 1 and 0 <= k <= l
    assert D * ((1 << l) + 1) <= (1 << (w - 1)) - 1
    assert D < 1 << ((M - 1) * l - 1)
    assert (l, k, D) == bigint.params(M, w)


def test_params_w64_table():
    # the closed form l = ceil(w/M), k = w - (M-1)l holds where it is feasible
    for M in range(3, 12):
        l, k, _ = oracle.params(M, 64)
        L = -(-64 // M)
        assert (l, k) == (L, 64 - (M - 1) * L)


# ------------------------------------------------------------- LSB ops

def _rand(seed, lo, hi, size):
    return np.random.default_rng(seed).integers(lo, hi, size=size, dtype=np.int64)


@pytest.mark.parametrize("n,K", [(1, 1), (5, 1), (1, 7), (3, 8), (64, 16), (1000, 333), (17, 64)])
def test_conv_matches_numpy(n, K):
    x = _rand(n * 31 + K, -1000, 1000, n)
    g = _rand(n + 7 * K, -1000, 1000, K)
    ref = np.convolve(x, g)
    assert np.array_equal(oracle.apply("conv", x, g), ref)
    if n * K < 5000:
        assert bigint.conv(x.tolist(), g.tolist()) == ref.tolist()


def test_conv_at_matches_full():
    x = _rand(1, -2048, 2048, 3000)
    g = _rand(2, -2048, 2048, 64)
    full = np.convolve(x, g)
    pos = np.array([0, 1, 62, 63, 64, 1500, 2999, 3000, 3062], np.int64)
    assert np.array_equal(oracle.conv_at(x, g, pos), full[pos])


def test_conv_empty():
    assert oracle.apply("conv", np.zeros(0, np.int64), np.ones(4, np.int64)).size == 0


def test_other_ops_match_numpy():
    x = _rand(3, -512, 512, 777)
    v = _rand(4, -512, 512, 777)
    perm = np.random.default_rng(5).permutation(777)
    assert np.array_equal(oracle.apply("scale", x, scalar=-37), -37 * x)
    assert np.array_equal(oracle.apply("add", x, v), x + v)
    assert oracle.apply("inner", x, v)[0] == int(np.dot(x, v))
    assert np.array_equal(oracle.apply("perm", x, perm), x[perm])
    with pytest.raises(oracle.OracleError):
        oracle.apply("perm", x, np.zeros(777, np.int64) + 800)


def test_exact_arithmetic_beyond_int64_intermediates():
    # products near 2^62 must not wrap; the final sum fits in 64 bits
    x = np.array([1 << 40, -(1 << 40)], np.int64)
    g = np.array([1 << 21, 1 << 21], np.int64)
    assert oracle.apply("inner", x, g)[0] == 0
    with pytest.raises(oracle.OracleError):
        oracle.apply("inner", x, np.array([1 << 23, 0], np.int64))


# --------------------------------------------------------- entanglement

def entangle_matrix(M, l):
    """The circulant operator of eq. (14) as an explicit integer matrix:
    cyclic shifts of the row [1 0 ... 0 2^l]."""
    first = np.zeros(M, dtype=object)
    first[0] = 1
    first[-1] = 1 << l
    return np.array([np.roll(first, m) for m in range(M)], dtype=object)


@pytest.mark.parametrize("M", [3, 4, 5, 8, 11])
def test_entangle_is_circulant_operator(M):
    l, _, _ = oracle.params(M, 64)
    c = _rand(M, -(1 << 11), 1 << 11, (M, 200))
    E = entangle_matrix(M, l)
    ref = (E.dot(c.astype(object))).astype(np.int64)
    assert np.array_equal(oracle.entangle(c, l), ref)
    assert bigint.entangle(c.tolist(), l, 64) == ref.tolist()


def test_entangle_m3_eq6():
    l, _, _ = oracle.params(3, 64)
    c = _rand(9, -100, 100, (3, 50))
    e = oracle.entangle(c, l)
    assert np.array_equal(e[0], c[2] * (1 << l) + c[0])
    assert np.array_equal(e[1], c[0] * (1 << l) + c[1])
    assert np.array_equal(e[2], c[1] * (1 << l) + c[2])


def test_entangle_overflow_detected():
    l, _, _ = oracle.params(3, 32)
    c = np.array([[1 << 21], [0], [0]], np.int64)
    with pytest.raises(oracle.OracleError):
        oracle.entangle(c, l, w=32)


OP_CASES = ["conv", "scale", "add", "inner", "perm"]


def _operand(op, n, seed):
    g = np.random.default_rng(seed)
    if op == "conv":
        return g.integers(-2048, 2048, 37, dtype=np.int64), 0
    if op in ("add", "inner"):
        return g.integers(-2048, 2048, n, dtype=np.int64), 0
    if op == "perm":
        return g.permutation(n).astype(np.int64), 0
    return np.zeros(0, np.int64), int(g.integers(-2048, 2048))


@pytest.mark.parametrize("op", OP_CASES)
@pytest.mark.parametrize("M", [3, 4, 6, 8])
def test_entangled_outputs_closed_form(op, M):
    """By linearity, delta_m = d_m + 2^l d_(m-1 mod M) (eq. (9) with eq. (15)),
    with d computed by numpy on the plain inputs."""
    l, _, _ = oracle.params(M, 64)
    n = 300
    c = _rand(M * 13, -2048, 2048, (M, n))
    g, s = _operand(op, n, M)
    eps = oracle.entangle(c, l)
    gop = oracle.entangle_operand(g, l) if op == "add" else g
    delta = oracle.apply(op, eps, gop, s)
    if op == "conv":
        d = np.stack([np.convolve(row, g) for row in c])
    elif op == "scale":
        d = s * c
    elif op == "add":
        d = c + g
    elif op == "inner":
        d = (c @ g)[:, None]
    else:
        d = c[:, g]
    assert np.array_equal(delta, d + (np.roll(d, 1, axis=0) << l))


# ------------------------------------------------------------ extraction

def _exhaustive(M, w):
    """Every output M-tuple in [-D, D]^M, each single loss r, recovers it."""
    l, k, D = oracle.params(M, w)
    vals = np.arange(-D, D + 1, dtype=np.int64)
    rest = np.stack(np.meshgrid(*([vals] * (M - 1)), indexing="ij"), 0).reshape(M - 1, -1)
    E = entangle_matrix(M, l).astype(np.int64)
    checked = 0
    for v0 in vals:
        d = np.concatenate([np.full((1, rest.shape[1]), v0, np.int64), rest], 0)
        delta = E @ d                              # closed form of the outputs
        assert np.abs(delta).max() < 1 << (w - 1)  # fits the w-bit word
        for r in range(M):
            dd = delta.copy()
            dd[r] = 0x5A5A5A5A5A5A5A5 if w == 64 else 0x5A5  # never read
            assert np.array_equal(oracle.extract(dd, r, l, w), d), (M, w, r, int(v0))
        checked += d.shape[1]
    return checked, D


def test_exhaustive_m3_w12():
    checked, D = _exhaustive(3, 12)
    assert D == 112 and checked == 225 ** 3


def test_exhaustive_m4_w10():
    checked, D = _exhaustive(4, 10)
    assert D == 48 and checked == 97 ** 4


def test_exhaustive_m5_w8():
    # k = 0 here: the headroom can vanish and the method still holds
    l, k, D = oracle.params(5, 8)
    assert (l, k, D) == (2, 0, 16)
    checked, _ = _exhaustive(5, 8)
    assert checked == 33 ** 5


def test_bound_is_needed_tiny_w():
    """Just past the largest magnitude whose entangled output fits w bits,
    the oracle refuses (the word would overflow): the range condition of
    eq. (11)/(13) is what keeps the method exact."""
    M, w = 3, 12
    l, _, D = oracle.params(M, w)
    tight = ((1 << (w - 1)) - 1) // ((1 << l) + 1)
    assert D <= tight
    c = np.array([[tight + 1], [tight + 1], [tight + 1]], np.int64)
    with pytest.raises(oracle.OracleError):
        oracle.entangle(c, l, w)


@pytest.mark.parametrize("M", list(range(3, 13)) + [16, 21, 32])
def test_all_subsets_boundary_w64(M):
    """Recovery from each of the M possible (M-1)-subsets returns exactly the
    outputs, with outputs at and near +-D (w = 64)."""
    l, _, D = oracle.params(M, 64)
    g = np.random.default_rng(M)
    n = 257
    d = g.integers(-D, D + 1, size=(M, n), dtype=np.int64)
    d[:, :6] = np.array([D, -D, 0, 1, -1, D - 1])[None, :]
    d[0, 6], d[M - 1, 7] = -D, D
    delta = (entangle_matrix(M, l).dot(d.astype(object))).astype(np.int64)
    for r in range(M):
        dd = delta.copy()
        dd[r] = g.integers(-(1 << 62), 1 << 62, n)
        assert np.array_equal(oracle.extract(dd, r, l), d)
    if M <= 8:
        small = [list(map(int, row[:24])) for row in delta]
        for r in range(M):
            small_r = [row if j != r else None for j, row in enumerate(small)]
            assert bigint.extract(small_r, r, l, 64) == [list(map(int, row[:24])) for row in d]


def test_m3_matches_eq10():
    """For M = 3 and a loss of stream 0, eq. (10) spells the extraction out:
    d_temp = delta_2 - S_l delta_1, d2 = sign-extension of its low 2l bits,
    d0 = -(d_temp - d2) >> 2l, d1 = delta_1 - S_l d0."""
    l, _, D = oracle.params(3, 64)
    g = np.random.default_rng(3)
    d = g.integers(-D, D + 1, size=(3, 100), dtype=np.int64)
    delta = (entangle_matrix(3, l).dot(d.astype(object)))
    out = []
    for i in range(100):
        dt = int(delta[2, i]) - (int(delta[1, i]) << l)
        low = dt & ((1 << (2 * l)) - 1)
        d2 = low - (1 << (2 * l)) if low >> (2 * l - 1) else low
        d0 = (-(dt - d2)) >> (2 * l)
        d1 = int(delta[1, i]) - (d0 << l)
        out.append((d0, d1, d2))
    assert np.array_equal(np.array(out).T, d)
    assert np.array_equal(oracle.extract(delta.astype(np.int64), 0, l), d)


@pytest.mark.parametrize("M", [3, 4, 5, 6, 7, 8])
def test_printed_sign_of_eq16_fails_for_odd_m(M):
    """Planted-mistake check: eq. (16) exactly as printed (no (-1)^M) breaks
    recovery for odd M and is harmless for even M, which is the evidence for
    the sign reading used by the oracle."""
    l, _, D = oracle.params(M, 64)
    d = np.random.default_rng(M).integers(-D // 4, D // 4, size=(M, 64), dtype=np.int64)
    d[:, 0] = 5
    delta = (entangle_matrix(M, l).dot(d.astype(object))).astype(np.int64)
    try:
        wrong = oracle.extract(delta, 0, l, printed_sign=True)
        same = np.array_equal(wrong, d)
    except oracle.OracleError:
        same = False
    assert same == (M % 2 == 0)
    assert np.array_equal(oracle.extract(delta, 0, l), d)


# ---------------------------------------------------------- whole method

@pytest.mark.parametrize("op", OP_CASES)
@pytest.mark.parametrize("M", [3, 5, 8])
def test_pipeline_recovers_plain_result(op, M):
    n = 257
    c = _rand(M * 7 + len(op), -2048, 2048, (M, n))
    g, s = _operand(op, n, 11)
    plain = oracle.apply(op, c, g, s)
    for r in range(M):
        dhat, _, _ = oracle.pipeline(c, op, g, s, r=r)
        assert np.array_equal(dhat, plain), (op, M, r)


def test_identity_storage_round_trip():
    """op = x with g = 1: data kept entangled at rest comes back unchanged."""
    c = _rand(21, -(1 << 20), 1 << 20, (4, 1000))
    for r in range(4):
        dhat, _, _ = oracle.pipeline(c, "scale", None, 1, r=r)
        assert np.array_equal(dhat, c)


def test_add_needs_entangled_operand():
    """Footnote 3: without entangling the added vector, recovery fails."""
    M = 3
    l, _, _ = oracle.params(M, 64)
    c = _rand(1, -100, 100, (M, 50))
    g = _rand(2, 1, 100, 50)
    eps = oracle.entangle(c, l)
    bad = oracle.extract(oracle.apply("add", eps, g), 0, l)
    good = oracle.extract(oracle.apply("add", eps, oracle.entangle_operand(g, l)), 0, l)
    assert np.array_equal(good, c + g)
    assert not np.array_equal(bad, c + g)


# ------------------------------------------- the other operators of eq. (2)

@pytest.mark.parametrize("n,K", [(1, 1), (7, 3), (100, 17), (40, 64), (257, 257)])
def test_more_operators_match_numpy(n, K):
    """Subtraction, element-by-element product, circular convolution,
    cross-correlation and outer product against numpy on Python integers."""
    x = _rand(n + K, -3000, 3000, n)
    v = _rand(n + K + 1, -3000, 3000, n)
    g = _rand(n + K + 2, -3000, 3000, K)
    xo, vo, go = x.astype(object), v.astype(object), g.astype(object)
    assert np.array_equal(oracle.apply("sub", x, v).astype(object), xo - vo)
    assert np.array_equal(oracle.apply("mul", x, v).astype(object), xo * vo)
    circ = [sum(go[j] * xo[(t - j) % n] for j in range(K)) for t in range(n)]
    assert oracle.apply("circ", x, g).tolist() == circ
    assert np.array_equal(oracle.apply("xcorr", x, g).astype(object),
                          np.correlate(xo, go, "full"))
    assert np.array_equal(oracle.apply("outer", x, g).astype(object), np.outer(xo, go).ravel())


def test_circular_convolution_is_folded_linear_convolution():
    """Circular convolution of length n = the linear convolution with its
    tail folded back (indices mod n), an identity independent of the
    definition above."""
    x = _rand(1, -500, 500, 50)
    g = _rand(2, -500, 500, 120)  # longer than the stream: folds twice
    lin = np.convolve(x, g).astype(object)
    fold = np.zeros(50, dtype=object)
    for t, v in enumerate(lin):
        fold[t % 50] += v
    assert np.array_equal(oracle.apply("circ", x, g).astype(object), fold)


@pytest.mark.parametrize("op", ["sub", "mul", "circ", "xcorr", "outer"])
@pytest.mark.parametrize("M", [3, 5, 8])
def test_more_operators_recover(op, M):
    """The method recovers each of them from any M-1 streams, and the
    entangled outputs hold d_m + 2^l d_(m-1) (all are linear in the
    stream; subtraction entangles its operand like addition)."""
    n = 90
    c = _rand(M + 5 * len(op), -2048, 2048, (M, n))
    g = _rand(M + 6 * len(op), -2048, 2048, 23 if op in ("circ", "xcorr", "outer") else n)
    plain = oracle.apply(op, c, g)
    l, _, _ = oracle.params(M, 64)
    for r in range(M):
        dhat, _, delta = oracle.pipeline(c, op, g, r=r)
        assert np.array_equal(dhat, plain), (op, M, r)
    want = plain.astype(object) + (np.roll(plain.astype(object), 1, axis=0) << l)
    assert np.array_equal(delta.astype(object), want)


# --------------------------------------------------- series of operations

def _numpy_series(c, ops):
    """The series by numpy on Python integers (object arrays): each
    operation restated from its definition, independently of the C oracle."""
    x = np.array(c, dtype=object)
    for op, g, s in ops:
        if op == "conv":
            x = np.array([np.convolve(row, np.array(g, dtype=object)) if row.size else row
                          for row in x], dtype=object)
        elif op == "scale":
            x = x * s
        elif op == "add":
            x = x + np.array(g, dtype=object)
        elif op == "inner":
            x = np.array([[sum(int(a) * int(b) for a, b in zip(row, g))] for row in x], dtype=object)
        else:
            x = x[:, np.asarray(g, dtype=np.int64)]
    return x


SERIES = [wl.CHAIN_RECIPE, ("conv", "conv"), ("scale", "perm", "inner", "scale"),
          ("perm", "add", "conv", "inner"), ("add",)]


@pytest.mark.parametrize("recipe", SERIES)
def test_series_matches_numpy(recipe):
    """The oracle's series equals numpy's composition of the definitions."""
    c = _rand(5, -512, 512, (3, 120))
    ops = wl.chain_series(wl.rng(17), 120, recipe, bits=10, K=9)
    assert np.array_equal(oracle.chain(c, ops).astype(object), _numpy_series(c, ops))


@pytest.mark.parametrize("recipe", SERIES)
@pytest.mark.parametrize("M", [3, 4, 7])
def test_series_recovers_plain_result(recipe, M):
    """One extraction after the whole series recovers the series' plain
    result from any M-1 streams, and the last stage still holds the
    closed form d_m + 2^l d_(m-1) (linearity of every operation)."""
    n = 150
    c = _rand(M * 3 + len(recipe), -512, 512, (M, n))
    ops = wl.chain_series(wl.rng(M + 40), n, recipe, bits=10, K=17)
    plain = oracle.chain(c, ops)
    l, _, _ = oracle.params(M, 64)
    for r in range(M):
        dhat, last = oracle.chain_pipeline(c, ops, r=r)
        assert np.array_equal(dhat, plain), (recipe, M, r)
    want = plain.astype(object) + (np.roll(plain.astype(object), 1, axis=0) << l)
    assert np.array_equal(last.astype(object), want)


def test_series_add_needs_entangled_operand():
    """Footnote 3 holds inside a series too: a plain added vector breaks
    recovery (planted on the CPU: the pipeline with the plain operand)."""
    M, n = 3, 60
    c = _rand(8, -100, 100, (M, n))
    ops = wl.chain_series(wl.rng(9), n, ("scale", "add", "conv"), bits=8, K=5)
    l, _, _ = oracle.params(M, 64)
    x = oracle.entangle(c, l)
    for op, g, s in ops:
        x = oracle.apply(op, x, g, s)  # add without entangling its operand
    assert not np.array_equal(oracle.extract(x, 0, l), oracle.chain(c, ops))


# ------------------------------------------------------- matrix product

@pytest.mark.parametrize("N,P,Q", [(1, 1, 1), (7, 5, 4), (16, 64, 16), (33, 70, 17), (0, 3, 2),
                                   (3, 0, 2), (2, 3, 0)])
def test_gemm_matches_numpy(N, P, Q):
    """Block matrix product against numpy's matmul on Python integers."""
    c = _rand(N + 3 * P, -2048, 2048, (2, N, P))
    g = _rand(P + 5 * Q, -2048, 2048, (P, Q))
    want = np.stack([blk.astype(object) @ g.astype(object) for blk in c]) if N * Q else \
        np.zeros((2, N, Q), dtype=object)
    assert np.array_equal(oracle.gemm(c, g).astype(object), want)


def test_gemm_at_matches_full():
    c = _rand(3, -2048, 2048, (40, 70))
    g = _rand(4, -2048, 2048, (70, 30))
    rows, cols = np.array([0, 39, 17, 5]), np.array([29, 0, 13, 5])
    assert np.array_equal(oracle.gemm_at(c, g, rows, cols), oracle.gemm(c, g)[rows, cols])


def test_gemm_exact_beyond_int64_intermediates():
    """Products near 2^62 that cancel: the sum is exact, and a sum that does
    not fit 64 bits is refused."""
    c = np.array([[1 << 40, -(1 << 40)]], np.int64)
    g = np.array([[1 << 21], [1 << 21]], np.int64)
    assert oracle.gemm(c, g)[0, 0] == 0
    with pytest.raises(oracle.OracleError):
        oracle.gemm(c, np.array([[1 << 23], [0]], np.int64))


@pytest.mark.parametrize("M", [3, 4, 8])
def test_gemm_entangled_closed_form_and_recovery(M):
    """Entangled blocks times G hold D_m + 2^l D_(m-1) (linearity of the
    product), and every block is recovered from any M-1 of them."""
    l, _, _ = oracle.params(M, 64)
    c = _rand(M + 60, -2048, 2048, (M, 9, 33))
    g = _rand(M + 61, -2048, 2048, (33, 11))
    plain = np.stack([blk.astype(object) @ g.astype(object) for blk in c])
    for r in range(M):
        dhat, delta = oracle.gemm_pipeline(c, g, r=r)
        assert np.array_equal(dhat.astype(object), plain), (M, r)
    want = plain + (np.roll(plain, 1, axis=0) << l)
    assert np.array_equal(delta.astype(object), want)


@pytest.mark.parametrize("w", [32, 64])
def test_c_oracle_matches_bigint_twin(w):
    g = np.random.default_rng(w)
    for M in (3, 4, 7):
        l, _, D = oracle.params(M, w)
        for op in OP_CASES:
            n = 23
            amp = 40 if w == 32 else 2000
            c = g.integers(-amp, amp, (M, n), dtype=np.int64)
            if op == "conv":
                opd, s = g.integers(-amp, amp, 5, dtype=np.int64), 0
            elif op in ("add", "inner"):
                opd, s = g.integers(-amp // 8, amp // 8, n, dtype=np.int64), 0
            elif op == "perm":
                opd, s = g.permutation(n).astype(np.int64), 0
            else:
                opd, s = np.zeros(0, np.int64), int(g.integers(-amp, amp))
            r = int(g.integers(0, M))
            dhat, eps, delta = oracle.pipeline(c, op, opd, s, r=r, w=w)
            e2 = bigint.entangle(c.tolist(), l, w)
            gop = bigint.entangle_operand(opd.tolist(), l, w) if op == "add" else opd.tolist()
            d2 = [bigint.apply(op, row, gop, s) for row in e2]
            x2 = bigint.extract([row if j != r else None for j, row in enumerate(d2)], r, l, w)
            assert eps.tolist() == e2 and delta.tolist() == d2 and dhat.tolist() == x2
            assert dhat.tolist() == [bigint.apply(op, row, opd.tolist(), s) for row in c.tolist()]


# ------------------------------------------------------- checksum method

@pytest.mark.parametrize("op", ["conv", "scale", "inner", "perm", "add"])
def test_checksum_recovery(op):
    M, n = 4, 120
    c = _rand(77, -2048, 2048, (M, n))
    g, s = _operand(op, n, 3)
    d = oracle.apply(op, c, g, s)
    rs = oracle.checksum(c)
    assert np.array_equal(rs, c.sum(0))
    gchk = M * g if op == "add" else g  # the checksum stream carries sum of M operands
    e = oracle.apply(op, rs, gchk, s)
    for r in range(M):
        dd = d.copy()
        dd[r] = 12345
        assert np.array_equal(oracle.checksum_recover(dd, e, r), d[r])
    assert bigint.checksum_recover([list(row) for row in d.tolist()], e.tolist(), 1) == d[1].tolist()


# ------------------------------------------------------------- workloads

def test_workload_shapes_and_ranges():
    g = wl.config_small()
    assert g.c.shape == (3, 65536) and g.operand.size == 16
    assert g.c.min() >= -128 and g.c.max() <= 127
    grp = wl.config_uneven(groups=40, n_hi=1 << 14)
    assert all(3 <= x.M <= 8 for x in grp)
    assert all((1 << 12) <= x.n <= (1 << 14) for x in grp)
    for x in grp:
        if x.op == "perm":
            assert np.array_equal(np.sort(x.operand), np.arange(x.n))
    v = wl.log_uniform_int(wl.rng(0), 8, 512, 10000)
    assert v.min() >= 8 and v.max() <= 512


def test_config_outputs_within_dynamic_range():
    """Worst-case output magnitude of every benchmark configuration is inside
    the admissible range of eq. (11)/(13) at w = 64."""
    D = {M: oracle.params(M, 64)[2] for M in range(3, 9)}
    assert 16 * 128 * 128 <= D[3]                      # M = 3, 16 taps, 8-bit
    assert 64 * (1 << 11) ** 2 <= D[3]                 # 64 taps, 12-bit
    assert 512 * (1 << 9) ** 2 <= D[3]                 # uneven conv
    assert (1 << 22) * (1 << 9) ** 2 <= D[3]           # uneven inner product
    assert 1024 * (1 << 15) ** 2 <= D[3]               # long kernel, 16-bit
    assert 1024 * (1 << 10) ** 2 <= D[3]               # serving
