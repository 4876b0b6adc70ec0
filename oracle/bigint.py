"""Pure-Python big-integer twin of the C oracle, for tiny inputs only.

TEST INFRASTRUCTURE: used by the test suite to cross-check the C oracle
(which could hide undefined behaviour in 128-bit arithmetic) on small cases.
Python integers are unbounded, so every register width the paper talks about
(w bits for the entangled words, 2w bits for the extraction temporary of
Sec. III-A) is modelled explicitly by reduction into a signed range.

Paper: Anam & Andreopoulos, "Failure Mitigation in Linear, Sesquilinear and
Bijective Operations On Integer Data Streams Via Numerical Entanglement",
IOLTS 2015.
"""
from __future__ import annotations


class RangeError(ValueError):
    """A value left the register the paper says it must fit in."""


def wrap(x: int, bits: int) -> int:
    """x modulo 2^bits, read as a signed `bits`-bit two's-complement word."""
    m = 1 << bits
    x %= m
    return x - m if x >= (m >> 1) else x


def fits(x: int, bits: int) -> bool:
    return -(1 << (bits - 1)) <= x < (1 << (bits - 1))


def shift(x: int, l: int, bits: int) -> int:
    """Shift operator S_l of eq. (7) in a `bits`-bit register (footnote 1):
    left by l (truncating at the top of the register) when l >= 0, else an
    arithmetic right shift by -l (Python's >> on ints is a floor shift)."""
    if l >= 0:
        return wrap(x << l, bits)
    return x >> (-l)


def params(M: int, w: int) -> tuple[int, int, int]:
    """(l, k, D) for M streams in w-bit words.

    l, k: among l >= 1, 0 <= k <= l with (M-1)l + k <= w (eq. (12); eq. (8)
    for M = 3) the pair maximising the output bit-width (M-2)l + k that
    Table I lists, larger l among equals.
    D: the admissible output magnitude, eq. (11) for M = 3, eq. (13) else.
    """
    if M < 3:
        raise ValueError("M >= 3")
    best = None
    for l in range(1, w + 1):
        for k in range(0, l + 1):
            if (M - 1) * l + k > w:
                continue
            key = ((M - 2) * l + k, l)
            if best is None or key > best[0]:
                best = (key, l, k)
    if best is None:
        raise ValueError("no (l, k) for this (M, w)")
    _, l, k = best
    if M == 3:
        D = (1 << (l + k - 1)) - (1 << l)
    else:
        D = (1 << ((M - 3) * l + k)) * ((1 << (l - 1)) - 1)
    return l, k, D


def entangle(c: list[list[int]], l: int, w: int) -> list[list[int]]:
    """eq. (14)-(15): eps_m = c_m + S_l{c_(m-1 mod M)}, position by position."""
    M = len(c)
    out = []
    for m in range(M):
        row = []
        for a, b in zip(c[m], c[(m - 1) % M]):
            e = a + (b << l)
            if not fits(e, w):
                raise RangeError("entangled word exceeds w bits")
            row.append(e)
        out.append(row)
    return out


def entangle_operand(g: list[int], l: int, w: int) -> list[int]:
    """Footnote 3: g <- S_l{g} + g (for op in {+, -})."""
    out = [(x << l) + x for x in g]
    if not all(fits(v, w) for v in out):
        raise RangeError("entangled operand exceeds w bits")
    return out


def conv(x: list[int], g: list[int]) -> list[int]:
    """Full linear convolution y[t] = sum_j g[j] x[t-j], t in [0, n+K-2]."""
    if not x or not g:
        return []
    n, K = len(x), len(g)
    return [sum(g[j] * x[t - j] for j in range(K) if 0 <= t - j < n) for t in range(n + K - 1)]


def apply(op: str, x: list[int], operand=None, scalar: int = 0) -> list[int]:
    """d = x op g (eq. (2)), exact."""
    if op == "conv":
        return conv(x, operand)
    if op == "scale":
        return [scalar * v for v in x]
    if op == "add":
        return [a + b for a, b in zip(x, operand, strict=True)]
    if op == "inner":
        return [sum(a * b for a, b in zip(x, operand, strict=True))]
    if op == "perm":
        assert sorted(operand) == list(range(len(x)))
        return [x[i] for i in operand]
    raise ValueError(op)


def extract(delta: list[list[int] | None], r: int, l: int, w: int,
            printed_sign: bool = False) -> list[list[int]]:
    """Recover d-hat from the M-1 entangled outputs other than delta[r]
    (eq. (16)-(19)); delta[r] is never touched and may be None.

    Readings: eq. (16) carries an extra (-1)^M (without it only even M
    recover; `printed_sign=True` keeps the printed form to demonstrate that);
    eq. (18) subtracts the value eq. (17) produced; eq. (19) covers
    1 <= m <= M-2.
    """
    M = len(delta)
    W2 = 2 * w
    sh = W2 - (M - 1) * l
    n = len(delta[(r + 1) % M])
    out = [[0] * n for _ in range(M)]
    for i in range(n):
        dtemp = 0
        for m in range(M - 1):
            term = shift(delta[(r + 1 + m) % M][i], (M - 2 - m) * l, W2)
            sgn = (-1) ** m if printed_sign else (-1) ** (M + m)
            dtemp = wrap(dtemp + sgn * term, W2)
        last = (r + M - 1) % M
        d_last = shift(shift(dtemp, sh, W2), -sh, W2)
        diff = wrap(dtemp - d_last, W2)
        if M % 2:
            diff = -diff
        d_r = shift(diff, -(M - 1) * l, W2)
        if (d_r << ((M - 1) * l)) != diff:
            raise RangeError("eq. (18) shift is not exact")
        out[last][i] = d_last
        out[r][i] = d_r
        prev = d_r
        for m in range(1, M - 1):
            j = (r + m) % M
            prev = wrap(delta[j][i] - shift(prev, l, W2), W2)
            out[j][i] = prev
    return out


def checksum(c: list[list[int]]) -> list[int]:
    """eq. (4): r_n = sum_m c_(m,n)."""
    return [sum(col) for col in zip(*c)]


def checksum_recover(d: list[list[int] | None], e: list[int], r: int) -> list[int]:
    """d_r = e - sum_(m != r) d_m (linearity of op; not printed in the paper)."""
    out = list(e)
    for m, row in enumerate(d):
        if m == r:
            continue
        out = [a - b for a, b in zip(out, row)]
    return out
