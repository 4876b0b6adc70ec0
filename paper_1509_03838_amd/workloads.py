"""Seeded synthetic workloads (inputs only).

This module draws random inputs and nothing else: it holds none of the
method's arithmetic (no entanglement, no LSB operation, no extraction), so
that the CPU oracle and the GPU path can both be fed from it without sharing
any computation. It imports only numpy.

The paper's own experiment (Sec. V) convolves M in {3, 8} streams of 10^6
32-bit integer samples with kernels of 100 to 4500 taps; its data are not
published, so every workload here is synthetic, with the shapes and value
ranges of the benchmark configurations below. Integers are drawn with
numpy's PCG64; "uniform in [a, b)" is numpy's ``integers(a, b)``;
"log-uniform in [a, b]" is floor(2^U), U ~ Uniform[log2 a, log2 b], clipped
to [a, b].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1509038380
OP_KINDS = ("conv", "scale", "add", "inner", "perm")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_i32(g: np.random.Generator, lo: int, hi: int, size) -> np.ndarray:
    """int32 samples uniform in [lo, hi)."""
    return g.integers(lo, hi, size=size, dtype=np.int64).astype(np.int32)


def log_uniform_int(g: np.random.Generator, a: int, b: int, size=None):
    u = g.uniform(np.log2(a), np.log2(b), size=size)
    v = np.clip(np.floor(np.exp2(u)).astype(np.int64), a, b)
    return v


@dataclass
class Group:
    """One group of M input streams sharing one operand.

    op       : one of OP_KINDS
    c        : (M, n) int32 input streams
    operand  : int32 array -- conv kernel (K taps), add/inner vector (n), or
               the permutation's source indices (n); empty for scale
    scalar   : the scale factor (scale only)
    fail     : index of the stream whose LSB operation is dropped (fail-stop),
               or -1 for none
    """
    op: str
    c: np.ndarray
    operand: np.ndarray
    scalar: int = 0
    fail: int = -1
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.c.shape[0])

    @property
    def n(self) -> int:
        return int(self.c.shape[1])


def conv_group(g: np.random.Generator, M: int, n: int, K: int, lo: int, hi: int,
               fail: int = -1) -> Group:
    c = uniform_i32(g, lo, hi, (M, n))
    k = uniform_i32(g, lo, hi, K)
    return Group("conv", c, k, 0, fail)


def config_small(seed: int = SEED_BASE + 0, fail: int = -1) -> Group:
    """M = 3 streams of 65,536 int32 samples uniform in [-128, 127] and one
    16-tap kernel in the same range; full linear convolution."""
    return conv_group(rng(seed), 3, 65536, 16, -128, 128, fail)


def config_batched(seed: int = SEED_BASE + 1, groups: int = 64, n: int = 1 << 20, K: int = 64,
                   fail: int = -1) -> list[Group]:
    """64 stream-triples of 1,048,576 int32 samples uniform in [-2^11, 2^11),
    each with its own 64-tap kernel in the same range."""
    g = rng(seed)
    return [conv_group(g, 3, n, K, -(1 << 11), 1 << 11, fail) for _ in range(groups)]


def permutation(g: np.random.Generator, n: int) -> np.ndarray:
    return g.permutation(n).astype(np.int32)


def config_uneven(seed: int = SEED_BASE + 2, groups: int = 512, n_lo: int = 1 << 12,
                  n_hi: int = 1 << 22, k_lo: int = 8, k_hi: int = 512,
                  ops=OP_KINDS) -> list[Group]:
    """512 groups; M uniform in {3..8}; lengths log-uniform in [2^12, 2^22];
    samples uniform in [-2^9, 2^9); conv taps log-uniform in [8, 512]; the
    operation of each group uniform over `ops`. Operand values (kernel taps,
    added and inner-product vectors, the scale factor) are drawn from the
    samples' range; the permutation is a seeded random bijection."""
    g = rng(seed)
    lo, hi = -(1 << 9), 1 << 9
    out = []
    for _ in range(groups):
        M = int(g.integers(3, 9))
        n = int(log_uniform_int(g, n_lo, n_hi))
        op = ops[int(g.integers(0, len(ops)))]
        c = uniform_i32(g, lo, hi, (M, n))
        scalar = 0
        if op == "conv":
            operand = uniform_i32(g, lo, hi, int(log_uniform_int(g, k_lo, k_hi)))
        elif op in ("add", "inner"):
            operand = uniform_i32(g, lo, hi, n)
        elif op == "perm":
            operand = permutation(g, n)
        else:
            operand = np.zeros(0, np.int32)
            scalar = int(g.integers(lo, hi))
        out.append(Group(op, c, operand, scalar, -1))
    return out


def config_long_kernel(seed: int = SEED_BASE + 3, groups: int = 256, n: int = 262144,
                       K: int = 1024) -> list[Group]:
    """256 stream-triples of 262,144 samples uniform in [-2^15, 2^15) held as
    int32, with 1024-tap kernels in the same range."""
    g = rng(seed)
    return [conv_group(g, 3, n, K, -(1 << 15), 1 << 15) for _ in range(groups)]


FIG2_M = (3, 8)
FIG2_TAPS = (100, 250, 500, 1000, 2000, 3000, 4500)
FIG2_N = 1_000_000
FIG2_BITS = 15


def config_fig2(M: int, K: int, seed: int = SEED_BASE + 5, n: int = FIG2_N) -> Group:
    """One group shaped as in the paper's experiment (Sec. V, Fig. 2): M
    streams of 10^6 samples and one K-tap kernel, samples and taps uniform in
    [-2^14, 2^14) held as int32 -- the widest range whose worst-case output
    at K = 4500 fits the M = 3 bound at w = 64. The streams depend on M and
    the seed only, the taps on M, K and the seed."""
    lo, hi = -(1 << (FIG2_BITS - 1)), 1 << (FIG2_BITS - 1)
    c = uniform_i32(rng(seed * 16 + M), lo, hi, (M, n))
    k = uniform_i32(rng((seed * 16 + M) * 8192 + K), lo, hi, K)
    return Group("conv", c, k, 0, -1)


CHAIN_RECIPE = ("add", "scale", "conv", "perm", "add")


def chain_series(g: np.random.Generator, n: int, recipe=CHAIN_RECIPE, bits: int = 10,
                 K: int = 64) -> list[tuple[str, np.ndarray | None, int]]:
    """Operands of a series of operations on streams of n samples: for each
    op of the recipe, (op, operand, scalar) with the operand drawn uniform
    in [-2^(bits-1), 2^(bits-1)) (conv, circ, xcorr: K taps; outer: K
    values; add, sub, mul, inner: a vector of the current length), a seeded
    permutation of the current length, or a scale factor in the same range
    (nonzero). The length after each op follows it (inner: 1; outer: n K)."""
    lo, hi = -(1 << (bits - 1)), 1 << (bits - 1)
    out = []
    for op in recipe:
        if op in ("conv", "xcorr"):
            out.append((op, uniform_i32(g, lo, hi, K), 0))
            n = n + K - 1 if n else 0
        elif op in ("circ", "outer"):
            out.append((op, uniform_i32(g, lo, hi, K), 0))
            n = n * K if op == "outer" else n
        elif op in ("add", "inner", "sub", "mul"):
            out.append((op, uniform_i32(g, lo, hi, n), 0))
            n = 1 if op == "inner" else n
        elif op == "perm":
            out.append((op, permutation(g, n), 0))
        else:
            s = int(g.integers(lo, hi))
            out.append((op, None, s if s else 1))
    return out


GEMM_BITS = 12


def config_gemm(seed: int = SEED_BASE + 8, M: int = 3, N: int = 4096, P: int = 1024,
                Q: int = 4096) -> tuple[np.ndarray, np.ndarray]:
    """M blocks of N x P int32 values and one P x Q kernel matrix, all
    uniform in [-2^11, 2^11) (the batched configuration's range)."""
    g = rng(seed)
    lo, hi = -(1 << (GEMM_BITS - 1)), 1 << (GEMM_BITS - 1)
    return uniform_i32(g, lo, hi, (M, N, P)), uniform_i32(g, lo, hi, (P, Q))


@dataclass
class Job:
    arrival_s: float
    group: Group


def serving_jobs(seed: int = SEED_BASE + 4, count: int = 2000, rate_hz: float = 2000.0,
                 n_lo: int = 1 << 10, n_hi: int = 1 << 20, k_lo: int = 16, k_hi: int = 1024,
                 drop_prob: float = 0.01) -> list[Job]:
    """Poisson arrivals (exponential gaps of mean 1/rate); each job has M
    uniform in {3, 4, 5}, length log-uniform in [2^10, 2^20] with samples
    uniform in [-2^10, 2^10), a conv kernel of log-uniform [16, 1024] taps in
    the same range, and with probability `drop_prob` one stream (uniform)
    whose operation is dropped."""
    g = rng(seed)
    t = 0.0
    jobs = []
    lo, hi = -(1 << 10), 1 << 10
    for _ in range(count):
        t += float(g.exponential(1.0 / rate_hz))
        M = int(g.integers(3, 6))
        n = int(log_uniform_int(g, n_lo, n_hi))
        K = int(log_uniform_int(g, k_lo, k_hi))
        fail = int(g.integers(0, M)) if g.uniform() < drop_prob else -1
        jobs.append(Job(t, conv_group(g, M, n, K, lo, hi, fail)))
    return jobs
