"""CPU oracle for numerical entanglement (Anam & Andreopoulos, IOLTS 2015).

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU library and imports nothing from it.

The arithmetic lives in ``ne_oracle.c`` (plain C with 128-bit integers, every
overflow checked); this module only marshals numpy arrays into it. The
pure-Python twin in ``bigint.py`` re-derives the same results with unbounded
integers for tiny inputs.

Conventions: a group of M streams of n samples is an int64 array of shape
(M, n). Integer op codes follow the paper's eq. (2): CONV (full linear
convolution), SCALE, ADD, INNER (inner product), PERM (fixed permutation),
SUB, MUL (element by element), CIRC (circular convolution), XCORR (full
cross-correlation), OUTER (outer product).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ne_oracle.c")
_LIB = os.path.join(_HERE, "libne_oracle.so")

CONV, SCALE, ADD, INNER, PERM = 0, 1, 2, 3, 4
SUB, MUL, CIRC, XCORR, OUTER = 5, 6, 7, 8, 9
OPS = {"conv": CONV, "scale": SCALE, "add": ADD, "inner": INNER, "perm": PERM,
       "sub": SUB, "mul": MUL, "circ": CIRC, "xcorr": XCORR, "outer": OUTER}
# operations whose vector operand is added or subtracted: on entangled data it
# is entangled with itself first (footnote 3)
ADDITIVE = ("add", "sub")

OK, EINVAL, EOVERFLOW, EINEXACT = 0, 1, 2, 3


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into oracle/libne_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        L.orc_params.argtypes = [i32, i32, P, P, P]
        L.orc_entangle.argtypes = [i32, i32, i32, i64, P, P]
        L.orc_entangle_operand.argtypes = [i32, i32, i64, P, P]
        L.orc_op.argtypes = [i32, i32, i64, P, P, i64, i64, P, i64]
        L.orc_conv_at.argtypes = [i32, i64, P, i64, P, i64, P, P]
        L.orc_extract.argtypes = [i32, i32, i32, i64, P, i32, P]
        L.orc_extract_printed_sign.argtypes = [i32, i32, i32, i64, P, i32, P]
        L.orc_checksum.argtypes = [i32, i32, i64, P, P]
        L.orc_checksum_recover.argtypes = [i32, i32, i64, P, P, i32, P]
        L.orc_gemm.argtypes = [i32, i64, i64, i64, P, P, P]
        L.orc_gemm_at.argtypes = [i32, i64, i64, i64, P, P, i64, P, P, P]
        for f in ("orc_params", "orc_entangle", "orc_entangle_operand", "orc_op", "orc_conv_at",
                  "orc_extract", "orc_extract_printed_sign", "orc_checksum",
                  "orc_checksum_recover", "orc_gemm", "orc_gemm_at"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _check(rc: int, what: str):
    if rc != OK:
        name = {EINVAL: "invalid argument", EOVERFLOW: "value outside the register",
                EINEXACT: "inexact shift"}.get(rc, str(rc))
        raise OracleError(f"{what}: {name}")


def params(M: int, w: int = 64) -> tuple[int, int, int]:
    """(l, k, D): shift, headroom and admissible output magnitude (Table I,
    eq. (11)-(13))."""
    l, k, D = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
    rc = lib().orc_params(M, w, ctypes.byref(l), ctypes.byref(k), ctypes.byref(D))
    _check(rc, f"params(M={M}, w={w})")
    return l.value, k.value, D.value


def entangle(c, l: int, w: int = 64) -> np.ndarray:
    """eq. (14)-(15) on an (M, n) group."""
    c = _i64(c)
    M, n = c.shape
    out = np.empty_like(c)
    _check(lib().orc_entangle(M, l, w, n, _p(c), _p(out)), "entangle")
    return out


def entangle_operand(g, l: int, w: int = 64) -> np.ndarray:
    """Footnote 3: g + S_l{g}."""
    g = _i64(g)
    out = np.empty_like(g)
    _check(lib().orc_entangle_operand(l, w, g.size, _p(g), _p(out)), "entangle_operand")
    return out


def n_out(op: str, n_in: int, n_operand: int) -> int:
    if op in ("conv", "xcorr"):
        return 0 if n_in == 0 or n_operand == 0 else n_in + n_operand - 1
    if op == "inner":
        return 1
    if op == "outer":
        return n_in * n_operand
    return n_in


def apply(op: str, x, operand=None, scalar: int = 0, w: int = 64) -> np.ndarray:
    """x op g for one stream (1-D) or each row of a 2-D group; exact."""
    x = _i64(x)
    if x.ndim == 2:
        return np.stack([apply(op, row, operand, scalar, w) for row in x]) if x.shape[0] else \
            np.zeros((0, 0), np.int64)
    operand = _i64(operand if operand is not None else np.zeros(0, np.int64))
    no = n_out(op, x.size, operand.size)
    out = np.empty(no, np.int64)
    rc = lib().orc_op(OPS[op], w, x.size, _p(x), _p(operand), operand.size, int(scalar),
                      _p(out), no)
    _check(rc, f"apply({op})")
    return out


def conv_at(x, g, pos, w: int = 64) -> np.ndarray:
    """Full-linear-convolution outputs at the given positions only."""
    x, g, pos = _i64(x), _i64(g), _i64(pos)
    out = np.empty(pos.size, np.int64)
    _check(lib().orc_conv_at(w, x.size, _p(x), g.size, _p(g), pos.size, _p(pos), _p(out)),
           "conv_at")
    return out


def extract(delta, r: int, l: int, w: int = 64, printed_sign: bool = False) -> np.ndarray:
    """eq. (16)-(19): recover all M outputs without reading delta[r]."""
    delta = _i64(delta)
    M, n = delta.shape
    out = np.empty_like(delta)
    f = lib().orc_extract_printed_sign if printed_sign else lib().orc_extract
    _check(f(M, l, w, n, _p(delta), r, _p(out)), "extract")
    return out


def checksum(c, w: int = 64) -> np.ndarray:
    """eq. (4)."""
    c = _i64(c)
    M, n = c.shape
    out = np.empty(n, np.int64)
    _check(lib().orc_checksum(M, w, n, _p(c), _p(out)), "checksum")
    return out


def checksum_recover(d, e, r: int, w: int = 64) -> np.ndarray:
    """d_r = e - sum_{m != r} d_m."""
    d, e = _i64(d), _i64(e)
    M, n = d.shape
    out = np.empty(n, np.int64)
    _check(lib().orc_checksum_recover(M, w, n, _p(d), _p(e), r, _p(out)), "checksum_recover")
    return out


def pipeline(c, op: str, operand=None, scalar: int = 0, r: int = 0, w: int = 64):
    """The whole method on one group: entangle, op on every entangled stream,
    drop stream r, extract. Returns (d_hat, eps, delta)."""
    c = _i64(c)
    M = c.shape[0]
    l, _, _ = params(M, w)
    eps = entangle(c, l, w)
    g = operand
    if op in ADDITIVE:
        g = entangle_operand(operand, l, w)
    delta = apply(op, eps, g, scalar, w)
    return extract(delta, r, l, w), eps, delta


def chain(c, ops, w: int = 64) -> np.ndarray:
    """A series of LSB operations applied one after another to every stream
    (Sec. II: operators in series before any extraction), exact. ops: a list
    of (op, operand, scalar)."""
    x = _i64(c)
    for op, operand, scalar in ops:
        x = apply(op, x, operand, scalar, w)
    return x


def chain_pipeline(c, ops, r: int = 0, w: int = 64):
    """The method with a series: entangle once (eq. (14)-(15)), run every
    operation on every entangled stream (an added vector entangled with
    itself, footnote 3), drop stream r, extract once (eq. (16)-(19)).
    Returns (d_hat, the last stage's entangled outputs)."""
    c = _i64(c)
    M = c.shape[0]
    l, _, _ = params(M, w)
    x = entangle(c, l, w)
    for op, operand, scalar in ops:
        g = entangle_operand(operand, l, w) if op in ADDITIVE else operand
        x = apply(op, x, g, scalar, w)
    return extract(x, r, l, w), x


def gemm(c, g, w: int = 64) -> np.ndarray:
    """Integer matrix product of every block: c (M, N, P) or (N, P), g (P, Q);
    exact (the multiplication operator of eq. (2) on matrix blocks)."""
    c, g = _i64(c), _i64(g)
    if c.ndim == 3:
        return np.stack([gemm(blk, g, w) for blk in c]) if c.shape[0] else \
            np.zeros((0, c.shape[1], g.shape[1]), np.int64)
    N, P = c.shape
    Q = g.shape[1]
    if g.shape[0] != P:
        raise ValueError("inner dimensions differ")
    out = np.empty((N, Q), np.int64)
    _check(lib().orc_gemm(w, N, P, Q, _p(np.ascontiguousarray(c)), _p(np.ascontiguousarray(g)),
                          _p(out)), "gemm")
    return out


def gemm_at(c, g, rows, cols, w: int = 64) -> np.ndarray:
    """Entries (rows[q], cols[q]) of c @ g for one block c (N, P)."""
    c, g = np.ascontiguousarray(_i64(c)), np.ascontiguousarray(_i64(g))
    rows, cols = _i64(rows), _i64(cols)
    out = np.empty(rows.size, np.int64)
    N, P = c.shape
    _check(lib().orc_gemm_at(w, N, P, g.shape[1], _p(c), _p(g), rows.size, _p(rows), _p(cols),
                             _p(out)), "gemm_at")
    return out


def gemm_pipeline(c, g, r: int = 0, w: int = 64):
    """The method on M matrix blocks: entangle the blocks element by element
    (eq. (14)-(15)), multiply every entangled block by g, drop block r,
    extract element by element (eq. (16)-(19)). Returns (d_hat, delta)."""
    c = _i64(c)
    M, N, P = c.shape
    l, _, _ = params(M, w)
    eps = entangle(c.reshape(M, N * P), l, w).reshape(M, N, P)
    delta = gemm(eps, g, w)
    Q = delta.shape[2]
    dhat = extract(delta.reshape(M, N * Q), r, l, w).reshape(M, N, Q)
    return dhat, delta
