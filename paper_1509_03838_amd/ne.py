"""ctypes binding of libne (include/ne.h).

Argument marshalling only: every step of the method runs in the HIP
library. Tensors must be contiguous device tensors of the stated dtype; the
binding passes their data pointers and the current HIP stream, and raises
``NeError`` with the library's status text on any non-zero status. If the
library has not been built, loading raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
# NE_LIB names another build of the library to load instead (to compare builds).
LIB_PATH = os.environ.get("NE_LIB") or os.path.join(HERE, "libne.so")

CONV, SCALE, ADD, INNER, PERM = 0, 1, 2, 3, 4
SUB, MUL, CIRC, XCORR, OUTER = 5, 6, 7, 8, 9
OPS = {"conv": CONV, "scale": SCALE, "add": ADD, "inner": INNER, "perm": PERM,
       "sub": SUB, "mul": MUL, "circ": CIRC, "xcorr": XCORR, "outer": OUTER}
MAX_M = 32
MAX_M32 = 17
CHAIN_SCRATCH_BYTES = 64 << 20  # NE_CHAIN_SCRATCH_BYTES: the fixed buffer of chain_apply_noalloc

EXPORTS = ("ne_strerror", "ne_last_hip_error", "ne_version", "ne_params", "ne_entangle",
           "ne_entangle_inplace", "ne_entangle_operand", "ne_lsb_apply", "ne_extract_recover",
           "ne_plain_apply", "ne_checksum", "ne_checksum_recover", "ne_plan_create",
           "ne_plan_run", "ne_plan_capture", "ne_plan_launch", "ne_plan_flags",
           "ne_plan_stats_get", "ne_plan_destroy", "ne_plan_workspace_size", "ne_plan_create_in",
           "ne_chain_check", "ne_chain_workspace_size", "ne_chain_apply", "ne_gemm",
           "ne_gemm_workspace_size", "ne_entangle32", "ne_entangle_operand32", "ne_lsb_apply32",
           "ne_extract_recover32", "ne_chain_check32", "ne_chain_workspace_size32",
           "ne_chain_apply32", "ne_device_flags", "ne_chain_apply_noalloc", "ne_stream_widen",
           "ne_mfma_i8_peak", "ne_wait_streams", "ne_stream_delay", "ne_chain_run_workspace_size",
           "ne_chain_run", "ne_chain_run_workspace_size32", "ne_chain_run32")

FUSED_MAX_M = 8
MODES = {"entangled": 0, "plain": 1, "plain_same": 2, "checksum": 3, "checksum_same": 4}
FLAG_INPUT_RANGE, FLAG_LIMBS, FLAG_MISMATCH, FLAG_PERM_INDEX, FLAG_STALL = 1, 2, 4, 8, 16


class GroupC(ctypes.Structure):
    """struct ne_group"""
    _fields_ = [("op", ctypes.c_int32), ("M", ctypes.c_int32), ("n", ctypes.c_int64),
                ("n_operand", ctypes.c_int64), ("scalar", ctypes.c_int64),
                ("lost", ctypes.c_int32), ("in_bits", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("ring_waves", ctypes.c_int32),
                ("tap_copies", ctypes.c_int32), ("word_bits", ctypes.c_int32),
                ("c", ctypes.c_void_p * FUSED_MAX_M), ("operand", ctypes.c_void_p),
                ("out", ctypes.c_void_p * FUSED_MAX_M)]


class ChainOpC(ctypes.Structure):
    """struct ne_chain_op"""
    _fields_ = [("op", ctypes.c_int32), ("operand_bits", ctypes.c_int32),
                ("operand", ctypes.c_void_p), ("n_operand", ctypes.c_int64),
                ("scalar", ctypes.c_int64)]


class TuningC(ctypes.Structure):
    _fields_ = [("conv_steps", ctypes.c_int32), ("stream_steps", ctypes.c_int32),
                ("single_launch", ctypes.c_int32)]


class StatsC(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("groups", "items", "launches", "in_bytes",
                                               "out_bytes", "out_samples", "macs", "mfma_macs",
                                               "lds_bytes", "limb_macs")]


class NeError(RuntimeError):
    def __init__(self, fn: str, status: int, text: str, hip: int = 0):
        super().__init__(f"{fn}: {text} (status {status}" + (f", hip error {hip})" if hip else ")"))
        self.status = status


_lib = None
_P = ctypes.c_void_p
_i32, _i64, _u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32


def load() -> ctypes.CDLL:
    """Load libne.so (built by paper_1509_03838_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing; build it with python -m paper_1509_03838_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "ne_strerror": (ctypes.c_char_p, [_i32]),
        "ne_last_hip_error": (_i32, []),
        "ne_version": (_i32, []),
        "ne_device_flags": (_i32, [ctypes.POINTER(ctypes.c_uint32), _i32]),
        "ne_params": (_i32, [_i32, _i32, _P, _P, _P]),
        "ne_entangle": (_i32, [_i32, _i32, _i64, _P, _P, _P]),
        "ne_entangle_inplace": (_i32, [_i32, _i32, _i64, _P, _P]),
        "ne_entangle_operand": (_i32, [_i32, _i64, _P, _P, _P]),
        "ne_lsb_apply": (_i32, [_i32, _i32, _i64, _P, _P, _i64, _i64, _P, _i64, _u32, _P]),
        "ne_extract_recover": (_i32, [_i32, _i32, _i64, _P, _i32, _P, _P]),
        "ne_plain_apply": (_i32, [_i32, _i32, _i64, _P, _P, _i64, _i64, _P, _i64, _P]),
        "ne_checksum": (_i32, [_i32, _i64, _P, _P, _P]),
        "ne_checksum_recover": (_i32, [_i32, _i64, _P, _P, _i32, _P, _P]),
        "ne_plan_create": (_i32, [ctypes.POINTER(GroupC), _i32, _i32, ctypes.POINTER(TuningC),
                                  ctypes.POINTER(ctypes.c_void_p)]),
        "ne_plan_run": (_i32, [_P, _P]),
        "ne_plan_capture": (_i32, [_P, _P]),
        "ne_plan_launch": (_i32, [_P, _P]),
        "ne_plan_flags": (_i32, [_P, ctypes.POINTER(ctypes.c_uint32), _i32]),
        "ne_plan_stats_get": (_i32, [_P, ctypes.POINTER(StatsC)]),
        "ne_plan_destroy": (_i32, [_P]),
        "ne_plan_workspace_size": (_i32, [ctypes.POINTER(GroupC), _i32, _i32,
                                          ctypes.POINTER(TuningC), ctypes.POINTER(ctypes.c_size_t)]),
        "ne_plan_create_in": (_i32, [ctypes.POINTER(GroupC), _i32, _i32, ctypes.POINTER(TuningC),
                                     _P, ctypes.c_size_t, _P, ctypes.POINTER(ctypes.c_void_p)]),
        "ne_chain_check": (_i32, [_i32, _i32, _i64, ctypes.POINTER(ChainOpC), _i32,
                                  ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
        "ne_chain_workspace_size": (_i32, [_i32, _i64, ctypes.POINTER(ChainOpC), _i32,
                                           ctypes.POINTER(ctypes.c_size_t)]),
        "ne_chain_apply": (_i32, [_i32, _i64, _P, ctypes.POINTER(ChainOpC), _i32, _P, _i64, _u32,
                                  _P, ctypes.c_size_t, _P]),
        "ne_chain_run_workspace_size": (_i32, [_i32, _i64, ctypes.POINTER(ChainOpC), _i32,
                                               ctypes.POINTER(ctypes.c_size_t)]),
        "ne_chain_run": (_i32, [_i32, _i64, _P, ctypes.POINTER(ChainOpC), _i32, _i32, _P, _i64,
                                _P, ctypes.c_size_t, _P]),
        "ne_chain_run_workspace_size32": (_i32, [_i32, _i64, ctypes.POINTER(ChainOpC), _i32,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
        "ne_chain_run32": (_i32, [_i32, _i64, _P, ctypes.POINTER(ChainOpC), _i32, _i32, _P, _i64,
                                  _P, ctypes.c_size_t, _P]),
        "ne_stream_widen": (_i32, [_P, _i64, _P, _P]),
        "ne_wait_streams": (_i32, [_i32, _P, _i64, ctypes.POINTER(_i32)]),
        "ne_stream_delay": (_i32, [_i64, _P]),
        "ne_mfma_i8_peak": (_i32, [_i32, _i64, _i32, _P, ctypes.POINTER(ctypes.c_double), _P]),
        "ne_chain_apply_noalloc": (_i32, [_i32, _i64, _P, ctypes.POINTER(ChainOpC), _i32, _P,
                                          _i64, _u32, _P]),
        "ne_gemm": (_i32, [_i32, _i32, _i64, _i64, _i64, _P, _P, _P, _i32, _i32, _P,
                           ctypes.c_size_t, _P, _P]),
        "ne_gemm_workspace_size": (_i32, [_i32, _i32, _i64, _i64, _i64, _i32,
                                          ctypes.POINTER(ctypes.c_size_t)]),
        "ne_entangle32": (_i32, [_i32, _i32, _i64, _P, _P, _P]),
        "ne_entangle_operand32": (_i32, [_i32, _i64, _P, _P, _P]),
        "ne_lsb_apply32": (_i32, [_i32, _i32, _i64, _P, _P, _i64, _i64, _P, _i64, _u32, _P]),
        "ne_extract_recover32": (_i32, [_i32, _i32, _i64, _P, _i32, _P, _P]),
        "ne_chain_check32": (_i32, [_i32, _i32, _i64, ctypes.POINTER(ChainOpC), _i32,
                                    ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
        "ne_chain_workspace_size32": (_i32, [_i32, _i64, ctypes.POINTER(ChainOpC), _i32,
                                             ctypes.POINTER(ctypes.c_size_t)]),
        "ne_chain_apply32": (_i32, [_i32, _i64, _P, ctypes.POINTER(ChainOpC), _i32, _P, _i64,
                                    _u32, _P, ctypes.c_size_t, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


def _check(fn: str, status: int):
    if status != 0:
        L = load()
        raise NeError(fn, status, L.ne_strerror(status).decode(), L.ne_last_hip_error())


def _ptr(t) -> int:
    """Device address of a tensor, or a raw integer address, or 0 for None."""
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _ptr_array(ts: Sequence) -> ctypes.Array:
    arr = (ctypes.c_void_p * max(1, len(ts)))()
    for i, t in enumerate(ts):
        arr[i] = _ptr(t)
    return arr


def _stream(stream) -> int:
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dtype(ts, dt, what):
    for t in ts:
        if t is not None and not isinstance(t, int) and t.dtype != dt:
            raise TypeError(f"{what} must be {dt}, got {t.dtype}")


def _tensors(ts) -> list:
    """The tensors among ts (None and raw integer addresses are the caller's
    responsibility and are skipped)."""
    return [t for t in ts if t is not None and not isinstance(t, int)]


def _on_device(what: str, ts, device=None):
    """Every tensor in ts must live on one GPU (the library dereferences the
    pointers on the device; a host tensor would be an out-of-bounds device
    access). Returns that device, or `device` if ts holds no tensor."""
    for t in _tensors(ts):
        if t.device.type != "cuda":
            raise ValueError(f"{what} must be on the GPU, got a tensor on {t.device}")
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if device is None:
            device = t.device
        elif t.device != device:
            raise ValueError(f"{what} is on {t.device}, other buffers on {device}")
    return device


def _lengths(what: str, ts, n: int, exact: bool):
    """Every tensor in ts holds n elements (exact) or at least n."""
    for i, t in enumerate(ts):
        if t is None or isinstance(t, int):
            continue
        k = t.numel()
        if (exact and k != n) or k < n:
            raise ValueError(f"{what}[{i}] holds {k} elements, "
                             f"{'exactly' if exact else 'at least'} {n} needed")


def _n_of(ts, n, what: str) -> int:
    """n if given, else the common length of the tensors in ts (which must
    agree: the C ABI takes one length for all of them)."""
    known = [t.numel() for t in _tensors(ts)]
    if n is None:
        if not known:
            raise ValueError(f"{what}: no tensor to take the length from; pass n")
        n = known[0]
        _lengths(what, ts, n, exact=True)
    else:
        _lengths(what, ts, n, exact=False)
    return n


def device_flags(clear: bool = False) -> int:
    """NE_FLAG_* bits the per-step kernels raised on the current device
    (synchronous: waits for the device); clear zeroes the word."""
    f = ctypes.c_uint32()
    _check("ne_device_flags", load().ne_device_flags(ctypes.byref(f), int(clear)))
    return f.value


def params(M: int, w: int = 64) -> tuple[int, int, int]:
    """(l, k, D) per Table I and eq. (11)/(13)."""
    l, k, D = _i32(), _i32(), _i64()
    _check("ne_params", load().ne_params(M, w, ctypes.byref(l), ctypes.byref(k), ctypes.byref(D)))
    return l.value, k.value, D.value


def entangle(c: Sequence, eps: Sequence, l: int, n: int | None = None, stream=None):
    """eps[m] = c[m] + 2^l c[m-1] (int32 -> int64), eq. (14)-(15)."""
    import torch
    _dtype(c, torch.int32, "c")
    _dtype(eps, torch.int64, "eps")
    if len(c) != len(eps):
        raise ValueError("c and eps differ in length")
    _on_device("c and eps", list(c) + list(eps))
    n = _n_of(c, n, "c")
    _lengths("eps", eps, n, exact=False)
    _check("ne_entangle", load().ne_entangle(len(c), l, n, _ptr_array(c), _ptr_array(eps),
                                             _stream(stream)))


def entangle_inplace(x: Sequence, l: int, n: int | None = None, stream=None):
    import torch
    _dtype(x, torch.int64, "x")
    _on_device("x", x)
    n = _n_of(x, n, "x")
    _check("ne_entangle_inplace", load().ne_entangle_inplace(len(x), l, n, _ptr_array(x),
                                                             _stream(stream)))


def entangle_operand(g, g_ent, l: int, stream=None):
    import torch
    _dtype([g], torch.int32, "g")
    _dtype([g_ent], torch.int64, "g_ent")
    _on_device("g and g_ent", [g, g_ent])
    _lengths("g_ent", [g_ent], g.numel(), exact=False)
    _check("ne_entangle_operand", load().ne_entangle_operand(l, g.numel(), _ptr(g), _ptr(g_ent),
                                                             _stream(stream)))


def n_out(op: str, n_in: int, n_operand: int) -> int:
    if op in ("conv", "xcorr"):
        return 0 if n_in == 0 else n_in + n_operand - 1
    if op == "inner":
        return 1
    if op == "outer":
        return n_in * n_operand
    return n_in


def lsb_apply(op: str, eps: Sequence, operand, delta: Sequence, scalar: int = 0,
              mask: int | None = None, n_in: int | None = None, n_operand: int | None = None,
              stream=None):
    """delta[m] = eps[m] op operand for every stream whose mask bit is set."""
    import torch
    _dtype(eps, torch.int64, "eps")
    _dtype(delta, torch.int64, "delta")
    if operand is not None and not isinstance(operand, int):
        _dtype([operand], torch.int64 if op in ("add", "sub") else torch.int32, "operand")
    M = len(eps)
    if len(delta) != M:
        raise ValueError("eps and delta differ in length")
    if mask is None:
        mask = (1 << M) - 1
    _on_device("eps, operand and delta", list(eps) + list(delta) + [operand])
    n_in = _n_of(eps, n_in, "eps")
    if n_operand is None:
        n_operand = 0 if operand is None or isinstance(operand, int) else operand.numel()
    elif operand is not None and not isinstance(operand, int):
        _lengths("operand", [operand], n_operand, exact=False)
    no = n_out(op, n_in, n_operand)
    _lengths("delta", [t for m, t in enumerate(delta) if (mask >> m) & 1], no, exact=False)
    _check("ne_lsb_apply", load().ne_lsb_apply(OPS[op], M, n_in, _ptr_array(eps), _ptr(operand),
                                               n_operand, int(scalar), _ptr_array(delta), no,
                                               mask & 0xFFFFFFFF, _stream(stream)))


def extract_recover(delta: Sequence, r: int, dhat: Sequence, l: int, n: int | None = None,
                    stream=None):
    """Recover all M outputs without reading delta[r] (eq. (16)-(19))."""
    import torch
    _dtype(delta, torch.int64, "delta")
    _dtype(dhat, torch.int64, "dhat")
    M = len(dhat)
    if len(delta) != M:
        raise ValueError("delta and dhat differ in length")
    _on_device("delta and dhat", list(delta) + list(dhat))
    n = _n_of(dhat, n, "dhat")
    _lengths("delta", [t for m, t in enumerate(delta) if m != r], n, exact=False)
    _check("ne_extract_recover", load().ne_extract_recover(M, l, n, _ptr_array(delta), r,
                                                           _ptr_array(dhat), _stream(stream)))


def entangle32(c: Sequence, eps: Sequence, l: int, n: int | None = None, stream=None):
    """eps[m] = c[m] + 2^l c[m-1] modulo 2^32 (int32 -> int32), eq. (14)-(15)
    in 32-bit words; l normally params(M, 32)[0]."""
    import torch
    _dtype(c, torch.int32, "c")
    _dtype(eps, torch.int32, "eps")
    if len(c) != len(eps):
        raise ValueError("c and eps differ in length")
    _on_device("c and eps", list(c) + list(eps))
    n = _n_of(c, n, "c")
    _lengths("eps", eps, n, exact=False)
    _check("ne_entangle32", load().ne_entangle32(len(c), l, n, _ptr_array(c), _ptr_array(eps),
                                                 _stream(stream)))


def entangle_operand32(g, g_ent, l: int, stream=None):
    import torch
    _dtype([g, g_ent], torch.int32, "g")
    _on_device("g and g_ent", [g, g_ent])
    _lengths("g_ent", [g_ent], g.numel(), exact=False)
    _check("ne_entangle_operand32", load().ne_entangle_operand32(l, g.numel(), _ptr(g),
                                                                 _ptr(g_ent), _stream(stream)))


def lsb_apply32(op: str, eps: Sequence, operand, delta: Sequence, scalar: int = 0,
                mask: int | None = None, n_in: int | None = None, stream=None):
    """delta[m] = eps[m] op operand modulo 2^32 for every stream whose mask
    bit is set; int32 words, int32 operand."""
    import torch
    _dtype(eps, torch.int32, "eps")
    _dtype(delta, torch.int32, "delta")
    if operand is not None and not isinstance(operand, int):
        _dtype([operand], torch.int32, "operand")
    M = len(eps)
    if len(delta) != M:
        raise ValueError("eps and delta differ in length")
    if mask is None:
        mask = (1 << M) - 1
    _on_device("eps, operand and delta", list(eps) + list(delta) + [operand])
    n_in = _n_of(eps, n_in, "eps")
    n_operand = 0 if operand is None or isinstance(operand, int) else operand.numel()
    no = n_out(op, n_in, n_operand)
    _lengths("delta", [t for m, t in enumerate(delta) if (mask >> m) & 1], no, exact=False)
    _check("ne_lsb_apply32", load().ne_lsb_apply32(OPS[op], M, n_in, _ptr_array(eps),
                                                   _ptr(operand), n_operand, int(scalar),
                                                   _ptr_array(delta), no, mask & 0xFFFFFFFF,
                                                   _stream(stream)))


def extract_recover32(delta: Sequence, r: int, dhat: Sequence, l: int, n: int | None = None,
                      stream=None):
    """Recover all M int32 outputs from the int32 words of the streams other
    than r (eq. (16)-(19) in 32-bit words)."""
    import torch
    _dtype(delta, torch.int32, "delta")
    _dtype(dhat, torch.int32, "dhat")
    M = len(dhat)
    if len(delta) != M:
        raise ValueError("delta and dhat differ in length")
    _on_device("delta and dhat", list(delta) + list(dhat))
    n = _n_of(dhat, n, "dhat")
    _lengths("delta", [t for m, t in enumerate(delta) if m != r], n, exact=False)
    _check("ne_extract_recover32", load().ne_extract_recover32(M, l, n, _ptr_array(delta), r,
                                                               _ptr_array(dhat), _stream(stream)))


def plain_apply(op: str, c: Sequence, operand, d: Sequence, scalar: int = 0, stream=None):
    import torch
    _dtype(c, torch.int32, "c")
    _dtype(d, torch.int64, "d")
    if operand is not None:
        _dtype([operand], torch.int32, "operand")
    if len(c) != len(d):
        raise ValueError("c and d differ in length")
    _on_device("c, operand and d", list(c) + list(d) + [operand])
    n_in = _n_of(c, None, "c")
    n_operand = 0 if operand is None else operand.numel()
    no = n_out(op, n_in, n_operand)
    _lengths("d", d, no, exact=False)
    _check("ne_plain_apply", load().ne_plain_apply(OPS[op], len(c), n_in, _ptr_array(c),
                                                   _ptr(operand), n_operand, int(scalar),
                                                   _ptr_array(d), no, _stream(stream)))


def checksum(c: Sequence, rsum, stream=None):
    import torch
    _dtype(c, torch.int32, "c")
    _dtype([rsum], torch.int64, "rsum")
    _on_device("c and rsum", list(c) + [rsum])
    n = _n_of(c, None, "c")
    _lengths("rsum", [rsum], n, exact=False)
    _check("ne_checksum", load().ne_checksum(len(c), n, _ptr_array(c), _ptr(rsum),
                                             _stream(stream)))


def checksum_recover(d: Sequence, e, r: int, d_r, stream=None):
    import torch
    _dtype(d, torch.int64, "d")
    _dtype([e, d_r], torch.int64, "e and d_r")
    _on_device("d, e and d_r", list(d) + [e, d_r])
    n = e.numel()
    _lengths("d", [t for m, t in enumerate(d) if m != r], n, exact=False)
    _lengths("d_r", [d_r], n, exact=False)
    _check("ne_checksum_recover", load().ne_checksum_recover(len(d), n, _ptr_array(d), _ptr(e), r,
                                                             _ptr(d_r), _stream(stream)))


class GroupSpec:
    """One group for a Plan: M int32 input tensors, an int32 operand (or None
    for scale), M output tensors of n_out elements: int64, or int32 with
    word_bits = 32 (the paper's 32-bit entangled words)."""

    def __init__(self, op: str, c: Sequence, operand, out: Sequence, scalar: int = 0,
                 lost: int = -1, in_bits: int = 32, steps: int = 0, ring_waves: int = 0,
                 tap_copies: int = 0, word_bits: int = 0):
        self.op, self.c, self.operand, self.out = op, list(c), operand, list(out)
        self.scalar, self.lost, self.in_bits = int(scalar), int(lost), int(in_bits)
        self.steps, self.ring_waves, self.tap_copies = int(steps), int(ring_waves), int(tap_copies)
        self.word_bits = int(word_bits)

    def to_c(self) -> GroupC:
        import torch
        _dtype(self.c, torch.int32, "c")
        _dtype(self.out, torch.int32 if self.word_bits == 32 else torch.int64, "out")
        if self.operand is not None:
            _dtype([self.operand], torch.int32, "operand")
        if len(self.out) != len(self.c):
            raise ValueError("a group needs one output per input stream")
        if len(self.c) > FUSED_MAX_M:
            raise ValueError(f"a group holds at most {FUSED_MAX_M} streams")
        if any(t is None or isinstance(t, int) for t in self.c + self.out):
            raise ValueError("every input and output of a group must be a tensor")
        _on_device("group inputs, operand and outputs", self.c + self.out + [self.operand])
        n = _n_of(self.c, None, "c") if self.c else 0
        n_operand = 0 if self.operand is None else self.operand.numel()
        _lengths("out", self.out, n_out(self.op, n, n_operand), exact=False)
        g = GroupC()
        g.op = OPS[self.op]
        g.M = len(self.c)
        g.n = n
        g.n_operand = n_operand
        g.scalar = self.scalar
        g.lost = self.lost
        g.in_bits = self.in_bits
        g.steps = self.steps
        g.ring_waves = self.ring_waves
        g.tap_copies = self.tap_copies
        g.word_bits = self.word_bits
        for m, t in enumerate(self.c):
            g.c[m] = _ptr(t)
        for m, t in enumerate(self.out):
            g.out[m] = _ptr(t)
        g.operand = _ptr(self.operand) if self.operand is not None else None
        return g


def workspace_size(groups: Sequence[GroupSpec], mode: str = "entangled", conv_steps: int = 0,
                   stream_steps: int = 0, single_launch: bool = False) -> int:
    arr = (GroupC * max(1, len(groups)))()
    for i, g in enumerate(groups):
        arr[i] = g.to_c()
    tun = TuningC(conv_steps, stream_steps, int(single_launch))
    size = ctypes.c_size_t()
    _check("ne_plan_workspace_size", load().ne_plan_workspace_size(
        arr, len(groups), MODES[mode], ctypes.byref(tun), ctypes.byref(size)))
    return size.value


class Plan:
    """A batched run of many groups (ne_plan_*). With `workspace` (a device
    uint8 tensor of at least workspace_size() bytes) and `stream`, the plan
    allocates nothing and uploads its tables asynchronously on that stream.
    single_launch: the whole run is one persistent launch (ne_tuning)."""

    def __init__(self, groups: Sequence[GroupSpec], mode: str = "entangled", conv_steps: int = 0,
                 stream_steps: int = 0, workspace=None, stream=None, single_launch: bool = False):
        L = load()
        self._groups = list(groups)  # keeps the tensors alive
        self._ws = workspace
        if workspace is not None:
            _on_device("workspace", [workspace])
        arr = (GroupC * max(1, len(self._groups)))()
        for i, g in enumerate(self._groups):
            arr[i] = g.to_c()
        tun = TuningC(conv_steps, stream_steps, int(single_launch))
        h = ctypes.c_void_p()
        if workspace is None:
            _check("ne_plan_create", L.ne_plan_create(arr, len(self._groups), MODES[mode],
                                                      ctypes.byref(tun), ctypes.byref(h)))
        else:
            _check("ne_plan_create_in", L.ne_plan_create_in(
                arr, len(self._groups), MODES[mode], ctypes.byref(tun), _ptr(workspace),
                workspace.numel() * workspace.element_size(), _stream(stream), ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check("ne_plan_run", load().ne_plan_run(self._h, _stream(stream)))

    def capture(self, stream):
        _check("ne_plan_capture", load().ne_plan_capture(self._h, _stream(stream)))

    def launch(self, stream=None):
        _check("ne_plan_launch", load().ne_plan_launch(self._h, _stream(stream)))

    def flags(self, clear: bool = False) -> int:
        f = ctypes.c_uint32()
        _check("ne_plan_flags", load().ne_plan_flags(self._h, ctypes.byref(f), int(clear)))
        return f.value

    def stats(self) -> dict:
        st = StatsC()
        _check("ne_plan_stats_get", load().ne_plan_stats_get(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in StatsC._fields_}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().ne_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ChainOp:
    """One operation of a series: op, its device operand (None for scale;
    for add on entangled streams the entangled int64 vector), the scale
    factor, and the bits of the plain operand's values (conv, add, inner)."""

    def __init__(self, op: str, operand=None, scalar: int = 0, operand_bits: int = 32,
                 n_operand: int | None = None):
        self.op, self.operand, self.scalar, self.operand_bits = op, operand, int(scalar), operand_bits
        if n_operand is None:
            n_operand = 0 if operand is None or isinstance(operand, int) else operand.numel()
        self.n_operand = int(n_operand)

    def to_c(self) -> ChainOpC:
        o = ChainOpC()
        o.op, o.operand_bits = OPS[self.op], int(self.operand_bits)
        o.operand = _ptr(self.operand) if self.operand is not None else None
        o.n_operand, o.scalar = self.n_operand, self.scalar
        return o


def _chain_c(ops: Sequence[ChainOp]):
    return (ChainOpC * max(1, len(ops)))(*[o.to_c() for o in ops])


def chain_check(M: int, in_bits: int, n_in: int, ops: Sequence[ChainOp],
                w: int = 64) -> tuple[int, int]:
    """(output length, worst-case |d| of the last stage) of a series in w-bit
    words (64 or 32); raises NeError (status -2) if some stage's bound
    exceeds D."""
    fn = "ne_chain_check32" if w == 32 else "ne_chain_check"
    no, b = _i64(), _i64()
    _check(fn, getattr(load(), fn)(M, in_bits, n_in, _chain_c(ops), len(ops), ctypes.byref(no),
                                   ctypes.byref(b)))
    return no.value, b.value


def chain_workspace_size(M: int, n_in: int, ops: Sequence[ChainOp], w: int = 64) -> int:
    fn = "ne_chain_workspace_size32" if w == 32 else "ne_chain_workspace_size"
    sz = ctypes.c_size_t()
    _check(fn, getattr(load(), fn)(M, n_in, _chain_c(ops), len(ops), ctypes.byref(sz)))
    return sz.value


def chain_apply(eps: Sequence, ops: Sequence[ChainOp], delta: Sequence, mask: int | None = None,
                workspace=None, n_in: int | None = None, stream=None, w: int = 64):
    """delta[m] = the series applied to eps[m], for every stream whose mask
    bit is set; int64 words, or int32 words with w = 32. workspace: a uint8
    device tensor of chain_workspace_size bytes (allocated here if None)."""
    import torch
    word = torch.int32 if w == 32 else torch.int64
    _dtype(eps, word, "eps")
    _dtype(delta, word, "delta")
    M = len(eps)
    if len(delta) != M:
        raise ValueError("eps and delta differ in length")
    if mask is None:
        mask = (1 << M) - 1
    live = [m for m in range(M) if (mask >> m) & 1]
    dev = _on_device("eps, operands, delta and workspace",
                     list(eps) + list(delta) + [o.operand for o in ops] + [workspace])
    n_in = _n_of([eps[m] for m in live], n_in, "eps")
    n = n_in
    for o in ops:
        n = n_out(o.op, n, o.n_operand)
    _lengths("delta", [delta[m] for m in live], n, exact=False)
    ws_bytes = chain_workspace_size(M, n_in, ops, w)
    if workspace is not None and not isinstance(workspace, int) and workspace.numel() < ws_bytes:
        raise ValueError(f"workspace holds {workspace.numel()} bytes, the series needs {ws_bytes}")
    if workspace is None and ws_bytes:
        workspace = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
        workspace = workspace[(-workspace.data_ptr()) % 256:]
    fn = "ne_chain_apply32" if w == 32 else "ne_chain_apply"
    _check(fn, getattr(load(), fn)(M, n_in, _ptr_array(eps), _chain_c(ops), len(ops),
                                   _ptr_array(delta), n, mask & 0xFFFFFFFF, _ptr(workspace),
                                   ws_bytes, _stream(stream)))


def chain_run_workspace_size(M: int, n_in: int, ops: Sequence[ChainOp], w: int = 64) -> int:
    sz = ctypes.c_size_t()
    fn = "ne_chain_run_workspace_size32" if w == 32 else "ne_chain_run_workspace_size"
    _check(fn, getattr(load(), fn)(M, n_in, _chain_c(ops), len(ops), ctypes.byref(sz)))
    return sz.value


def chain_run(c: Sequence, ops: Sequence[ChainOp], dhat: Sequence, lost: int = -1,
              workspace=None, stream=None, w: int = 64):
    """The whole method on a series: entangle the int32 streams c, run the
    series on every stream but `lost`, recover all outputs into dhat (int64,
    or int32 with w = 32; one per stream); entanglement and recovery fused
    into the first and last runs of element-wise operations where the series
    allows (ne_chain_run, ne_chain_run32). workspace: a uint8 device tensor
    of chain_run_workspace_size bytes (allocated here if None)."""
    import torch
    _dtype(c, torch.int32, "c")
    _dtype(dhat, torch.int32 if w == 32 else torch.int64, "dhat")
    M = len(c)
    if len(dhat) != M:
        raise ValueError("c and dhat differ in length")
    dev = _on_device("c, operands, dhat and workspace",
                     list(c) + list(dhat) + [o.operand for o in ops] + [workspace])
    n_in = _n_of(c, None, "c")
    n = n_in
    for o in ops:
        n = n_out(o.op, n, o.n_operand)
    _lengths("dhat", dhat, n, exact=False)
    ws_bytes = chain_run_workspace_size(M, n_in, ops, w)
    if workspace is not None and workspace.numel() < ws_bytes:
        raise ValueError(f"workspace holds {workspace.numel()} bytes, the series needs {ws_bytes}")
    if workspace is None and ws_bytes:
        workspace = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
        workspace = workspace[(-workspace.data_ptr()) % 256:]
    fn = "ne_chain_run32" if w == 32 else "ne_chain_run"
    _check(fn, getattr(load(), fn)(M, n_in, _ptr_array(c), _chain_c(ops), len(ops), int(lost),
                                   _ptr_array(dhat), n, _ptr(workspace), ws_bytes,
                                   _stream(stream)))


def chain_apply_noalloc(eps: Sequence, ops: Sequence[ChainOp], delta: Sequence,
                        mask: int | None = None, n_in: int | None = None, stream=None):
    """chain_apply in 64-bit words with the intermediates in the library's
    fixed device buffer (CHAIN_SCRATCH_BYTES per device) instead of a
    workspace: nothing is allocated, here or in the library. Calls that
    overlap on one device race on that buffer. Raises NeError (status -7)
    when the series needs more than the buffer holds."""
    import torch
    _dtype(eps, torch.int64, "eps")
    _dtype(delta, torch.int64, "delta")
    M = len(eps)
    if len(delta) != M:
        raise ValueError("eps and delta differ in length")
    if mask is None:
        mask = (1 << M) - 1
    live = [m for m in range(M) if (mask >> m) & 1]
    _on_device("eps, operands and delta", list(eps) + list(delta) + [o.operand for o in ops])
    n_in = _n_of([eps[m] for m in live], n_in, "eps")
    n = n_in
    for o in ops:
        n = n_out(o.op, n, o.n_operand)
    _lengths("delta", [delta[m] for m in live], n, exact=False)
    _check("ne_chain_apply_noalloc",
           load().ne_chain_apply_noalloc(M, n_in, _ptr_array(eps), _chain_c(ops), len(ops),
                                         _ptr_array(delta), n, mask & 0xFFFFFFFF,
                                         _stream(stream)))


def wait_streams(events: Sequence, deadline_us: int) -> int:
    """Fail-stop identification by deadline: waits until every stream's
    completion event (torch.cuda.Event, or None for a stream never launched)
    has completed or deadline_us has passed; returns the index of the one
    late stream, or -1. Raises NeError (status -8) if two or more are late."""
    arr = (ctypes.c_void_p * max(1, len(events)))(
        *[None if e is None else e.cuda_event for e in events])
    lost = _i32()
    _check("ne_wait_streams", load().ne_wait_streams(len(events), arr, int(deadline_us),
                                                     ctypes.byref(lost)))
    return lost.value


def stream_delay(microseconds: int, stream=None):
    """Enqueues a bounded wait (a slow core) on `stream`."""
    _check("ne_stream_delay", load().ne_stream_delay(int(microseconds), _stream(stream)))


def stream_widen(src, dst, stream=None):
    """dst[i] = src[i] widened to int64: the HBM ceiling reference (4 bytes
    read, 8 written per element, the fused convolution's mix)."""
    import torch
    _dtype([src], torch.int32, "src")
    _dtype([dst], torch.int64, "dst")
    _on_device("src and dst", [src, dst])
    n = src.numel()
    _lengths("dst", [dst], n, exact=False)
    _check("ne_stream_widen", load().ne_stream_widen(_ptr(src), n, _ptr(dst), _stream(stream)))


def mfma_i8_peak(sink, blocks: int, iters: int, varied: bool = False, stream=None) -> float:
    """Launches the i8 matrix-core rate reference (blocks x 4 waves, iters x 8
    independent products each; varied: pseudo-random operands changing every
    product) on `stream`; returns the integer operations launched. sink: an
    int32 device tensor of at least 4 * blocks values."""
    import torch
    _dtype([sink], torch.int32, "sink")
    _on_device("sink", [sink])
    _lengths("sink", [sink], 4 * blocks, exact=False)
    ops = ctypes.c_double()
    _check("ne_mfma_i8_peak", load().ne_mfma_i8_peak(blocks, iters, int(bool(varied)), _ptr(sink),
                                                     ctypes.byref(ops), _stream(stream)))
    return ops.value


def gemm_workspace_size(mode: str, M: int, N: int, P: int, Q: int, in_bits: int) -> int:
    sz = ctypes.c_size_t()
    _check("ne_gemm_workspace_size", load().ne_gemm_workspace_size(MODES[mode], M, N, P, Q, in_bits,
                                                                   ctypes.byref(sz)))
    return sz.value


def gemm(c: Sequence, g, out: Sequence, mode: str = "entangled", lost: int = -1,
         in_bits: int = 16, flags=None, stream=None, workspace=None):
    """out[m] = c[m] @ g for M int32 blocks c[m] (N x P) and an int32 kernel
    matrix g (P x Q), int64 outputs (N x Q), by the method of `mode`.
    workspace: None (one fused launch) or a 256-byte aligned uint8 device
    tensor of gemm_workspace_size bytes (two-phase form)."""
    import torch
    _dtype(c, torch.int32, "c")
    _dtype([g], torch.int32, "g")
    _dtype(out, torch.int64, "out")
    if g.dim() != 2:
        raise ValueError("g must be a matrix")
    if len(out) != len(c):
        raise ValueError("one output per block")
    _on_device("blocks, kernel matrix, outputs, flags and workspace",
               list(c) + [g] + list(out) + [flags, workspace])
    P, Q = g.shape
    N = out[0].shape[0] if out[0].dim() == 2 else 0
    for t in c:
        if t.dim() != 2 or t.shape[1] != P or t.shape[0] != N:
            raise ValueError("every block must be N x P")
    for t in out:
        if t.dim() != 2 or tuple(t.shape) != (N, Q):
            raise ValueError("every output must be N x Q")
    ws_bytes = 0 if workspace is None else workspace.numel()
    _check("ne_gemm", load().ne_gemm(MODES[mode], len(c), N, P, Q, _ptr_array(c), _ptr(g),
                                     _ptr_array(out), lost, in_bits, _ptr(workspace), ws_bytes,
                                     _ptr(flags), _stream(stream)))
