"""The C-ABI library loads, exports every symbol include/ne.h declares, and
its host-only logic (parameters, argument validation) is right. No kernel is
launched here: every call below returns before enqueueing work."""
import ctypes
import os
import re

import pytest

import oracle
from paper_1509_03838_amd import ne

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(ne_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return ne.load()


def test_header_declares_the_binding_exports():
    assert set(declared_symbols()) == set(ne.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_version_and_strerror(lib):
    assert lib.ne_version() >= 100
    assert lib.ne_strerror(0) == b"ok"
    assert b"index" in lib.ne_strerror(-3)


@pytest.mark.parametrize("w", [8, 10, 12, 16, 24, 32, 48, 63, 64])
def test_params_match_oracle(w):
    for M in range(3, 33):
        try:
            l, k, D = oracle.params(M, w)
        except oracle.OracleError:  # no (l, k) at all: M - 1 > w
            l, k, D = 0, 0, 0
        if D < 1:
            with pytest.raises(ne.NeError):
                ne.params(M, w)
            continue
        assert ne.params(M, w) == (l, k, D), (M, w)


def test_params_rejects(lib):
    out = ctypes.c_int32()
    assert lib.ne_params(2, 64, ctypes.byref(out), None, None) == -1
    assert lib.ne_params(33, 64, ctypes.byref(out), None, None) == -1
    assert lib.ne_params(3, 65, ctypes.byref(out), None, None) == -1
    assert lib.ne_params(3, 64, None, None, None) == -1


def _ptrs(vals):
    a = (ctypes.c_void_p * len(vals))()
    for i, v in enumerate(vals):
        a[i] = v
    return a


FAKE = 0x100000  # never dereferenced: every call below fails validation first


def test_validation_before_launch(lib):
    p3 = _ptrs([FAKE, FAKE + 64, FAKE + 128])
    # M < 3 for entanglement
    assert lib.ne_entangle(2, 22, 10, p3, p3, None) == -1
    # l out of range
    assert lib.ne_entangle(3, 0, 10, p3, p3, None) == -1
    # NULL stream entry
    assert lib.ne_entangle(3, 22, 10, _ptrs([FAKE, 0, FAKE]), p3, None) == -1
    # failed index out of range
    assert lib.ne_extract_recover(3, 22, 10, p3, 3, p3, None) == -3
    assert lib.ne_extract_recover(3, 22, 10, p3, -2, p3, None) == -3
    # (M-1) l > 64
    assert lib.ne_extract_recover(3, 33, 10, p3, 0, p3, None) == -1
    # NULL among the M-1 streams that recovery reads
    assert lib.ne_extract_recover(3, 22, 10, _ptrs([FAKE, 0, FAKE]), 0, p3, None) == -1
    # conv: n_out must be n + K - 1
    assert lib.ne_lsb_apply(0, 3, 10, p3, FAKE, 4, 0, p3, 12, 7, None) == -1
    # inner: n_out must be 1
    assert lib.ne_lsb_apply(3, 3, 10, p3, FAKE, 10, 0, p3, 10, 7, None) == -1
    # unknown op
    assert lib.ne_lsb_apply(10, 3, 10, p3, FAKE, 10, 0, p3, 10, 7, None) == -4
    # a NULL output for a stream that is computed
    assert lib.ne_lsb_apply(1, 3, 10, p3, 0, 0, 2, _ptrs([FAKE, 0, FAKE]), 10, 7, None) == -1
    # checksum recovery: bad index
    assert lib.ne_checksum_recover(3, 10, p3, FAKE, 3, FAKE, None) == -3


def test_empty_inputs_enqueue_nothing(lib):
    p3 = _ptrs([FAKE, FAKE + 64, FAKE + 128])
    assert lib.ne_entangle(3, 22, 0, p3, p3, None) == 0
    assert lib.ne_extract_recover(3, 22, 0, p3, 1, p3, None) == 0
    assert lib.ne_lsb_apply(0, 3, 0, p3, FAKE, 16, 0, p3, 0, 7, None) == 0
    # every stream masked off (all lost): nothing to compute
    assert lib.ne_lsb_apply(1, 3, 10, p3, 0, 0, 2, p3, 10, 0, None) == 0


def test_word32_validation_before_launch(lib):
    """The 32-bit word calls check their own limits: M up to 17 (the largest
    group with an admissible l at w = 32), l up to 31, (M - 1) l <= 32."""
    p3 = _ptrs([FAKE, FAKE + 64, FAKE + 128])
    p18 = _ptrs([FAKE + 64 * i for i in range(18)])
    assert ne.MAX_M32 == 17 and ne.params(17, 32)[0] == 2
    with pytest.raises(ne.NeError):
        ne.params(18, 32)
    assert lib.ne_entangle32(2, 11, 10, p3, p3, None) == -1
    assert lib.ne_entangle32(18, 2, 10, p18, p18, None) == -1
    assert lib.ne_entangle32(3, 32, 10, p3, p3, None) == -1
    assert lib.ne_entangle32(3, 11, 10, _ptrs([FAKE, 0, FAKE]), p3, None) == -1
    assert lib.ne_entangle_operand32(0, 10, FAKE, FAKE, None) == -1
    assert lib.ne_entangle_operand32(11, 10, 0, FAKE, None) == -1
    assert lib.ne_extract_recover32(3, 11, 10, p3, 3, p3, None) == -3
    assert lib.ne_extract_recover32(3, 11, 10, p3, -2, p3, None) == -3
    assert lib.ne_extract_recover32(3, 17, 10, p3, 0, p3, None) == -1   # (M-1) l = 34 > 32
    assert lib.ne_extract_recover32(18, 2, 10, p18, 0, p18, None) == -1
    assert lib.ne_extract_recover32(3, 11, 10, _ptrs([FAKE, 0, FAKE]), 0, p3, None) == -1
    assert lib.ne_lsb_apply32(0, 3, 10, p3, FAKE, 4, 0, p3, 12, 7, None) == -1
    assert lib.ne_lsb_apply32(3, 3, 10, p3, FAKE, 10, 0, p3, 10, 7, None) == -1
    assert lib.ne_lsb_apply32(10, 3, 10, p3, FAKE, 10, 0, p3, 10, 7, None) == -4
    assert lib.ne_lsb_apply32(1, 3, 10, p3, 0, 0, 2, _ptrs([FAKE, 0, FAKE]), 10, 7, None) == -1
    # zero lengths and all-lost masks enqueue nothing
    assert lib.ne_entangle32(3, 11, 0, p3, p3, None) == 0
    assert lib.ne_extract_recover32(3, 11, 0, p3, 1, p3, None) == 0
    assert lib.ne_lsb_apply32(1, 3, 10, p3, 0, 0, 2, p3, 10, 0, None) == 0
    assert lib.ne_lsb_apply32(0, 3, 0, p3, FAKE, 16, 0, p3, 0, 7, None) == 0


def _group(**kw):
    g = ne.GroupC()
    g.op, g.M, g.n, g.n_operand, g.scalar, g.lost, g.in_bits = 0, 3, 100, 16, 0, -1, 12
    for m in range(3):
        g.c[m] = FAKE + 256 * m
        g.out[m] = FAKE + 4096 + 1024 * m
    g.operand = FAKE + 8192
    for k, v in kw.items():
        setattr(g, k, v)
    return g


@pytest.mark.parametrize("kw,status", [
    ({"M": 2}, -1),                      # entangled needs M >= 3
    ({"M": 9}, -1),                      # above the fused limit
    ({"lost": 3}, -3),                   # failed index out of range
    ({"op": 9, "n_operand": -1}, -1),    # the outer product needs K >= 0
    ({"op": 10}, -4),                    # unknown operation
    ({"n_operand": 0}, -1),              # convolution without taps
    ({"in_bits": 32}, -1),               # 32-bit convolution operands
    ({"in_bits": 31, "n_operand": 1 << 20}, -2),  # worst case above D
])
def test_plan_validation_before_allocation(lib, kw, status):
    arr = (ne.GroupC * 1)(_group(**kw))
    h = ctypes.c_void_p()
    assert lib.ne_plan_create(arr, 1, 0, None, ctypes.byref(h)) == status
    assert not h.value


def test_plan_rejects_misaligned_inputs(lib):
    g = _group()
    g.c[1] = FAKE + 4  # int32 streams must be 16-byte aligned
    h = ctypes.c_void_p()
    assert lib.ne_plan_create((ne.GroupC * 1)(g), 1, 0, None, ctypes.byref(h)) == -1


@pytest.mark.parametrize("word_bits", [0, 32])
@pytest.mark.parametrize("mode,m_lo", [(0, 3), (1, 1), (2, 1), (3, 2), (4, 2)])
def test_every_planned_convolution_has_a_kernel_variant(lib, mode, m_lo, word_bits):
    """The planner picks the digit counts of a convolution group from its
    declared input bits (and, for entangled and plain-same groups, the word
    width's shift l); a kernel variant must exist for every choice it can
    make (sizing only: ne_plan_workspace_size touches no device)."""
    accepted = 0
    for M in range(m_lo, 9):
        for bits in range(1, 32):
            g = _group(M=M, in_bits=bits, n_operand=1, word_bits=word_bits)
            for m in range(M):
                g.c[m] = FAKE + 256 * m
                g.out[m] = FAKE + 4096 + 1024 * m
            size = ctypes.c_size_t()
            st = lib.ne_plan_workspace_size((ne.GroupC * 1)(g), 1, mode, None, ctypes.byref(size))
            assert st in (0, -2), (mode, M, bits, st)  # OK, or the range check (never EUNSUP)
            accepted += st == 0
    assert accepted > 0


def _ws(lib, groups, mode=0):
    size = ctypes.c_size_t()
    st = lib.ne_plan_workspace_size((ne.GroupC * len(groups))(*groups), len(groups), mode, None,
                                    ctypes.byref(size))
    return st, size.value


def test_workspace_holds_permutation_rows(lib):
    """A permutation group adds n rows of 16 bytes (<= 4 slots) or 32 bytes
    (more slots) to the plan's workspace; other operations add none."""
    n = 10_000
    st0, base = _ws(lib, [_group(op=1, n=n, n_operand=0, scalar=3)])  # scale
    st1, perm3 = _ws(lib, [_group(op=4, n=n, n_operand=n)])
    g6 = _group(op=4, M=6, n=n, n_operand=n)
    for m in range(6):
        g6.c[m] = FAKE + 256 * m
        g6.out[m] = FAKE + 4096 + 1024 * m
    st2, perm6 = _ws(lib, [g6])
    assert st0 == st1 == st2 == 0
    up = lambda x: (x + 255) // 256 * 256
    assert perm3 - base >= up(16 * n) and perm3 - base < up(16 * n) + 4096
    assert perm6 - base >= up(32 * n) and perm6 - base < up(32 * n) + 4096


@pytest.mark.parametrize("rw,status", [(0, 0), (1, 0), (4, 0), (2, -1), (-1, -1)])
def test_ring_waves_values(lib, rw, status):
    g = _group(ring_waves=rw)
    assert _ws(lib, [g])[0] == status


@pytest.mark.parametrize("rw,tc,status", [(0, 0, 0), (0, 1, 0), (0, 4, 0), (4, 1, 0), (4, 4, 0),
                                          (1, 4, 0), (1, 1, -1), (0, 2, -1), (0, -1, -1)])
def test_tap_copies_values(lib, rw, tc, status):
    """One tap copy exists only with a block ring."""
    g = _group(ring_waves=rw, tap_copies=tc)
    assert _ws(lib, [g])[0] == status


def test_outer_product_plans(lib):
    """The batched executor plans the outer product over its n K outputs:
    the worst case 2^(b-1) 2^(b-1), no taps needed (K = 0 plans nothing),
    and an n K beyond the work-item table is refused."""
    assert _ws(lib, [_group(op=9, n_operand=8)])[0] == 0
    assert _ws(lib, [_group(op=9, n_operand=0, operand=0)])[0] == 0
    assert _ws(lib, [_group(op=9, n_operand=8, in_bits=32)], 1)[0] == 0      # plain: 2^62
    assert _ws(lib, [_group(op=9, n_operand=8, in_bits=22)])[0] == -2        # 2^42 > D(3)
    assert _ws(lib, [_group(op=9, n=1 << 40, n_operand=1 << 10, in_bits=4)])[0] == -4


@pytest.mark.parametrize("wb,status", [(0, 0), (64, 0), (32, 0), (1, -1), (16, -1), (128, -1)])
def test_word_bits_values(lib, wb, status):
    assert _ws(lib, [_group(word_bits=wb, in_bits=6)])[0] == status


def test_word32_groups_check_the_narrower_range(lib):
    """At w = 32 an entangled group's worst case must stay within
    D = 1,046,528 (M = 3), a plain one within 2^31 - 1; the 64-bit width
    accepts both. Output bytes per sample halve."""
    def ws(mode, wb, bits, K, op=0):
        g = _group(word_bits=wb, in_bits=bits, n_operand=K, op=op)
        return _ws(lib, [g], mode)[0]
    assert ws(0, 32, 7, 64) == 0          # 64 * 2^12 = 2^18
    assert ws(0, 32, 10, 3) == 0          # 3 * 2^18 = 786,432
    assert ws(0, 32, 10, 4) == -2         # 4 * 2^18 = 1,048,576 > D
    assert ws(0, 32, 11, 1) == -2         # 2^20 > D
    assert ws(0, 64, 11, 1) == 0
    assert ws(1, 32, 16, 1) == 0 and ws(1, 32, 16, 2) == -2   # 2^30, 2^31
    assert ws(3, 32, 12, 256) == -2       # checksum stream: 3 * 256 * 2^22 > 2^31 - 1
    assert ws(3, 32, 12, 128) == 0        # 3 * 128 * 2^22 = 3 * 2^29


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("M", [3, 8])
def test_paper_experiment_shapes_plan(lib, mode, M):
    """The paper's experiment (Sec. V) convolves M in {3, 8} streams of 10^6
    samples with up to 4500 taps: every mode plans at 15-bit inputs (the
    widest whose worst case fits D for M = 3 at K = 4500); far longer
    kernels are refused as unsupported (their windows exceed LDS), not
    mis-planned."""
    def grp(K):
        g = _group(M=M, in_bits=15, n=10**6, n_operand=K)
        for m in range(M):
            g.c[m] = FAKE + 256 * m
            g.out[m] = FAKE + 4096 + 1024 * m
        return g
    for K in (100, 1000, 4500):
        assert _ws(lib, [grp(K)], mode)[0] == 0, K
    assert _ws(lib, [grp(16000)], mode)[0] in (-2, -4)


# ------------------------------------------------ series of operations (host)

def _series(*ops):
    """ChainOp list from (op, n_operand, scalar, operand_bits) tuples, with
    fake operand addresses (sizing and range checks read no operand)."""
    return [ne.ChainOp(op, FAKE + 4096 * i, scalar, bits, n_operand=nop)
            for i, (op, nop, scalar, bits) in enumerate(ops)]


def test_series_lengths_and_bound():
    """Lengths follow each operation (conv grows by K - 1, inner makes 1);
    the bound composes stage by stage: 2^9 inputs, + 2^9 (add), x 37
    (scale), x 64 taps x 2^9 (conv), unchanged (perm), then x n x 2^3 for
    an inner product with 4-bit values."""
    n = 100
    ops = _series(("add", n, 0, 10), ("scale", 0, -37, 0), ("conv", 64, 0, 10),
                  ("perm", n + 63, 0, 0))
    no, b = ne.chain_check(3, 10, n, ops)
    assert no == n + 63
    assert b == (2**9 + 2**9) * 37 * 64 * 2**9
    ops2 = ops + _series(("inner", n + 63, 0, 4))
    no2, b2 = ne.chain_check(3, 10, n, ops2)
    assert no2 == 1 and b2 == b * (n + 63) * 2**3


def test_series_bound_against_d():
    """Every stage must stay within D(M): M = 3 (D = 2^41 - 2^22) accepts a
    bound of 2^40 and refuses 2^42, even when a later scale by 1 would not
    change it; M = 8 (D above 2^55) accepts the latter."""
    ok = _series(("conv", 4, 0, 16), ("scale", 0, 1 << 8, 0))     # 2^15 * 2^15 * 4 * 2^8
    bad = _series(("conv", 16, 0, 16), ("scale", 0, 1 << 8, 0))   # 2^15 * 2^15 * 16 * 2^8
    assert ne.chain_check(3, 16, 100, ok)[1] == 1 << 40
    with pytest.raises(ne.NeError) as e:
        ne.chain_check(3, 16, 100, bad)
    assert e.value.status == -2
    assert ne.chain_check(8, 16, 100, bad)[1] == 1 << 42


@pytest.mark.parametrize("ops,status", [
    ([("add", 99, 0, 10)], -1),                  # operand length differs
    ([("conv", 0, 0, 10)], -1),                  # no taps
    ([("conv", 5, 0, 0)], -1),                   # operand bits missing
    ([("conv", 5, 0, 33)], -1),                  # operand bits above 32
    ([("perm", 100, 0, 0), ("inner", 100, 0, 8), ("add", 100, 0, 8)], -1),  # length 1 after inner
    ([(10, 0, 0, 0)], -4),                       # unknown operation
])
def test_series_validation(ops, status):
    L = ne.load()
    arr = (ne.ChainOpC * len(ops))()
    for i, (op, nop, sc, bits) in enumerate(ops):
        arr[i].op = ne.OPS[op] if isinstance(op, str) else op
        arr[i].n_operand, arr[i].scalar, arr[i].operand_bits = nop, sc, bits
        arr[i].operand = FAKE
    no, b = ctypes.c_int64(), ctypes.c_int64()
    assert L.ne_chain_check(3, 10, 100, arr, len(ops), ctypes.byref(no), ctypes.byref(b)) == status


def test_series_argument_checks():
    L = ne.load()
    ops = ne._chain_c(_series(("scale", 0, 3, 0)))
    no = ctypes.c_int64()
    assert L.ne_chain_check(2, 10, 100, ops, 1, ctypes.byref(no), None) == -1   # M < 3
    assert L.ne_chain_check(3, 0, 100, ops, 1, ctypes.byref(no), None) == -1   # in_bits
    assert L.ne_chain_check(3, 10, -1, ops, 1, ctypes.byref(no), None) == -1   # n_in
    assert L.ne_chain_check(3, 10, 100, ops, 0, ctypes.byref(no), None) == -1  # no ops
    assert L.ne_chain_check(3, 10, 100, ops, 65, ctypes.byref(no), None) == -1  # too many
    assert L.ne_chain_check(3, 10, 100, None, 1, ctypes.byref(no), None) == -1


def test_series_run_workspace_and_checks():
    """ne_chain_run: nothing for a series that is one run of element-wise
    operations (one pass); the entangled inputs too when the series starts
    with another operation; the intermediates otherwise. Bad arguments are
    refused before the device is touched."""
    n = 1000
    up = lambda x: (x + 255) // 256 * 256
    run = _series(("perm", n, 0, 0), ("add", n, 0, 8), ("scale", 0, 3, 0))  # one run
    assert ne.chain_run_workspace_size(3, n, run) == 0
    two = _series(("add", n, 0, 8), ("scale", 0, 3, 0), ("perm", n, 0, 0))  # a permutation leads
    assert ne.chain_run_workspace_size(3, n, two) == 2 * 3 * up(8 * n)
    conv = _series(("conv", 64, 0, 10))
    assert ne.chain_run_workspace_size(3, n, conv) == 2 * 3 * up(8 * n)
    mixed = _series(("add", n, 0, 8), ("scale", 0, 3, 0), ("conv", 64, 0, 10),
                    ("perm", n + 63, 0, 0), ("add", n + 63, 0, 8))
    assert ne.chain_run_workspace_size(5, n, mixed) == 2 * 5 * up(8 * (n + 63))
    lead = _series(("conv", 64, 0, 10), ("perm", n + 63, 0, 0))
    assert ne.chain_run_workspace_size(4, n, lead) == 2 * 4 * up(8 * (n + 63))
    L = ne.load()
    c = ne._ptr_array([FAKE + 64 * m for m in range(3)])
    out = ne._ptr_array([FAKE + (1 << 20) + 64 * m for m in range(3)])
    arr = ne._chain_c(conv)
    ws = ne.chain_run_workspace_size(3, n, conv)
    assert L.ne_chain_run(3, n, c, arr, 1, -1, out, n + 63, None, 0, None) == -1     # no workspace
    assert L.ne_chain_run(3, n, c, arr, 1, -1, out, n + 63, FAKE, ws - 1, None) == -1
    assert L.ne_chain_run(3, n, c, arr, 1, -1, out, n + 62, FAKE, ws, None) == -1    # wrong n_out
    assert L.ne_chain_run(3, n, c, arr, 1, 3, out, n + 63, FAKE, ws, None) == -3     # lost index
    assert L.ne_chain_run(2, n, c, arr, 1, -1, out, n + 63, FAKE, ws, None) == -1    # M < 3
    assert L.ne_chain_run(3, n, c, arr, 1, -1, out, n + 63, FAKE + 8, ws, None) == -1


def test_series_run32_workspace_and_checks():
    """ne_chain_run32: the same passes in int32 words (planes of 4-byte
    words), groups of up to NE_MAX_M32 = 17 streams; bad arguments refused
    before the device is touched."""
    n = 1000
    up = lambda x: (x + 255) // 256 * 256
    run = _series(("perm", n, 0, 0), ("add", n, 0, 4), ("scale", 0, 3, 0))
    assert ne.chain_run_workspace_size(3, n, run, w=32) == 0
    mixed = _series(("add", n, 0, 4), ("scale", 0, 3, 0), ("conv", 16, 0, 4),
                    ("perm", n + 15, 0, 0), ("add", n + 15, 0, 4))
    assert ne.chain_run_workspace_size(5, n, mixed, w=32) == 2 * 5 * up(4 * (n + 15))
    assert ne.chain_run_workspace_size(17, n, mixed, w=32) == 2 * 17 * up(4 * (n + 15))
    with pytest.raises(ne.NeError) as e:
        ne.chain_run_workspace_size(18, n, mixed, w=32)
    assert e.value.status == -1
    L = ne.load()
    c = ne._ptr_array([FAKE + 64 * m for m in range(3)])
    out = ne._ptr_array([FAKE + (1 << 20) + 64 * m for m in range(3)])
    conv = _series(("conv", 16, 0, 4))
    arr = ne._chain_c(conv)
    ws = ne.chain_run_workspace_size(3, n, conv, w=32)
    assert ws == 2 * 3 * up(4 * (n + 15))
    assert L.ne_chain_run32(3, n, c, arr, 1, -1, out, n + 15, None, 0, None) == -1    # no workspace
    assert L.ne_chain_run32(3, n, c, arr, 1, -1, out, n + 14, FAKE, ws, None) == -1   # wrong n_out
    assert L.ne_chain_run32(3, n, c, arr, 1, 3, out, n + 15, FAKE, ws, None) == -3    # lost index
    assert L.ne_chain_run32(18, n, c, arr, 1, -1, out, n + 15, FAKE, ws, None) == -1  # M > 17


def test_series_workspace_size():
    """Two buffers of M streams of the longest intermediate (256-byte
    rounded); nothing for a single operation. ne_chain_apply refuses a
    missing or short workspace before touching the device."""
    n = 1000
    one = _series(("conv", 64, 0, 10))
    assert ne.chain_workspace_size(3, n, one) == 0
    ops = _series(("conv", 64, 0, 10), ("scale", 0, 3, 0), ("inner", n + 63, 0, 8))
    up = lambda x: (x + 255) // 256 * 256
    assert ne.chain_workspace_size(5, n, ops) == 2 * 5 * up(8 * (n + 63))
    L = ne.load()
    eps = ne._ptr_array([FAKE + 64 * m for m in range(3)])
    out = ne._ptr_array([FAKE + (1 << 20) + 64 * m for m in range(3)])
    arr = ne._chain_c(ops)
    assert L.ne_chain_apply(3, n, eps, arr, 3, out, 1, 7, None, 0, None) == -1
    ws = ne.chain_workspace_size(3, n, ops)
    assert L.ne_chain_apply(3, n, eps, arr, 3, out, 1, 7, FAKE, ws - 1, None) == -1
    assert L.ne_chain_apply(3, n, eps, arr, 3, out, 2, 7, FAKE, ws, None) == -1   # wrong n_out
    assert L.ne_chain_apply(3, n, eps, arr, 3, out, 1, 7, FAKE + 8, ws, None) == -1  # misaligned


def test_series_in_32_bit_words():
    """The 32-bit series bounds every stage by D of w = 32 (1,046,528 for
    M = 3; 2^28 for M = 17, the largest group w = 32 admits), counts int32
    intermediates, and refuses a short workspace before touching the device."""
    n = 1000
    ok = _series(("conv", 16, 0, 8), ("scale", 0, 3, 0))        # 16 * 2^14 * 3 < D
    bad = _series(("conv", 16, 0, 8), ("scale", 0, 5, 0))       # 16 * 2^14 * 5 > D
    assert ne.chain_check(3, 8, n, ok, w=32) == (n + 15, 16 * 2**14 * 3)
    with pytest.raises(ne.NeError) as e:
        ne.chain_check(3, 8, n, bad, w=32)
    assert e.value.status == -2
    assert ne.chain_check(3, 8, n, bad)[1] == 16 * 2**14 * 5      # fits 64-bit words
    assert ne.chain_check(17, 8, n, bad, w=32)[1] == 16 * 2**14 * 5
    with pytest.raises(ne.NeError) as e:
        ne.chain_check(18, 8, n, ok, w=32)
    assert e.value.status == -1
    up = lambda x: (x + 255) // 256 * 256
    assert ne.chain_workspace_size(5, n, ok, w=32) == 2 * 5 * up(4 * (n + 15))
    assert ne.chain_workspace_size(5, n, ok) == 2 * 5 * up(8 * (n + 15))
    L = ne.load()
    eps = ne._ptr_array([FAKE + 64 * m for m in range(3)])
    out = ne._ptr_array([FAKE + (1 << 20) + 64 * m for m in range(3)])
    arr = ne._chain_c(ok)
    ws = ne.chain_workspace_size(3, n, ok, w=32)
    assert L.ne_chain_apply32(3, n, eps, arr, 2, out, n + 15, 7, FAKE, ws - 1, None) == -1
    assert L.ne_chain_apply32(3, n, eps, arr, 2, out, n + 14, 7, FAKE, ws, None) == -1


def test_series_bound_saturates():
    """An absurd operand length cannot wrap the 128-bit bound below D:
    2^40 (after scaling 2^31 by 2^9) times 2^31 times 2^62 taps is 2^133,
    which modulo 2^128 would be 32."""
    ops = _series(("scale", 0, 1 << 9, 0), ("conv", 1 << 62, 0, 32))
    with pytest.raises(ne.NeError) as e:
        ne.chain_check(3, 32, 1, ops)
    assert e.value.status == -2


def test_series_of_empty_streams_needs_no_workspace(lib):
    """Streams of length 0: every stage is empty, the workspace size is 0,
    NULL stream and workspace pointers are accepted and nothing is
    launched."""
    ops = _series(("conv", 5, 0, 8), ("scale", 0, 3, 0))
    assert ne.chain_workspace_size(3, 0, ops) == 0
    nulls = ne._ptr_array([None, None, None])
    assert lib.ne_chain_apply(3, 0, nulls, ne._chain_c(ops), 2, nulls, 0, 7, None, 0, None) == 0


# ---------------------------------------------------- matrix product (host)

@pytest.mark.parametrize("args,status", [
    (dict(mode=4), -1),                      # unknown mode
    (dict(M=2), -1),                         # the method needs M >= 3
    (dict(M=9), -1),                         # above the fused limit
    (dict(N=-1), -1),
    (dict(lost=3), -3),                      # lost block out of range
    (dict(in_bits=0), -1),
    (dict(in_bits=17), -4),                  # beyond the supported values
    (dict(P=1 << 20, in_bits=16), -2),       # worst case above D
    (dict(Q=(1 << 26) + 1), -4),
    (dict(N=0), 0),                          # no outputs: nothing to do
    (dict(Q=0), 0),
])
def test_gemm_validation(lib, args, status):
    a = dict(mode=0, M=3, N=8, P=8, Q=8, lost=-1, in_bits=12)
    a.update(args)
    c = ne._ptr_array([FAKE + 4096 * m for m in range(8)])
    out = ne._ptr_array([FAKE + (1 << 20) + 4096 * m for m in range(8)])
    assert lib.ne_gemm(a["mode"], a["M"], a["N"], a["P"], a["Q"], c, FAKE, out, a["lost"],
                       a["in_bits"], None, 0, None, None) == status


def test_gemm_null_blocks_refused(lib):
    c = ne._ptr_array([FAKE, 0, FAKE])
    out = ne._ptr_array([FAKE, FAKE, FAKE])
    assert lib.ne_gemm(0, 3, 8, 8, 8, c, FAKE, out, -1, 12, None, 0, None, None) == -1
    assert lib.ne_gemm(0, 3, 8, 8, 8, out, 0, out, -1, 12, None, 0, None, None) == -1


def test_gemm_workspace_size_and_checks(lib):
    """Digit planes of every slot (rows padded to 32, the inner dimension to
    64) and of G (columns padded to 64); a short or misaligned workspace is
    refused before anything is launched."""
    # entangled M = 3, 12-bit values: each word split at bit l = 22 into two
    # fields of 2 digits (4 planes instead of 5 for the whole word), 2 digits
    # per kernel value
    size = ne.gemm_workspace_size("entangled", 3, 100, 70, 90, 12)
    up = lambda x, m: (x + m - 1) // m * m
    assert size == up(3 * 4 * 128 * 128, 256) + 2 * 128 * 128
    # plain: 12-bit values need 2 digits, no split
    assert ne.gemm_workspace_size("plain", 3, 100, 70, 90, 12) == up(3 * 2 * 128 * 128, 256) + 2 * 128 * 128
    assert ne.gemm_workspace_size("entangled", 3, 0, 70, 90, 12) == 0
    c = ne._ptr_array([FAKE + 4096 * m for m in range(3)])
    out = ne._ptr_array([FAKE + (1 << 20) + 4096 * m for m in range(3)])
    assert lib.ne_gemm(0, 3, 100, 70, 90, c, FAKE, out, -1, 12, FAKE, size - 1, None, None) == -1
    assert lib.ne_gemm(0, 3, 100, 70, 90, c, FAKE, out, -1, 12, FAKE + 16, size, None, None) == -1


def test_chain_noalloc_refuses_series_past_its_buffer(lib):
    """ne_chain_apply_noalloc checks the series against its fixed buffer
    before anything touches the device: the pointers here are never read."""
    import ctypes
    M = 3
    n = ne.CHAIN_SCRATCH_BYTES // (2 * M) // 8 + 1
    ops = [ne.ChainOp("scale", None, 3), ne.ChainOp("scale", None, 5)]
    assert ne.chain_workspace_size(M, n, ops) > ne.CHAIN_SCRATCH_BYTES
    assert ne.chain_workspace_size(M, n - 64, ops) <= ne.CHAIN_SCRATCH_BYTES
    fake = (ctypes.c_void_p * M)(*([0x1000] * M))
    st = lib.ne_chain_apply_noalloc(M, n, fake, ne._chain_c(ops), len(ops), fake, n, 7, None)
    assert st == -7 and b"scratch" in lib.ne_strerror(st)
    # argument errors come first as well (a wrong n_out)
    st = lib.ne_chain_apply_noalloc(M, 100, fake, ne._chain_c(ops), len(ops), fake, 99, 7, None)
    assert st == -1


def test_stream_widen_argument_checks(lib):
    """Misaligned, overlapping or missing buffers are refused before any
    launch (the addresses are never dereferenced)."""
    assert lib.ne_stream_widen(FAKE, -1, FAKE + 4096, None) == -1
    assert lib.ne_stream_widen(None, 0, None, None) == 0        # nothing to copy
    assert lib.ne_stream_widen(None, 16, FAKE, None) == -1
    assert lib.ne_stream_widen(FAKE + 4, 16, FAKE + 4096, None) == -1   # misaligned input
    assert lib.ne_stream_widen(FAKE, 16, FAKE + 8, None) == -1          # misaligned output
    assert lib.ne_stream_widen(FAKE, 16, FAKE + 32, None) == -1         # overlapping


def test_wait_streams_and_delay_argument_checks(lib):
    """Refused before any device or event access."""
    import ctypes
    lost = ctypes.c_int32(7)
    ev = (ctypes.c_void_p * 3)(None, None, None)
    assert lib.ne_wait_streams(0, ev, 10, ctypes.byref(lost)) == -1
    assert lib.ne_wait_streams(3, None, 10, ctypes.byref(lost)) == -1
    assert lib.ne_wait_streams(3, ev, -1, ctypes.byref(lost)) == -1
    assert lib.ne_wait_streams(3, ev, 10, None) == -1
    # no stream launched at all: every one is late
    assert lib.ne_wait_streams(3, ev, 0, ctypes.byref(lost)) == -8 and lost.value == -1
    one = (ctypes.c_void_p * 1)(None)
    assert lib.ne_wait_streams(1, one, 0, ctypes.byref(lost)) == 0 and lost.value == 0
    assert lib.ne_stream_delay(-1, None) == -1
    assert lib.ne_stream_delay(1_000_001, None) == -1
    assert lib.ne_stream_delay(0, None) == 0      # nothing enqueued
    assert b"deadline" in lib.ne_strerror(-8)


def _gm(**kw):
    """_group with a stream and an output pointer for each of M streams."""
    g = _group(**kw)
    for m in range(g.M):
        g.c[m] = FAKE + 256 * m
        g.out[m] = FAKE + 4096 + 1024 * m
    return g


def _ws_single(lib, groups, mode=0, single=1):
    size = ctypes.c_size_t()
    tun = ne.TuningC(0, 0, single)
    st = lib.ne_plan_workspace_size((ne.GroupC * len(groups))(*groups), len(groups), mode,
                                    ctypes.byref(tun), ctypes.byref(size))
    return st, size.value


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4])
def test_single_launch_menu(lib, mode):
    """The single launch takes convolutions of 9..12-bit samples and scale,
    add, inner and perm groups of 3..8 data streams in every mode; 16-bit
    convolutions, other operations, the one-copy tap layout and more or fewer
    streams are refused (NE_EUNSUP) before anything touches a device, and
    single_launch must be 0 or 1."""
    ok = [_gm(in_bits=b, M=M) for b in (9, 10, 11, 12) for M in (3, 5, 8)]
    ok += [_gm(op=op, n_operand=0 if op == 1 else 100, in_bits=10, M=M)
           for op in (1, 2, 3, 4) for M in (3, 8)]  # scale, add, inner, perm
    for g in ok:
        assert _ws_single(lib, [g], mode)[0] == 0
    st, both = _ws_single(lib, ok, mode)
    assert st == 0
    st, multi = _ws_single(lib, ok, mode, single=0)
    # the queue (16 bytes a task), 8 bytes of counters a group and the queue head
    assert st == 0 and both > multi
    for bad in (_gm(in_bits=16), _gm(in_bits=8), _gm(op=9, n_operand=4),
                _gm(op=5, n_operand=100, in_bits=10), _gm(tap_copies=1, ring_waves=4)):
        assert _ws_single(lib, [bad], mode)[0] == -4
    if mode in (1, 2):  # plain groups may hold 1 or 2 streams, outside the menu
        assert _ws_single(lib, [_gm(M=2, op=1, n_operand=0, in_bits=10)], mode)[0] == -4
    assert _ws_single(lib, ok[:1], mode, single=2)[0] == -1
