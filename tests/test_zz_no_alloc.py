"""The no-allocation series call (ne_chain_apply_noalloc) against the one
with caller workspace (ne_chain_apply), bit for bit, through the C ABI:
two calls in a row on the library's fixed device buffer, the second with a
smaller input, so that stale contents of the first call would show. Both
are also checked against the CPU oracle after one extraction."""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
POISON = -0x5A5A5A5A5A5A5A5A

RECIPES = [wl.CHAIN_RECIPE, ("perm", "add", "conv", "inner"), ("sub", "mul", "circ", "xcorr"),
           ("outer", "sub", "perm"), ("conv", "conv")]


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def device_ops(ops, l, bits):
    out = []
    for op, g, s in ops:
        if op == "scale":
            out.append(ne.ChainOp(op, None, s))
            continue
        dg = dev32(g)
        if op in ("add", "sub"):  # footnote 3: the added vector is entangled too
            ge = torch.empty(g.size, dtype=torch.int64, device=DEV)
            ne.entangle_operand(dg, ge, l)
            dg = ge
        out.append(ne.ChainOp(op, dg, s, operand_bits=bits))
    return out


def both_ways(c, ops, lost, bits):
    """(outputs of ne_chain_apply, of ne_chain_apply_noalloc, recovered
    outputs of the latter) on the same entangled streams."""
    M, n = c.shape
    l = ne.params(M)[0]
    dops = device_ops(ops, l, bits)
    no, _ = ne.chain_check(M, bits, n, dops)
    eps = [torch.empty(n, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.entangle([dev32(r) for r in c], eps, l)
    mask = ((1 << M) - 1) & ~(1 << lost if lost >= 0 else 0)
    ref = [torch.full((no,), POISON, dtype=torch.int64, device=DEV) for _ in range(M)]
    got = [torch.full((no,), POISON, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.chain_apply(eps, dops, ref, mask=mask)
    ne.chain_apply_noalloc(eps, dops, got, mask=mask)
    dhat = [torch.empty(no, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.extract_recover([None if m == lost else got[m] for m in range(M)], lost, dhat, l, n=no)
    torch.cuda.synchronize()
    host = lambda ts: np.stack([t.cpu().numpy() for t in ts])  # noqa: E731
    return host(ref), host(got), host(dhat)


@pytest.mark.parametrize("recipe", RECIPES)
@pytest.mark.parametrize("M", [3, 5])
def test_noalloc_matches_workspace_call_twice(recipe, M):
    """A large call, then a smaller one: both equal the workspace call and
    recover the oracle's plain result."""
    g = wl.rng(5150 + M + len(recipe))
    lost = 1
    first = 20_011 if "outer" in recipe else 200_003  # outer: 23 outputs per sample
    for n in (first, 4_099):
        c = wl.uniform_i32(g, -32, 32, (M, n))
        ops = wl.chain_series(g, n, recipe, bits=6, K=23)
        ref, got, dhat = both_ways(c, ops, lost, 6)
        live = [m for m in range(M) if m != lost]
        assert np.array_equal(got[live], ref[live]), (recipe, M, n)
        assert np.array_equal(dhat, oracle.chain(c, ops)), (recipe, M, n)


def test_noalloc_at_the_buffer_limit_and_past_it():
    """The longest three-stream series the buffer holds runs; one sample
    more is refused with NE_ESCRATCH before anything is launched."""
    M = 3
    plane = ne.CHAIN_SCRATCH_BYTES // (2 * M)
    n_fit = plane // 8 - 64  # two scale stages: intermediates of n words
    g = wl.rng(5199)
    for n in (n_fit, 1000):
        ops = [("scale", None, 3), ("scale", None, -5)]
        c = wl.uniform_i32(g, -32, 32, (M, n))
        ref, got, dhat = both_ways(c, ops, -1, 6)
        assert np.array_equal(got, ref)
        assert np.array_equal(dhat, c.astype(np.int64) * -15)
    n_big = plane // 8 + 1
    eps = [torch.zeros(n_big, dtype=torch.int64, device=DEV) for _ in range(M)]
    out = [torch.zeros(n_big, dtype=torch.int64, device=DEV) for _ in range(M)]
    ops = [ne.ChainOp("scale", None, 3), ne.ChainOp("scale", None, 5)]
    with pytest.raises(ne.NeError) as e:
        ne.chain_apply_noalloc(eps, ops, out)
    assert e.value.status == -7
    ne.chain_apply_noalloc(eps[:1] * 3, [ne.ChainOp("scale", None, 3)], out)  # one stage: no buffer
    torch.cuda.synchronize()
