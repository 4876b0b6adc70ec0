"""A permutation index outside [0, n) is reported, not clamped (the
operation is a fixed bijection, eq. (2) and footnote 2): the per-step calls
raise NE_FLAG_PERM_INDEX in the library's device flag word and write 0
there; the fused executor raises it in the plan's flag word. Every other
output still equals the oracle's."""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def dev(a, dt=np.int32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(DEV)


def inputs(M=3, n=5000, seed=71):
    g = wl.rng(seed)
    c = wl.uniform_i32(g, -512, 512, (M, n))
    p = wl.permutation(g, n)
    return c, p


@pytest.mark.parametrize("bad", [-1, 5000, 2**31 - 1])
@pytest.mark.parametrize("width", [64, 32])
def test_per_step_permutation_flags_bad_index(bad, width):
    ne.device_flags(clear=True)
    c, p = inputs()
    M, n = c.shape
    at = 1234
    ref = oracle.apply("perm", c, p).copy()
    p_bad = p.copy()
    p_bad[at] = bad
    word = torch.int32 if width == 32 else torch.int64
    l = ne.params(M, width)[0]
    cd = [dev(r) for r in c]
    eps = [torch.empty(n, dtype=word, device=DEV) for _ in range(M)]
    delta = [torch.empty(n, dtype=word, device=DEV) for _ in range(M)]
    out = [torch.empty(n, dtype=word, device=DEV) for _ in range(M)]
    pd = dev(p_bad)
    if width == 32:
        ne.entangle32(cd, eps, l)
        ne.lsb_apply32("perm", eps, pd, delta)
        ne.extract_recover32(delta, -1, out, l)
    else:
        ne.entangle(cd, eps, l)
        ne.lsb_apply("perm", eps, pd, delta)
        ne.extract_recover(delta, -1, out, l)
    assert ne.device_flags(clear=True) & ne.FLAG_PERM_INDEX
    got = np.stack([t.cpu().numpy() for t in out]).astype(np.int64)
    keep = np.ones(n, bool)
    keep[at] = False
    assert np.array_equal(got[:, keep], ref[:, keep])
    assert np.all(got[:, at] == 0)  # every entangled word there is 0, so is its recovery
    assert ne.device_flags() == 0


def test_per_step_plain_permutation_flags_bad_index():
    ne.device_flags(clear=True)
    c, p = inputs()
    M, n = c.shape
    p_bad = p.copy()
    p_bad[0] = n
    out = [torch.empty(n, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.plain_apply("perm", [dev(r) for r in c], dev(p_bad), out)
    assert ne.device_flags(clear=True) == ne.FLAG_PERM_INDEX
    got = np.stack([t.cpu().numpy() for t in out])
    ref = oracle.apply("perm", c, p)
    assert np.array_equal(got[:, 1:], ref[:, 1:]) and np.all(got[:, 0] == 0)


def test_valid_permutation_raises_nothing():
    ne.device_flags(clear=True)
    c, p = inputs()
    M, n = c.shape
    out = [torch.empty(n, dtype=torch.int64, device=DEV) for _ in range(M)]
    ne.plain_apply("perm", [dev(r) for r in c], dev(p), out)
    assert ne.device_flags() == 0
    assert np.array_equal(np.stack([t.cpu().numpy() for t in out]), oracle.apply("perm", c, p))


@pytest.mark.parametrize("mode", ["entangled", "plain", "checksum"])
@pytest.mark.parametrize("M", [3, 6])
def test_fused_permutation_flags_bad_index(mode, M):
    c, p = inputs(M=M, n=7001, seed=72)
    n = c.shape[1]
    at = [0, 4097, n - 1]
    p_bad = p.copy()
    p_bad[at] = [-5, n, 1 << 30]
    cd = [dev(r) for r in c]
    out = [torch.empty(n, dtype=torch.int64, device=DEV) for _ in range(M)]
    plan = ne.Plan([ne.GroupSpec("perm", cd, dev(p_bad), out, 0, -1, 10)], mode)
    plan.run()
    torch.cuda.synchronize()
    assert plan.flags() & ne.FLAG_PERM_INDEX
    got = np.stack([t.cpu().numpy() for t in out])
    keep = np.ones(n, bool)
    keep[at] = False
    assert np.array_equal(got[:, keep], oracle.apply("perm", c, p)[:, keep])
    # a valid permutation in the same plan shape raises nothing
    plan2 = ne.Plan([ne.GroupSpec("perm", cd, dev(p), out, 0, -1, 10)], mode)
    plan2.run()
    torch.cuda.synchronize()
    assert plan2.flags() == 0
    assert np.array_equal(np.stack([t.cpu().numpy() for t in out]), oracle.apply("perm", c, p))
