"""GPU parity of the single-launch executor (ne_tuning.single_launch): a whole
uneven batch in one persistent launch whose blocks take work items from a
device queue -- every mode, every operation of its menu, single-stream
losses, repeated runs and captured replays (the queue and the per-group
counters must return to zero within each run), against the CPU oracle bit
for bit and against the per-variant launches."""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
POISON = 0x3C3C3C3C3C3C3C3C
MODES = ["entangled", "plain", "plain_same", "checksum", "checksum_same"]
LOSS_MODES = ("entangled", "checksum", "checksum_same")


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


class DevGroup:
    def __init__(self, grp, in_bits, lost=-1):
        self.grp = grp
        self.c = [dev32(row) for row in grp.c]
        self.operand = None if grp.op == "scale" else dev32(grp.operand)
        self.n_out = ne.n_out(grp.op, grp.n, 0 if grp.operand is None else grp.operand.size)
        self.out = [torch.full((max(self.n_out, 1),), POISON, dtype=torch.int64, device=DEV)[:self.n_out]
                    for _ in range(grp.M)]
        self.spec = ne.GroupSpec(grp.op, self.c, self.operand, self.out, grp.scalar, lost, in_bits)

    def poison(self):
        for t in self.out:
            t.fill_(POISON)

    def result(self):
        return np.stack([t.cpu().numpy() for t in self.out])

    def reference(self):
        g = self.grp
        return oracle.apply(g.op, g.c, g.operand if g.op != "scale" else None, g.scalar)


def group(op, M, n, K, bits, seed):
    g = wl.rng(seed)
    lo, hi = -(1 << (bits - 1)), 1 << (bits - 1)
    c = wl.uniform_i32(g, lo, hi, (M, n))
    s = 0
    if op == "conv":
        operand = wl.uniform_i32(g, lo, hi, K)
    elif op in ("add", "inner"):
        operand = wl.uniform_i32(g, lo, hi, n)
    elif op == "perm":
        operand = wl.permutation(g, n)
    else:
        operand, s = np.zeros(0, np.int32), int(g.integers(lo, hi))
    return wl.Group(op, c, operand, s)


def edge_groups(bits):
    """Tiny and ragged groups of every menu operation, both permutation row
    widths (<= 4 and > 4 slots), several strips per group."""
    gs = []
    for i, (op, M, n, K) in enumerate([
            ("conv", 3, 1, 1), ("conv", 8, 5000, 300), ("conv", 4, 2049, 512), ("conv", 5, 70001, 9),
            ("scale", 3, 1, 0), ("scale", 8, 70001, 0), ("add", 4, 255, 0), ("add", 7, 40001, 0),
            ("inner", 3, 1, 0), ("inner", 6, 70001, 0), ("perm", 3, 1, 0), ("perm", 4, 4097, 0),
            ("perm", 5, 70001, 0), ("perm", 8, 16385, 0)]):
        gs.append(group(op, M, n, K, bits, seed=7100 + i))
    return gs


def check(devs):
    for dg in devs:
        got = dg.result()
        ref = dg.reference()
        assert np.array_equal(got, ref), (dg.grp.op, dg.grp.M, dg.grp.n, dg.spec.lost)


@pytest.mark.parametrize("mode", MODES)
def test_single_launch_uneven_batch(mode):
    """An uneven batch (M 3..8, lengths 2^12..2^15, taps 8..512, all five
    operations) and the edge groups in one launch: every output equals the
    oracle, and the plan reports one launch."""
    groups = wl.config_uneven(seed=31, groups=28, n_hi=1 << 15) + edge_groups(10)
    rng = wl.rng(77)
    lost = [int(rng.integers(-1, g.M)) if mode in LOSS_MODES else -1 for g in groups]
    devs = [DevGroup(g, 10, r) for g, r in zip(groups, lost)]
    plan = ne.Plan([d.spec for d in devs], mode, single_launch=True)
    assert plan.stats()["launches"] == 1
    plan.run()
    torch.cuda.synchronize()
    assert plan.flags() == 0
    check(devs)
    plan.close()


@pytest.mark.parametrize("bits", [9, 11, 12])
def test_single_launch_sample_widths(bits):
    """The menu's other sample widths (split words at 11 and 12 bits, M = 3),
    every loss of a group of 3."""
    groups = [group(op, M, n, K, bits, seed=7300 + bits * 10 + i) for i, (op, M, n, K) in
              enumerate([("conv", 3, 9001, 64), ("conv", 4, 3000, 200), ("conv", 6, 5000, 33),
                         ("conv", 8, 2100, 130), ("inner", 3, 5000, 0), ("perm", 3, 6000, 0),
                         ("add", 5, 3001, 0), ("scale", 4, 3001, 0)])]
    for lost in (-1, 0, 1, 2):
        devs = [DevGroup(g, bits, lost) for g in groups]
        plan = ne.Plan([d.spec for d in devs], "entangled", single_launch=True)
        plan.run()
        torch.cuda.synchronize()
        assert plan.flags() == 0
        check(devs)
        plan.close()


def test_single_launch_matches_per_variant_launches_and_replays():
    """The same batch through the per-variant launches and through the single
    launch gives the same bits; the single launch run eagerly twice and
    captured and replayed three times, with the outputs poisoned and other
    device work between runs, gives the oracle's result every time."""
    groups = wl.config_uneven(seed=47, groups=24, n_hi=1 << 14) + edge_groups(10)[4:]
    rng = wl.rng(5)
    lost = [int(rng.integers(-1, g.M)) for g in groups]
    multi = [DevGroup(g, 10, r) for g, r in zip(groups, lost)]
    p = ne.Plan([d.spec for d in multi])
    p.run()
    torch.cuda.synchronize()
    p.close()
    single = [DevGroup(g, 10, r) for g, r in zip(groups, lost)]
    plan = ne.Plan([d.spec for d in single], single_launch=True)
    for _ in range(2):
        for d in single:
            d.poison()
        plan.run()
        torch.cuda.synchronize()
        assert plan.flags() == 0
        for a, b in zip(multi, single):
            assert np.array_equal(a.result(), b.result()), (a.grp.op, a.grp.M, a.grp.n)
    check(single)
    s = torch.cuda.Stream()
    plan.capture(s)
    for _ in range(3):
        for d in single:
            d.poison()
        torch.cuda.synchronize()
        scratch = torch.arange(1 << 20, device=DEV).sum()  # other device work in between
        plan.launch(s)
        s.synchronize()
        assert int(scratch) == (1 << 20) * ((1 << 20) - 1) // 2
        assert plan.flags() == 0
        check(single)
    plan.close()


def test_single_launch_refuses_groups_outside_its_menu():
    """16-bit samples and the outer product are outside the single launch's
    menu: plan creation fails with NE_EUNSUP; the per-variant plan accepts
    them."""
    g16 = DevGroup(group("conv", 3, 500, 20, 16, seed=7400), 16)
    outer = DevGroup(group("scale", 3, 100, 0, 10, seed=7401), 10)
    outer_spec = ne.GroupSpec("outer", outer.c, dev32(np.arange(4, dtype=np.int32)),
                              [torch.empty(400, dtype=torch.int64, device=DEV) for _ in range(3)],
                              0, -1, 10)
    for spec in (g16.spec, outer_spec):
        with pytest.raises(ne.NeError) as e:
            ne.Plan([spec], single_launch=True)
        assert e.value.status == -4
        ne.Plan([spec]).close()


def test_single_launch_replay_reads_new_inputs():
    """A captured single launch replayed after the inputs and operands were
    overwritten in place (new samples, new taps, new added vectors, a new
    permutation): each replay's outputs are those of its own inputs, so no
    permutation row or partial sum of an earlier run is read again."""
    base = wl.config_uneven(seed=53, groups=16, n_hi=1 << 14) + edge_groups(10)

    def redraw(grp, seed):
        g = wl.rng(seed)
        c = wl.uniform_i32(g, -(1 << 9), 1 << 9, grp.c.shape)
        if grp.op == "perm":
            operand = wl.permutation(g, grp.n)
        elif grp.op == "scale":
            operand = grp.operand
        else:
            operand = wl.uniform_i32(g, -(1 << 9), 1 << 9, grp.operand.size)
        return wl.Group(grp.op, c, operand, grp.scalar)

    other = [redraw(g, 7500 + i) for i, g in enumerate(base)]
    rng = wl.rng(11)
    lost = [int(rng.integers(-1, g.M)) for g in base]
    devs = [DevGroup(g, 10, r) for g, r in zip(base, lost)]
    plan = ne.Plan([d.spec for d in devs], single_launch=True)
    s = torch.cuda.Stream()
    plan.capture(s)

    def load(src):
        for d, g in zip(devs, src):
            for t, row in zip(d.c, g.c):
                t.copy_(torch.from_numpy(np.ascontiguousarray(row)))
            if d.operand is not None:
                d.operand.copy_(torch.from_numpy(np.ascontiguousarray(g.operand)))
            d.grp = g
            d.poison()
        torch.cuda.synchronize()

    for src in (base, other, base, other):
        load(src)
        plan.launch(s)
        s.synchronize()
        assert plan.flags() == 0
        check(devs)
    plan.close()


@pytest.mark.parametrize("mode", ["entangled", "plain", "checksum"])
def test_single_launch_32_bit_words(mode):
    """Element-wise groups with 32-bit entangled words (int32 outputs) in one
    launch: the gathers and inner products take 8 or 4 positions per lane
    there (int32 stores of 16 bytes), every loss of a group of 3, and ragged
    lengths; all equal the oracle."""
    bits = 7
    # (inner products short enough for D of w = 32: 64 * 64 * n <= D)
    cases = [("perm", 3, 70001), ("perm", 4, 4097), ("perm", 6, 40003), ("inner", 3, 255),
             ("inner", 8, 20001), ("scale", 3, 5001), ("add", 5, 3003)]
    for lost in ((-1, 0, 1, 2) if mode != "plain" else (-1,)):
        devs, refs = [], []
        for i, (op, M, n) in enumerate(cases):
            grp = group(op, M, n, 0, bits, seed=7600 + i)
            c = [dev32(row) for row in grp.c]
            operand = None if op == "scale" else dev32(grp.operand)
            n_out = ne.n_out(op, n, 0 if grp.operand is None else grp.operand.size)
            out = [torch.full((n_out,), 0x3C3C3C3C, dtype=torch.int32, device=DEV) for _ in range(M)]
            r = lost if lost < M else -1
            devs.append((ne.GroupSpec(op, c, operand, out, grp.scalar, r, bits, word_bits=32), out))
            refs.append(oracle.apply(op, grp.c, grp.operand if op != "scale" else None, grp.scalar))
        plan = ne.Plan([d[0] for d in devs], mode, single_launch=True)
        plan.run()
        torch.cuda.synchronize()
        assert plan.flags() == 0
        for (spec, out), ref, case in zip(devs, refs, cases):
            got = np.stack([t.cpu().numpy() for t in out]).astype(np.int64)
            assert np.array_equal(got, ref), (mode, lost, case)
        plan.close()
