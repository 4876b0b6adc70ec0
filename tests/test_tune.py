"""Autotuner: class keys and the on-disk cache (CPU), and on the GPU that
tuned plans give the same bits as untuned ones."""
import json
import types

import numpy as np
import pytest

from paper_1509_03838_amd import tune


class FakeTensor:
    def __init__(self, n):
        self.n = n

    def numel(self):
        return self.n


def spec(op, M, n, K=0, bits=12):
    return types.SimpleNamespace(op=op, c=[FakeTensor(n)] * M,
                                 operand=FakeTensor(K) if K else None, in_bits=bits, steps=0,
                                 ring_waves=0)


def test_class_keys_bucket_sizes():
    a = tune.class_key(spec("conv", 3, 1 << 20, 64), "entangled")
    b = tune.class_key(spec("conv", 3, (1 << 20) + 5, 100), "entangled")
    c = tune.class_key(spec("conv", 3, 1 << 20, 128), "entangled")
    d = tune.class_key(spec("conv", 3, 1 << 20, 64), "plain")
    assert a == b and a != c and a != d
    assert tune.class_key(spec("scale", 5, 4096), "entangled") == "entangled|scale|M>4|n6"
    assert tune.class_key(spec("scale", 3, 8191), "entangled") == "entangled|scale|M<=4|n6"


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    t = tune.Tuner(path)
    t.cache = {"entangled|conv|M3|b12|K6|n10": (8, 1)}
    t.save()
    assert json.load(open(path))["steps"]["entangled|conv|M3|b12|K6|n10"] == [8, 1]
    t2 = tune.Tuner(path)
    sp = [spec("conv", 3, 1 << 20, 64) for _ in range(3)]
    table = t2.tune(sp, "entangled")  # cached: no timing, no GPU
    assert table == {"entangled|conv|M3|b12|K6|n10": (8, 1)}
    assert all(s.steps == 8 and s.ring_waves == 1 for s in sp)


def test_cached_per_wave_ring_falls_back_where_it_does_not_fit(tmp_path, monkeypatch):
    """A per-wave ring chosen on one member of a K bucket can exceed LDS on
    a longer member: that member goes back to the planner's own layout
    choice; the members it fits keep the cached choice."""
    from paper_1509_03838_amd import ne
    limit = 2100  # M = 3, 12-bit samples: the planner refuses per-wave rings at K = 2200

    def fake_size(groups, mode="entangled", *a, **k):
        (g,) = groups
        if g.ring_waves == 1 and g.operand.numel() > limit:
            raise ne.NeError("ne_plan_workspace_size", -4, "unsupported")
        return 0

    monkeypatch.setattr(ne, "workspace_size", fake_size)
    path = str(tmp_path / "t.json")
    t = tune.Tuner(path)
    t.cache = {"entangled|conv|M3|b12|K11|n10": (4, 1)}
    sp = [ne.GroupSpec("conv", [FakeTensor(1 << 20)] * 3, FakeTensor(K), [], 0, -1, 12)
          for K in (2048, 2200)]
    t.tune(sp, "entangled")
    assert [(s.steps, s.ring_waves) for s in sp] == [(4, 1), (4, 0)]


@pytest.mark.parametrize("verdict", [0, 1])
def test_whole_plan_verdict_from_the_cache(tmp_path, verdict):
    """A batch of several classes: the cached whole-plan verdict keeps the
    classes' choices (0) or gives every group the planner's defaults (1)."""
    sp = [spec("conv", 3, 1 << 20, 64), spec("scale", 5, 4096)]
    keys = [tune.class_key(s, "entangled") for s in sp]
    t = tune.Tuner(str(tmp_path / "t.json"))
    t.cache = {keys[0]: (8, 1), keys[1]: (2, 0),
               tune.plan_key(dict.fromkeys(keys), "entangled"): (verdict, 0)}
    table = t.tune(sp, "entangled")
    want = [(0, 0), (0, 0)] if verdict else [(8, 1), (2, 0)]
    assert [(s.steps, s.ring_waves) for s in sp] == want
    assert table[tune.plan_key(dict.fromkeys(keys), "entangled")] == (
        "planner defaults" if verdict else "tuned")


def test_cache_reads_bare_step_counts(tmp_path):
    path = tmp_path / "old.json"
    path.write_text(json.dumps({"steps": {"entangled|scale|M<=4|n6": 4}}))
    assert tune.Tuner(str(path)).cache == {"entangled|scale|M<=4|n6": (4, 0)}


@pytest.mark.gpu
def test_tuned_plan_is_bit_identical(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_1509_03838_amd import ne
    from paper_1509_03838_amd import workloads as wl
    groups = wl.config_uneven(seed=3, groups=12, n_hi=1 << 15)
    dev = "cuda:0"

    def specs(out):
        res = []
        for g, o in zip(groups, out):
            c = [torch.from_numpy(np.ascontiguousarray(r)).to(dev) for r in g.c]
            k = None if g.op == "scale" else torch.from_numpy(g.operand).to(dev)
            res.append(ne.GroupSpec(g.op, c, k, o, g.scalar, -1, 10))
        return res

    def outs():
        return [[torch.zeros(max(ne.n_out(g.op, g.n, 0 if g.operand is None else g.operand.size), 1),
                             dtype=torch.int64, device=dev) for _ in range(g.M)] for g in groups]

    o1, o2 = outs(), outs()
    s1 = specs(o1)
    ne.Plan(s1).run()
    s2 = specs(o2)
    table = tune.Tuner(str(tmp_path / "c.json")).tune(s2)
    verdicts = {k: v for k, v in table.items() if "|plan|" in k}
    assert list(verdicts.values()) in (["tuned"], ["planner defaults"])  # several classes
    assert all(v in tune.CONV_CANDIDATES + tune.STREAM_CANDIDATES
               for k, v in table.items() if k not in verdicts)
    ne.Plan(s2).run()
    torch.cuda.synchronize()
    for a, b in zip(o1, o2):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
