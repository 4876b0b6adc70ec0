"""The serving loop's device pool bookkeeping (host only)."""
import random

from paper_1509_03838_amd.serve import _Pool, _up


def test_pool_first_fit_and_merge():
    p = _Pool(4096)
    a = p.alloc(100)
    b = p.alloc(300)
    c = p.alloc(256)
    assert a == (0, 256) and b == (256, 512) and c == (768, 256)
    assert p.alloc(4096) is None
    p.release(*b)
    assert p.alloc(512) == (256, 512)  # first fit reuses the hole
    p.release(256, 512)
    p.release(*a)
    p.release(*c)
    assert p.free == [(0, 4096)]  # neighbours merged back into one range


def test_pool_random_never_overlaps():
    rng = random.Random(5)
    p = _Pool(1 << 20)
    live = []
    for _ in range(2000):
        if live and rng.random() < 0.45:
            p.release(*live.pop(rng.randrange(len(live))))
        else:
            r = p.alloc(rng.randrange(1, 40000))
            if r is not None:
                assert r[0] % 256 == 0 and r[1] == _up(r[1])
                live.append(r)
        spans = sorted(live + p.free)
        for (o1, s1), (o2, _) in zip(spans, spans[1:]):
            assert o1 + s1 <= o2  # live and free ranges are disjoint
        assert sum(s for _, s in spans) == 1 << 20  # and cover the pool
    for r in live:
        p.release(*r)
    assert p.free == [(0, 1 << 20)]
