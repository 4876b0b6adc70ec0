"""The serving loop: every job's recovered outputs are the same in the mix
as when the job runs alone, and equal the CPU oracle's convolution."""
import numpy as np
import pytest

import oracle
from paper_1509_03838_amd import ne
from paper_1509_03838_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def alone(job, in_bits=11):
    g = job.group
    dev = "cuda:0"
    c = [torch.from_numpy(np.ascontiguousarray(r)).to(dev) for r in g.c]
    k = torch.from_numpy(g.operand).to(dev)
    out = [torch.empty(g.n + g.operand.size - 1, dtype=torch.int64, device=dev) for _ in range(g.M)]
    plan = ne.Plan([ne.GroupSpec("conv", c, k, out, 0, g.fail, in_bits)])
    plan.run()
    torch.cuda.synchronize()
    assert plan.flags() == 0
    return [t.cpu().numpy() for t in out]


def test_serving_results_alone_equal_in_the_mix():
    from paper_1509_03838_amd.serve import Server
    jobs = wl.serving_jobs(seed=7, count=80, n_hi=1 << 15, drop_prob=0.2)
    assert any(j.group.fail >= 0 for j in jobs)
    srv = Server(hbm_budget=24 << 20, lanes=3, max_batch=8, keep_outputs=True)
    rep = srv.run(jobs)
    assert rep.jobs == 80 and rep.peak_bytes <= 24 << 20
    assert 0 < rep.p50_ms <= rep.p99_ms <= rep.max_ms
    assert rep.batches >= 2 and rep.lost_jobs == sum(j.group.fail >= 0 for j in jobs)
    torch.cuda.synchronize()
    for r, job in zip(rep.records, jobs):
        mixed = [t.cpu().numpy() for t in r.outputs]
        solo = alone(job)
        for a, b in zip(mixed, solo):
            assert np.array_equal(a, b), r.index
        g = job.group
        if g.n <= 5000:
            ref = oracle.apply("conv", g.c, g.operand)
            assert np.array_equal(np.stack(mixed), ref), r.index
        else:  # every stream at both ends and 1000 seeded positions between
            n_out = g.n + g.operand.size - 1
            pos = np.unique(np.concatenate([
                np.arange(64), np.arange(n_out - 64, n_out),
                wl.rng(r.index).integers(0, n_out, 1000)]))
            for m in range(g.M):
                assert np.array_equal(mixed[m][pos], oracle.conv_at(g.c[m], g.operand, pos)), \
                    (r.index, m)


def test_serving_defers_by_footprint_and_batches():
    """Under a load the device cannot absorb job by job (a burst of 60
    jobs, one lane, a budget of a few jobs), the server forms batches of
    several jobs and defers admissions on the HBM budget; every result is
    still the oracle's."""
    from paper_1509_03838_amd.serve import Server
    jobs = wl.serving_jobs(seed=11, count=60, rate_hz=200_000.0, n_hi=1 << 14, drop_prob=0.1)
    srv = Server(hbm_budget=4 << 20, lanes=1, max_batch=16, keep_outputs=True)
    rep = srv.run(jobs)
    assert rep.jobs == 60 and rep.peak_bytes <= 4 << 20
    assert rep.mean_batch > 1 and rep.deferred_jobs > 0
    torch.cuda.synchronize()
    for r, job in zip(rep.records, jobs):
        ref = oracle.apply("conv", job.group.c, job.group.operand)
        assert np.array_equal(np.stack([t.cpu().numpy() for t in r.outputs]), ref), r.index
