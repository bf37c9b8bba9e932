"""Serving loop: arrival process, statistics and admission logic (CPU, fake engine)."""
import time
import types

import numpy as np
import pytest

from paper_1705_10218_amd import inputs, serve


def test_poisson_arrivals():
    rng = np.random.default_rng(0)
    t = serve.poisson_arrivals(20000, 50.0, rng)
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 50.0) < 0.03 / 50.0 * 10   # within a few standard errors
    assert np.all(serve.poisson_arrivals(5, 0.0, rng) == 0.0)


def test_percentiles():
    p = serve.percentiles(np.arange(1, 101))
    assert p["p50"] == pytest.approx(50.5) and p["p99"] == pytest.approx(99.01)


def test_footprint_terms():
    a, b, _ = inputs.dft_like_pair(150, config=97, sizes=(5, 13), cutoff=5.0)
    ob = serve.operand_bytes(a, b)
    assert ob >= 8 * (a.n_values() + b.n_values())
    a2, b2, _ = inputs.dft_like_pair(150, config=97, sizes=(5, 13), cutoff=5.5)
    assert serve.operand_bytes(a2, b2) > ob
    assert serve.plan_bytes(10, 2, 30, 256) == 8 * 10 + 48 * 2 + 8 * 30 + 256


class _FakeServer(serve.Server):
    """The loop with a fake engine: a batch 'runs' for a fixed time after its
    launch; planned bytes are the operand bytes times a per-request factor."""

    def __init__(self, *a, run_s=0.01, factor=None, **k):
        super().__init__(0, *a, **k)
        self.run_s = run_s
        self.factor = factor or {}
        self.launches = []

    def _new_lane(self):
        return types.SimpleNamespace(planned=[], inflight=None)

    def _plan(self, lane, r):
        r.flops = 1.0
        return int(self.factor.get(r.rid, 2.0) * serve.operand_bytes(r.a, r.b))

    def _launch(self, lane, reqs):
        self.launches.append([r.rid for r in reqs])
        return time.perf_counter() + self.run_s

    def _finished(self, lane, event):
        return time.perf_counter() >= event

    def _complete(self, lane, r):
        pass


def _reqs(n, arrivals, atoms=60):
    out = []
    for i in range(n):
        a, b, _ = inputs.dft_like_pair(atoms, config=98, sizes=(5,), cutoff=4.0, request=i)
        out.append(serve.Request(rid=i, a=a, b=b, arrival=arrivals[i]))
    return out


def test_loop_batches_overlap_and_respect_the_budget():
    """Requests arriving while a batch runs are planned on the other lane and
    launched before the running batch ends; every request completes after
    its arrival; the planned bytes in flight never exceed the budget once
    more than one request is in flight."""
    arrivals = [0.0] * 4 + [0.002 * k for k in range(1, 13)]
    reqs = _reqs(16, arrivals)
    ob = serve.operand_bytes(reqs[0].a, reqs[0].b)
    srv = _FakeServer(budget_bytes=20 * ob, max_batch=4, run_s=0.01, max_wait_s=0.001)
    done = srv.run(reqs)
    assert len(done) == 16 and sorted(r.rid for r in done) == list(range(16))
    assert all(r.done >= r.launched >= r.planned >= r.admitted >= r.arrival for r in done)
    assert max(srv.batches) <= 4 and len(srv.batches) >= 4
    assert srv.overlapping_batches() > 0, srv.batch_times
    assert srv.peak_used <= 20 * ob


def test_loop_admits_by_planned_size():
    """A request whose plan turns out large keeps later ones waiting until
    memory frees up: no two large requests are in flight together."""
    reqs = _reqs(6, [0.0] * 6)
    ob = serve.operand_bytes(reqs[0].a, reqs[0].b)
    factor = {0: 9.0, 3: 9.0}
    srv = _FakeServer(budget_bytes=12 * ob, max_batch=8, run_s=0.005, factor=factor)
    done = srv.run(reqs)
    assert len(done) == 6
    for k in range(len(srv.batches)):
        members = {r.rid for r in done if r.batch == k}
        assert not {0, 3} <= members
    t = {r.rid: r for r in done}
    assert t[3].launched >= t[0].done or t[0].launched >= t[3].done


def test_three_lanes_run_three_batches_at_once():
    """With three lanes, requests arriving while two batches run are planned
    on the third and launched before either ends; every request completes;
    fewer than two lanes are rejected."""
    arrivals = [0.0] * 2 + [0.003] * 2 + [0.006] * 2
    reqs = _reqs(6, arrivals)
    ob = serve.operand_bytes(reqs[0].a, reqs[0].b)
    srv = _FakeServer(budget_bytes=100 * ob, max_batch=2, run_s=0.05, max_wait_s=0.001, lanes=3)
    done = srv.run(reqs)
    assert sorted(r.rid for r in done) == list(range(6))
    assert all(r.done >= r.arrival for r in done)
    # some batch launched while two others were still running
    bt = srv.batch_times
    assert any(sum(1 for j, (a, c) in enumerate(bt) if j != k and a < l < c) >= 2 for k, (l, _) in enumerate(bt))
    with pytest.raises(ValueError):
        _FakeServer(budget_bytes=ob, lanes=1)
