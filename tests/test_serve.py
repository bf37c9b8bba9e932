"""Serving loop: arrival process, statistics and admission logic (CPU, fake engine)."""
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


def test_footprint_counts_result_blocks():
    a, b, _ = inputs.dft_like_pair(150, config=97, sizes=(5, 13), cutoff=5.0)
    small = serve.footprint_bytes(a, b)
    assert small > 8 * (a.n_values() + b.n_values())
    a2, b2, _ = inputs.dft_like_pair(150, config=97, sizes=(5, 13), cutoff=5.5)
    assert serve.footprint_bytes(a2, b2) > small


class _FakeBsmm(types.SimpleNamespace):
    pass


def test_admission_respects_budget(monkeypatch):
    """Drive Server.run with a fake engine: every batch fits the budget, every
    request completes after it arrived, and arrivals during a batch join a
    later batch."""
    import paper_1705_10218_amd as pkg
    batches = []

    class M:
        def __init__(self, *a, **k):
            pass

        @classmethod
        def from_host(cls, ctx, m):
            return cls()

        def close(self):
            pass

        def to_host(self):
            return None

    class P:
        def __init__(self, ctx, ta, tb, alpha, a, b, beta=0.0, c=None, filter_eps=0.0):
            self.info = types.SimpleNamespace(useful_flops=1.0)

        def result(self):
            return M()

        def close(self):
            pass

    fake = _FakeBsmm(Matrix=M, Plan=P, plans_execute=lambda plans: batches.append(len(plans)),
                     _torch=lambda: types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None)))
    monkeypatch.setattr(pkg, "bsmm", fake, raising=False)
    monkeypatch.setitem(__import__("sys").modules, "paper_1705_10218_amd.bsmm", fake)
    sizes = {}
    monkeypatch.setattr(serve, "footprint_bytes", lambda a, b: sizes[id(a)])
    reqs = []
    for i in range(12):
        a = object()
        sizes[id(a)] = 10 if i % 3 else 25
        reqs.append(serve.Request(rid=i, a=a, b=None, arrival=0.0 if i < 8 else 0.02 * (i - 7)))
    srv = serve.Server(ctx=None, budget_bytes=40, max_batch=4)
    done = srv.run(reqs)
    assert len(done) == 12 and sorted(r.rid for r in done) == list(range(12))
    assert all(r.done >= r.arrival for r in done)
    for k in range(len(srv.batches)):
        members = [r for r in done if r.batch == k]
        assert sum(sizes[id(r.a)] for r in members) <= 40 and len(members) <= 4
    assert max(batches) > 1
