"""Serving loop on the GPU (needs an MI355X): requests that arrive while
others run are planned on the other lane and launched while the running
batch is still on the device; every result is bitwise the one the request
gets alone, and matches the oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_1705_10218_amd import inputs, serve
from _util import rel_fro


pytestmark = pytest.mark.gpu


def _log(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def test_results_identical_alone_and_in_the_mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1705_10218_amd import bsmm
    # two large requests first (their batch runs for a while), then small
    # ones arriving while it runs
    big = inputs.serving_requests(2, atoms=(1500, 1600), occupancy=(0.15, 0.2), seed=7)
    small = inputs.serving_requests(10, atoms=(150, 600), occupancy=(0.03, 0.2), seed=8)
    arrivals = [0.0, 0.0] + [0.002 * (k + 1) for k in range(10)]
    reqs = [serve.Request(rid=i, a=a, b=b, eps=1e-10, arrival=arrivals[i])
            for i, (a, b, _) in enumerate(big + small)]
    srv = serve.Server(0, budget_bytes=64 << 30, max_batch=8, keep_results=True, max_wait_s=0.001)
    done = srv.run(reqs)
    _log(f"batches {srv.batches}, overlapping {srv.overlapping_batches()}, "
         f"times {[(round(a, 4), round(c, 4)) for a, c in srv.batch_times]}")
    assert len(done) == 12 and max(srv.batches) > 1
    assert srv.overlapping_batches() > 0, "a batch should start while another is on the device"
    assert all(r.done >= r.launched >= r.planned >= r.admitted >= r.arrival for r in done)
    ctx = bsmm.Context(0)
    for r in done:
        A, B = bsmm.Matrix.from_host(ctx, r.a), bsmm.Matrix.from_host(ctx, r.b)
        C, _ = bsmm.multiply(ctx, "N", "N", 1.0, A, B, filter_eps=r.eps)
        alone = C.to_host()
        for m in (C, A, B):
            m.close()
        assert np.array_equal(alone.row_ptr, r.result.row_ptr) and np.array_equal(alone.col_idx, r.result.col_idx)
        assert np.array_equal(alone.values.view(np.uint64), r.result.values.view(np.uint64)), \
            f"request {r.rid} differs in the mix"
        if r.rid in (2, 3, 4):
            ref = oracle.multiply("N", "N", 1.0, r.a, r.b, eps=r.eps, nthreads=8)
            assert np.array_equal(ref.col_idx, r.result.col_idx)
            assert rel_fro(r.result.values, ref.values) <= 1e-12
    stats = serve.summary(done)
    _log(f"{stats}")
    assert stats["latency_p99_ms"] >= stats["latency_p50_ms"] > 0
    ctx.close()
