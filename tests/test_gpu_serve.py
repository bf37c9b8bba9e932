"""Serving loop on the GPU (needs an MI355X): requests batched into shared
launches give bitwise the results they get alone, and match the oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_1705_10218_amd import inputs, serve
from _util import rel_fro

pytestmark = pytest.mark.gpu


def test_results_identical_alone_and_in_the_mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1705_10218_amd import bsmm
    ctx = bsmm.Context(0)
    gen = inputs.serving_requests(10, atoms=(150, 600), occupancy=(0.03, 0.2), seed=7)
    arrivals = [0.0] * 6 + [0.05, 0.06, 0.3, 0.31]
    reqs = [serve.Request(rid=i, a=a, b=b, eps=1e-10, arrival=arrivals[i]) for i, (a, b, _) in enumerate(gen)]
    srv = serve.Server(ctx, budget_bytes=8 << 30, max_batch=8, keep_results=True)
    done = srv.run(reqs)
    sys.stdout.write(f"batches {srv.batches}\n")
    assert max(srv.batches) > 1 and len(done) == 10
    for r in done:
        A, B = bsmm.Matrix.from_host(ctx, r.a), bsmm.Matrix.from_host(ctx, r.b)
        C, _ = bsmm.multiply(ctx, "N", "N", 1.0, A, B, filter_eps=r.eps)
        alone = C.to_host()
        for m in (C, A, B):
            m.close()
        assert np.array_equal(alone.row_ptr, r.result.row_ptr) and np.array_equal(alone.col_idx, r.result.col_idx)
        assert np.array_equal(alone.values, r.result.values), f"request {r.rid} differs in the mix"
        if r.rid < 3:
            ref = oracle.multiply("N", "N", 1.0, r.a, r.b, eps=r.eps, nthreads=8)
            assert np.array_equal(ref.col_idx, r.result.col_idx)
            assert rel_fro(r.result.values, ref.values) <= 1e-12
    stats = serve.summary(done)
    sys.stdout.write(f"{stats}\n")
    assert stats["latency_p99_ms"] >= stats["latency_p50_ms"] > 0
    ctx.close()
