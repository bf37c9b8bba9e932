"""bsmm_filter_noalloc (the filter for callers that cannot allocate) against
bsmm_filter, through the C ABI: bitwise equal index and values, on two calls
in a row whose second input is smaller, with the output buffers of the first
call reused (and left holding its results) for the second."""
import sys

import numpy as np
import pytest

from _util import random_bcsr

pytestmark = pytest.mark.gpu


def _log(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1705_10218_amd import bsmm
    return bsmm


def _reference(B, X, eps):
    F = B.filter(X, eps)
    host = F.to_host()
    F.close()
    return host


def _noalloc(B, ctx, X, eps, bufs):
    rp, ci, vals, counts = bufs
    held0 = ctx.memory()[0]
    B.filter_noalloc(X, eps, rp, ci, vals, counts)
    ctx.synchronize()
    assert ctx.memory()[0] == held0, "the library allocated device memory"
    nbr = X.info()[0]
    kb, kv = (int(x) for x in counts.cpu().numpy())
    return rp[:nbr + 1].cpu().numpy(), ci[:kb].cpu().numpy(), vals[:kv].cpu().numpy(), kb, kv


def test_noalloc_matches_filter_twice(B):
    import torch
    ctx = B.Context(0)
    rng = np.random.default_rng(7301)
    big = random_bcsr(rng, 700, 650, p=0.04, max_bs=32, empty_rows=(3, 4, 699))
    small = random_bcsr(rng, 41, 37, p=0.5, max_bs=13)
    dev = f"cuda:{ctx.device}"
    bufs = (torch.full((big.nbr + 1,), -7, dtype=torch.int64, device=dev),
            torch.full((max(big.nnzb, 1),), -7, dtype=torch.int32, device=dev),
            torch.full((max(big.n_values(), 1),), float("nan"), dtype=torch.float64, device=dev),
            torch.full((2,), -7, dtype=torch.int64, device=dev))
    for name, x in (("700x650 blocks, sizes 1-32", big), ("41x37 blocks, sizes 1-13", small)):
        X = B.Matrix.from_host(ctx, x)
        norms = B.block_norms(X).cpu().numpy()
        for eps in (float(np.median(norms)), 0.0):
            _log(f"filter_noalloc: {name}, nnzb {x.nnzb}, eps {eps:.6g}")
            ref = _reference(B, X, eps)
            rp, ci, vals, kb, kv = _noalloc(B, ctx, X, eps, bufs)
            assert kb == ref.nnzb and kv == ref.values.shape[0]
            assert np.array_equal(rp, ref.row_ptr), "row_ptr differs"
            assert np.array_equal(ci, ref.col_idx), "col_idx differs"
            assert np.array_equal(vals.view(np.uint64), ref.values.view(np.uint64)), "values differ"
            if eps > 0:
                assert 0 < kb < x.nnzb, "the threshold should drop some blocks and keep others"
        X.close()
    ctx.close()


def test_noalloc_rejects(B):
    import torch
    ctx = B.Context(0)
    rng = np.random.default_rng(7302)
    x = random_bcsr(rng, 5, 5, p=0.6, max_bs=4)
    X = B.Matrix.from_host(ctx, x)
    dev = f"cuda:{ctx.device}"
    rp = torch.zeros(x.nbr + 1, dtype=torch.int64, device=dev)
    ci = torch.zeros(x.nnzb, dtype=torch.int32, device=dev)
    vals = torch.zeros(x.n_values(), dtype=torch.float64, device=dev)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    with pytest.raises(B.BsmmError) as e:
        B.filter_noalloc(X, -1.0, rp, ci, vals, counts)
    assert e.value.status == 1
    with pytest.raises(B.BsmmError) as e:
        B.filter_noalloc(X, 0.5, rp, None, vals, counts)
    assert e.value.status == 1
    X.close()
    ctx.close()
