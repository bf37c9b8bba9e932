"""The edge-subtile GEMM variant (variant 4: result blocks with both edges
in 9..24 and one above 16, covered by one 16x16x4 MFMA tile plus 4x4x4 MFMA
subtiles along the edges beyond 16, with lane rotations between k-groups'
lanes) against the FP64 oracle, through the C ABI (needs an MI355X).

Bar as for the other parity tests: pattern, product and candidate counts
and useful flops exact; values within relative Frobenius error 1e-12.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1705_10218_amd import inputs
from _util import random_bcsr, rel_fro

pytestmark = pytest.mark.gpu
TOL = 1e-12
EDGE_CLASSES = ((13, 23), (23, 13), (23, 23))   # (m, n) classes the variant serves


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


@pytest.fixture
def ctx(B):
    c = B.Context(0)
    for m, n in EDGE_CLASSES:
        c.set_gemm_variant(m, n, 4)
    yield c
    c.close()


def _mul(B, ctx, ta, tb, alpha, a, b, beta=0.0, c=None, eps=0.0, retain=False):
    A = B.Matrix.from_host(ctx, a)
    Bm = B.Matrix.from_host(ctx, b)
    C0 = B.Matrix.from_host(ctx, c) if c is not None else None
    C, info = B.multiply(ctx, ta, tb, alpha, A, Bm, beta, C0, eps, retain)
    host = C.to_host()
    for m in (C, A, Bm, C0):
        if m is not None:
            m.close()
    return host, info


def _check(host, info, ref):
    assert np.array_equal(host.row_ptr, ref.row_ptr)
    assert np.array_equal(host.col_idx, ref.col_idx)
    assert info.n_products == ref.n_products
    assert info.n_candidates == ref.n_candidates
    assert info.useful_flops == ref.useful_flops
    err = rel_fro(host.values, ref.values) if ref.values.size else 0.0
    assert err <= TOL, f"relative Frobenius error {err:.3e}"
    return err


@pytest.mark.parametrize("m,n", [(5, 23), (13, 13), (23, 5), (25, 23), (23, 32)])
def test_rejects_other_edges(B, ctx, m, n):
    with pytest.raises(Exception):
        ctx.set_gemm_variant(m, n, 4)


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
@pytest.mark.parametrize("menu", [(9, 16, 17, 20, 24), (1, 5, 13, 17, 23, 24, 29)])
def test_random_grids(B, ctx, ta, tb, menu):
    """Edges 9..24 (every shape the variant serves: one or both edges above
    16, each edge-subtile row or column group partly or fully used) and a
    mix with edges the variant leaves to the others, in one launch."""
    rng = np.random.default_rng(400 + len(menu))
    sz = np.array(menu, dtype=np.int32)
    ar, ac, nc = rng.choice(sz, 27), rng.choice(sz, 19), rng.choice(sz, 25)
    a = random_bcsr(rng, 27, 19, rbs=ar, cbs=ac, p=0.4) if ta == "N" else random_bcsr(rng, 19, 27, rbs=ac, cbs=ar, p=0.4)
    b = random_bcsr(rng, 19, 25, rbs=ac, cbs=nc, p=0.4) if tb == "N" else random_bcsr(rng, 25, 19, rbs=nc, cbs=ac, p=0.4)
    ref = oracle.multiply(ta, tb, 1.0, a, b)
    host, info = _mul(B, ctx, ta, tb, 1.0, a, b)
    err = _check(host, info, ref)
    _log(f"{ta}{tb} menu={menu}: rel err {err:.2e}")


def test_every_element_placed(B, ctx):
    """A 24 x 24 result from one product of rank-one-free data: every
    element of C = A·B lands in its own place (a lane or register mix-up in
    the edge subtiles would move or drop a value, and the check is exact
    for integer-valued inputs)."""
    rng = np.random.default_rng(7)
    for m, k, n in ((24, 24, 24), (17, 5, 24), (24, 3, 17), (20, 13, 16), (16, 7, 21)):
        a = random_bcsr(rng, 1, 1, rbs=np.array([m], np.int32), cbs=np.array([k], np.int32), p=1.0)
        b = random_bcsr(rng, 1, 1, rbs=np.array([k], np.int32), cbs=np.array([n], np.int32), p=1.0)
        a.values[:] = rng.integers(-8, 9, a.values.size)
        b.values[:] = rng.integers(-8, 9, b.values.size)
        ref = oracle.multiply("N", "N", 1.0, a, b)
        host, info = _mul(B, ctx, "N", "N", 1.0, a, b)
        assert np.array_equal(host.values, ref.values), f"{m}x{k}x{n}"


def test_dft_like_filter_and_c_old(B, ctx):
    a, b, _ = inputs.dft_like_pair(300, config=97, sizes=(5, 13, 23), cutoff=6.0)
    rng = np.random.default_rng(12)
    for eps in (0.0, 1e-6):
        ref = oracle.multiply("N", "N", 1.0, a, b, eps=eps, nthreads=8)
        host, info = _mul(B, ctx, "N", "N", 1.0, a, b, eps=eps)
        _check(host, info, ref)
    c = random_bcsr(rng, a.nbr, b.nbc, p=0.05, rbs=a.rbs, cbs=b.cbs)
    ref = oracle.multiply("N", "N", -0.5, a, b, 1.5, c, nthreads=8)
    host, info = _mul(B, ctx, "N", "N", -0.5, a, b, 1.5, c)
    _check(host, info, ref)
    ref = oracle.multiply("N", "N", 1.0, a, b, 0.5, c, retain_sparsity=True, nthreads=8)
    host, info = _mul(B, ctx, "N", "N", 1.0, a, b, 0.5, c, retain=True)
    _check(host, info, ref)


def test_same_as_other_variants(B, ctx):
    """Variant 4 sums the same products as the 16x16 tiles and the 4x4
    subtiles: results agree to rounding, and each is deterministic."""
    a, b, _ = inputs.dft_like_pair(250, config=98, sizes=(13, 23), cutoff=6.0)
    h4a, _ = _mul(B, ctx, "N", "N", 1.0, a, b)
    h4b, _ = _mul(B, ctx, "N", "N", 1.0, a, b)
    assert np.array_equal(h4a.values, h4b.values)
    for v in (1, 2):
        for m, n in EDGE_CLASSES:
            ctx.set_gemm_variant(m, n, v)
        h, _ = _mul(B, ctx, "N", "N", 1.0, a, b)
        assert np.array_equal(h.col_idx, h4a.col_idx)
        assert rel_fro(h4a.values, h.values) <= 1e-14, f"variant {v}"
