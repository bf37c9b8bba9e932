"""FP32 and split-FP32 compute modes vs the FP64 CPU oracle (needs an MI355X).

Bar: the block pattern, product counts and useful flops equal the oracle's
exactly (norms and thresholds stay FP64, so every filter decision is the
FP64 one); values within relative Frobenius error 1e-5 for FP32 and 1e-6
for split-FP32 (FP32 hi + lo operands, FP64 accumulation across k), and the
split form is never less accurate than plain FP32 on the same input.  Each
step's MFMA result is an FP32 number, so split keeps an error of about
2^-24 relative per step: it does not grow with the number of k-steps (plain
FP32 accumulation grows like its square root), but it does not reach FP64.
The measured errors are printed.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1705_10218_amd import inputs
from _util import random_bcsr, rel_fro

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split": 1e-6}
MODES = {"fp64": 0, "fp32": 1, "split": 2}


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
    yield c
    c.close()


def _mul(B, ctx, mode, ta, tb, alpha, a, b, beta=0.0, c=None, eps=0.0):
    ctx.set_compute_mode(MODES[mode])
    A = B.Matrix.from_host(ctx, a)
    Bm = B.Matrix.from_host(ctx, b)
    C0 = B.Matrix.from_host(ctx, c) if c is not None else None
    C, info = B.multiply(ctx, ta, tb, alpha, A, Bm, beta, C0, eps, False)
    host = C.to_host()
    for m in (C, A, Bm, C0):
        if m is not None:
            m.close()
    ctx.set_compute_mode(0)
    return host, info


def _check(host, info, ref, mode):
    assert np.array_equal(host.row_ptr, ref.row_ptr)
    assert np.array_equal(host.col_idx, ref.col_idx)
    assert info.n_products == ref.n_products
    assert info.useful_flops == ref.useful_flops
    err = rel_fro(host.values, ref.values) if ref.values.size else 0.0
    assert err <= TOL[mode], f"{mode}: relative Frobenius error {err:.3e}"
    return err


# block-size menus: the low-precision kernels run on the quad path, which
# takes at most 8 distinct contraction block sizes
MENUS = {7: [1, 2, 3, 4, 5, 6, 7], 16: [1, 2, 5, 8, 9, 13, 15, 16], 32: [1, 5, 13, 16, 17, 23, 29, 32]}


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
@pytest.mark.parametrize("max_bs", [7, 16, 32])
def test_random_grids(B, ctx, ta, tb, max_bs):
    rng = np.random.default_rng(100 + max_bs)
    menu = np.array(MENUS[max_bs], dtype=np.int32)
    ar, ac, nc = rng.choice(menu, 23), rng.choice(menu, 19), rng.choice(menu, 17)
    if ta == "N":   # op(A) = A: 23 x 19 blocks
        a = random_bcsr(rng, 23, 19, rbs=ar, cbs=ac, p=0.35)
    else:           # op(A) = A^T: A is 19 x 23
        a = random_bcsr(rng, 19, 23, rbs=ac, cbs=ar, p=0.35)
    if tb == "N":   # op(B) = B: 19 x 17
        b = random_bcsr(rng, 19, 17, rbs=ac, cbs=nc, p=0.35)
    else:
        b = random_bcsr(rng, 17, 19, rbs=nc, cbs=ac, p=0.35)
    ref = oracle.multiply(ta, tb, 1.0, a, b)
    errs = {}
    for mode in ("fp32", "split"):
        host, info = _mul(B, ctx, mode, ta, tb, 1.0, a, b)
        errs[mode] = _check(host, info, ref, mode)
    _log(f"{ta}{tb} max_bs={max_bs}: fp32 {errs['fp32']:.2e} split {errs['split']:.2e}")
    assert errs["split"] <= errs["fp32"]


def test_dft_like_and_filters(B, ctx):
    a, b, _ = inputs.dft_like_pair(700, config=90, sizes=(5, 13), cutoff=7.0)
    for eps in (0.0, 1e-10):
        ref = oracle.multiply("N", "N", 1.0, a, b, eps=eps, nthreads=8)
        errs = {}
        for mode in ("fp32", "split"):
            host, info = _mul(B, ctx, mode, "N", "N", 1.0, a, b, eps=eps)
            errs[mode] = _check(host, info, ref, mode)
        _log(f"dft-like 700 atoms eps={eps}: fp32 {errs['fp32']:.2e} split {errs['split']:.2e}")
        assert errs["split"] <= errs["fp32"]


def test_alpha_beta_c_old(B, ctx):
    rng = np.random.default_rng(7)
    sz = rng.choice(np.array([5, 13], dtype=np.int32), 20)
    a = random_bcsr(rng, 20, 20, p=0.3, rbs=sz, cbs=sz)
    b = random_bcsr(rng, 20, 20, p=0.3, rbs=sz, cbs=sz)
    c = random_bcsr(rng, 20, 20, p=0.3, rbs=sz, cbs=sz)
    ref = oracle.multiply("N", "N", -0.75, a, b, beta=1.5, c=c)
    for mode in ("fp32", "split"):
        host, info = _mul(B, ctx, mode, "N", "N", -0.75, a, b, beta=1.5, c=c)
        _check(host, info, ref, mode)


def test_deterministic_and_mode_switch(B, ctx):
    a, b, _ = inputs.dft_like_pair(300, config=91, sizes=(5, 13), cutoff=7.0)
    h64a, _ = _mul(B, ctx, "fp64", "N", "N", 1.0, a, b)
    for mode in ("fp32", "split"):
        x, _ = _mul(B, ctx, mode, "N", "N", 1.0, a, b)
        y, _ = _mul(B, ctx, mode, "N", "N", 1.0, a, b)
        assert np.array_equal(x.values, y.values), f"{mode} not deterministic"
    h64b, _ = _mul(B, ctx, "fp64", "N", "N", 1.0, a, b)
    assert np.array_equal(h64a.values, h64b.values), "FP64 result changed after a mode switch"
