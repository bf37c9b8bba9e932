"""Newton-Schulz sign iteration on the GPU vs the oracle's iteration (needs an MI355X).

Same starting matrix, same iteration count and filter: the block counts
after every step and the final pattern equal the oracle's exactly, the
residual traces agree to 1e-9 relative, the final values within relative
Frobenius error 1e-11 (FP64 rounding differences compound over the steps).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1705_10218_amd import inputs
from _util import rel_fro

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


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c


def _run(B, ctx, x, n, eps, tol):
    X = B.Matrix.from_host(ctx, x)
    Y, info, res, nnz = B.sign_newton_schulz(ctx, X, n, eps, tol)
    host = Y.to_host()
    Y.close()
    X.close()
    return host, info, res, nnz


@pytest.mark.parametrize("case", [
    dict(atoms=80, sizes=(2, 3), cutoff=4.0, n=8, eps=0.0, tol=0.0),
    dict(atoms=150, sizes=(5, 13), cutoff=5.0, n=6, eps=0.0, tol=0.0),
    dict(atoms=150, sizes=(5, 13), cutoff=5.0, n=12, eps=1e-8, tol=1e-9),
    dict(atoms=300, sizes=(5, 13, 23), cutoff=6.0, n=5, eps=1e-6, tol=0.0),
])
def test_matches_oracle_iteration(B, ctx, case):
    x = inputs.symmetric_dft_like(case["atoms"], config=6, sizes=case["sizes"], cutoff=case["cutoff"])
    _log(f"sign iteration {case}")
    ref, rres, rnnz, rconv, rflops = oracle.newton_schulz(x, case["n"], eps=case["eps"], tol=case["tol"], nthreads=8)
    host, info, res, nnz = _run(B, ctx, x, case["n"], case["eps"], case["tol"])
    assert info.iterations == len(rres) and bool(info.converged) == rconv
    assert np.array_equal(nnz, rnnz)
    assert np.max(np.abs(res - rres) / np.maximum(rres, 1e-300)) <= 1e-9
    assert np.array_equal(host.row_ptr, ref.row_ptr) and np.array_equal(host.col_idx, ref.col_idx)
    err = rel_fro(host.values, ref.values)
    _log(f"  iterations {info.iterations} residual {info.residual:.3e} rel err {err:.2e} nnzb {nnz.tolist()} "
         f"plan reuses {info.plan_reuses}")
    assert err <= 1e-11
    assert info.useful_flops == rflops
    assert info.nnzb == host.row_ptr[-1]


@pytest.mark.parametrize("eps,reuse", [(0.0, True), (1e-8, True), (1e-4, None)])
def test_plan_reuse_on_settled_pattern(B, ctx, eps, reuse):
    """Once the pattern of X settles, the multiplications re-execute the
    previous step's plans (eps > 0: only where every filter decision is the
    same under the new norms -- by the norm-ratio bound, else by deciding
    every candidate again; at 1e-4 whether they hold depends on the
    iterates); the iteration equals the oracle's, step by step, either way."""
    x = inputs.symmetric_dft_like(120, config=6, sizes=(5, 13), cutoff=5.0, request=2)
    n = 10
    ref, rres, rnnz, rconv, rflops = oracle.newton_schulz(x, n, eps=eps, tol=0.0, nthreads=8)
    host, info, res, nnz = _run(B, ctx, x, n, eps, 0.0)
    _log(f"  eps {eps}: plan reuses {info.plan_reuses} of {2 * info.iterations}, nnzb {nnz.tolist()}")
    if reuse:
        assert info.plan_reuses > 0, "the pattern settles: the plans should be re-executed"
    assert np.array_equal(nnz, rnnz)
    assert np.max(np.abs(res - rres) / np.maximum(rres, 1e-300)) <= 1e-9
    assert np.array_equal(host.row_ptr, ref.row_ptr) and np.array_equal(host.col_idx, ref.col_idx)
    assert rel_fro(host.values, ref.values) <= 1e-11
    assert info.useful_flops == rflops


def test_zero_iterations_copy(B, ctx):
    x = inputs.symmetric_dft_like(80, config=6, sizes=(2, 3), cutoff=4.0, request=1)
    host, info, res, nnz = _run(B, ctx, x, 0, 0.0, 0.0)
    assert info.iterations == 0 and res.size == 0
    assert np.array_equal(host.values, x.values) and np.array_equal(host.col_idx, x.col_idx)


def test_rejects_non_square(B, ctx):
    rng = np.random.default_rng(0)
    from _util import random_bcsr
    a = random_bcsr(rng, 5, 6, p=0.5)
    X = B.Matrix.from_host(ctx, a)
    with pytest.raises(B.BsmmError) as e:
        B.sign_newton_schulz(ctx, X, 3)
    assert e.value.status == 3
    X.close()
