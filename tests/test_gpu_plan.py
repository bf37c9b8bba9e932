"""Plans: structural part once, numeric part re-executed on new values, and
the numeric part replayed from a HIP graph (needs an MI355X).

A plan's numeric part runs the same kernels on the same stacks as a one-shot
multiplication, so its result must be bitwise equal to bsmm_multiply on the
same values whenever the filter decisions are the same (always at eps = 0).
Graph replays are checked one by one against the eager result, with eager
work and synchronisations between them.
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
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.fixture(scope="module")
def B(torch_mod):
    from paper_1705_10218_amd import bsmm
    return bsmm


def _same(h1, h2):
    return (np.array_equal(h1.row_ptr, h2.row_ptr) and np.array_equal(h1.col_idx, h2.col_idx)
            and np.array_equal(h1.values, h2.values))


@pytest.mark.parametrize("eps,beta", [(0.0, 0.0), (1e-10, 0.0), (0.0, 0.5), (1e-3, 0.0)])
def test_plan_equals_multiply(B, eps, beta):
    ctx = B.Context(0)
    a, b, _ = inputs.dft_like_pair(300, config=93, sizes=(5, 13), cutoff=6.0, decay=1.0 if eps >= 1e-3 else 2.0)
    A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
    C0 = None
    if beta != 0.0:
        c0, _ = B.multiply(ctx, "N", "T", 1.0, A, Bm)   # any matrix of C's block sizes
        C0 = c0
    want, winfo = B.multiply(ctx, "N", "N", 1.25, A, Bm, beta, C0, eps)
    plan = B.Plan(ctx, "N", "N", 1.25, A, Bm, beta, C0, eps)
    assert plan.info.n_products == winfo.n_products and plan.info.useful_flops == winfo.useful_flops
    plan.execute()
    got = plan.result()
    assert _same(got.to_host(), want.to_host())
    for m in (got, want):
        m.close()
    plan.close()
    for m in (C0, A, Bm):
        if m is not None:
            m.close()
    ctx.close()


def test_plan_reexecutes_on_new_values(B, torch_mod):
    ctx = B.Context(0)
    a, b, _ = inputs.dft_like_pair(250, config=94, sizes=(5, 13), cutoff=6.0)
    A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
    plan = B.Plan(ctx, "N", "N", 1.0, A, Bm)
    for step in range(3):
        A._values.mul_(-0.75).add_(0.125)   # new values, same pattern
        torch_mod.cuda.synchronize()
        plan.execute()
        got = plan.result().to_host()
        want_m, _ = B.multiply(ctx, "N", "N", 1.0, A, Bm)
        assert _same(got, want_m.to_host()), f"step {step}"
        want_m.close()
    ha = A.to_host()
    ref = oracle.multiply("N", "N", 1.0, ha, b)
    assert rel_fro(got.values, ref.values) <= 1e-12
    plan.close()
    A.close()
    Bm.close()
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_graph_replays_match_eager(B, torch_mod, mode):
    torch = torch_mod
    st = torch.cuda.Stream()   # default priority; graphs need a non-default stream
    with torch.cuda.stream(st):
        ctx = B.Context(0, stream=st)
        ctx.set_compute_mode(mode)
        a, b, _ = inputs.dft_like_pair(250, config=95, sizes=(5, 13), cutoff=6.0)
        A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
        st.synchronize()
        plan = B.Plan(ctx, "N", "N", 1.0, A, Bm)
        plan.capture()
        for rep in range(4):
            A._values.mul_(1.5).sub_(0.25)   # eager work on the same stream between replays
            Bm._values.mul_(-1.0)
            plan.execute()                   # graph replay
            got = plan.result().to_host()
            st.synchronize()
            want_m, _ = B.multiply(ctx, "N", "N", 1.0, A, Bm)
            want = want_m.to_host()
            want_m.close()
            _log(f"mode {mode} replay {rep}: max |diff| {np.max(np.abs(got.values - want.values)):.3e}")
            assert _same(got, want), f"replay {rep}"
        plan.close()
        A.close()
        Bm.close()
        ctx.close()


def test_capture_needs_a_stream(B):
    ctx = B.Context(0)
    a, b, _ = inputs.dft_like_pair(120, config=96, sizes=(5,), cutoff=5.0)
    A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
    plan = B.Plan(ctx, "N", "N", 1.0, A, Bm)
    assert ctx.stream.cuda_stream == 0   # the default stream cannot be captured
    with pytest.raises(B.BsmmError) as e:
        plan.capture()
    assert e.value.status == 7
    plan.close()
    A.close()
    Bm.close()
    ctx.close()


def test_plan_filter_holds(B, torch_mod):
    """bsmm_plan_filter_holds against fresh multiplies: unchanged values;
    blocks scaled by 1e3 and 1e-3 where every product stays on its side of
    the threshold (the norm-ratio bound is then inconclusive and every
    candidate is decided again: the decisions hold, and re-executing the
    plan gives a fresh multiply's bits); and a block scaled so that one of
    its products crosses the threshold (the decisions do not hold)."""
    from _util import random_bcsr
    torch = torch_mod
    rng = np.random.default_rng(730)
    a = random_bcsr(rng, 30, 26, p=0.3, max_bs=6)
    b = random_bcsr(rng, 26, 28, a.cbs, None, p=0.3, max_bs=6)
    off, rows = a.block_offsets(), a.block_rows()
    for p in range(a.nnzb):
        a.values[off[p]:off[p + 1]] *= 10.0 ** (-(rows[p] % 7))
    na, nb = oracle.block_norms(a), oracle.block_norms(b)
    # products per A block (stored id) through its column k
    a_col, b_rows = a.col_idx, b.block_rows()
    prod = {p: na[p] * nb[b_rows == a_col[p]] for p in range(a.nnzb)}
    allp = np.sort(np.concatenate([v for v in prod.values() if v.size]))
    eps = float(0.5 * (allp[len(allp) // 2] + allp[len(allp) // 2 + 1]))
    assert np.min(np.abs(allp - eps)) > 1e-6 * eps
    hi = [p for p, v in prod.items() if v.size and v.min() >= eps]     # every product kept: stays kept when scaled up
    lo = [p for p, v in prod.items() if v.size and v.max() < eps]      # every product dropped: stays dropped when scaled down
    near = [p for p, v in prod.items() if v.size and np.any((v >= eps) & (v < 1.5 * eps))]
    assert hi and lo and near, (len(hi), len(lo), len(near))
    ctx = B.Context(0)
    A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
    plan = B.Plan(ctx, "N", "N", 1.0, A, Bm, filter_eps=eps)
    assert plan.filter_holds()   # values as planned

    def block(p):
        return A._values[int(off[p]):int(off[p + 1])]

    # kept products scaled up and dropped ones scaled down: same decisions
    block(hi[0]).mul_(1e3)
    block(lo[0]).mul_(1e-3)
    torch.cuda.synchronize()
    assert plan.filter_holds()
    plan.execute()
    got = plan.result()
    want, winfo = B.multiply(ctx, "N", "N", 1.0, A, Bm, filter_eps=eps)
    assert _same(got.to_host(), want.to_host())
    assert winfo.n_products == plan.info.n_products
    got.close()
    want.close()
    # a product just above the threshold falls below it
    block(near[0]).mul_(0.5)
    torch.cuda.synchronize()
    assert not plan.filter_holds()
    want, winfo = B.multiply(ctx, "N", "N", 1.0, A, Bm, filter_eps=eps)
    assert winfo.n_products < plan.info.n_products
    want.close()
    plan.close()
    A.close()
    Bm.close()
    ctx.close()
