"""Per-unit addressing of the packed operand copies (gemm_path 5), through
the C ABI (needs an MI355X).

With per-unit addressing the packed blocks of every row of op(A) and every
column of op(B) are contiguous and the stack entries hold offsets from
their start, so the copies may exceed 2 GB.  The products and their order
are unchanged, so results must be bitwise those of the default addressing
(every transpose pair, alpha/beta, both filters, retain_sparsity, the
kernel variants, plans and batched plans) and within the FP64 bar of the
oracle.  In automatic mode a product whose copies reach 2 GB (a 128-row
panel of the mixed-size 20,000-atom workload: B alone is 2.3 GB) takes it
by itself; sampled rows are checked against the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1705_10218_amd import inputs
from _util import as_bcsr, random_bcsr, rel_fro

pytestmark = pytest.mark.gpu

TOL = 1e-12
PACKED, UNITS = 0, 5


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


def _run(B, mode, ta, tb, alpha, a, b, beta=0.0, c=None, eps=0.0, retain=False, variants=()):
    ctx = B.Context(0)
    ctx.set_packed_addressing(mode)
    for m, n, v in variants:
        ctx.set_gemm_variant(m, n, v)
    A = B.Matrix.from_host(ctx, a)
    Bm = B.Matrix.from_host(ctx, b)
    C0 = B.Matrix.from_host(ctx, c) if c is not None else None
    C, info = B.multiply(ctx, ta, tb, alpha, A, Bm, beta, C0, eps, retain)
    host = C.to_host()
    for m in (C, A, Bm, C0):
        if m is not None:
            m.close()
    ctx.close()
    return host, info


def _same(h1, h2):
    return (np.array_equal(h1.row_ptr, h2.row_ptr) and np.array_equal(h1.col_idx, h2.col_idx)
            and np.array_equal(h1.values, h2.values))


def _both(B, *args, **kw):
    """Default and per-unit addressing; asserts the paths and equal bits."""
    h0, i0 = _run(B, 0, *args, **kw)
    h1, i1 = _run(B, 1, *args, **kw)
    assert i0.gemm_path == PACKED, f"default addressing ran path {i0.gemm_path}"
    assert i1.gemm_path == UNITS, f"per-unit addressing ran path {i1.gemm_path}"
    assert i0.n_products == i1.n_products and i0.useful_flops == i1.useful_flops
    assert _same(h0, h1), "per-unit addressing changed the result bits"
    return h1, i1


def _check(host, info, ref, tol=TOL):
    assert np.array_equal(host.row_ptr, ref.row_ptr), "row_ptr differs"
    assert np.array_equal(host.col_idx, ref.col_idx), "col_idx differs"
    assert info.n_products == ref.n_products and info.useful_flops == ref.useful_flops
    assert rel_fro(host.values, ref.values) <= tol


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_units_transposes(B, ta, tb):
    a, b, _ = inputs.dft_like_pair(300, config=95, sizes=(5, 13), cutoff=6.0)
    _log(f"units {ta}{tb}: {a.nnzb} x {b.nnzb} blocks")
    host, info = _both(B, ta, tb, 1.0, a, b)
    _check(host, info, oracle.multiply(ta, tb, 1.0, a, b))
    host, info = _both(B, ta, tb, 1.0, a, b, eps=1e-10)   # filters: bitwise against the default


@pytest.mark.parametrize("seed", [0, 1])
def test_units_variants_alpha_beta(B, seed):
    """Sizes {5, 13, 23} with the diagonal-pair, 4x4-subtile and edge-subtile
    variants in force, alpha and beta with C_old."""
    rng = np.random.default_rng(600 + seed)
    sizes = np.array([5, 13, 23], np.int32)
    nb = 40
    bs = rng.choice(sizes, nb).astype(np.int32)
    a = random_bcsr(rng, nb, nb, bs, bs, p=0.3)
    b = random_bcsr(rng, nb, nb, bs, bs, p=0.3)
    c = random_bcsr(rng, nb, nb, bs, bs, p=0.2)
    variants = ((5, 5, 3), (5, 13, 2), (13, 23, 4), (23, 13, 4), (23, 23, 4))
    _log(f"units variants seed={seed}: {a.nnzb} x {b.nnzb} blocks")
    host, info = _both(B, "N", "N", 1.5, a, b, 0.5, c, variants=variants)
    _check(host, info, oracle.multiply("N", "N", 1.5, a, b, 0.5, c))


def test_units_retain_sparsity(B):
    rng = np.random.default_rng(610)
    bs = rng.choice(np.array([5, 13], np.int32), 30).astype(np.int32)
    a = random_bcsr(rng, 30, 30, bs, bs, p=0.35)
    b = random_bcsr(rng, 30, 30, bs, bs, p=0.35)
    c = random_bcsr(rng, 30, 30, bs, bs, p=0.25)
    host, info = _both(B, "N", "N", 1.0, a, b, 0.75, c, retain=True)
    _check(host, info, oracle.multiply("N", "N", 1.0, a, b, 0.75, c, retain_sparsity=True))


def test_units_plan_reexecutes_and_batches(B):
    """A per-unit plan re-executed on new values equals a one-shot multiply
    with the default addressing; in one batch with a default-addressed plan,
    both equal their results alone."""
    import torch
    a, b, _ = inputs.dft_like_pair(250, config=96, sizes=(5, 13), cutoff=6.0)
    ctx = B.Context(0)
    A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
    ctx.set_packed_addressing(1)
    pu = B.Plan(ctx, "N", "N", 1.0, A, Bm)
    ctx.set_packed_addressing(0)
    p0 = B.Plan(ctx, "N", "T", 1.0, A, Bm)
    assert pu.info.gemm_path == UNITS and p0.info.gemm_path == PACKED
    for step in range(2):
        A._values.mul_(-0.75).add_(0.125)   # new values, same pattern
        torch.cuda.synchronize()
        pu.execute()
        got = pu.result().to_host()
        want, _ = B.multiply(ctx, "N", "N", 1.0, A, Bm)
        assert _same(got, want.to_host()), f"step {step}"
        want.close()
    B.plans_execute([pu, p0])
    got_u, got_0 = pu.result().to_host(), p0.result().to_host()
    want_u, _ = B.multiply(ctx, "N", "N", 1.0, A, Bm)
    want_0, _ = B.multiply(ctx, "N", "T", 1.0, A, Bm)
    assert _same(got_u, want_u.to_host()) and _same(got_0, want_0.to_host())
    for m in (want_u, want_0):
        m.close()
    pu.close()
    p0.close()
    A.close()
    Bm.close()
    ctx.close()


def test_units_mode_rejected(B):
    ctx = B.Context(0)
    for mode in (-1, 2):
        with pytest.raises(B.BsmmError) as e:
            ctx.set_packed_addressing(mode)
        assert e.value.status == 1   # BSMM_ERR_INVALID_ARG
    ctx.close()


def test_units_automatic_past_2gb(B):
    """Copies above 2 GB: the default mode addresses them per unit; a seeded
    6 of the 128 result rows against the oracle."""
    pb = inputs.batching_problem(20000, 0.03, sizes=(5, 13, 23))
    a = inputs.batching_matrix(pb, 1, (0, 128))
    b = inputs.batching_matrix(pb, 2, None, row_mask=inputs.reachable_rows(a, pb.n))
    assert b.values.nbytes >= (1 << 31)
    _log(f"units past 2 GB: A {a.nnzb} blocks, B {b.nnzb} blocks ({b.values.nbytes / 1e9:.2f} GB)")
    host, info = _run(B, 0, "N", "N", 1.0, a, b, eps=1e-10)
    assert info.gemm_path == UNITS
    rows = np.sort(np.random.default_rng(7).choice(128, 6, replace=False)).astype(np.int32)
    ref = oracle.multiply("N", "N", 1.0, a, b, eps=1e-10, nthreads=8, rows=rows)
    go, ro = as_bcsr(host).block_offsets(), as_bcsr(ref).block_offsets()
    num = den = 0.0
    for i in rows:
        g0, g1 = host.row_ptr[i], host.row_ptr[i + 1]
        r0, r1 = ref.row_ptr[i], ref.row_ptr[i + 1]
        assert np.array_equal(host.col_idx[g0:g1], ref.col_idx[r0:r1]), f"row {i} pattern"
        d = host.values[go[g0]:go[g1]] - ref.values[ro[r0]:ro[r1]]
        num += float(d @ d)
        den += float(ref.values[ro[r0]:ro[r1]] @ ref.values[ro[r0]:ro[r1]])
    assert den > 0 and (num / den) ** 0.5 <= TOL


def test_units_graph_replays(B):
    """A per-unit plan captured in a HIP graph: every replay, with eager work
    on the stream between replays, equals a one-shot multiply."""
    import torch
    st = torch.cuda.Stream()   # default priority; graphs need a non-default stream
    with torch.cuda.stream(st):
        ctx = B.Context(0, stream=st)
        ctx.set_packed_addressing(1)
        a, b, _ = inputs.dft_like_pair(250, config=97, sizes=(5, 13), cutoff=6.0)
        A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
        st.synchronize()
        plan = B.Plan(ctx, "N", "N", 1.0, A, Bm)
        assert plan.info.gemm_path == UNITS
        plan.capture()
        for rep in range(3):
            A._values.mul_(1.5).sub_(0.25)
            plan.execute()   # graph replay
            got = plan.result().to_host()
            st.synchronize()
            want_m, _ = B.multiply(ctx, "N", "N", 1.0, A, Bm)
            assert _same(got, want_m.to_host()), f"replay {rep}"
            want_m.close()
        plan.close()
        A.close()
        Bm.close()
        ctx.close()


def test_units_sign_iteration(B):
    """The sign iteration (eq. (3)) with every product addressed per unit
    gives the bits of the default addressing."""
    x = inputs.symmetric_dft_like(200, config=6, sizes=(5, 13), cutoff=5.0)
    out = []
    for mode in (0, 1):
        ctx = B.Context(0)
        ctx.set_packed_addressing(mode)
        X = B.Matrix.from_host(ctx, x)
        Y, info, res, nnz = B.sign_newton_schulz(ctx, X, 6, 1e-8, 0.0)
        out.append((Y.to_host(), list(res), list(nnz)))
        Y.close()
        X.close()
        ctx.close()
    (h0, r0, n0), (h1, r1, n1) = out
    assert n0 == n1 and r0 == r1 and _same(h0, h1)


@pytest.mark.parametrize("seed", [0, 1])
def test_units_edges_to_32_and_empty_units(B, seed):
    """Block edges up to 32 (the widest kernel instance), empty rows of
    op(A) and empty columns of op(B) (units with no packed block), and a
    transposed op(B)."""
    rng = np.random.default_rng(620 + seed)
    nbr, nk, nbc = 30, 26, 34
    ks = rng.choice(np.array([3, 9, 17, 25, 29, 32], np.int32), nk)   # at most 8 k sizes: the packed path
    a = random_bcsr(rng, nbr, nk, rng.integers(1, 33, nbr).astype(np.int32), ks, p=0.3, empty_rows=(0, 7, 19))
    bt = random_bcsr(rng, nbc, nk, rng.integers(1, 33, nbc).astype(np.int32), ks, p=0.3, empty_rows=(3, 11))
    _log(f"units edges to 32 seed={seed}: {a.nnzb} x {bt.nnzb} blocks")
    host, info = _both(B, "N", "T", 0.75, a, bt)
    _check(host, info, oracle.multiply("N", "T", 0.75, a, bt))
