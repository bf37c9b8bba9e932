"""The plan boundary through the C ABI (needs an MI355X): sizes known before
anything of the result is allocated, the numeric part in caller-owned torch
buffers (result bitwise equal to the one-shot multiply), and budget failures
that leave the stream idle and the caller's buffers untouched."""
import sys

import numpy as np
import pytest

from paper_1705_10218_amd import inputs
from _util import random_bcsr, same_pattern

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


def _bits(x):
    return np.ascontiguousarray(x).view(np.uint64)


def _one_shot(B, ctx, A, Bm, eps):
    C, info = B.multiply(ctx, "N", "N", 1.0, A, Bm, filter_eps=eps)
    h = C.to_host()
    C.close()
    return h, info


def _cases():
    rng = np.random.default_rng(820)
    dft_a, dft_b, _ = inputs.dft_like_pair(250, config=8, sizes=(5, 13), cutoff=6.0, decay=1.0)
    big_a, big_b, _ = inputs.dft_like_pair(200, config=8, sizes=(23,), cutoff=6.0)
    r = random_bcsr(rng, 30, 25, p=0.3, max_bs=9)
    s = random_bcsr(rng, 25, 28, r.cbs, None, p=0.3, max_bs=9)
    return [("dft 5/13, post-filter drops", dft_a, dft_b, 1e-3),
            ("dft 5/13, eps 0", dft_a, dft_b, 0.0),
            ("23x23 tile path, eps 1e-10", big_a, big_b, 1e-10),
            ("random 1..9", r, s, 0.0)]


@pytest.mark.parametrize("case", range(4))
def test_execute_into_torch_buffers_equals_one_shot(B, case):
    import torch
    name, a, b, eps = _cases()[case]
    ctx = B.Context(0)
    A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
    ref, rinfo = _one_shot(B, ctx, A, Bm, eps)
    P = B.Plan(ctx, "N", "N", 1.0, A, Bm, filter_eps=eps)
    c_nnzb, c_nval, ws_bytes = P.sizes()
    _log(f"{name}: c_nnzb {c_nnzb} c_values {c_nval} workspace {ws_bytes} B, result nnzb {ref.nnzb}")
    assert c_nnzb == rinfo.c_nnzb_symbolic and c_nnzb >= ref.nnzb and c_nval >= ref.values.size
    dev = f"cuda:{ctx.device}"
    cvals = torch.full((max(c_nval, 1),), float("nan"), dtype=torch.float64, device=dev)
    ws = torch.empty(max(ws_bytes, 256) + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256   # 256-byte aligned view
    wsv = ws[off:off + max(ws_bytes, 256)]
    for rep in range(2):   # twice: the same buffers are reused
        R = P.execute_into(cvals, wsv)
        h = R.to_host()
        assert same_pattern(h, ref), f"pattern differs (run {rep})"
        assert np.array_equal(_bits(h.values), _bits(ref.values)), f"values differ (run {rep})"
        # the result's values are the caller's buffer itself
        assert R.values_ptr() == cvals.data_ptr()
        got = cvals[:h.values.size].cpu().numpy()
        assert np.array_equal(_bits(got), _bits(ref.values))
        R.close()
    # library-owned execution of the same plan gives the same bits
    P.execute()
    R2 = P.result()
    h2 = R2.to_host()
    R2.close()
    assert np.array_equal(_bits(h2.values), _bits(ref.values))
    P.close()
    A.close()
    Bm.close()
    ctx.close()


def test_execute_into_rejects_bad_buffers(B):
    import torch
    rng = np.random.default_rng(821)
    a = random_bcsr(rng, 10, 10, p=0.4, max_bs=6)
    b = random_bcsr(rng, 10, 10, a.cbs, None, p=0.4, max_bs=6)
    ctx = B.Context(0)
    A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
    P = B.Plan(ctx, "N", "N", 1.0, A, Bm)
    _, nval, ws_bytes = P.sizes()
    dev = f"cuda:{ctx.device}"
    ws = torch.empty(ws_bytes + 512, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    cvals = torch.empty(nval, dtype=torch.float64, device=dev)
    with pytest.raises(B.BsmmError) as e:   # misaligned workspace
        P.execute_into(cvals, ws[off + 8:off + 8 + ws_bytes])
    assert e.value.status == 1
    with pytest.raises(B.BsmmError) as e:   # the result over an operand's values
        P.execute_into(A._values, ws[off:off + ws_bytes])
    assert e.value.status == 4
    P.close()
    A.close()
    Bm.close()
    ctx.close()


def test_budget_failures_leave_the_stream_idle(B):
    """A context budget below the plan's needs fails bsmm_plan_create with
    BSMM_ERR_OUT_OF_MEMORY, the stream idle and no plan; a budget that holds
    the plan but not its numeric buffers fails bsmm_plan_execute before any
    launch, while caller buffers (bsmm_plan_execute_into) still work."""
    import torch
    a, b, _ = inputs.dft_like_pair(300, config=8, sizes=(5, 13), cutoff=6.0)
    stream = torch.cuda.Stream()
    # reference result, in a context of its own
    ctxr = B.Context(0, stream=stream)
    Ar, Br = B.Matrix.from_host(ctxr, a), B.Matrix.from_host(ctxr, b)
    ref, _ = _one_shot(B, ctxr, Ar, Br, 0.0)
    Ar.close()
    Br.close()
    ctxr.close()
    # the plan's memory, from an unlimited context: matrices, peak while
    # planning, the plan alone, its numeric buffers
    ctx0 = B.Context(0, stream=stream)
    A0, B0 = B.Matrix.from_host(ctx0, a), B.Matrix.from_host(ctx0, b)
    stream.synchronize()
    held_mats = ctx0.memory()[0]
    P0 = B.Plan(ctx0, "N", "N", 1.0, A0, B0)
    _, nval, ws_bytes = P0.sizes()
    peak_plan = ctx0.memory()[1]
    ctx0.trim()
    held_plan = ctx0.memory()[0]
    P0.close()
    A0.close()
    B0.close()
    ctx0.close()
    _log(f"matrices {held_mats} B, planning peak {peak_plan} B, plan {held_plan} B, "
         f"result values {8 * nval} B, workspace {ws_bytes} B")
    assert held_plan > held_mats
    # 1) budget below the plan
    ctx = B.Context(0, stream=stream, budget_bytes=held_mats + (held_plan - held_mats) // 4)
    A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
    stream.synchronize()
    with pytest.raises(B.BsmmError) as e:
        B.Plan(ctx, "N", "N", 1.0, A, Bm)
    assert e.value.status == 5, e.value
    assert stream.query(), "the stream should be idle after the failure"
    A.close()
    Bm.close()
    ctx.close()
    # 2) budget that holds the plan but not its numeric buffers
    budget = max(peak_plan, held_plan) + (1 << 20)
    if budget >= held_plan + 8 * nval:
        pytest.skip("planning peak leaves no room between the plan and its numeric buffers")
    ctx = B.Context(0, stream=stream, budget_bytes=budget)
    A, Bm = B.Matrix.from_host(ctx, a), B.Matrix.from_host(ctx, b)
    P = B.Plan(ctx, "N", "N", 1.0, A, Bm)
    with pytest.raises(B.BsmmError) as e:
        P.execute()
    assert e.value.status == 5, e.value
    assert stream.query(), "the stream should be idle after the failure"
    dev = f"cuda:{ctx.device}"
    cvals = torch.full((nval,), 7.0, dtype=torch.float64, device=dev)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    torch.cuda.synchronize()
    R = P.execute_into(cvals, ws[off:off + ws_bytes])
    h = R.to_host()
    assert same_pattern(h, ref) and np.array_equal(_bits(h.values), _bits(ref.values))
    R.close()
    P.close()
    A.close()
    Bm.close()
    ctx.close()
