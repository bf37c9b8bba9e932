"""Autotuner table handling (CPU) and GEMM kernel variants vs the oracle (GPU)."""
import json

import numpy as np
import pytest

import oracle
from paper_1705_10218_amd import autotune, inputs
from _util import rel_fro


def test_size_classes():
    assert [autotune.size_class(e) for e in (1, 8, 9, 16, 17, 24, 25, 32)] == [0, 0, 1, 1, 2, 2, 3, 3]
    with pytest.raises(ValueError):
        autotune.size_class(33)


def test_apply_sets_every_class(tmp_path):
    calls = []

    class FakeCtx:
        def set_gemm_variant(self, m, n, v):
            calls.append((autotune.size_class(m), autotune.size_class(n), v))

        def set_tile_shape(self, ti, tj):
            calls.append(("shape", ti, tj))

        def set_tile_schedule(self, persistent, chunk):
            calls.append(("chunk", persistent, chunk))

    t1 = {"sizes": [5, 23], "classes": [{"m_class": 0, "n_class": 2, "variant": 1},
                                        {"m_class": 2, "n_class": 2, "variant": 2}]}
    t2 = {"sizes": [13], "classes": [{"m_class": 1, "n_class": 1, "variant": 2}]}
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"tables": [t2, t1]}))
    assert autotune.apply(FakeCtx(), str(p), sizes=(23, 5)) == 2
    assert calls == [(0, 2, 1), (2, 2, 2), ("shape", 2, 2), ("chunk", False, 0)]   # no tile entry: defaults
    calls.clear()
    assert autotune.apply(FakeCtx(), str(p), sizes=(5, 13)) == 0   # no table for that set
    assert calls == []
    assert autotune.apply(FakeCtx(), t2) == 1 and calls[0] == (1, 1, 2)


def test_apply_sets_the_tile_schedule():
    calls = []

    class FakeCtx:
        def set_gemm_variant(self, m, n, v):
            calls.append(("variant", m, n, v))

        def set_tile_shape(self, ti, tj):
            calls.append(("shape", ti, tj))

        def set_tile_schedule(self, persistent, chunk):
            calls.append(("chunk", persistent, chunk))

    t = {"sizes": [23], "classes": [{"m_class": 2, "n_class": 2, "m": 23, "n": 23, "variant": 5,
                                     "variant_name": "tile_path_lds_staged"}],
         "tile": {"m": 23, "n": 23, "variant": 5, "shape": [2, 2], "xcd_chunk": 2048}}
    assert autotune.apply(FakeCtx(), t) == 1
    assert calls == [("variant", 17, 17, 5), ("shape", 2, 2), ("chunk", False, 2048)]
    d = autotune.describe({"tables": [t]}, (23,))
    assert "23x23: tile_path_lds_staged" in d and "2048 tiles per XCD chunk" in d
    assert autotune.describe({"tables": [t]}, (5,)).startswith("default")


def test_class_workload_shapes():
    a, b = autotune.class_workload(13, 23, (5, 13), atoms=200, cutoff=5.0)
    assert set(a.rbs.tolist()) == {13} and set(b.cbs.tolist()) == {23}
    assert np.array_equal(a.cbs, b.rbs)


def test_variant_edges():
    """Which variants exist for which block edges (as the library checks)."""
    assert autotune.applies(3, 8, 5) and not autotune.applies(3, 9, 5)
    assert autotune.applies(4, 13, 23) and autotune.applies(4, 24, 9) and autotune.applies(4, 17, 17)
    assert not autotune.applies(4, 16, 16) and not autotune.applies(4, 5, 23) and not autotune.applies(4, 25, 23)
    assert all(autotune.applies(v, m, n) for v in (1, 2) for m in (1, 32) for n in (1, 32))
    # the tile-path variants only for sets whose sizes all lie in 17..24
    assert autotune.applies(5, 23, 23, (23,)) and autotune.applies(6, 17, 24, (17, 24))
    assert not autotune.applies(5, 23, 23, (5, 13, 23)) and not autotune.applies(6, 23, 23)


@pytest.mark.gpu
def test_variants_agree_with_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1705_10218_amd import bsmm
    a, b, _ = inputs.dft_like_pair(400, config=92, sizes=(5, 13, 23), cutoff=6.0)
    ref = oracle.multiply("N", "N", 1.0, a, b, nthreads=8)
    ctx = bsmm.Context(0)
    A = bsmm.Matrix.from_host(ctx, a)
    B = bsmm.Matrix.from_host(ctx, b)
    results = {}
    for v in (0, 1, 2, 3, 4):
        for m in (5, 13, 23, 32):
            for n in (5, 13, 23, 32):   # variants 3 and 4 exist for some edges only
                ctx.set_gemm_variant(m, n, v if autotune.applies(v, m, n) else 0)
        C, info = bsmm.multiply(ctx, "N", "N", 1.0, A, B)
        h = C.to_host()
        C.close()
        assert np.array_equal(h.col_idx, ref.col_idx) and np.array_equal(h.row_ptr, ref.row_ptr)
        err = rel_fro(h.values, ref.values)
        print(f"variant {v}: rel err {err:.2e}, gemm {info.ms_gemm:.3f} ms", flush=True)
        assert err <= 1e-12
        results[v] = h.values
    A.close()
    B.close()
    ctx.close()


def test_schedule_keeps_the_default_within_the_margin():
    d = autotune.DEFAULT_SCHEDULE
    assert autotune.pick_schedule({d: 10.0, ((2, 2), 2048): 9.9}) == d          # 1 % faster: noise
    assert autotune.pick_schedule({d: 10.0, ((2, 2), 2048): 9.5}) == ((2, 2), 2048)
    assert autotune.pick_schedule({((2, 4), 2048): 9.0, ((4, 4), 8192): 8.0}) == ((4, 4), 8192)
