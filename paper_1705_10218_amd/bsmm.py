"""Thin ctypes binding of libbsmm.so (the C ABI declared in include/bsmm.h).

Argument marshalling only: every step of a multiplication runs in the
library's HIP kernels.  PyTorch supplies device memory (value buffers) and
the stream the library enqueues on.  The names follow the C entry points
without their ``bsmm_`` prefix (``multiply`` -> ``bsmm_multiply`` ...).

Loading fails loudly when the library has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsmm.so")

OK = 0
STATUS = {
    0: "BSMM_OK", 1: "BSMM_ERR_INVALID_ARG", 2: "BSMM_ERR_BAD_INDEX", 3: "BSMM_ERR_SHAPE",
    4: "BSMM_ERR_ALIAS", 5: "BSMM_ERR_OUT_OF_MEMORY", 6: "BSMM_ERR_DEVICE", 7: "BSMM_ERR_UNSUPPORTED",
}
COMPUTE_FP64, COMPUTE_FP32, COMPUTE_SPLIT = 0, 1, 2

# every symbol include/bsmm.h declares
SYMBOLS = (
    "bsmm_status_string", "bsmm_last_error", "bsmm_ctx_create", "bsmm_ctx_set_stream",
    "bsmm_ctx_set_timing", "bsmm_ctx_set_compute_mode", "bsmm_ctx_set_gemm_variant", "bsmm_ctx_memory",
    "bsmm_ctx_trim",
    "bsmm_ctx_synchronize", "bsmm_ctx_destroy", "bsmm_mat_create", "bsmm_mat_info",
    "bsmm_mat_get_index", "bsmm_mat_get_block_sizes", "bsmm_mat_values", "bsmm_mat_copy_values",
    "bsmm_mat_destroy", "bsmm_block_norms", "bsmm_multiply", "bsmm_filter", "bsmm_sign_newton_schulz",
    "bsmm_plan_create", "bsmm_plan_execute", "bsmm_plan_capture", "bsmm_plan_result", "bsmm_plan_destroy",
    "bsmm_plans_execute", "bsmm_filter_noalloc", "bsmm_ctx_set_tile_shape", "bsmm_plan_sizes",
    "bsmm_plan_execute_into", "bsmm_ctx_set_tile_schedule", "bsmm_plan_filter_holds",
    "bsmm_ctx_set_packed_addressing", "bsmm_ctx_set_row_order",
)


class BsmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class MultiplyInfo(ctypes.Structure):
    _fields_ = [
        ("c_nnzb_symbolic", ctypes.c_int64), ("c_nnzb", ctypes.c_int64), ("c_n_values", ctypes.c_int64),
        ("n_candidates", ctypes.c_int64), ("n_products", ctypes.c_int64), ("useful_flops", ctypes.c_double),
        ("ms_index", ctypes.c_float), ("ms_norms", ctypes.c_float), ("ms_symbolic", ctypes.c_float),
        ("ms_stacks", ctypes.c_float), ("ms_gemm", ctypes.c_float), ("ms_filter", ctypes.c_float),
        ("ms_total", ctypes.c_float), ("gemm_path", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class SignInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("residual", ctypes.c_double),
        ("nnzb", ctypes.c_int64), ("nnzb_max", ctypes.c_int64), ("useful_flops", ctypes.c_double),
        ("ms_total", ctypes.c_float), ("plan_reuses", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


def lib() -> ctypes.CDLL:
    """The loaded libbsmm.so; raises if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                               "g.build()'` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        L.bsmm_status_string.restype = ctypes.c_char_p
        L.bsmm_status_string.argtypes = [ctypes.c_int]
        L.bsmm_last_error.restype = ctypes.c_char_p
        L.bsmm_last_error.argtypes = []
        for name in SYMBOLS[2:]:
            getattr(L, name).restype = ctypes.c_int
        L.bsmm_ctx_create.argtypes = [ctypes.c_int, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]
        L.bsmm_ctx_set_stream.argtypes = [_vp, _vp]
        L.bsmm_ctx_set_timing.argtypes = [_vp, ctypes.c_int]
        L.bsmm_ctx_set_compute_mode.argtypes = [_vp, ctypes.c_int]
        L.bsmm_ctx_set_gemm_variant.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.bsmm_ctx_set_tile_shape.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
        L.bsmm_ctx_set_tile_schedule.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64]
        L.bsmm_ctx_set_packed_addressing.argtypes = [_vp, ctypes.c_int32]
        L.bsmm_ctx_set_row_order.argtypes = [_vp, ctypes.c_int32]
        L.bsmm_ctx_memory.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
        L.bsmm_ctx_trim.argtypes = [_vp]
        L.bsmm_ctx_synchronize.argtypes = [_vp]
        L.bsmm_ctx_destroy.argtypes = [_vp]
        L.bsmm_mat_create.argtypes = [_vp, _i32, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _i64, ctypes.POINTER(_vp)]
        L.bsmm_mat_info.argtypes = [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                                    ctypes.POINTER(_i64)]
        L.bsmm_mat_get_index.argtypes = [_vp, _vp, _vp]
        L.bsmm_mat_get_block_sizes.argtypes = [_vp, _vp, _vp]
        L.bsmm_mat_values.argtypes = [_vp, ctypes.POINTER(_vp)]
        L.bsmm_mat_copy_values.argtypes = [_vp, _vp]
        L.bsmm_mat_destroy.argtypes = [_vp]
        L.bsmm_block_norms.argtypes = [_vp, _vp]
        L.bsmm_multiply.argtypes = [_vp, ctypes.c_char, ctypes.c_char, ctypes.c_double, _vp, _vp, ctypes.c_double,
                                    _vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_vp),
                                    ctypes.POINTER(MultiplyInfo)]
        L.bsmm_filter.argtypes = [_vp, ctypes.c_double, ctypes.POINTER(_vp)]
        L.bsmm_filter_noalloc.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp]
        L.bsmm_plan_create.argtypes = [_vp, ctypes.c_char, ctypes.c_char, ctypes.c_double, _vp, _vp,
                                       ctypes.c_double, _vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_vp),
                                       ctypes.POINTER(MultiplyInfo)]
        L.bsmm_plan_execute.argtypes = [_vp]
        L.bsmm_plan_sizes.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_size_t)]
        L.bsmm_plan_filter_holds.argtypes = [_vp, ctypes.POINTER(_i32)]
        L.bsmm_plan_execute_into.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_vp)]
        L.bsmm_plan_capture.argtypes = [_vp]
        L.bsmm_plan_result.argtypes = [_vp, ctypes.POINTER(_vp)]
        L.bsmm_plan_destroy.argtypes = [_vp]
        L.bsmm_plans_execute.argtypes = [ctypes.c_int32, ctypes.POINTER(_vp)]
        L.bsmm_sign_newton_schulz.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                              ctypes.POINTER(_vp), ctypes.POINTER(SignInfo),
                                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise BsmmError(status, lib().bsmm_last_error().decode(errors="replace"))


def _torch():
    import torch  # device memory and streams only
    return torch


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_vp)


class Context:
    """A library context on one device and one (borrowed) stream."""

    def __init__(self, device: int = 0, stream=None, budget_bytes: int = 0):
        torch = _torch()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = _vp()
        _check(lib().bsmm_ctx_create(device, _vp(stream.cuda_stream), budget_bytes, ctypes.byref(h)))
        self.handle = h

    def set_stream(self, stream):
        _check(lib().bsmm_ctx_set_stream(self.handle, _vp(stream.cuda_stream)))
        self.stream = stream

    def set_timing(self, enable: bool):
        _check(lib().bsmm_ctx_set_timing(self.handle, 1 if enable else 0))

    def set_compute_mode(self, mode: int):
        _check(lib().bsmm_ctx_set_compute_mode(self.handle, mode))

    def set_gemm_variant(self, m: int, n: int, variant: int):
        _check(lib().bsmm_ctx_set_gemm_variant(self.handle, int(m), int(n), int(variant)))

    def set_tile_shape(self, ti: int, tj: int):
        _check(lib().bsmm_ctx_set_tile_shape(self.handle, int(ti), int(tj)))

    def set_tile_schedule(self, persistent: bool = False, xcd_chunk: int = 0):
        _check(lib().bsmm_ctx_set_tile_schedule(self.handle, int(bool(persistent)), int(xcd_chunk)))

    def set_row_order(self, mode: int):
        """0: automatic (square operands of 2,048+ block rows); 1: always (64+ rows); 2: never."""
        _check(lib().bsmm_ctx_set_row_order(self.handle, int(mode)))

    def set_packed_addressing(self, mode: int):
        """0: automatic (per unit only when a packed copy reaches 2 GB); 1: per unit."""
        _check(lib().bsmm_ctx_set_packed_addressing(self.handle, int(mode)))

    def memory(self):
        held, peak = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().bsmm_ctx_memory(self.handle, ctypes.byref(held), ctypes.byref(peak)))
        return held.value, peak.value

    def trim(self):
        _check(lib().bsmm_ctx_trim(self.handle))

    def synchronize(self):
        _check(lib().bsmm_ctx_synchronize(self.handle))

    def close(self):
        if self.handle:
            _check(lib().bsmm_ctx_destroy(self.handle))
            self.handle = None


class Matrix:
    """Handle of a library matrix.  `values` keeps a borrowed torch buffer alive."""

    def __init__(self, ctx: Context, handle, values=None):
        self.ctx = ctx
        self.handle = handle
        self._values = values

    # -- creation --------------------------------------------------------
    @classmethod
    def create(cls, ctx: Context, rbs, cbs, row_ptr, col_idx, values) -> "Matrix":
        """bsmm_mat_create: host index arrays (copied) + a device FP64 torch tensor (borrowed)."""
        torch = _torch()
        rbs = np.ascontiguousarray(rbs, dtype=np.int32)
        cbs = np.ascontiguousarray(cbs, dtype=np.int32)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        if not isinstance(values, torch.Tensor) or values.device.type != "cuda" or values.dtype != torch.float64:
            raise TypeError("values must be a float64 CUDA (HIP) tensor")
        values = values.contiguous()
        h = _vp()
        _check(lib().bsmm_mat_create(ctx.handle, rbs.shape[0], cbs.shape[0], _ptr(rbs), _ptr(cbs),
                                     int(rp[-1]), _ptr(rp), _ptr(ci), _vp(values.data_ptr() if values.numel() else 0),
                                     values.numel(), ctypes.byref(h)))
        return cls(ctx, h, values)

    @classmethod
    def from_host(cls, ctx: Context, m) -> "Matrix":
        """Upload a host block-CSR matrix (values copied into a new torch tensor)."""
        torch = _torch()
        vals = torch.from_numpy(np.ascontiguousarray(m.values, dtype=np.float64)).to(f"cuda:{ctx.device}")
        return cls.create(ctx, m.rbs, m.cbs, m.row_ptr, m.col_idx, vals)

    # -- queries ---------------------------------------------------------
    def info(self):
        nbr, nbc, nnzb, nval = _i32(), _i32(), _i64(), _i64()
        _check(lib().bsmm_mat_info(self.handle, ctypes.byref(nbr), ctypes.byref(nbc), ctypes.byref(nnzb),
                                   ctypes.byref(nval)))
        return nbr.value, nbc.value, nnzb.value, nval.value

    def index(self):
        nbr, _, nnzb, _ = self.info()
        rp = np.zeros(nbr + 1, np.int64)
        ci = np.zeros(max(nnzb, 1), np.int32)
        _check(lib().bsmm_mat_get_index(self.handle, _ptr(rp), _ptr(ci)))
        return rp, ci[:nnzb]

    def block_sizes(self):
        nbr, nbc, _, _ = self.info()
        r = np.zeros(max(nbr, 1), np.int32)
        c = np.zeros(max(nbc, 1), np.int32)
        _check(lib().bsmm_mat_get_block_sizes(self.handle, _ptr(r), _ptr(c)))
        return r[:nbr], c[:nbc]

    def values(self):
        """A new torch tensor holding a copy of the values (ordered on the stream)."""
        torch = _torch()
        _, _, _, nval = self.info()
        out = torch.empty(nval, dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        _check(lib().bsmm_mat_copy_values(self.handle, _vp(out.data_ptr() if nval else 0)))
        return out

    def values_ptr(self) -> int:
        p = _vp()
        _check(lib().bsmm_mat_values(self.handle, ctypes.byref(p)))
        return p.value or 0

    def to_host(self):
        """(rbs, cbs, row_ptr, col_idx, values) as numpy arrays."""
        rp, ci = self.index()
        rbs, cbs = self.block_sizes()
        v = self.values()
        self.ctx.synchronize()
        return HostMat(rbs, cbs, rp, ci, v.cpu().numpy())

    def close(self):
        if self.handle:
            _check(lib().bsmm_mat_destroy(self.handle))
            self.handle = None
            self._values = None

    def __del__(self):
        try:
            if self.handle and self.ctx is not None and self.ctx.handle:
                lib().bsmm_mat_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


@dataclass
class HostMat:
    rbs: np.ndarray
    cbs: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray

    @property
    def nnzb(self) -> int:
        return int(self.row_ptr[-1])


def block_norms(m: Matrix):
    """bsmm_block_norms -> torch float64 tensor of nnzb norms."""
    torch = _torch()
    _, _, nnzb, _ = m.info()
    out = torch.empty(max(nnzb, 1), dtype=torch.float64, device=f"cuda:{m.ctx.device}")
    _check(lib().bsmm_block_norms(m.handle, _vp(out.data_ptr())))
    return out[:nnzb]


def multiply(ctx: Context, transa: str, transb: str, alpha: float, a: Matrix, b: Matrix, beta: float = 0.0,
             c: Matrix | None = None, filter_eps: float = 0.0, retain_sparsity: bool = False):
    """bsmm_multiply: returns (C matrix, MultiplyInfo)."""
    out = _vp()
    info = MultiplyInfo()
    _check(lib().bsmm_multiply(ctx.handle, transa.encode(), transb.encode(), float(alpha), a.handle, b.handle,
                               float(beta), c.handle if c is not None else None, float(filter_eps),
                               1 if retain_sparsity else 0, ctypes.byref(out), ctypes.byref(info)))
    return Matrix(ctx, out), info


def filter(m: Matrix, eps: float) -> Matrix:  # noqa: A001 - mirrors bsmm_filter
    """bsmm_filter: new matrix of the blocks with Frobenius norm >= eps."""
    out = _vp()
    _check(lib().bsmm_filter(m.handle, float(eps), ctypes.byref(out)))
    return Matrix(m.ctx, out)


def filter_noalloc(m: Matrix, eps: float, row_ptr_out, col_idx_out, values_out, counts_out) -> None:
    """bsmm_filter_noalloc: the filter into caller-owned torch tensors
    (int64 nbr+1, int32 >= nnzb, float64 >= n_values, int64 2); ordered on
    the context's stream, no allocation inside the library."""
    def p(t):
        return _vp(t.data_ptr() if t is not None and t.numel() else 0)
    _check(lib().bsmm_filter_noalloc(m.handle, float(eps), p(row_ptr_out), p(col_idx_out), p(values_out),
                                     p(counts_out)))


class Plan:
    """bsmm_plan_*: a multiplication whose structure is fixed once; execute()
    reruns its numeric part on the current values of A, B and C_old (which
    must stay alive), capture() records that part in a HIP graph."""

    def __init__(self, ctx: Context, transa: str, transb: str, alpha: float, a: Matrix, b: Matrix,
                 beta: float = 0.0, c: Matrix | None = None, filter_eps: float = 0.0, retain_sparsity: bool = False):
        self.ctx = ctx
        self.handle = _vp()
        self.info = MultiplyInfo()
        self._keep = (a, b, c)
        _check(lib().bsmm_plan_create(ctx.handle, transa.encode(), transb.encode(), float(alpha), a.handle,
                                      b.handle, float(beta), c.handle if c is not None else None,
                                      float(filter_eps), 1 if retain_sparsity else 0, ctypes.byref(self.handle),
                                      ctypes.byref(self.info)))

    def execute(self):
        _check(lib().bsmm_plan_execute(self.handle))

    def capture(self):
        _check(lib().bsmm_plan_capture(self.handle))

    def sizes(self):
        """bsmm_plan_sizes: (c_nnzb, c_n_values, workspace_bytes) before the post-filter."""
        nb, nv, ws = _i64(), _i64(), ctypes.c_size_t()
        _check(lib().bsmm_plan_sizes(self.handle, ctypes.byref(nb), ctypes.byref(nv), ctypes.byref(ws)))
        return nb.value, nv.value, ws.value

    def filter_holds(self) -> bool:
        """bsmm_plan_filter_holds: the plan's filter decisions equal those a
        new plan would take on the operands' current values."""
        h = _i32()
        _check(lib().bsmm_plan_filter_holds(self.handle, ctypes.byref(h)))
        return bool(h.value)

    def execute_into(self, c_values, workspace) -> Matrix:
        """bsmm_plan_execute_into: numeric part and post-filter in caller
        tensors (float64 with room for c_n_values; a byte tensor of
        workspace_bytes, 256-byte aligned).  The result matrix borrows c_values."""
        out = _vp()
        _check(lib().bsmm_plan_execute_into(self.handle, _vp(c_values.data_ptr() if c_values.numel() else 0),
                                            _vp(workspace.data_ptr() if workspace.numel() else 0), ctypes.byref(out)))
        return Matrix(self.ctx, out, c_values)

    def result(self) -> Matrix:
        out = _vp()
        _check(lib().bsmm_plan_result(self.handle, ctypes.byref(out)))
        return Matrix(self.ctx, out)

    def close(self):
        if self.handle:
            _check(lib().bsmm_plan_destroy(self.handle))
            self.handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plans_execute(plans) -> None:
    """bsmm_plans_execute: the numeric parts of several plans in one batch."""
    arr = (_vp * max(len(plans), 1))(*[p.handle for p in plans])
    _check(lib().bsmm_plans_execute(len(plans), arr))


def sign_newton_schulz(ctx: Context, x0: Matrix, max_iter: int, filter_eps: float = 0.0, tol: float = 0.0):
    """bsmm_sign_newton_schulz: returns (X matrix, SignInfo, residual per
    iteration, blocks after each iteration) -- the two traces cut to the
    iterations run."""
    import numpy as np
    out = _vp()
    info = SignInfo()
    n = max(int(max_iter), 1)
    res = np.zeros(n, dtype=np.float64)
    nnz = np.zeros(n, dtype=np.int64)
    _check(lib().bsmm_sign_newton_schulz(ctx.handle, x0.handle, int(max_iter), float(filter_eps), float(tol),
                                         ctypes.byref(out), ctypes.byref(info),
                                         res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         nnz.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    k = info.iterations
    return Matrix(ctx, out), info, res[:k].copy(), nnz[:k].copy()


def status_string(s: int) -> str:
    return lib().bsmm_status_string(s).decode()
