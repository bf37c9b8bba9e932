"""CPU FP64 oracle for the local block-sparse multiply (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.  The arithmetic lives in ``oracle.c`` (plain C,
``-O2 -ffp-contract=off``); this module only marshals numpy arrays.

Paper: arXiv:1705.10218, Section 2 (blocked CSR storage, non-fixed result
pattern, on-the-fly norm filter during the block products) and Section 1
(two-phase filtering: on the fly and after each multiplication).  The
readings taken where the paper is silent are listed at the top of
``oracle.c``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)


class _Result(ctypes.Structure):
    _fields_ = [
        ("nbr", ctypes.c_int32), ("nbc", ctypes.c_int32),
        ("rbs", _i32p), ("cbs", _i32p),
        ("nnzb", ctypes.c_int64),
        ("row_ptr", _i64p), ("col_idx", _i32p),
        ("val", _f64p), ("n_val", ctypes.c_int64),
        ("n_products", ctypes.c_int64), ("n_candidates", ctypes.c_int64),
        ("useful_flops", ctypes.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no GPU, no HIP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_block_norms.restype = ctypes.c_int
        lib.oracle_multiply.restype = ctypes.c_int
        lib.oracle_filter.restype = ctypes.c_int
        lib.oracle_free.restype = None
        lib.oracle_free.argtypes = [ctypes.POINTER(_Result)]
        _lib = lib
    return _lib


@dataclass
class Mat:
    """Host block-CSR matrix as the oracle returns it."""
    rbs: np.ndarray
    cbs: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    n_products: int = 0
    n_candidates: int = 0
    useful_flops: float = 0.0

    @property
    def nbr(self) -> int:
        return int(self.rbs.shape[0])

    @property
    def nbc(self) -> int:
        return int(self.cbs.shape[0])

    @property
    def nnzb(self) -> int:
        return int(self.row_ptr[-1])


def _arr(x, dt):
    return np.ascontiguousarray(np.asarray(x), dtype=dt)


def _p(a, t):
    return a.ctypes.data_as(t)


def _mat_args(m):
    rbs = _arr(m.rbs, np.int32)
    cbs = _arr(m.cbs, np.int32)
    rp = _arr(m.row_ptr, np.int64)
    ci = _arr(m.col_idx, np.int32)
    v = _arr(m.values, np.float64)
    keep = (rbs, cbs, rp, ci, v)
    args = [ctypes.c_int32(rbs.shape[0]), ctypes.c_int32(cbs.shape[0]),
            _p(rbs, _i32p), _p(cbs, _i32p), _p(rp, _i64p), _p(ci, _i32p), _p(v, _f64p)]
    return args, keep


def _take(res_ptr) -> Mat:
    r = res_ptr.contents
    nbr, nbc, nnzb, nval = r.nbr, r.nbc, r.nnzb, r.n_val
    out = Mat(
        rbs=np.ctypeslib.as_array(r.rbs, shape=(max(nbr, 1),))[:nbr].copy(),
        cbs=np.ctypeslib.as_array(r.cbs, shape=(max(nbc, 1),))[:nbc].copy(),
        row_ptr=np.ctypeslib.as_array(r.row_ptr, shape=(nbr + 1,)).copy(),
        col_idx=np.ctypeslib.as_array(r.col_idx, shape=(max(nnzb, 1),))[:nnzb].copy(),
        values=np.ctypeslib.as_array(r.val, shape=(max(nval, 1),))[:nval].copy(),
        n_products=int(r.n_products), n_candidates=int(r.n_candidates),
        useful_flops=float(r.useful_flops))
    _load().oracle_free(res_ptr)
    return out


def block_norms(m) -> np.ndarray:
    """Frobenius norm of every stored block (storage order), FP64."""
    lib = _load()
    args, keep = _mat_args(m)
    out = np.zeros(max(int(np.asarray(m.row_ptr)[-1]), 1), dtype=np.float64)
    rc = lib.oracle_block_norms(*args, _p(out, _f64p))
    assert rc == 0
    del keep
    return out[: int(np.asarray(m.row_ptr)[-1])]


def multiply(transa: str, transb: str, alpha: float, a, b, beta: float = 0.0, c=None,
             eps: float = 0.0, retain_sparsity: bool = False, nthreads: int = 1,
             rows=None) -> Mat:
    """C = alpha*op(A)*op(B) + beta*C_old with on-the-fly and post filtering.

    ``rows`` (optional) restricts the work to those result block rows; the
    other rows come back empty.
    """
    lib = _load()
    aa, ka = _mat_args(a)
    ba, kb = _mat_args(b)
    if c is None:
        z32 = np.zeros(1, np.int32)
        z64 = np.zeros(1, np.int64)
        zf = np.zeros(1, np.float64)
        ca = [ctypes.c_int32(-1), ctypes.c_int32(-1), _p(z32, _i32p), _p(z32, _i32p),
              _p(z64, _i64p), _p(z32, _i32p), _p(zf, _f64p)]
        kc = (z32, z64, zf)
    else:
        ca, kc = _mat_args(c)
    if rows is not None:
        rs = _arr(rows, np.int32)
        rs_p, n_rs = _p(rs, _i32p), ctypes.c_int64(rs.shape[0])
    else:
        rs = None
        rs_p, n_rs = _i32p(), ctypes.c_int64(0)
    res = ctypes.POINTER(_Result)()
    rc = lib.oracle_multiply(
        ctypes.c_char(transa.encode()), ctypes.c_char(transb.encode()), ctypes.c_double(alpha),
        *aa, *ba, ctypes.c_double(beta), *ca,
        ctypes.c_double(eps), ctypes.c_int(1 if retain_sparsity else 0), ctypes.c_int(nthreads),
        rs_p, n_rs, ctypes.byref(res))
    del ka, kb, kc, rs
    if rc != 0:
        raise ValueError(f"oracle_multiply: bad arguments (code {rc})")
    return _take(res)


def filter_blocks(m, eps: float) -> Mat:
    """Drop the blocks whose Frobenius norm is below eps (kept iff >= eps)."""
    lib = _load()
    args, keep = _mat_args(m)
    res = ctypes.POINTER(_Result)()
    rc = lib.oracle_filter(*args, ctypes.c_double(eps), ctypes.byref(res))
    del keep
    assert rc == 0
    return _take(res)


# ------------------------------------------------------------------ sign
def _identity(sizes) -> Mat:
    """Block-diagonal identity with the given block sizes."""
    sizes = np.asarray(sizes, dtype=np.int32)
    n = sizes.shape[0]
    vals = np.concatenate([np.eye(int(s)).reshape(-1, order="F") for s in sizes]) if n else np.zeros(0)
    return Mat(sizes.copy(), sizes.copy(), np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), vals)


def _shift_dist(t: Mat, shift: float) -> float:
    """||T - shift * I||_F for a square block matrix T (block rows in order)."""
    sizes = t.rbs.astype(np.int64)
    ss = 0.0
    off = 0
    for i in range(t.nbr):
        has_diag = False
        for p in range(int(t.row_ptr[i]), int(t.row_ptr[i + 1])):
            j = int(t.col_idx[p])
            n = int(sizes[i] * t.cbs[j])
            blk = t.values[off:off + n].reshape((int(sizes[i]), int(t.cbs[j])), order="F").copy()
            off += n
            if j == i:
                has_diag = True
                blk[np.diag_indices(int(sizes[i]))] -= shift
            ss += float(np.sum(blk * blk))
        if not has_diag:
            ss += shift * shift * float(sizes[i])
    return math.sqrt(ss)


def newton_schulz(x0, max_iter: int, eps: float = 0.0, tol: float = 0.0, nthreads: int = 1):
    """Newton-Schulz iteration for the matrix sign function, X <- X (3I - X^2) / 2
    (arXiv:1705.10218, Section 1, eq. (3) and the iteration after it), each
    product a filtered block-sparse multiplication of this oracle:
    T = 3I - X X (C_old = I, beta = 3), residual ||T - 2I||_F / sqrt(N) =
    ||X^2 - I||_F / sqrt(N), stop if it is below tol (> 0), else
    X = 0.5 X T.  Returns (X, residuals, nnzb after each step, converged,
    useful flops)."""
    ident = _identity(x0.rbs)
    ndim = float(np.sum(np.asarray(x0.rbs, dtype=np.int64)))
    x = x0
    res, nnz = [], []
    flops = 0.0
    converged = False
    for _ in range(max_iter):
        t = multiply("N", "N", -1.0, x, x, beta=3.0, c=ident, eps=eps, nthreads=nthreads)
        flops += t.useful_flops
        r = _shift_dist(t, 2.0) / math.sqrt(ndim) if ndim > 0 else 0.0
        res.append(r)
        if tol > 0.0 and r < tol:
            nnz.append(int(x.row_ptr[-1]))
            converged = True
            break
        x = multiply("N", "N", 0.5, x, t, eps=eps, nthreads=nthreads)
        flops += x.useful_flops
        nnz.append(int(x.row_ptr[-1]))
    if x is x0:
        x = multiply("N", "N", 1.0, x0, ident, nthreads=nthreads)
    return x, np.array(res), np.array(nnz, dtype=np.int64), converged, flops
