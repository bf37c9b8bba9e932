"""Shared helpers for the test suite (layout conversions and comparisons only)."""
from __future__ import annotations

import numpy as np

from paper_1705_10218_amd.inputs import BlockCSR, from_pattern, to_dense


def random_bcsr(rng, nbr, nbc, rbs=None, cbs=None, p=0.4, max_bs=7, empty_rows=(), dist="normal"):
    if rbs is None:
        rbs = rng.integers(1, max_bs + 1, nbr)
    if cbs is None:
        cbs = rng.integers(1, max_bs + 1, nbc)
    mask = rng.random((nbr, nbc)) < p
    for r in empty_rows:
        if r < nbr:
            mask[r, :] = False
    r, c = np.nonzero(mask)
    return from_pattern(np.asarray(rbs, np.int32), np.asarray(cbs, np.int32), r, c, rng, dist=dist)


def as_bcsr(m) -> BlockCSR:
    if isinstance(m, BlockCSR):
        return m
    return BlockCSR(np.asarray(m.rbs), np.asarray(m.cbs), np.asarray(m.row_ptr),
                    np.asarray(m.col_idx), np.asarray(m.values))


def pattern_dense(m) -> np.ndarray:
    m = as_bcsr(m)
    pat = np.zeros((m.nbr, m.nbc), dtype=bool)
    pat[m.block_rows(), m.col_idx] = True
    return pat


def transpose_host(m: BlockCSR) -> BlockCSR:
    """Block-CSR of the transpose (grid and blocks), by layout moves only."""
    off = m.block_offsets()
    rows = m.block_rows()
    order = np.lexsort((rows, m.col_idx))
    new_rp = np.zeros(m.nbc + 1, dtype=np.int64)
    np.cumsum(np.bincount(m.col_idx, minlength=m.nbc), out=new_rp[1:])
    new_ci = rows[order].astype(np.int32)
    vals = []
    for p in order:
        i, j = rows[p], m.col_idx[p]
        mm, nn = int(m.rbs[i]), int(m.cbs[j])
        blk = m.values[off[p]:off[p] + mm * nn].reshape((mm, nn), order="F")
        vals.append(blk.T.reshape(-1, order="F"))
    v = np.concatenate(vals) if vals else np.zeros(0)
    return BlockCSR(m.cbs.copy(), m.rbs.copy(), new_rp, new_ci, v)


def permute(m: BlockCSR, prow, pcol) -> BlockCSR:
    """Block-permuted copy: new block (prow[i], pcol[j]) = old block (i, j)."""
    off = m.block_offsets()
    rows = m.block_rows()
    nr = np.asarray(prow)[rows]
    nc = np.asarray(pcol)[m.col_idx]
    order = np.lexsort((nc, nr))
    rbs = np.empty_like(m.rbs)
    rbs[np.asarray(prow)] = m.rbs
    cbs = np.empty_like(m.cbs)
    cbs[np.asarray(pcol)] = m.cbs
    rp = np.zeros(m.nbr + 1, dtype=np.int64)
    np.cumsum(np.bincount(nr, minlength=m.nbr), out=rp[1:])
    vals = [m.values[off[p]:off[p + 1]] for p in order]
    v = np.concatenate(vals) if vals else np.zeros(0)
    return BlockCSR(rbs, cbs, rp, nc[order].astype(np.int32), v)


def rel_fro(x: np.ndarray, ref: np.ndarray) -> float:
    den = np.linalg.norm(ref)
    num = np.linalg.norm(x - ref)
    if den == 0:
        return float(num)
    return float(num / den)


def dense(m) -> np.ndarray:
    return to_dense(as_bcsr(m))


def same_pattern(x, y) -> bool:
    return (np.array_equal(np.asarray(x.row_ptr), np.asarray(y.row_ptr))
            and np.array_equal(np.asarray(x.col_idx), np.asarray(y.col_idx)))
