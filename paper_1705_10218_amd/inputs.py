"""Seeded synthetic inputs: block-CSR matrices shaped like the paper's workloads.

This module is shared by the GPU path's tests and benchmark and by the CPU
oracle's tests.  It only *draws* inputs (patterns, block sizes, values); it
performs none of the multiply's arithmetic (no products, no norms, no
filtering), so that the two sides stay independent.

Workloads (arXiv:1705.10218, Section 4 and Table 1): the H2O-DFT-LS
benchmark has matrices of 23x23 blocks, one per molecule, at liquid-water
density and 7-15 % occupancy; block sizes in general follow the atomic
kinds (Section 1).  The CP2K inputs are not available, so the generator
places "atoms" uniformly in a periodic cube at 0.1 atoms per cubic
Angstrom, gives each a block size, keeps block (i,j) when the
minimum-image distance r_ij is below a cutoff, and fills the block with
i.i.d. N(0,1) entries scaled by exp(-r_ij / decay).  Seeds come from
``numpy.random.default_rng([config, matrix, request])``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DENSITY = 0.1  # atoms per cubic Angstrom


@dataclass
class BlockCSR:
    """Host block-CSR matrix.

    rbs[i] / cbs[j]: row / column block sizes; row_ptr (int64, nbr+1) and
    col_idx (int32, strictly increasing inside a row) index the stored
    blocks; values (float64) holds the blocks contiguously in CSR order,
    each block column-major with leading dimension rbs[i].
    """
    rbs: np.ndarray
    cbs: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nbr(self) -> int:
        return int(self.rbs.shape[0])

    @property
    def nbc(self) -> int:
        return int(self.cbs.shape[0])

    @property
    def nnzb(self) -> int:
        return int(self.row_ptr[-1])

    def block_rows(self) -> np.ndarray:
        return np.repeat(np.arange(self.nbr, dtype=np.int32), np.diff(self.row_ptr))

    def block_offsets(self) -> np.ndarray:
        """Element offset of every block (nnzb+1 entries, int64)."""
        sizes = self.rbs[self.block_rows()].astype(np.int64) * self.cbs[self.col_idx].astype(np.int64)
        off = np.zeros(self.nnzb + 1, dtype=np.int64)
        np.cumsum(sizes, out=off[1:])
        return off

    def n_values(self) -> int:
        return int(self.block_offsets()[-1])


def rng_for(config: int, matrix: int, request: int = 0) -> np.random.Generator:
    return np.random.default_rng([config, matrix, request])


def _csr_from_mask_rows(nbr: int, rows: np.ndarray, cols: np.ndarray):
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(nbr + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=nbr), out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), order


def from_pattern(rbs, cbs, rows, cols, rng, scale=None, dist="normal") -> BlockCSR:
    """Block-CSR with the given (row, col) pattern and random values.

    ``scale`` (one factor per pattern entry, in the order given) multiplies
    every element of that block.  ``dist`` is 'normal' (N(0,1)) or
    'uniform' (U[-1,1)).
    """
    rbs = np.asarray(rbs, dtype=np.int32)
    cbs = np.asarray(cbs, dtype=np.int32)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    row_ptr, col_idx, order = _csr_from_mask_rows(rbs.shape[0], rows, cols)
    sizes = rbs[rows[order]].astype(np.int64) * cbs[col_idx].astype(np.int64)
    total = int(sizes.sum())
    if dist == "normal":
        vals = rng.standard_normal(total)
    elif dist == "uniform":
        vals = rng.uniform(-1.0, 1.0, total)
    else:
        raise ValueError(dist)
    if scale is not None:
        s = np.asarray(scale, dtype=np.float64)[order]
        vals *= np.repeat(s, sizes)
    return BlockCSR(rbs, cbs, row_ptr, col_idx, vals)


def bernoulli_pattern(nbr, nbc, p, rng, diag=True):
    mask = rng.random((nbr, nbc)) < p
    if diag:
        d = np.arange(min(nbr, nbc))
        mask[d, d] = True
    r, c = np.nonzero(mask)
    return r, c


def config_tiny(matrix: int = 0, nb: int = 100, bs: int = 5, p: float = 0.2) -> BlockCSR:
    """100x100 blocks of 5x5, diagonal always present, off-diagonal blocks
    present with probability 0.2, N(0,1) entries."""
    rng = rng_for(1, matrix)
    r, c = bernoulli_pattern(nb, nb, p, rng, diag=True)
    sizes = np.full(nb, bs, dtype=np.int32)
    m = from_pattern(sizes, sizes, r, c, rng)
    m.meta = dict(workload="tiny", nb=nb, bs=bs, p=p)
    return m


@dataclass
class Atoms:
    pos: np.ndarray      # (n, 3) Angstrom
    box: float           # cube edge, Angstrom
    sizes: np.ndarray    # (n,) block size per atom


def make_atoms(n: int, rng: np.random.Generator, sizes=(5, 13), probs=None,
               density: float = DENSITY) -> Atoms:
    box = (n / density) ** (1.0 / 3.0)
    pos = rng.random((n, 3)) * box
    sz = rng.choice(np.asarray(sizes, dtype=np.int32), size=n, p=probs).astype(np.int32)
    return Atoms(pos, box, sz)


def neighbour_pairs(atoms: Atoms, cutoff: float, chunk: int = 512):
    """All (i, j, r_ij) with minimum-image distance r_ij < cutoff (i == j
    included, r = 0), sorted by (i, j)."""
    n = atoms.pos.shape[0]
    box = atoms.box
    rows, cols, dist = [], [], []
    c2 = cutoff * cutoff
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        d = atoms.pos[r0:r1, None, :] - atoms.pos[None, :, :]
        d -= box * np.round(d / box)
        d2 = np.einsum("ijk,ijk->ij", d, d)
        ii, jj = np.nonzero(d2 < c2)
        rows.append(ii + r0)
        cols.append(jj)
        dist.append(np.sqrt(d2[ii, jj]))
    rows = np.concatenate(rows).astype(np.int64)
    cols = np.concatenate(cols).astype(np.int64)
    dist = np.concatenate(dist)
    return rows, cols, dist


def cutoff_for_occupancy(n: int, occupancy: float, density: float = DENSITY) -> float:
    """Cutoff radius whose expected blocks per row equal occupancy * n:
    1 + density * 4/3 pi r^3 = occupancy * n."""
    want = max(occupancy * n - 1.0, 0.0)
    return (3.0 * want / (4.0 * math.pi * density)) ** (1.0 / 3.0)


def dft_like_pair(n_atoms: int, config: int, sizes=(5, 13), probs=None, cutoff: float = 7.0,
                  decay: float = 2.0, request: int = 0, dist: str = "normal"):
    """Two matrices A, B on the same atoms (same pattern and block sizes),
    with independent value streams."""
    rng_atoms = rng_for(config, 0, request)
    atoms = make_atoms(n_atoms, rng_atoms, sizes=sizes, probs=probs)
    if cutoff >= atoms.box / 2:
        raise ValueError("cutoff must stay below half the box edge for minimum-image distances")
    r, c, d = neighbour_pairs(atoms, cutoff)
    scale = np.exp(-d / decay)
    mats = []
    for mid in (1, 2):
        m = from_pattern(atoms.sizes, atoms.sizes, r, c, rng_for(config, mid, request), scale=scale, dist=dist)
        m.meta = dict(workload="dft_like", n_atoms=n_atoms, sizes=tuple(sizes), cutoff=cutoff,
                      decay=decay, box=atoms.box, config=config, request=request)
        mats.append(m)
    return mats[0], mats[1], atoms


def config_dft(n_atoms: int = 4000):
    """4,000 atoms at 0.1 /A^3, block sizes 50/50 from {5,13}, cutoff 7 A,
    values N(0,1) exp(-r/2 A).  Used with eps = 1e-10 for both filters."""
    return dft_like_pair(n_atoms, config=2, sizes=(5, 13), cutoff=7.0, decay=2.0)


def config_big23(n_atoms: int = 20000, occupancy: float = 0.03, sizes=(23,)):
    """20,000 atoms, 23x23 blocks (or a mix), cutoff tuned to ~3 % occupancy."""
    rc = cutoff_for_occupancy(n_atoms, occupancy)
    return dft_like_pair(n_atoms, config=3, sizes=sizes, cutoff=rc, decay=2.0)


def morton_order(pos: np.ndarray, box: float, bits: int = 10) -> np.ndarray:
    """Permutation that sorts positions along a Morton (Z-order) curve of the
    periodic box: neighbouring indices are neighbouring points."""
    q = np.clip(np.floor(pos / box * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(pos.shape[0], dtype=np.int64)
    for bit in range(bits):
        for d in range(3):
            code |= ((q[:, d] >> bit) & 1) << (3 * bit + d)
    return np.argsort(code, kind="stable")


PANEL_CHUNK = 256   # block rows per value stream of the batching workload


@dataclass
class BatchingProblem:
    """Geometry of the batching workload: atoms on a Morton curve (so that a
    contiguous range of block rows, a process's panel, is a compact region),
    their block sizes and the cutoff."""
    pos: np.ndarray
    box: float
    sizes: np.ndarray
    cutoff: float
    decay: float
    config: int

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def batching_problem(n_atoms: int = 20000, occupancy: float = 0.03, sizes=(23,), config: int = 3,
                     decay: float = 2.0) -> BatchingProblem:
    """20,000 atoms at 0.1 /A^3 (box 58.5 A), block sizes drawn from `sizes`,
    cutoff giving `occupancy` of the block grid on average; atoms renumbered
    along a Morton curve."""
    rc = cutoff_for_occupancy(n_atoms, occupancy)
    at = make_atoms(n_atoms, rng_for(config, 0, 0), sizes=sizes)
    if rc >= at.box / 2:
        raise ValueError("cutoff must stay below half the box edge for minimum-image distances")
    perm = morton_order(at.pos, at.box)
    return BatchingProblem(at.pos[perm], at.box, at.sizes[perm].astype(np.int32), rc, decay, config)


def _pairs_of_rows(pb: BatchingProblem, r0: int, r1: int):
    """(local row, column, distance) of every block of rows [r0, r1) within
    the cutoff (minimum image, diagonal included), sorted by (row, column)."""
    from scipy.spatial import cKDTree   # neighbour search only
    full = cKDTree(pb.pos, boxsize=pb.box)
    part = cKDTree(pb.pos[r0:r1], boxsize=pb.box)
    pr = part.sparse_distance_matrix(full, pb.cutoff, output_type="ndarray")
    keep = pr["v"] < pb.cutoff
    rows, cols, dist = pr["i"][keep].astype(np.int64), pr["j"][keep].astype(np.int64), pr["v"][keep]
    order = np.lexsort((cols, rows))
    return rows[order], cols[order], dist[order]


def batching_matrix(pb: BatchingProblem, matrix: int, row_range=None, row_mask=None,
                    threads: int | None = None) -> BlockCSR:
    """Rows [r0, r1) of matrix `matrix` (1 = A, 2 = B) of the batching
    workload, over all n block columns: block (i, j) present when the
    minimum-image distance is below the cutoff, values N(0,1) exp(-r/decay).
    The values of every chunk of PANEL_CHUNK block rows come from their own
    stream default_rng([config, matrix, chunk]) in storage order, so a panel
    holds exactly the rows of the whole matrix.  row_mask (optional, n
    booleans) leaves the unmasked rows empty (their products are never
    formed when the other operand does not reach them)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    n = pb.n
    r0, r1 = row_range if row_range is not None else (0, n)
    c0, c1 = (r0 // PANEL_CHUNK) * PANEL_CHUNK, min(n, -(-r1 // PANEL_CHUNK) * PANEL_CHUNK)
    rows, cols, dist = _pairs_of_rows(pb, c0, c1)
    rows += c0
    sizes_all = pb.sizes[rows].astype(np.int64) * pb.sizes[cols].astype(np.int64)
    boff = np.zeros(rows.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes_all, out=boff[1:])
    row_start = np.searchsorted(rows, np.arange(c0, c1 + 1))
    nchunk = (c1 - c0 + PANEL_CHUNK - 1) // PANEL_CHUNK
    # the blocks kept: rows in [r0, r1) (and in the mask)
    sel_rows = np.zeros(n, dtype=bool)
    sel_rows[r0:r1] = True
    if row_mask is not None:
        sel_rows &= np.asarray(row_mask, dtype=bool)
    keep_blk = sel_rows[rows]
    kept_sizes = sizes_all[keep_blk]
    koff = np.zeros(int(keep_blk.sum()) + 1, dtype=np.int64)
    np.cumsum(kept_sizes, out=koff[1:])
    vals = np.empty(int(koff[-1]), dtype=np.float64)
    kidx = np.cumsum(keep_blk) - 1   # position of a kept block among kept blocks

    def fill(ch: int):
        a0 = c0 + ch * PANEL_CHUNK
        a1 = min(c1, a0 + PANEL_CHUNK)
        b0, b1 = int(row_start[a0 - c0]), int(row_start[a1 - c0])
        if b0 == b1:
            return
        v = rng_for(pb.config, matrix, a0 // PANEL_CHUNK).standard_normal(int(boff[b1] - boff[b0]))
        v *= np.repeat(np.exp(-dist[b0:b1] / pb.decay), sizes_all[b0:b1])
        for r in range(a0, a1):
            if not sel_rows[r]:
                continue
            p0, p1 = int(row_start[r - c0]), int(row_start[r - c0 + 1])
            if p0 == p1:
                continue
            d0 = int(koff[kidx[p0]])
            vals[d0:d0 + int(boff[p1] - boff[p0])] = v[boff[p0] - boff[b0]:boff[p1] - boff[b0]]

    nt = threads or min(16, len(os.sched_getaffinity(0)))
    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(fill, range(nchunk)))
    kr, kc = rows[keep_blk] - r0, cols[keep_blk]
    row_ptr = np.zeros(r1 - r0 + 1, dtype=np.int64)
    np.cumsum(np.bincount(kr, minlength=r1 - r0), out=row_ptr[1:])
    m = BlockCSR(pb.sizes[r0:r1].copy(), pb.sizes.copy(), row_ptr, kc.astype(np.int32), vals)
    m.meta = dict(workload="batching", atoms=n, rows=(r0, r1), cutoff=pb.cutoff, box=pb.box, matrix=matrix)
    return m


def reachable_rows(a_panel: BlockCSR, n: int) -> np.ndarray:
    """Block rows k of the other operand that some stored block (i, k) of the
    panel reaches (a mask of n booleans)."""
    mask = np.zeros(n, dtype=bool)
    mask[np.asarray(a_panel.col_idx)] = True
    return mask


def symmetric_dft_like(n_atoms: int, config: int = 4, sizes=(5, 13), cutoff: float = 7.0, decay: float = 2.0,
                       gap: float = 10.0, request: int = 0) -> BlockCSR:
    """Symmetric DFT-like start matrix for the sign iteration (Section 1,
    eq. (3)): the DFT-like pattern, off-diagonal blocks N(0,1) exp(-r/decay)
    with block (j,i) the transpose of block (i,j), diagonal blocks symmetric
    N(0,1) plus +-gap on the diagonal (a random sign per orbital, so the
    spectrum has eigenvalues on both sides of 0, away from it), the whole
    matrix divided by its largest absolute row sum (a Gershgorin bound), so
    every eigenvalue lies in (-1, 1).  Input preparation only."""
    rng = rng_for(config, 0, request)
    atoms = make_atoms(n_atoms, rng, sizes=sizes)
    if cutoff >= atoms.box / 2:
        raise ValueError("cutoff must stay below half the box edge for minimum-image distances")
    r, c, d = neighbour_pairs(atoms, cutoff)
    vrng = rng_for(config, 1, request)
    sz = atoms.sizes
    blocks = {}
    for i, j, dist in zip(r.tolist(), c.tolist(), d.tolist()):
        if i < j:
            blocks[(i, j)] = vrng.standard_normal((sz[i], sz[j])) * math.exp(-dist / decay)
        elif i == j:
            g = vrng.standard_normal((sz[i], sz[i]))
            g = 0.5 * (g + g.T)
            g[np.diag_indices(sz[i])] += gap * vrng.choice([-1.0, 1.0], size=sz[i])
            blocks[(i, i)] = g
    for (i, j) in list(blocks):
        if i < j:
            blocks[(j, i)] = blocks[(i, j)].T
    keys = sorted(blocks)
    rows = np.array([k[0] for k in keys], dtype=np.int64)
    cols = np.array([k[1] for k in keys], dtype=np.int64)
    row_ptr = np.zeros(n_atoms + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n_atoms), out=row_ptr[1:])
    rowsum = np.zeros(int(sz.sum()))
    first = np.concatenate([[0], np.cumsum(sz)[:-1]])
    for (i, j) in keys:
        rowsum[first[i]:first[i] + sz[i]] += np.abs(blocks[(i, j)]).sum(axis=1)
    scale = 1.0 / float(rowsum.max()) if rowsum.size else 1.0
    vals = np.concatenate([(blocks[k] * scale).reshape(-1, order="F") for k in keys]) if keys else np.zeros(0)
    m = BlockCSR(sz.copy(), sz.copy(), row_ptr, cols.astype(np.int32), vals)
    m.meta = dict(workload="sign_start", atoms=n_atoms, sizes=list(sizes), cutoff=cutoff, gap=gap, scale=scale)
    return m


def serving_request_params(n: int, atoms=(200, 8000), occupancy=(0.02, 0.20), seed: int = 0, config: int = 5):
    """(atoms, occupancy, cutoff) of the n requests of serving_requests, from
    the same draws, without building the matrices."""
    rng = np.random.default_rng([config, 99, seed])
    out = []
    for _ in range(n):
        na = int(round(math.exp(rng.uniform(math.log(atoms[0]), math.log(atoms[1])))))
        occ = float(rng.uniform(occupancy[0], occupancy[1]))
        box = (na / DENSITY) ** (1.0 / 3.0)
        rc = min(cutoff_for_occupancy(na, occ), 0.49 * box)
        out.append((na, occ, rc))
    return out


def serving_requests(n: int, atoms=(200, 8000), occupancy=(0.02, 0.20), sizes=(5, 13, 23), config: int = 5,
                     seed: int = 0):
    """Independent multiplication requests: atom count log-uniform in atoms,
    block sizes uniform over sizes, cutoff giving an occupancy uniform in
    occupancy (capped below half the box edge), DFT-like A and B from
    default_rng([config, matrix, request])."""
    out = []
    for rid, (na, occ, rc) in enumerate(serving_request_params(n, atoms, occupancy, seed, config)):
        a, b, _ = dft_like_pair(na, config=config, sizes=sizes, cutoff=rc, request=seed * 100000 + rid)
        out.append((a, b, {"atoms": na, "occupancy": occ, "cutoff": rc}))
    return out


def identity(sizes) -> BlockCSR:
    sizes = np.asarray(sizes, dtype=np.int32)
    n = sizes.shape[0]
    row_ptr = np.arange(n + 1, dtype=np.int64)
    col_idx = np.arange(n, dtype=np.int32)
    vals = np.concatenate([np.eye(int(s)).reshape(-1, order="F") for s in sizes]) if n else np.zeros(0)
    return BlockCSR(sizes.copy(), sizes.copy(), row_ptr, col_idx, vals)


def to_dense(m: BlockCSR) -> np.ndarray:
    """Dense copy (zeros outside stored blocks); a layout conversion only."""
    ro = np.zeros(m.nbr + 1, dtype=np.int64)
    np.cumsum(m.rbs, out=ro[1:])
    co = np.zeros(m.nbc + 1, dtype=np.int64)
    np.cumsum(m.cbs, out=co[1:])
    d = np.zeros((int(ro[-1]), int(co[-1])))
    off = m.block_offsets()
    for i in range(m.nbr):
        for p in range(int(m.row_ptr[i]), int(m.row_ptr[i + 1])):
            j = int(m.col_idx[p])
            mm, nn = int(m.rbs[i]), int(m.cbs[j])
            d[ro[i]:ro[i] + mm, co[j]:co[j] + nn] = m.values[off[p]:off[p] + mm * nn].reshape((mm, nn), order="F")
    return d
