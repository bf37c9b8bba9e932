"""Autotuner for the block GEMM's kernel variant per (m, n) size class and
the tile path's schedule.

The FP64 block GEMM has several ways to cover a result block on the matrix
cores: 16x16x4 MFMA tiles (few loads per k-step, padding to 16), 4x4x4
MFMA subtiles (padding to 4, more loads), for edges up to 8 one 16x16x4
tile carrying two products per k-slice in its diagonal quadrants, and for
edges in 9..24 one 16x16x4 tile plus 4x4x4 subtiles along the edges beyond
16.
Which is faster depends on the block edges, so it is chosen per size class
(edges 1-8, 9-16, 17-24, 25-32) by timing: for every (m, n) pair of a block-size set, a synthetic DFT-like
workload whose result blocks all have that shape (contraction sizes drawn
from the same set) is multiplied with each variant, and the fastest GEMM
time wins.  The best variant depends on the contraction-size mix as well,
so the JSON file holds one table per block-size set and :func:`apply` picks
the table of the workload's set.  A wavefront (packed path) or a tile (tile
path) owns result blocks whose products have every k size of the set, so the
choice is made per (m, n) class with the set's k mix, not per (m, n, k).
For sets whose sizes all lie in 17..24 the tile path is a candidate too, and
when it wins, its tile shape and the number of consecutive tiles per XCD
chunk are tuned as well.

Usage::

    python -m paper_1705_10218_amd.autotune --size-sets 5,13 23 5,13,23 --out tuning.json
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys

import numpy as np

VARIANTS = {1: "mfma16x16x4_tiles", 2: "mfma4x4x4_subtiles", 3: "mfma16x16x4_diagonal_pairs",
            4: "mfma16x16x4_with_4x4x4_edges", 5: "tile_path_lds_staged", 6: "tile_path_general_kernel"}
TILE_SHAPES = ((2, 2), (2, 4), (4, 2), (4, 4))
XCD_CHUNKS = (2048, 8192, 32768)


def applies(v: int, m: int, n: int, sizes=None) -> bool:
    """Variant 3 exists for blocks with both edges at most 8, variant 4 for
    both edges in 9..24 with one above 16.  The tile-path variants 5 and 6
    take a whole product or none of it: they are tried only for block-size
    sets whose sizes all lie in 17..24 (in a mixed set they would never
    run)."""
    if v == 3:
        return m <= 8 and n <= 8
    if v == 4:
        return 9 <= m <= 24 and 9 <= n <= 24 and max(m, n) > 16
    if v in (5, 6):
        return sizes is not None and all(17 <= x <= 24 for x in sizes)
    return True
DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "mi355x.json")


def size_class(edge: int) -> int:
    """0: 1-8, 1: 9-16, 2: 17-24, 3: 25-32."""
    if not 1 <= edge <= 32:
        raise ValueError("block edge outside 1..32")
    return (edge + 7) // 8 - 1


def class_workload(m: int, n: int, ks, atoms: int = 1500, cutoff: float = 7.0, seed: int = 0):
    """A (rows of size m) and B (columns of size n) on a DFT-like pattern;
    contraction sizes drawn from ks.  Every result block is m x n."""
    from . import inputs
    rng = inputs.rng_for(70, 0, seed)
    at = inputs.make_atoms(atoms, rng, sizes=tuple(ks))
    r, c, d = inputs.neighbour_pairs(at, cutoff)
    scale = np.exp(-d / 2.0)
    ms = np.full(atoms, m, dtype=np.int32)
    ns = np.full(atoms, n, dtype=np.int32)
    a = inputs.from_pattern(ms, at.sizes, r, c, inputs.rng_for(70, 1, seed), scale=scale)
    b = inputs.from_pattern(at.sizes, ns, r, c, inputs.rng_for(70, 2, seed), scale=scale)
    return a, b


def time_gemm(bsmm, ctx, A, B, reps: int = 3) -> float:
    """Median GEMM time (ms) over reps multiplies after one warm-up."""
    C, _ = bsmm.multiply(ctx, "N", "N", 1.0, A, B)
    C.close()
    ts = []
    for _ in range(reps):
        C, info = bsmm.multiply(ctx, "N", "N", 1.0, A, B)
        ts.append(info.ms_gemm)
        C.close()
    return statistics.median(ts)


def tune(sizes=(5, 13, 23), atoms: int = 1500, reps: int = 3, log=None) -> dict:
    """Time every variant for every (m, n) in sizes x sizes; returns the table."""
    import torch

    from . import bsmm
    ctx = bsmm.Context(0)
    ctx.set_timing(True)
    entries = {}
    tile = None
    for m in sizes:
        for n in sizes:
            key = (size_class(m), size_class(n))
            a, b = class_workload(m, n, sizes, atoms=atoms)
            A = bsmm.Matrix.from_host(ctx, a)
            B = bsmm.Matrix.from_host(ctx, b)
            times = {}
            for v in VARIANTS:
                if not applies(v, m, n, sizes):
                    continue
                ctx.set_gemm_variant(m, n, v)
                times[v] = time_gemm(bsmm, ctx, A, B, reps)
            best = min(times, key=times.get)
            entries[key] = {"m_class": key[0], "n_class": key[1], "m": m, "n": n, "variant": best,
                            "variant_name": VARIANTS[best], "gemm_ms": {VARIANTS[v]: round(t, 4) for v, t in times.items()}}
            if log:
                log(f"m={m} n={n}: " + ", ".join(f"{VARIANTS[v]} {t:.3f} ms" for v, t in times.items())
                    + f" -> {VARIANTS[best]}")
            if best in (5, 6) and tile is None:
                ctx.set_gemm_variant(m, n, best)
                tile = tune_tile(bsmm, ctx, A, B, m, n, best, reps, log)
            ctx.set_gemm_variant(m, n, 0)
            A.close()
            B.close()
            torch.cuda.synchronize()
    ctx.close()
    out = {"device": torch.cuda.get_device_name(0), "sizes": sorted(set(sizes)),
           "workload": f"dft-like {atoms} atoms, block sizes {list(sizes)}",
           "classes": sorted(entries.values(), key=lambda e: (e["m_class"], e["n_class"]))}
    if tile is not None:
        out["tile"] = tile
    return out


DEFAULT_SCHEDULE = ((2, 2), 8192)
MARGIN = 0.02   # a schedule replaces the default only when this much faster


def pick_schedule(times: dict):
    """The fastest (shape, chunk), unless the default is within MARGIN of it:
    timings on the small tuning workload differ by about 1-2 % between runs,
    and larger workloads need not follow such small differences."""
    best = min(times, key=times.get)
    base = times.get(DEFAULT_SCHEDULE)
    if base is not None and times[best] > (1.0 - MARGIN) * base:
        return DEFAULT_SCHEDULE
    return best


def tune_tile(bsmm, ctx, A, B, m: int, n: int, variant: int, reps: int, log=None) -> dict:
    """Schedule of the tile path for the class (m, n) with the chosen tile
    variant: the result-block tile shape (the general kernel takes 2x2 to
    4x4; the uniform-size kernel 2x2 only) and the number of consecutive
    tiles handed to one XCD at a time."""
    shapes = TILE_SHAPES if variant == 6 else ((2, 2),)
    times = {}
    for sh in shapes:
        ctx.set_tile_shape(*sh)
        for ch in XCD_CHUNKS:
            ctx.set_tile_schedule(False, ch)
            times[(sh, ch)] = time_gemm(bsmm, ctx, A, B, reps)
    ctx.set_tile_shape(2, 2)
    ctx.set_tile_schedule(False, 0)
    (sh, ch) = pick_schedule(times)
    if log:
        log(f"tile schedule m={m} n={n}: " + ", ".join(f"{s[0]}x{s[1]}/{c} {t:.3f} ms" for (s, c), t in times.items())
            + f" -> {sh[0]}x{sh[1]}, chunk {ch}")
    return {"m": m, "n": n, "variant": variant, "shape": list(sh), "xcd_chunk": ch,
            "gemm_ms": {f"{s[0]}x{s[1]}/{c}": round(t, 4) for (s, c), t in times.items()}}


def pick(doc: dict, sizes) -> dict | None:
    """The table of doc tuned on exactly this block-size set, if any."""
    want = sorted(set(int(x) for x in sizes))
    for t in doc.get("tables", []):
        if sorted(t["sizes"]) == want:
            return t
    return None


def apply(ctx, table, sizes=None) -> int:
    """Set the tuned variant of every class on ctx.  table: a table dict, or a
    JSON document (dict or path) holding several; with a document, the table
    of `sizes` is used (none applied if there is no such table)."""
    if isinstance(table, (str, os.PathLike)):
        with open(table) as f:
            table = json.load(f)
    if "tables" in table:
        table = pick(table, sizes or ())
        if table is None:
            return 0
    for e in table["classes"]:
        edge = lambda cls: 8 * cls + 1   # noqa: E731 - any edge of the class
        ctx.set_gemm_variant(edge(e["m_class"]), edge(e["n_class"]), int(e["variant"]))
    t = table.get("tile")
    ctx.set_tile_shape(*(t["shape"] if t else (2, 2)))
    ctx.set_tile_schedule(False, int(t["xcd_chunk"]) if t else 0)
    return len(table["classes"])


def describe(table, sizes=None) -> str:
    """The tuned choices of the table of `sizes` in one line (for reports)."""
    if isinstance(table, (str, os.PathLike)):
        with open(table) as f:
            table = json.load(f)
    if "tables" in table:
        table = pick(table, sizes or ())
        if table is None:
            return "default (no tuned table for these block sizes)"
    parts = [f"{e['m']}x{e['n']}: {e['variant_name']}" for e in table["classes"]]
    t = table.get("tile")
    if t:
        parts.append(f"tile path {t['shape'][0]}x{t['shape'][1]} tiles, {t['xcd_chunk']} tiles per XCD chunk")
    return "; ".join(parts)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--size-sets", nargs="+", default=["5,13", "23", "5,13,23"])
    ap.add_argument("--atoms", type=int, default=1500)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    args = ap.parse_args(argv)
    doc = {"tables": []}
    for spec in args.size_sets:
        sizes = tuple(int(x) for x in spec.split(","))
        print(f"block sizes {sizes}", flush=True)
        doc["tables"].append(tune(sizes, args.atoms, args.reps, log=lambda s: print("  " + s, flush=True)))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {args.out}")


if __name__ == "__main__":
    sys.exit(main())
