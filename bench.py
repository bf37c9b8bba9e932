#!/usr/bin/env python3
"""Benchmark of the local block-sparse multiply on one MI355X.

One step = one whole multiplication C = A*B through the C ABI (index views,
block norms, symbolic phase, stack generation, FP64 MFMA block GEMM,
post-filter), with A and B already resident in HBM.  Workload: 4,000 atoms
in a periodic cube at 0.1 atoms/A^3, block sizes 5/13 (50/50), blocks kept
within 7 A, values N(0,1) exp(-r/2), on-the-fly and post filter eps 1e-10.

Prints ONE JSON line.  `value` is useful FP64 GFLOP/s (sum of 2*m*k*n over
kept block products divided by the step time).  `roofline` reports the
block-GEMM kernel against the FP64 matrix-core peak, timed with HIP events
the library records on the stream it launches on.  `cpu_baseline` times the
CPU oracle on a seeded sample of block rows.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
SIGN_ATOMS, SIGN_EPS, SIGN_TOL, SIGN_MAX_ITER = 1000, 1e-6, 1e-4, 20
SERVE_ATOMS, SERVE_BUDGET_GB = (200, 1500), 64   # serving stand-in: atoms log-uniform in this range
BATCH_ATOMS, BATCH_OCC, BATCH_PANEL = 20000, 0.03, 2500   # batching workload: one process's panel of C rows
PANEL_SAMPLE = 0.01   # fraction of the panel's rows the oracle checks
HBM_PEAK_GBS = 8000.0
METRIC = "useful FP64 GFLOP/s of block-sparse C+=A·B, % MFMA peak; p99 serve latency"


def _log(msg: str):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def workload(name: str):
    from paper_1705_10218_amd import inputs
    if name == "dft4000":
        a, b, atoms = inputs.config_dft(4000)
        cfg = {"workload": "dft_like_4000_atoms_blocks_5_13", "atoms": 4000, "block_sizes": [5, 13],
               "cutoff_A": 7.0, "density_per_A3": 0.1, "filter_eps": 1e-10, "box_A": round(atoms.box, 3)}
        return a, b, 1e-10, cfg
    if name == "tiny":
        a, b = inputs.config_tiny(0), inputs.config_tiny(1)
        return a, b, 0.0, {"workload": "tiny_100x100_blocks_5", "filter_eps": 0.0}
    if name in ("panel23", "panel_mixed"):   # a batching workload's panel, as the timed step (profiling)
        sizes = (23,) if name == "panel23" else (5, 13, 23)
        pb = inputs.batching_problem(BATCH_ATOMS, BATCH_OCC, sizes=sizes)
        a = inputs.batching_matrix(pb, 1, (0, BATCH_PANEL))
        b = inputs.batching_matrix(pb, 2)
        tag = "_".join(str(x) for x in sizes)
        return a, b, 1e-10, {"workload": f"batching_{BATCH_ATOMS}_atoms_blocks_{tag}_panel_{BATCH_PANEL}_rows",
                             "atoms": BATCH_ATOMS, "block_sizes": list(sizes), "panel_rows": [0, BATCH_PANEL],
                             "filter_eps": 1e-10, "box_A": round(pb.box, 3), "cutoff_A": round(pb.cutoff, 3)}
    raise SystemExit(f"unknown workload {name}")


# block-GEMM path (bsmm_multiply_info.gemm_path) -> name, and the kernel
# whose roofline a path reports
PATH_NAMES = {0: "packed", 1: "walker", 2: "tile", 3: "lowp", 4: "tile_uniform", 5: "packed_per_unit"}
ROOFLINE_KERNEL = {0: "packed", 2: "tile", 4: "tile_uniform", 5: "packed"}

CSRC = os.path.join(ROOT, "paper_1705_10218_amd", "csrc")
PROFILE_DIR = os.path.join(ROOT, "profiles")
# block-GEMM kernels: (source file, counter summaries per workload under profiles/)
GEMM_KERNELS = {
    "packed": ("k_gemm_f64 (batched block GEMM, all size classes in one launch)", "gemm_kernels.hip", "k_gemm_f64"),
    "tile": ("k_tile_gemm<2,2> (block GEMM over tiles of C blocks, operands staged in LDS)", "tile_gemm.hip",
             "k_tile_gemm"),
    "tile_uniform": ("k_tile_uni<23,false,false> (tile GEMM, every block 23x23, sizes fixed at compile time)",
                     "tile_gemm.hip",
                     "k_tile_uni"),
    "lowp": ("k_gemm_lowp (FP32 / split-FP32 block GEMM, packed FP32 operands)", "gemm_lowp.hip", "k_gemm_lowp"),
}


def source_digest(name: str) -> str:
    with open(os.path.join(CSRC, name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def profile_values(path_name: str, workload: str, what: str) -> dict:
    """Values of a committed counter summary (profiles/<kernel>_<workload>_<what>.md).

    A summary lists its figures as "- key: `value`" lines, among them the
    digest of the kernel's source file it was taken on; the values are used
    only while that source is unchanged, otherwise {} (the counters would
    describe another kernel).
    """
    _, src, kname = GEMM_KERNELS[path_name]
    try:
        text = open(os.path.join(PROFILE_DIR, f"{kname}_{workload}_{what}.md")).read()
    except OSError:
        return {}
    kv = dict(re.findall(r"^- ([a-z_0-9]+): `([^`]*)`", text, re.M))
    if kv.get("source_sha256_16") != source_digest(src):
        return {}
    out = {}
    for k, v in kv.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


def roofline(path_name: str, workload: str, flops: float, gemm_ms: float, compulsory: int) -> dict:
    """Roofline of the dominant kernel: useful flops per launch over its
    measured launch time against the FP64 MFMA peak, with the HBM traffic
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated) and the matrix-core counters
    of the committed summaries for this kernel and workload (null when the
    kernel changed since they were taken)."""
    tr = profile_values(path_name, workload, "traffic")
    mf = profile_values(path_name, workload, "mfma")
    tflops = flops / (gemm_ms * 1e-3) / 1e12
    issued = mf.get("mfma_f64_flops_per_launch") or mf.get("mfma_f32_flops_per_launch")
    peak = FP32_MFMA_PEAK_TFLOPS if path_name == "lowp" else FP64_MFMA_PEAK_TFLOPS
    return {"bound": "mfma", "kernel": GEMM_KERNELS[path_name][0], "achieved": round(tflops, 3),
            "peak": peak, "unit": "TFLOP/s", "frac": round(tflops / peak, 4),
            "traffic": tr.get("hbm_bytes_per_launch"), "traffic_unit": "bytes per launch (HBM, counter-calibrated)",
            "compulsory_bytes": compulsory, "ms_per_launch": round(gemm_ms, 4),
            "mfma_busy": mf.get("mfma_busy_frac"),
            "padding_ratio": round(issued / flops, 4) if issued else None,
            "clock_ghz_under_load": mf.get("clock_ghz")}


def copy_calibration(mib: int, reps: int):
    """Plain device-to-device copies of a known size (counter calibration)."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.randn(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8,
                      "copies": reps}))


def oracle_sample(a, b, eps, target_s: float, threads: int):
    """Time the oracle on a seeded sample of block rows (about target_s seconds)."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(12345)
    order = rng.permutation(a.nbr).astype(np.int32)
    # calibrate on a few rows, then size the sample to about target_s seconds
    probe = np.sort(order[: max(threads, 8)])
    t0 = time.perf_counter()
    oracle.multiply("N", "N", 1.0, a, b, eps=eps, nthreads=threads, rows=probe)
    dt = time.perf_counter() - t0
    per_row = dt / len(probe)
    n = int(min(a.nbr, max(len(probe), target_s / max(per_row, 1e-9))))
    rows = np.sort(order[:n])
    t0 = time.perf_counter()
    r = oracle.multiply("N", "N", 1.0, a, b, eps=eps, nthreads=threads, rows=rows)
    dt = time.perf_counter() - t0
    return r, rows, dt


def sample_parity(gpu_host, r, rows):
    """Pattern equality and relative Frobenius error of the sampled rows."""
    import numpy as np

    from paper_1705_10218_amd.inputs import BlockCSR
    go = BlockCSR(gpu_host.rbs, gpu_host.cbs, gpu_host.row_ptr, gpu_host.col_idx, gpu_host.values).block_offsets()
    ro = BlockCSR(r.rbs, r.cbs, r.row_ptr, r.col_idx, r.values).block_offsets()
    num = den = 0.0
    pattern_ok = True
    for i in rows:
        g0, g1 = gpu_host.row_ptr[i], gpu_host.row_ptr[i + 1]
        r0, r1 = r.row_ptr[i], r.row_ptr[i + 1]
        if not np.array_equal(gpu_host.col_idx[g0:g1], r.col_idx[r0:r1]):
            pattern_ok = False
            continue
        d = gpu_host.values[go[g0]:go[g1]] - r.values[ro[r0]:ro[r1]]
        num += float(d @ d)
        den += float(r.values[ro[r0]:ro[r1]] @ r.values[ro[r0]:ro[r1]])
    rel = math.sqrt(num / den) if den > 0 else 0.0
    return {"rows": int(len(rows)), "pattern_equal": bool(pattern_ok), "rel_fro_err": rel}


def time_mode(bsmm, ctx, A, Bm, eps, steps, warmup):
    """Warm-up, then `steps` whole multiplies, each bracketed by HIP events on
    the stream; returns the mean, the per-step times, the infos and the last
    result."""
    import torch
    for _ in range(warmup):
        C, info = bsmm.multiply(ctx, "N", "N", 1.0, A, Bm, filter_eps=eps)
        C.close()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    infos = []
    torch.cuda.synchronize()
    evs[0].record(stream)
    last = None
    for t in range(steps):
        C, info = bsmm.multiply(ctx, "N", "N", 1.0, A, Bm, filter_eps=eps)
        evs[t + 1].record(stream)
        infos.append(info)
        if last is not None:
            last.close()
        last = C
    torch.cuda.synchronize()
    per = [evs[t].elapsed_time(evs[t + 1]) for t in range(steps)]
    return sum(per) / steps, per, infos, last


def step_stats(per) -> dict:
    import statistics
    return {"ms_per_step_median": round(statistics.median(per), 4), "ms_per_step_min": round(min(per), 4),
            "ms_per_step_max": round(max(per), 4)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def panel_leg(bsmm, ctx, sizes, rows, steps: int, threads: int, variants: str) -> dict:
    """The batching workload at its real shape: a panel of C block rows of
    the 20,000-atom matrices against all of B, parity-checked against the
    oracle on a seeded sample of the panel's rows."""
    import numpy as np
    import torch

    import oracle
    from paper_1705_10218_amd import inputs
    t0 = time.perf_counter()
    pb = inputs.batching_problem(BATCH_ATOMS, BATCH_OCC, sizes=sizes)
    a = inputs.batching_matrix(pb, 1, rows)
    b = inputs.batching_matrix(pb, 2)
    gen_s = time.perf_counter() - t0
    _log(f"batching {sizes}: generated A panel {a.nnzb} blocks, B {b.nnzb} blocks "
         f"({(a.values.nbytes + b.values.nbytes) / 1e9:.1f} GB) in {gen_s:.1f} s")
    A, Bm = bsmm.Matrix.from_host(ctx, a), bsmm.Matrix.from_host(ctx, b)
    torch.cuda.synchronize()
    ms, per, infos, last = time_mode(bsmm, ctx, A, Bm, 1e-10, steps, 1)
    info = infos[-1]
    fl = info.useful_flops
    g = sorted(i.ms_gemm for i in infos)
    gemm_ms = g[len(g) // 2]
    # sampled parity: the oracle on a seeded 1 % of the panel's rows
    rng = np.random.default_rng(2024)
    n_s = max(1, int(round(PANEL_SAMPLE * a.nbr)))
    sample = np.sort(rng.choice(a.nbr, n_s, replace=False)).astype(np.int32)
    gpu_host = last.to_host()
    last.close()
    t1 = time.perf_counter()
    r = oracle.multiply("N", "N", 1.0, a, b, eps=1e-10, nthreads=threads, rows=sample)
    oracle_s = time.perf_counter() - t1
    parity = sample_parity(gpu_host, r, sample)
    A.close()
    Bm.close()
    ctx.trim()
    out = {"atoms": BATCH_ATOMS, "block_sizes": list(sizes), "occupancy_target": BATCH_OCC,
           "cutoff_A": round(pb.cutoff, 3), "box_A": round(pb.box, 3), "panel_rows": [int(rows[0]), int(rows[1])],
           "a_panel_nnzb": int(a.nnzb), "b_nnzb": int(b.nnzb), "b_gb": round(b.values.nbytes / 1e9, 2),
           "c_nnzb": int(info.c_nnzb), "n_products": int(info.n_products), "useful_flops": fl,
           "ms_per_step": round(ms, 3), **step_stats(per), "gemm_ms": round(gemm_ms, 3),
           "value": round(fl / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
           "gemm_tflops": round(fl / (gemm_ms * 1e-3) / 1e12, 3),
           "gemm_frac_of_fp64_mfma_peak": round(fl / (gemm_ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4),
           "gemm_path": PATH_NAMES.get(info.gemm_path, "?"),
           "roofline": (roofline(ROOFLINE_KERNEL[info.gemm_path],
                                 "panel23" if tuple(sizes) == (23,) else "panel_mixed", fl, gemm_ms,
                                 int(8 * (a.n_values() + b.n_values() + info.c_n_values)))
                        if info.gemm_path in ROOFLINE_KERNEL else None),
           "gemm_variants": variants, "generation_s": round(gen_s, 1),
           "sample_parity": parity,
           "oracle": {"rows": int(n_s), "threads": threads, "s": round(oracle_s, 2),
                      "gflops": round(r.useful_flops / oracle_s / 1e9, 3),
                      "extrapolated_panel_s": round(oracle_s * a.nbr / n_s, 1),
                      "note": "linear extrapolation from the sampled rows to the whole panel"}}
    _log(f"batching {sizes}: {ms:.1f} ms/step, GEMM {gemm_ms:.1f} ms ({out['gemm_tflops']} TF/s), "
         f"parity {parity}")
    return out


def tiny_latency(bsmm, torch, reps: int = 50) -> dict:
    from paper_1705_10218_amd import inputs
    st = torch.cuda.Stream()
    res = {"workload": "tiny_100x100_blocks_5", "reps": reps}
    with torch.cuda.stream(st):
        ctx = bsmm.Context(0, stream=st)
        a, b = inputs.config_tiny(0), inputs.config_tiny(1)
        A, Bm = bsmm.Matrix.from_host(ctx, a), bsmm.Matrix.from_host(ctx, b)
        st.synchronize()

        def timed(fn):
            fn()
            st.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            st.synchronize()
            return (time.perf_counter() - t0) / reps * 1e6

        def one_shot():
            C, _ = bsmm.multiply(ctx, "N", "N", 1.0, A, Bm)
            C.close()

        plan = bsmm.Plan(ctx, "N", "N", 1.0, A, Bm)
        res["useful_flops"] = plan.info.useful_flops
        res["multiply_us"] = round(timed(one_shot), 2)
        res["plan_execute_us"] = round(timed(plan.execute), 2)
        plan.capture()
        res["graph_replay_us"] = round(timed(plan.execute), 2)
        plan.close()
        A.close()
        Bm.close()
        ctx.close()
    _log(f"tiny latency: {res}")
    return res


def config5_estimate(n: int = 512, atoms=(200, 8000), sizes=(5, 13, 23)) -> dict:
    """Expected size of the full serving configuration from its request
    parameters (no matrices built): blocks per row 1 + rho 4/3 pi r^3 (at most
    the atom count), block areas and product flops from the uniform size mix."""
    import numpy as np

    from paper_1705_10218_amd import inputs
    ms = np.asarray(sizes, dtype=np.float64)
    area, cube = float(np.mean(ms) ** 2), float(np.mean(ms) ** 3)
    vals = flops = 0.0
    for na, occ, rc in inputs.serving_request_params(n, atoms=atoms, seed=1):
        per_row = min(na, 1.0 + inputs.DENSITY * 4.0 / 3.0 * math.pi * rc ** 3)
        vals += 2.0 * na * per_row * area
        flops += 2.0 * cube * na * per_row * per_row
    return {"requests": n, "atoms_log_uniform": list(atoms), "block_sizes": list(sizes),
            "input_bytes_estimate": round(8.0 * vals), "useful_flops_estimate": float(f"{flops:.3e}")}


def serving_leg(bsmm, n: int, configure=None, lanes: int = 2) -> dict:
    import numpy as np

    from paper_1705_10218_amd import inputs, serve
    t0 = time.perf_counter()
    gen = inputs.serving_requests(n, atoms=SERVE_ATOMS, occupancy=(0.02, 0.20), seed=1)
    gen_s = time.perf_counter() - t0
    budget = SERVE_BUDGET_GB << 30

    def requests(arrivals):
        return [serve.Request(rid=i, a=a, b=b, eps=1e-10, arrival=float(t)) for i, ((a, b, _), t) in
                enumerate(zip(gen, arrivals))]

    srv = serve.Server(0, budget, max_batch=64, configure=configure, lanes=lanes)
    sat = serve.summary(srv.run(requests(np.zeros(n))))
    rate = 0.7 * sat["requests_per_s"]
    # a seeded three of the requests (among those of at most 500 atoms, so
    # that the oracle takes seconds) are read back and checked against the
    # oracle; only those are read back inside the loop
    small = [i for i, (a, _, _) in enumerate(gen) if a.nbr <= 500]
    pick = sorted(int(x) for x in np.random.default_rng(7).choice(small, size=min(3, len(small)), replace=False)) \
        if small else []
    srv2 = serve.Server(0, budget, max_batch=64, configure=configure, keep_results=pick, lanes=lanes)
    done = srv2.run(requests(serve.poisson_arrivals(n, rate, np.random.default_rng(5))))
    st = serve.summary(done)
    import oracle
    checks = []
    byid = {r.rid: r for r in done}
    for rid in pick:
        r = byid[rid]
        ref = oracle.multiply("N", "N", 1.0, r.a, r.b, eps=r.eps, nthreads=len(os.sched_getaffinity(0)))
        same = bool(np.array_equal(ref.row_ptr, r.result.row_ptr) and np.array_equal(ref.col_idx, r.result.col_idx))
        err = float(np.linalg.norm(r.result.values - ref.values) / max(np.linalg.norm(ref.values), 1e-300)) \
            if same else None
        checks.append({"request": rid, "atoms": int(r.a.nbr), "pattern_equal": same, "rel_fro_err": err})
    for r in done:
        r.result = None
    _log(f"serving: saturation {sat['requests_per_s']:.1f} req/s, at 0.7x: p50 {st['latency_p50_ms']:.1f} ms "
         f"p99 {st['latency_p99_ms']:.1f} ms, {len(srv2.batches)} batches, {srv2.overlapping_batches()} overlapping")
    full = config5_estimate()
    return {"workload": "stand-in for the serving configuration (fewer, smaller requests)",
            "requests": n, "atoms_log_uniform": list(SERVE_ATOMS), "occupancy_uniform": [0.02, 0.20],
            "block_sizes": [5, 13, 23], "filter_eps": 1e-10, "hbm_budget_gb": SERVE_BUDGET_GB, "lanes": lanes,
            "generation_s": round(gen_s, 1),
            "saturation": {"requests_per_s": round(sat["requests_per_s"], 3),
                           "gflops": round(sat["throughput_gflops"], 2), "batches": len(srv.batches)},
            "arrival_rate_per_s": round(rate, 3), "arrival_rate_rule": "0.7 x measured saturation",
            "latency_p50_ms": round(st["latency_p50_ms"], 3), "latency_p99_ms": round(st["latency_p99_ms"], 3),
            "latency_parts_ms": st["latency_parts_ms"],
            "throughput_gflops": round(st["throughput_gflops"], 2), "batches": len(srv2.batches),
            "overlapping_batches": srv2.overlapping_batches(),
            "mean_batch": round(float(np.mean(srv2.batches)), 2), "useful_flops": st["useful_flops"],
            "sample_parity": checks,
            "full_configuration": dict(full, run=False,
                                       reason="512 requests up to 8,000 atoms need about "
                                              f"{full['input_bytes_estimate'] / 1e12:.1f} TB of generated input and "
                                              f"{full['useful_flops_estimate']:.2e} useful flops: far beyond the "
                                              "bench's few minutes; the stream above is scaled down, not the "
                                              "configuration")}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="dft4000", choices=["dft4000", "tiny", "panel23", "panel_mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--fp64-only", action="store_true",
                    help="only the headline FP64 workload (no precision, batching or sign-iteration legs)")
    ap.add_argument("--no-tuning", action="store_true", help="default GEMM kernel variants instead of the tuned table")
    ap.add_argument("--serve-requests", type=int, default=64, help="requests of the serving leg (0: skip it)")
    ap.add_argument("--no-batching", dest="batching", action="store_false",
                    help="skip the 20,000-atom batching legs (about 70 GB of host data)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--compute-mode", choices=["fp64", "fp32", "split"], default="fp64",
                    help="arithmetic of the timed workload's block products (profiling the FP32 and split "
                         "paths; with fp32 or split only that workload runs, as with --fp64-only)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run plain device copies of this size (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multiply runs on a single MI355X).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1705_10218_amd import bsmm, inputs
    if not torch.cuda.is_available():
        raise SystemExit("no HIP device visible")
    if args.calibrate_copy_mib > 0:
        copy_calibration(args.calibrate_copy_mib, 3)
        return

    _log("generating workload")
    a, b, eps, cfg = workload(args.workload)
    ctx = bsmm.Context(0)
    from paper_1705_10218_amd import autotune
    def tune_for(sizes):
        """Tuned GEMM variants and tile-path schedule of this block-size set,
        if the table has them; returns what was set."""
        for m in (5, 13, 23, 32):
            for n in (5, 13, 23, 32):
                ctx.set_gemm_variant(m, n, 0)
        ctx.set_tile_shape(2, 2)
        ctx.set_tile_schedule(False, 0)
        if args.no_tuning or not os.path.exists(autotune.DEFAULT_TABLE):
            return "default"
        if autotune.apply(ctx, autotune.DEFAULT_TABLE, sizes) == 0:
            return "default (no tuned table for these block sizes)"
        return (f"autotuned ({os.path.relpath(autotune.DEFAULT_TABLE, ROOT)}): "
                + autotune.describe(autotune.DEFAULT_TABLE, sizes))

    cfg["gemm_variants"] = tune_for(cfg.get("block_sizes", [5]))
    A = bsmm.Matrix.from_host(ctx, a)
    Bm = bsmm.Matrix.from_host(ctx, b)
    torch.cuda.synchronize()
    ctx.set_timing(True)

    mode = {"fp64": 0, "fp32": 1, "split": 2}[args.compute_mode]
    if mode:
        args.fp64_only = True   # the other legs measure FP64 (and the precision leg both modes)
        ctx.set_compute_mode(mode)
    _log(f"warmup {args.warmup}, timing {args.steps} steps ({args.compute_mode})")
    ms_step, per_step, infos, last = time_mode(bsmm, ctx, A, Bm, eps, args.steps, args.warmup)
    _log(f"{ms_step:.3f} ms/step")

    flops = infos[-1].useful_flops
    value = flops / (ms_step * 1e-3) / 1e9
    gemm_ms = sum(i.ms_gemm for i in infos) / len(infos)
    phases = {k: round(sum(getattr(i, k) for i in infos) / len(infos), 4)
              for k in ("ms_index", "ms_norms", "ms_symbolic", "ms_stacks", "ms_gemm", "ms_filter", "ms_total")}
    gemm_tflops = flops / (gemm_ms * 1e-3) / 1e12
    gpu_host = last.to_host()
    last.close()
    # compulsory HBM bytes of the GEMM launch: A and B values once, C values once
    compulsory = int(8 * (a.n_values() + b.n_values() + infos[-1].c_n_values))
    path_name = {**ROOFLINE_KERNEL, 3: "lowp"}.get(infos[-1].gemm_path, "packed")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        **step_stats(per_step),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "split": "f32x2 (split FP64)"}[args.compute_mode],
        "data": "synthetic (seeded generator, DFT-like block pattern)",
        "config": cfg,
        "pct_fp64_mfma_peak": round(100.0 * value / (FP64_MFMA_PEAK_TFLOPS * 1e3), 2),
        "useful_flops_per_step": flops,
        "c_nnzb": int(infos[-1].c_nnzb),
        "n_products": int(infos[-1].n_products),
        "phases_ms": phases,
        "roofline": roofline(path_name, args.workload if not mode else f"{args.workload}_{args.compute_mode}", flops,
                             gemm_ms, compulsory),
    }
    # FP32 and split-FP32 modes on the same matrices (norms and filters FP64)
    lowp_hosts = {}
    if not args.fp64_only:
        prec = {}
        for name, mode in (("fp32", 1), ("split", 2)):
            ctx.set_compute_mode(mode)
            ms_m, _, inf_m, last_m = time_mode(bsmm, ctx, A, Bm, eps, args.steps, 1)
            ctx.set_compute_mode(0)
            g_m = sum(i.ms_gemm for i in inf_m) / len(inf_m)
            prec[name] = {"value": round(inf_m[-1].useful_flops / (ms_m * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
                          "ms_per_step": round(ms_m, 4), "gemm_ms": round(g_m, 4),
                          "speedup_vs_fp64": round(ms_step / ms_m, 3),
                          "gemm_tflops": round(inf_m[-1].useful_flops / (g_m * 1e-3) / 1e12, 3),
                          "frac_of_fp32_mfma_peak": round(inf_m[-1].useful_flops / (g_m * 1e-3) / 1e12
                                                          / FP32_MFMA_PEAK_TFLOPS, 4)}
            _log(f"{name}: {ms_m:.3f} ms/step")
            lowp_hosts[name] = last_m.to_host()
            last_m.close()
        out["precision"] = prec
    # batching workloads at their real shape: a panel of 2,500 C block rows of
    # the 20,000-atom matrices (23x23 blocks, and sizes {5, 13, 23}) against
    # all of B, each parity-checked on a seeded sample of its rows
    threads = len(os.sched_getaffinity(0))
    if not args.fp64_only and args.batching:
        A.close()
        Bm.close()
        ctx.trim()
        torch.cuda.empty_cache()
        batching = {}
        for name, sizes in (("blocks_23", (23,)), ("blocks_5_13_23", (5, 13, 23))):
            batching[name] = panel_leg(bsmm, ctx, sizes, (0, BATCH_PANEL), 5, threads, tune_for(sizes))
            torch.cuda.empty_cache()
        out["batching"] = batching
        A = bsmm.Matrix.from_host(ctx, a)
        Bm = bsmm.Matrix.from_host(ctx, b)
    # latency of the tiny multiply (100x100 blocks of 5): one-shot multiply,
    # re-execution of its plan's numeric part, and the same part replayed
    # from a HIP graph (fixed pattern, values changing between calls)
    if not args.fp64_only:
        out["tiny_latency"] = tiny_latency(bsmm, torch)
    # serving: independent requests (DFT-like, sizes {5, 13, 23}, 2-20 %
    # occupancy) through the continuous-batching loop; first all at once
    # (saturation throughput), then Poisson arrivals at 0.7 of that rate
    if not args.fp64_only and args.serve_requests > 0:
        variants = tune_for((5, 13, 23))
        tuned = not (args.no_tuning or not os.path.exists(autotune.DEFAULT_TABLE))
        out["serving"] = serving_leg(
            bsmm, args.serve_requests,
            configure=(lambda c: autotune.apply(c, autotune.DEFAULT_TABLE, (5, 13, 23))) if tuned else None)
        out["serving"]["gemm_variants"] = variants
    # second workload: Newton-Schulz sign iteration (two filtered multiplies
    # per step, pattern evolving then stabilising)
    if not args.fp64_only:
        tune_for((5, 13))
        x0 = inputs.symmetric_dft_like(SIGN_ATOMS, config=4, sizes=(5, 13), cutoff=7.0)
        X0 = bsmm.Matrix.from_host(ctx, x0)
        torch.cuda.synchronize()
        Y, sinfo, sres, snnz = bsmm.sign_newton_schulz(ctx, X0, SIGN_MAX_ITER, SIGN_EPS, SIGN_TOL)
        torch.cuda.synchronize()
        out["sign_iteration"] = {
            "workload": f"symmetric_dft_like_{SIGN_ATOMS}_atoms_blocks_5_13", "filter_eps": SIGN_EPS, "tol": SIGN_TOL,
            "iterations": sinfo.iterations, "converged": bool(sinfo.converged), "residual": sinfo.residual,
            "ms_total": round(sinfo.ms_total, 3), "ms_per_iteration": round(sinfo.ms_total / max(sinfo.iterations, 1), 3),
            "value": round(sinfo.useful_flops / (sinfo.ms_total * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
            "x0_nnzb": int(x0.nnzb), "nnzb_trace": [int(v) for v in snnz],
            "plan_reuses": int(sinfo.plan_reuses),
            "residual_trace": [float(f"{v:.4g}") for v in sres],
        }
        _log(f"sign iteration: {sinfo.iterations} steps, {sinfo.ms_total:.1f} ms")
        Y.close()
        X0.close()
    if not args.no_cpu_baseline:
        _log(f"cpu baseline on {threads} threads")
        r, rows, dt = oracle_sample(a, b, eps, args.cpu_seconds, threads)
        out["cpu_baseline"] = {
            "value": round(r.useful_flops / dt / 1e9, 3),
            "unit": "GFLOP/s",
            "cores": threads,
            "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": (f"{len(rows)} of {a.nbr} seeded block rows of C ({r.useful_flops:.3e} useful flops, "
                       f"{100.0 * len(rows) / a.nbr:.1f}% of rows), {dt:.2f} s wall"),
            "sample_parity": sample_parity(gpu_host, r, rows),
        }
        for name, h in lowp_hosts.items():
            out["precision"][name]["sample_parity"] = sample_parity(h, r, rows)
    A.close()
    Bm.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
