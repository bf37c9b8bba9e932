"""Continuous-batching loop for independent block-sparse multiplications on one GPU.

Requests (C = A*B with a filter threshold) arrive over time.  The loop keeps
admitting arrived requests while their estimated device footprint fits the
HBM budget, uploads their matrices and builds their plans (the structural
part of the multiplication), then runs the numeric parts of every admitted
request as ONE batch -- a single block-GEMM launch over the result blocks of
all of them (bsmm_plans_execute) -- and returns each result as soon as its
batch is done.  Requests that arrive while a batch is on the GPU join the
next batch as memory frees up, so the device keeps working on a changing
mix of requests.  Each result is bitwise the one the request gets alone: a
result block is computed by one wavefront in a fixed order whatever else
shares the launch.

Latency of a request = completion time of its result on the device (read
back to the host) minus its arrival time; it includes waiting for admission,
the host-to-device upload of A and B, planning and execution.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    a: object                 # host block-CSR (inputs.BlockCSR)
    b: object
    eps: float = 0.0
    arrival: float = 0.0      # seconds after the start of the run
    admitted: float = math.nan
    done: float = math.nan
    flops: float = 0.0
    batch: int = -1
    nbytes: int = 0
    result: object = None     # host copy of C when keep_results
    _dev: tuple = field(default=(), repr=False)


def poisson_arrivals(n: int, rate: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate (per second)."""
    if rate <= 0:
        return np.zeros(n)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return t - t[0]   # the first request arrives at the start


def percentiles(x, qs=(50, 99)) -> dict:
    x = np.asarray(x, dtype=np.float64)
    return {f"p{q}": float(np.percentile(x, q)) for q in qs} if x.size else {f"p{q}": math.nan for q in qs}


def footprint_bytes(a, b) -> int:
    """Device bytes one request needs while it is in flight: its operands,
    their packed copies, the result (values, index, offsets, norms, work
    list) and the stacks -- from the symbolic product of the two patterns."""
    import scipy.sparse as sp
    pa = sp.csr_matrix((np.ones(a.nnzb, dtype=np.int8), a.col_idx, a.row_ptr), shape=(a.nbr, a.nbc))
    pb = sp.csr_matrix((np.ones(b.nnzb, dtype=np.int8), b.col_idx, b.row_ptr), shape=(b.nbr, b.nbc))
    pc = (pa.astype(np.int64) @ pb.astype(np.int64)).tocoo()
    c_vals = int(np.sum(a.rbs[pc.row].astype(np.int64) * b.cbs[pc.col].astype(np.int64)))
    n_prod = int(np.sum(np.diff(b.row_ptr)[a.col_idx]))
    ab = 8 * (a.n_values() + b.n_values())
    return int(ab + 1.2 * ab + 8 * c_vals + 40 * pc.nnz + 8 * n_prod + (1 << 20))


class Server:
    """The request loop on one context (one device, one stream)."""

    def __init__(self, ctx, budget_bytes: int, max_batch: int = 64, keep_results: bool = False):
        self.ctx = ctx
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.keep = keep_results
        self.batches = []      # number of requests per batch

    def run(self, requests) -> list:
        from . import bsmm
        torch = bsmm._torch()
        queue = deque(sorted(requests, key=lambda r: r.arrival))
        for r in queue:
            r.nbytes = footprint_bytes(r.a, r.b)
            if r.nbytes > self.budget:
                raise ValueError(f"request {r.rid} needs {r.nbytes} bytes, above the budget {self.budget}")
        t0 = time.perf_counter()
        done = []
        while queue:
            now = time.perf_counter() - t0
            if queue[0].arrival > now:
                time.sleep(min(queue[0].arrival - now, 0.05))
                continue
            # admit arrived requests while they fit the budget
            batch, used = [], 0
            while queue and queue[0].arrival <= time.perf_counter() - t0 and len(batch) < self.max_batch:
                r = queue[0]
                if used + r.nbytes > self.budget:
                    break
                queue.popleft()
                used += r.nbytes
                r.admitted = time.perf_counter() - t0
                A = bsmm.Matrix.from_host(self.ctx, r.a)
                B = bsmm.Matrix.from_host(self.ctx, r.b)
                plan = bsmm.Plan(self.ctx, "N", "N", 1.0, A, B, filter_eps=r.eps)
                r.flops = plan.info.useful_flops
                r._dev = (A, B, plan)
                batch.append(r)
            # one batched execution of every admitted request
            bsmm.plans_execute([r._dev[2] for r in batch])
            self.batches.append(len(batch))
            for r in batch:
                A, B, plan = r._dev
                C = plan.result()           # post filter, synchronises the stream
                if self.keep:
                    r.result = C.to_host()
                r.done = time.perf_counter() - t0
                r.batch = len(self.batches) - 1
                C.close()
                plan.close()
                A.close()
                B.close()
                r._dev = ()
                done.append(r)
            torch.cuda.synchronize()
        return done


def summary(done, makespan: float | None = None) -> dict:
    lat = [r.done - r.arrival for r in done]
    flops = sum(r.flops for r in done)
    span = makespan if makespan is not None else (max(r.done for r in done) - min(r.arrival for r in done))
    out = {"requests": len(done), "useful_flops": flops, "makespan_s": span,
           "throughput_gflops": flops / span / 1e9 if span > 0 else math.nan,
           "requests_per_s": len(done) / span if span > 0 else math.nan}
    out.update({f"latency_{k}_ms": v * 1e3 for k, v in percentiles(lat).items()})
    return out
