"""Continuous-batching loop for independent block-sparse multiplications on one GPU.

Requests (C = A*B with a filter threshold) arrive over time.  The loop works
on two lanes, each a library context with a stream of its own:

* admission -- an arrived request is admitted while the device memory of the
  requests in flight stays within the HBM budget.  Before the upload the
  request is counted with its operand bytes times the largest footprint /
  operand ratio seen so far; once its plan exists (the structural part of the
  multiplication: symbolic phase, stacks) it is counted with the sizes the
  library reports (bsmm_plan_sizes: result values and workspace, plus the
  stacks and the result index of its product counts);
* planning -- admitted requests are uploaded and planned on the lane that is
  not executing, so planning and uploads overlap the other lane's batch on
  the device;
* execution -- the planned requests of a lane run as ONE batch: a single
  block-GEMM launch over the result blocks of all of them
  (bsmm_plans_execute).  A lane launches when no batch is running, when its
  batch is full, or when its oldest request has waited max_wait_s; so the
  two lanes' batches can run on the device at the same time;
* completion -- an event per batch is polled; a finished batch's results are
  returned (post-filter, read back) and its memory is released, which lets
  waiting requests in.

Every result is bitwise the one the request gets alone: a result block is
computed by one wavefront in a fixed order whatever else shares the launch.

Latency of a request = the time its result is ready on the device (after
the post-filter) minus its arrival time; it includes waiting for admission,
the host-to-device upload of A and B, planning and execution.  With
keep_results the result is then also read back to the host (not counted).
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
    planned: float = math.nan
    launched: float = math.nan
    done: float = math.nan
    flops: float = 0.0
    batch: int = -1
    nbytes: int = 0           # device bytes counted against the budget
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


def operand_bytes(a, b) -> int:
    """Device bytes of a request's operands: FP64 values and the block index."""
    return int(8 * (a.n_values() + b.n_values()) + 16 * (a.nnzb + b.nnzb) + 8 * (a.nbr + b.nbr) + 4096)


def plan_bytes(n_products: int, c_nnzb: int, c_n_values: int, workspace: int) -> int:
    """Device bytes of a planned request beyond its operands: stacks (8 bytes
    a product), the result's index, offsets, counts and work list (48 bytes a
    block), its values and the numeric part's workspace."""
    return int(8 * n_products + 48 * c_nnzb + 8 * c_n_values + workspace)


@dataclass
class _Batch:
    reqs: list
    event: object
    launched: float
    index: int


class Lane:
    """A library context with its own stream; requests planned on it run in
    its batches."""

    def __init__(self, device: int, configure=None):
        from . import bsmm
        torch = bsmm._torch()
        self.stream = torch.cuda.Stream(device)
        self.ctx = bsmm.Context(device, stream=self.stream)
        if configure is not None:   # e.g. tuned kernel variants
            configure(self.ctx)
        self.planned = []
        self.inflight: _Batch | None = None

    def close(self):
        self.ctx.close()


class Server:
    """The request loop on one device.  The engine hooks (_new_lane, _plan,
    _launch, _finished, _complete) are the only places that touch the
    library; tests substitute them."""

    def __init__(self, device: int, budget_bytes: int, max_batch: int = 64, keep_results=False,
                 max_wait_s: float = 0.002, poll_s: float = 0.0002, configure=None, lanes: int = 2):
        if lanes < 2:
            raise ValueError("the loop needs at least two lanes (one plans while another executes)")
        self.device = device
        self.n_lanes = int(lanes)
        self.configure = configure   # called with each lane's context
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.keep = keep_results if keep_results is True else set(keep_results or ())   # True, or rids to keep
        self.max_wait = float(max_wait_s)
        self.poll = float(poll_s)
        self.batches = []          # requests per batch
        self.batch_times = []      # (launched, completed) per batch, seconds after the start
        self.expansion = 4.0       # largest footprint / operand bytes seen
        self.peak_used = 0

    # ------------------------------------------------------------ engine
    def _new_lane(self):
        return Lane(self.device, self.configure)

    def _plan(self, lane, r) -> int:
        """Upload and plan r on the lane; returns its planned device bytes."""
        from . import bsmm
        torch = bsmm._torch()
        with torch.cuda.stream(lane.stream):   # the uploads are ordered before the planning on the lane
            A = bsmm.Matrix.from_host(lane.ctx, r.a)
            B = bsmm.Matrix.from_host(lane.ctx, r.b)
        plan = bsmm.Plan(lane.ctx, "N", "N", 1.0, A, B, filter_eps=r.eps)
        nb, nv, ws = plan.sizes()
        r.flops = plan.info.useful_flops
        r._dev = (A, B, plan)
        return operand_bytes(r.a, r.b) + plan_bytes(plan.info.n_products, nb, nv, ws)

    def _launch(self, lane, reqs):
        from . import bsmm
        torch = bsmm._torch()
        bsmm.plans_execute([r._dev[2] for r in reqs])
        ev = torch.cuda.Event()
        ev.record(lane.stream)
        return ev

    def _finished(self, lane, event) -> bool:
        return bool(event.query())

    def _complete(self, lane, r):
        A, B, plan = r._dev
        C = plan.result()              # post-filter; the batch is done, so this waits for nothing else
        r.done = self._clock()         # the result is ready on the device
        if self.keep is True or (self.keep and r.rid in self.keep):
            r.result = C.to_host()
        C.close()
        plan.close()
        A.close()
        B.close()
        r._dev = ()

    # -------------------------------------------------------------- loop
    def run(self, requests) -> list:
        lanes = [self._new_lane() for _ in range(self.n_lanes)]
        try:
            return self._run(lanes, requests)
        finally:
            for ln in lanes:
                if hasattr(ln, "close"):
                    ln.close()

    def _run(self, lanes, requests) -> list:
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        for r in pending:
            if operand_bytes(r.a, r.b) > self.budget:
                raise ValueError(f"request {r.rid}: its operands alone exceed the budget {self.budget}")
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0   # noqa: E731
        self._clock = clock
        done, used, plan_lane = [], 0, 0
        while pending or any(ln.planned or ln.inflight for ln in lanes):
            progressed = False
            # completions
            for ln in lanes:
                b = ln.inflight
                if b is not None and self._finished(ln, b.event):
                    for r in b.reqs:
                        self._complete(ln, r)
                        if math.isnan(r.done):
                            r.done = clock()
                        used -= r.nbytes
                        done.append(r)
                    self.batch_times[b.index] = (b.launched, clock())
                    ln.inflight = None
                    progressed = True
            # admission and planning on a lane that is not executing
            # (planning synchronises the lane's stream)
            if lanes[plan_lane].inflight is not None:
                plan_lane = next((k for k, x in enumerate(lanes) if x.inflight is None), plan_lane)
            ln = lanes[plan_lane]
            if ln.inflight is None:
                while pending and pending[0].arrival <= clock() and len(ln.planned) < self.max_batch:
                    r = pending[0]
                    est = int(self.expansion * operand_bytes(r.a, r.b))
                    busy = any(x.planned or x.inflight for x in lanes)
                    if busy and used + est > self.budget:
                        break
                    pending.popleft()
                    r.admitted = clock()
                    used += est
                    r.nbytes = est
                    real = self._plan(ln, r)
                    used += real - est
                    r.nbytes = real
                    self.expansion = max(self.expansion, real / max(operand_bytes(r.a, r.b), 1))
                    self.peak_used = max(self.peak_used, used)
                    r.planned = clock()
                    ln.planned.append(r)
                    progressed = True
            # launch: a lane with planned requests and no batch running goes
            # when nothing else runs, its batch is full, or it waited enough
            for k in [plan_lane] + [j for j in range(len(lanes)) if j != plan_lane]:
                ln = lanes[k]
                if not ln.planned or ln.inflight is not None:
                    continue
                others = any(x.inflight is not None for x in lanes)
                waited = clock() - min(r.planned for r in ln.planned)
                arrived = bool(pending) and pending[0].arrival <= clock()
                if others and len(ln.planned) < self.max_batch and waited < self.max_wait and arrived:
                    continue
                now = clock()
                for r in ln.planned:
                    r.launched = now
                    r.batch = len(self.batches)
                ev = self._launch(ln, ln.planned)
                ln.inflight = _Batch(ln.planned, ev, now, len(self.batches))
                self.batches.append(len(ln.planned))
                self.batch_times.append((now, math.nan))
                ln.planned = []
                # plan next on another lane that is not executing
                plan_lane = next((j for j in range(len(lanes)) if lanes[j].inflight is None), plan_lane)
                progressed = True
            if not progressed:
                wait = self.poll
                if pending and not any(x.planned or x.inflight for x in lanes):
                    wait = max(0.0, min(pending[0].arrival - clock(), 0.05))
                time.sleep(wait)
        return done

    def overlapping_batches(self) -> int:
        """Batches launched while another batch was still running on the device."""
        n = 0
        for k, (l, _) in enumerate(self.batch_times):
            if any(j != k and a < l < c for j, (a, c) in enumerate(self.batch_times)):
                n += 1
        return n


def summary(done, makespan: float | None = None) -> dict:
    lat = [r.done - r.arrival for r in done]
    flops = sum(r.flops for r in done)
    span = makespan if makespan is not None else (max(r.done for r in done) - min(r.arrival for r in done))
    out = {"requests": len(done), "useful_flops": flops, "makespan_s": span,
           "throughput_gflops": flops / span / 1e9 if span > 0 else math.nan,
           "requests_per_s": len(done) / span if span > 0 else math.nan}
    out.update({f"latency_{k}_ms": v * 1e3 for k, v in percentiles(lat).items()})
    # where the latency goes: waiting for admission, upload and planning,
    # waiting for the launch, and the batch on the device up to the result
    parts = {"admission": [r.admitted - r.arrival for r in done], "upload_plan": [r.planned - r.admitted for r in done],
             "launch_wait": [r.launched - r.planned for r in done], "device": [r.done - r.launched for r in done]}
    out["latency_parts_ms"] = {name: {k: round(v * 1e3, 3) for k, v in percentiles(x).items()}
                               for name, x in parts.items()}
    return out
