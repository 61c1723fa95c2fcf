"""Continuous-batching service of PIC runs on one GPU.

Requests (a run's parameters, initial particles and step count) arrive over
time.  The server admits each one into a batch (the C ABI's pic_batch_*) as
soon as its HBM footprint fits the arena and a run-table slot is free, keeps
its state resident, steps every admitted run together (one persistent
particle launch plus one solve launch per step, replayed from a captured
graph), and retires each run the moment the device has finished it: its
diagnostics are read (without waiting for the other runs' queued work) and
its slot and memory go to the next waiting request.  Runs that arrive while
others are on the device join the very next launch, so their work overlaps.

All device work is in the HIP engine; this module only decides when to call
it and keeps the clock.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import inputs as I
from . import pic as P


@dataclass
class Request:
    """One simulation request: parameters, host payload and step count."""
    index: int
    arrival: float                 # seconds after the start of the load
    spec: I.RunSpec
    nsteps: int
    x: np.ndarray                  # x^0 [np], FP64
    v: np.ndarray                  # v^{-1/2} [np], FP64

    @property
    def work(self) -> int:
        return self.spec.np_ * self.nsteps


@dataclass
class Result:
    index: int
    np_: int
    ng: int
    nsteps: int
    arrival: float
    admitted: float
    completed: float
    diag: dict
    history: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.completed - self.arrival

    @property
    def wait(self) -> float:
        return self.admitted - self.arrival


class VirtualClock:
    """A clock that advances by `tick` seconds each time the server loop
    turns (and jumps forward when the server would sleep).  With it, the
    order of admissions depends only on the arrival schedule and the budget,
    not on how fast the device is."""

    def __init__(self, tick: float):
        self.t = 0.0
        self.tick = tick

    def now(self) -> float:
        return self.t

    def advance(self) -> None:
        self.t += self.tick

    def sleep_until(self, t: float) -> None:
        self.t = max(self.t, t)


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def advance(self) -> None:
        pass

    def sleep_until(self, t: float) -> None:
        d = t - self.now()
        if d > 0:
            time.sleep(min(d, 0.002))


def make_requests(nruns: int, rate: float = 50.0, seed_runs: int = 4, seed_arrivals: int = 4,
                  steps_range=(100, 2000), np_scale: float = 1.0, workers: int = 16) -> List[Request]:
    """The serving load: runs drawn as the batched ensemble with step counts
    uniform in `steps_range`, Poisson arrivals at `rate` per second; payloads
    are generated up front (they are the clients' data)."""
    from concurrent.futures import ThreadPoolExecutor
    specs = I.ensemble(nruns=nruns, seed=seed_runs, np_scale=np_scale, steps_range=steps_range)
    arrivals = I.arrival_times(nruns, rate=rate, seed=seed_arrivals)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(lambda s: s.particles(), specs))
    return [Request(k, float(arrivals[k]), s, s.nsteps, x, v)
            for k, (s, (x, v)) in enumerate(zip(specs, parts))]


class Server:
    """Admission, stepping and retirement around one batch.

    budget       bytes of the device arena shared by all resident runs
    chunk        steps issued per turn of the loop
    depth        chunks allowed in flight before the host waits (0: wait for
                 each chunk, which makes retirement order deterministic)
    keep_history copy each run's per-step history out when it retires
    """

    def __init__(self, budget: int, ng_max: int = 2048, max_runs: int = 256, chunk: int = 10,
                 graph_steps: int = 10, depth: int = 2, stream: Optional[int] = None,
                 keep_history: bool = False, clock=None):
        import torch
        self.torch = torch
        if stream is None:
            self._stream_obj = torch.cuda.Stream()      # non-blocking, default priority
            stream = self._stream_obj.cuda_stream
            self._tstream = self._stream_obj
        else:
            self._stream_obj = None
            self._tstream = torch.cuda.ExternalStream(stream)
        self.stream = stream
        self.batch = P.pic_batch_create(budget, ng_max, max_runs=max_runs, graph_steps=graph_steps,
                                        stream=stream)
        self.budget = budget
        self.ng_max = ng_max
        self.chunk = chunk
        self.depth = depth
        self.keep_history = keep_history
        self.clock = clock or WallClock()
        self.waiting: deque = deque()         # arrived, not admitted
        self.active: Dict[int, tuple] = {}     # run id -> (request, admitted time, last launch)
        self.issued = 0                        # batch launches issued
        self.inflight: deque = deque()         # events of issued chunks
        self.results: List[Result] = []
        self.max_resident = 0
        self.admit_blocked = 0                 # turns on which the head request did not fit

    # -------------------------------------------------------------- steps
    def _admit(self) -> None:
        now = self.clock.now()
        while self.waiting:
            req = self.waiting[0]
            p = P.make_params(req.spec.L, req.spec.ng, req.spec.np_, req.spec.dt, req.spec.qm,
                              req.spec.rho0, history_cap=req.nsteps if self.keep_history else 0)
            try:
                rid = P.pic_batch_admit(self.batch, p, req.x, req.v, req.nsteps)
            except P.PicBudget:
                self.admit_blocked += 1
                break                                     # first come, first served
            self.waiting.popleft()
            self.active[rid] = (req, now, self.issued + req.nsteps)
        self.max_resident = max(self.max_resident, len(self.active))

    def _remaining(self) -> int:
        return max((last - self.issued for (_, _, last) in self.active.values()), default=0)

    def _issue(self) -> bool:
        n = min(self.chunk, self._remaining())
        if n <= 0:
            return False
        P.pic_batch_step(self.batch, n)
        self.issued += n
        ev = self.torch.cuda.Event()
        ev.record(self._tstream)
        self.inflight.append(ev)
        while len(self.inflight) > self.depth:
            self.inflight.popleft().synchronize()
        return True

    def _retire(self) -> None:
        done = P.pic_batch_poll(self.batch)
        if not done:
            return
        now = self.clock.now()
        for rid in done:
            req, admitted, _ = self.active.pop(rid)
            view = P.pic_batch_run(self.batch, rid)
            diag, _, _ = P.pic_diagnostics(view)
            hist = P.pic_read_history(view, 0, req.nsteps) if (self.keep_history and req.nsteps) else None
            P.pic_batch_release(self.batch, rid)
            self.results.append(Result(req.index, req.spec.np_, req.spec.ng, req.nsteps, req.arrival,
                                       admitted, now, diag, hist))

    # ---------------------------------------------------------------- loop
    def run(self, requests: Sequence[Request]) -> List[Result]:
        for r in requests:
            # a run larger than the whole arena would wait at the head forever
            need = P.pic_footprint(P.make_params(r.spec.L, r.spec.ng, r.spec.np_, r.spec.dt, r.spec.qm, r.spec.rho0,
                                                 history_cap=r.nsteps if self.keep_history else 0)) - 256
            if need > self.budget:
                raise ValueError(f"request {r.index} needs {need} bytes, more than the {self.budget}-byte budget")
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.index)))
        total = len(pending)
        while len(self.results) < total:
            now = self.clock.now()
            while pending and pending[0].arrival <= now:
                self.waiting.append(pending.popleft())
            if self.waiting:
                self._admit()
            issued = self._issue()
            self._retire()
            if not issued:
                if self.active:
                    # everything is issued: wait for the device, then retire
                    while self.inflight:
                        self.inflight.popleft().synchronize()
                    self._retire()
                    if self.active:
                        time.sleep(0)
                elif pending and not self.waiting:
                    self.clock.sleep_until(pending[0].arrival)
            self.clock.advance()
        return sorted(self.results, key=lambda r: r.index)

    def close(self) -> None:
        if self.batch is not None:
            P.pic_batch_destroy(self.batch)
            self.batch = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def summarize(results: Sequence[Result], budget: int) -> dict:
    lat = np.array([r.latency for r in results])
    wait = np.array([r.wait for r in results])
    work = sum(r.np_ * r.nsteps for r in results)
    t_end = max(r.completed for r in results)
    t_start = min(r.arrival for r in results)
    span = t_end - t_start
    return {
        "runs": len(results),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "p99_admission_wait_s": float(np.percentile(wait, 99)),
        "particle_steps": int(work),
        "aggregate_particle_steps_per_s": work / span if span > 0 else math.nan,
        "span_s": span,
        "budget_bytes": int(budget),
    }


def serve_load(nruns: int = 1000, rate: float = 50.0, budget: int = 200 << 30, np_scale: float = 1.0,
               stream: Optional[int] = None, requests: Optional[List[Request]] = None,
               log: Optional[Callable[[str], None]] = None) -> dict:
    """Replay the Poisson serving load on the wall clock and report p50/p99
    completion latency and aggregate particle-steps/s."""
    if requests is None:
        t = time.perf_counter()
        requests = make_requests(nruns, rate=rate, np_scale=np_scale)
        if log:
            log(f"serving: generated {len(requests)} requests in {time.perf_counter() - t:.1f} s")
    ng_max = max(r.spec.ng for r in requests)
    with Server(budget, ng_max=ng_max, stream=stream) as srv:
        results = srv.run(requests)
        out = summarize(results, budget)
        out["max_resident_runs"] = srv.max_resident
        out["admission_blocked_turns"] = srv.admit_blocked
    offered = sum(r.work for r in requests) / max(r.arrival for r in requests)
    out["offered_particle_steps_per_s"] = offered
    out["rate_per_s"] = rate
    return out
