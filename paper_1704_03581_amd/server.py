"""Continuous-batching fold-in server loop.

Requests are new documents whose topic proportions theta are inferred
against a fixed, device-resident Phi (fold-in).  The loop admits every
request that has arrived as soon as a slot and enough arena tokens are free
(admission by device memory), advances all resident requests together by the
same budget of token draws in one launch (a request resumes mid-sweep where
the previous step stopped, so long and short requests take the same time per
step), collects the finished ones and admits more: requests that arrive
while others are on the GPU join the running batch.

Pipelined (the default): after launching step s the loop collects the
requests finished by step s-1 and admits new ones while step s runs, so the
host's work overlaps the GPU's instead of leaving it idle between steps.

The loop drives any backend with the FoldIn interface (submit / step / poll /
occupancy), so its bookkeeping is testable without a GPU.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclass
class ServeReport:
    results: Dict[int, dict]                 # request id -> result
    latency_s: np.ndarray                    # completion - arrival, per request
    wall_s: float
    steps: int = 0
    max_resident: int = 0
    admission_waits: int = 0                 # submits refused for capacity
    order_admitted: List[int] = field(default_factory=list)
    completion_s: np.ndarray = field(default_factory=lambda: np.zeros(0))  # completion time, per request

    @property
    def docs_per_s(self) -> float:
        return len(self.results) / self.wall_s if self.wall_s > 0 else float("inf")

    def percentile_ms(self, q: float) -> float:
        return float(np.percentile(self.latency_s, q) * 1e3) if len(self.latency_s) else 0.0

    def arrival_window(self, arrivals, lo: float = 0.1, hi: float = 0.9):
        """Open-loop steady state: the requests arriving between the lo and
        hi quantiles of the arrival times.  Returns (delivered docs/s over
        that window: completions inside it per second, p50 ms, p99 ms of
        the requests arriving inside it)."""
        arr = np.asarray(arrivals, dtype=np.float64)
        n = len(arr)
        if n < 10:
            return self.docs_per_s, self.percentile_ms(50), self.percentile_ms(99)
        t_a, t_b = arr[int(lo * n)], arr[int(hi * n) - 1]
        done = self.completion_s
        delivered = float(((done >= t_a) & (done <= t_b)).sum()) / (t_b - t_a) if t_b > t_a else float("inf")
        inside = (arr >= t_a) & (arr <= t_b)
        lat = self.latency_s[inside]
        return (delivered, float(np.percentile(lat, 50) * 1e3) if len(lat) else 0.0,
                float(np.percentile(lat, 99) * 1e3) if len(lat) else 0.0)

    def steady_docs_per_s(self, lo: float = 0.1, hi: float = 0.9) -> float:
        """Completions per second between the lo and hi quantiles of the
        completion times: the service rate with the start-up and the drain
        of the last (longest) requests left out."""
        done = np.sort(self.completion_s)
        if len(done) < 10:
            return self.docs_per_s
        a, b = int(lo * len(done)), int(hi * len(done)) - 1
        span = done[b] - done[a]
        return (b - a) / span if span > 0 else float("inf")


def serve(backend, requests: Sequence[np.ndarray], arrivals: Optional[Sequence[float]] = None,
          draws: int = 2048, clock: Callable[[], float] = time.perf_counter,
          sleep: Callable[[float], None] = time.sleep, max_poll: int = 4096,
          pipelined: bool = True) -> ServeReport:
    """Serve requests[i] arriving at arrivals[i] seconds (None: all at 0).

    Request ids are the indices into `requests`.  Admission is first come,
    first served: a request that does not fit waits (and blocks those behind
    it) until a poll frees a slot and arena space.  pipelined: each step's
    poll collects the previous step's finished requests (backend.poll with
    previous=True) while the step runs; otherwise it waits for the step.
    """
    n = len(requests)
    arr = np.zeros(n) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    if n and np.any(np.diff(arr) < 0):
        raise ValueError("arrivals must be non-decreasing")
    t0 = clock()
    lat = np.zeros(n)
    results: Dict[int, dict] = {}
    pending: deque = deque()
    nxt = 0
    rep = ServeReport(results, lat, 0.0, completion_s=np.zeros(n))
    while len(results) < n:
        now = clock() - t0
        while nxt < n and arr[nxt] <= now:
            pending.append(nxt)
            nxt += 1
        while pending:
            rid = pending[0]
            if not backend.submit(rid, requests[rid]):
                rep.admission_waits += 1
                break
            rep.order_admitted.append(rid)
            pending.popleft()
        occ = backend.occupancy()
        rep.max_resident = max(rep.max_resident, occ["resident"])
        if occ["resident"] == 0:
            if pending:
                raise RuntimeError(f"request {pending[0]} can never be admitted (larger than the arena?)")
            if nxt < n:
                sleep(max(0.0, min(arr[nxt] - (clock() - t0), 0.001)))
            continue
        backend.step(draws)
        rep.steps += 1
        for r in (backend.poll(cap=max_poll, previous=True) if pipelined else backend.poll(cap=max_poll)):
            rid = r["request_id"]
            now = clock() - t0
            rep.completion_s[rid] = now
            lat[rid] = now - arr[rid]
            results[rid] = r
    rep.wall_s = clock() - t0
    return rep


def serve_plain(backend, requests: Sequence[np.ndarray], arrivals: Optional[Sequence[float]] = None,
                clock: Callable[[], float] = time.perf_counter,
                sleep: Callable[[float], None] = time.sleep) -> ServeReport:
    """The plain per-document sampler: one request at a time, all sweeps in
    one launch, in arrival order."""
    n = len(requests)
    arr = np.zeros(n) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    t0 = clock()
    lat = np.zeros(n)
    results: Dict[int, dict] = {}
    for rid in range(n):
        now = clock() - t0
        if arr[rid] > now:
            sleep(arr[rid] - now)
        results[rid] = backend.run_one(rid, requests[rid])
        lat[rid] = clock() - t0 - arr[rid]
    return ServeReport(results, lat, clock() - t0, steps=n)


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Open-loop arrival times of a Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
