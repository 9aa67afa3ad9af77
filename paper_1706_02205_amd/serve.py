"""Serving loop: factor-and-solve requests of uneven size with continuous admission.

Each request carries points (n x d), right-hand sides (n x nrhs) and an arrival
time.  Its life:

1. host analysis (ordering, pattern, schedule: ``kc_analyze``) on a thread pool;
2. admission, in the order the analyses finish, as soon as an in-flight slot is
   free and the device bytes of its factor fit in the budget next to the
   resident factors -- the budget is the nnz(S)-proportional workspace reported
   by ``kc_factor_bytes``.  A request at the head that does not fit may be
   passed by later ones that do, at most ``max_bypass`` times, after which
   admission waits for it (so a large request is delayed boundedly, and small
   ones do not queue behind it meanwhile);
3. factorization and solve enqueued at once on one of several streams, so it
   runs on the device alongside requests admitted earlier (there is no batch
   boundary: a request never waits for others to finish unless the budget or
   the slots are exhausted);
4. completion detected through an event; the solution is copied to the host
   and the factor stays resident (least recently completed evicted first when
   the budget needs room).

Results do not depend on what runs beside a request: every request owns its
workspace and the kernels have a fixed operation order.
"""
from __future__ import annotations

import threading
import time
from collections import OrderedDict, deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import Factor, analyze


@dataclass
class RequestResult:
    rid: int
    n: int
    nnz: int
    arrival: float
    analyzed: float = 0.0
    admitted: float = 0.0
    done: float = 0.0
    solution: Optional[np.ndarray] = None
    bytes: int = 0
    bypassed: int = 0  # times later requests were admitted before this one while it waited at the head

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServeStats:
    results: List[RequestResult]
    wall_s: float
    peak_resident_bytes: int
    peak_inflight: int
    budget_bytes: int

    def percentile_ms(self, q: float) -> float:
        return float(np.percentile([r.latency for r in self.results], q) * 1e3)

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.results])
        nnz = sum(r.nnz for r in self.results)
        return {"requests": len(self.results), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "throughput_req_s": len(self.results) / self.wall_s, "s_entries_per_s": nnz / self.wall_s,
                "wall_s": self.wall_s, "peak_resident_bytes": self.peak_resident_bytes,
                "peak_inflight": self.peak_inflight, "budget_bytes": self.budget_bytes,
                "bypasses": int(sum(r.bypassed for r in self.results)),
                "max_bypassed": int(max(r.bypassed for r in self.results))}


class Server:
    def __init__(self, nu: float, lengthscale: float, rho: float, prec: str = "mixed", budget_bytes: float = 64e9,
                 max_inflight: int = 8, nstreams: int = 4, analysis_threads: int = 8,
                 analysis_nthreads: Optional[int] = None, max_bypass: int = 8,
                 max_analysis_threads: int = 16, points_per_thread: int = 12_500):
        import torch
        self.nu, self.ell, self.rho, self.prec = nu, lengthscale, rho, prec
        self.pivot, self.tau = ("zero", 0.0) if prec == "fp64" else ("shift", 1e-6)
        self.budget = int(budget_bytes)
        # host threads inside one request's analysis; None: by size, one per points_per_thread points (1 to
        # max_analysis_threads), so that the largest requests -- the latency tail -- get the most threads
        self.analysis_nthreads = analysis_nthreads
        self.max_analysis_threads = max_analysis_threads
        self.points_per_thread = points_per_thread
        self.max_inflight = max_inflight
        self.max_bypass = max_bypass
        self._bypassed = 0      # times the current head of the ready queue has been passed
        self._head_rid = None
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.pool = ThreadPoolExecutor(max_workers=analysis_threads)
        self._lock = threading.Lock()
        self._ready: deque = deque()        # analysed, waiting for admission (arrival order)
        self._inflight: List[tuple] = []    # (result, factor, event, x_out, tensors)
        self._resident: "OrderedDict[int, tuple]" = OrderedDict()  # rid -> (factor, bytes)
        self._used = 0
        self._peak_used = 0
        self._peak_inflight = 0
        self._next_stream = 0
        self.results: Dict[int, RequestResult] = {}

    # -- submission ----------------------------------------------------------
    def submit(self, rid: int, points: np.ndarray, b: np.ndarray, arrival: Optional[float] = None):
        res = RequestResult(rid, len(points), 0, arrival if arrival is not None else time.perf_counter())
        self.results[rid] = res

        nth = self.analysis_nthreads or max(1, min(self.max_analysis_threads, len(points) // self.points_per_thread))

        def work():
            plan = analyze(points, self.rho, nthreads=nth)
            res.analyzed = time.perf_counter()
            res.nnz = plan.nnz
            with self._lock:
                self._ready.append((res, plan, points, b))

        return self.pool.submit(work)

    # -- scheduling ------------------------------------------------------------
    def _evict_for(self, need: int) -> bool:
        while self._used + need > self.budget and self._resident:
            _, (f, nbytes) = self._resident.popitem(last=False)
            self._used -= nbytes
            del f
        return self._used + need <= self.budget

    def _need(self, plan, b) -> int:
        from . import _lib
        import ctypes as C
        nb = C.c_size_t()
        _lib.check(_lib.load().kc_factor_bytes(plan.handle, 0 if self.prec == "fp64" else 1, C.byref(nb)),
                   "kc_factor_bytes")
        return int(nb.value) + b.size * 8 * 4  # workspace + points/rhs/solution/scratch

    def _admit(self) -> bool:
        import torch
        with self._lock:
            if not self._ready or len(self._inflight) >= self.max_inflight:
                return False
            head = self._ready[0][0].rid
            if head != self._head_rid:
                self._head_rid, self._bypassed = head, 0
            pick = None
            for q, (res, plan, points, b) in enumerate(self._ready):
                need = self._need(plan, b)
                if need > self.budget:
                    raise RuntimeError(f"request {res.rid} needs {need} bytes, above the whole budget {self.budget}")
                if self._evict_for(need):
                    pick = q
                    break
                if q == 0 and self._bypassed >= self.max_bypass:
                    return False  # the head has waited long enough: nothing passes it
            if pick is None:
                return False
            if pick > 0:
                self._bypassed += 1
                self._ready[0][0].bypassed += 1
            res, plan, points, b = self._ready[pick]
            del self._ready[pick]
        s = self.streams[self._next_stream % len(self.streams)]
        self._next_stream += 1
        with torch.cuda.stream(s):
            f = Factor(plan, self.prec, stream=s)
            xd = torch.from_numpy(points).to("cuda", non_blocking=False)
            bd = torch.from_numpy(np.ascontiguousarray(b)).to("cuda", non_blocking=False)
            f.factorize(xd, self.nu, self.ell, self.pivot, self.tau, stream=s)
            out = f.solve(bd, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        res.admitted = time.perf_counter()
        res.bytes = need
        with self._lock:
            self._used += need
            self._peak_used = max(self._peak_used, self._used)
            self._inflight.append((res, f, ev, out, (xd, bd)))
            self._peak_inflight = max(self._peak_inflight, len(self._inflight))
        return True

    def _reap(self) -> int:
        done = 0
        keep = []
        for item in self._inflight:
            res, f, ev, out, _ = item
            if ev.query():
                res.solution = out.cpu().numpy()
                res.done = time.perf_counter()
                self._resident[res.rid] = (f, res.bytes)  # factor stays on the device
                done += 1
            else:
                keep.append(item)
        with self._lock:
            self._inflight = keep
        return done

    def run(self, requests, time_scale: float = 1.0) -> ServeStats:
        """Replay requests [(arrival_s, points, b)] in real time and serve them."""
        t0 = time.perf_counter()
        futures = []
        pending = deque(enumerate(requests))
        total = len(requests)
        finished = 0
        while finished < total:
            now = time.perf_counter() - t0
            while pending and pending[0][1][0] * time_scale <= now:
                rid, (arr, pts, b) = pending.popleft()
                futures.append(self.submit(rid, pts, b, t0 + arr * time_scale))
            progressed = False
            while self._admit():
                progressed = True
            got = self._reap()
            finished += got
            if not progressed and not got:
                time.sleep(0.0005)
            for fu in futures:
                if fu.done() and fu.exception() is not None:
                    raise fu.exception()
        wall = time.perf_counter() - t0
        return ServeStats([self.results[i] for i in range(total)], wall, self._peak_used, self._peak_inflight,
                          self.budget)

    def close(self):
        self.pool.shutdown(wait=True)
        self._resident.clear()
