"""Continuous-batching service for Picard-step solve requests.

Each request carries one linearized system (a harness-style Problem: CSR K and
maps on the host, right-hand side b) and solver options.  The server admits a
waiting request as soon as a slot is free and its estimated device footprint
(gdsw_footprint_bytes) fits in the remaining budget; every admitted request
runs gdsw_setup + gdsw_solve on its own HIP stream from a worker thread, so
requests that arrive while others are on the GPU overlap with them on the
device.  The library's kernels take no atomics and no cross-request state,
so each result is the same alone and in the mix.

Latency of a request = completion time - arrival time (host clock).
"""
import collections
import threading
import time

import numpy as np

from . import gdsw
from .metrics import percentile


class Request:
    def __init__(self, rid, problem, arrival=None, **options):
        self.id = rid
        self.problem = problem
        self.options = options
        self.arrival = time.perf_counter() if arrival is None else arrival
        self.t_start = None
        self.t_done = None
        self.x = None
        self.info = None
        self.error = None
        self.footprint = None
        self.oom_retries = 0
        self._done = threading.Event()

    def wait(self, timeout=None):
        self._done.wait(timeout)
        return self

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival


class Server:
    """Admission by footprint and slot count; one worker thread and HIP stream per running request."""

    def __init__(self, budget_bytes=200 * 2 ** 30, max_active=4, device=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.used = 0
        self.active = 0
        self.queue = collections.deque()
        self.lock = threading.Condition()
        self.finished = []
        self.peak_active = 0
        self._footprints = {}
        self._closed = False
        self._scheduler = threading.Thread(target=self._schedule, daemon=True)
        self._scheduler.start()

    def footprint(self, req):
        key = (id(req.problem), tuple(sorted(req.options.items())))
        if key not in self._footprints:
            fp = gdsw.footprint_bytes(req.problem, **req.options)
            if fp == 0:
                raise gdsw.GdswError(gdsw.EINVAL, gdsw.load_library().gdsw_last_error().decode())
            # the request's K, b and x, and the library's private copy of K
            fp += 2 * (12 * len(req.problem.col) + 8 * (req.problem.n + 1)) + 16 * req.problem.n
            self._footprints[key] = fp
        return self._footprints[key]

    def submit(self, req):
        req.footprint = self.footprint(req)
        if req.footprint > self.budget:
            raise ValueError(f"request {req.id} needs {req.footprint} bytes, more than the whole budget")
        with self.lock:
            self.queue.append(req)
            self.lock.notify_all()
        return req

    def _schedule(self):
        while True:
            with self.lock:
                while not self._closed and not self._admissible():
                    self.lock.wait()
                if self._closed and not self.queue:
                    return
                if not self._admissible():
                    continue
                req = self.queue.popleft()
                self.used += req.footprint
                self.active += 1
                self.peak_active = max(self.peak_active, self.active)
            threading.Thread(target=self._run, args=(req,), daemon=True).start()

    def _admissible(self):
        # first come, first served: the head of the queue waits until it fits
        return bool(self.queue) and self.active < self.max_active and \
            self.used + self.queue[0].footprint <= self.budget

    def _run(self, req):
        torch = self.torch
        req.t_start = time.perf_counter()
        try:
            torch.cuda.set_device(self.device)
            stream = torch.cuda.Stream(device=self.device)
            P = req.problem
            with torch.cuda.stream(stream):
                K = (torch.as_tensor(np.asarray(P.rowptr, dtype=np.int64)).to(self.device),
                     torch.as_tensor(np.asarray(P.col, dtype=np.int32)).to(self.device),
                     torch.as_tensor(np.asarray(P.val, dtype=np.float64)).to(self.device))
                b = torch.as_tensor(np.asarray(P.b, dtype=np.float64)).to(self.device)
                ctx = gdsw.Context(P, K=K, stream=stream, **req.options)
                try:
                    x, info = ctx.solve(b, stream=stream)
                    stream.synchronize()
                    req.x = x.cpu().numpy()
                    req.info = info
                finally:
                    ctx.close()
                del K, b
        except Exception as e:          # reported on the request, the server keeps serving
            req.error = e
        retry = False
        with self.lock:
            self.used -= req.footprint
            self.active -= 1
            # out of device memory while others run (their memory, or cached blocks, was not yet
            # free): back to the head of the queue, admitted again when a running request ends;
            # alone on the device it fails for good
            if (isinstance(req.error, gdsw.GdswError) and req.error.code == gdsw.ENOMEM and self.active > 0
                    and req.oom_retries < 8):
                req.oom_retries += 1
                req.error = None
                req.x = req.info = None
                self.queue.appendleft(req)
                retry = True
            else:
                req.t_done = time.perf_counter()
                self.finished.append(req)
            self.lock.notify_all()
        if not retry:
            req._done.set()

    def close(self):
        with self.lock:
            self._closed = True
            self.lock.notify_all()
        self._scheduler.join()

    def drain(self, reqs, timeout=None):
        for r in reqs:
            r.wait(timeout)
        return reqs


def run_stream(server, problems, n_requests, rate_hz, seed=0, **options):
    """Submit n_requests drawn from `problems` with Poisson arrivals at rate_hz; wait for all."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    t = time.perf_counter()
    for k in range(n_requests):
        P = problems[int(rng.integers(0, len(problems)))]
        reqs.append(server.submit(Request(k, P, arrival=time.perf_counter(), **options)))
        t += rng.exponential(1.0 / rate_hz)
        delay = t - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
    server.drain(reqs)
    return reqs


def summarize(reqs, t0, t1):
    lat = [r.latency * 1e3 for r in reqs if r.error is None]
    return {"requests": len(reqs), "failed": sum(r.error is not None for r in reqs),
            "out_of_memory_requeues": sum(r.oom_retries for r in reqs),
            "errors": sorted({str(r.error)[:160] for r in reqs if r.error is not None}),
            "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
            "solves_per_s": len(lat) / (t1 - t0),
            "iterations_mean": float(np.mean([r.info["iterations"] for r in reqs if r.error is None]))}
