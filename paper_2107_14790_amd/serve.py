"""Serving loop for block solves: continuous batching under a memory budget.

Blocks (octree leaves, Sec. 4.3-4.5) arrive as requests.  The server keeps
every admitted block's state resident in HBM and advances all active blocks
together, a few iterations per tick, with one batched solve call (one
persistent launch per iteration, or pair of iterations, over all their
tiles).  Between ticks it retires finished blocks (freeing their memory)
and admits waiting ones in arrival order as the memory budget allows; the
histograms of newly admitted blocks are built on a side stream while the
current tick runs on the device.  Ticks are issued ahead: the host queues
the next tick while the device still runs the current one (at most `depth`
ticks in flight) and learns that a tick has ended from an event, so the
device does not wait for the host between ticks.  Because a solve resumed
from its state is bit-identical to an uninterrupted one, and a batched
solve is bit-identical to a solo one, a served block's result does not
depend on what else was in flight.

The scheduling logic talks to a backend (GPU backend below; tests use a
host-only fake), so it is testable without a GPU.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    grid: object            # anything with origin, h, n, halo
    arrival: float          # seconds since the start of the run
    iters: int = 500
    cancelled: bool = False


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    ok: bool = True
    error: str = ""
    output: object = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class _Job:
    req: Request
    handle: object
    nbytes: int
    remaining: int
    result: Result


class Server:
    """Continuous-batching server.

    backend must provide: nbytes(grid) -> int, prepare(request) -> handle
    (may raise), step(handles, k) -> None (queue k iterations; returns before
    the device finishes), finish(handle) -> output (queued after the steps),
    release(handle) (the handle's memory may be reused by work queued later),
    mark() -> token (marks the work queued so far) and done(token) -> bool.
    """

    def __init__(self, backend, budget_bytes: int, tick_iters: int = 50, max_active: int = 1 << 30,
                 clock: Callable[[], float] = None, sleep: Callable[[float], None] = None, depth: int = 2,
                 poll_s: float = 1e-4):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.tick_iters = int(tick_iters)
        self.max_active = int(max_active)
        self.depth = max(1, int(depth))
        self.poll_s = float(poll_s)
        self._clock = clock or time.perf_counter
        self._sleep = sleep or time.sleep
        self.used = 0
        self.peak_used = 0
        self.ticks = 0
        self.max_active_seen = 0

    def run(self, requests: List[Request]) -> List[Result]:
        reqs = sorted(requests, key=lambda r: r.arrival)
        results = {r.rid: Result(r.rid, r.arrival) for r in reqs}
        t0 = self._clock()
        now = lambda: self._clock() - t0  # noqa: E731
        nxt = 0                      # next request not yet arrived
        pending: deque = deque()     # arrived, waiting for admission
        active: List[_Job] = []

        def admit():
            while pending and len(active) < self.max_active:
                r = pending[0]
                if r.cancelled:
                    pending.popleft()
                    results[r.rid].ok = False
                    results[r.rid].error = "cancelled"
                    results[r.rid].finished = now()
                    continue
                try:
                    nb = int(self.backend.nbytes(r.grid))
                except Exception as e:  # invalid block: fail the request, keep serving
                    pending.popleft()
                    results[r.rid].ok = False
                    results[r.rid].error = f"invalid block: {e}"
                    results[r.rid].finished = now()
                    continue
                if nb > self.budget:
                    pending.popleft()
                    results[r.rid].ok = False
                    results[r.rid].error = f"block needs {nb} bytes > budget {self.budget}"
                    results[r.rid].finished = now()
                    continue
                if self.used + nb > self.budget:
                    break  # wait for memory to free up (FIFO: no overtaking)
                pending.popleft()
                try:
                    h = self.backend.prepare(r)
                except Exception as e:
                    results[r.rid].ok = False
                    results[r.rid].error = f"prepare failed: {e}"
                    results[r.rid].finished = now()
                    continue
                self.used += nb
                self.peak_used = max(self.peak_used, self.used)
                results[r.rid].admitted = now()
                if r.iters <= 0:
                    results[r.rid].output = self.backend.finish(h)
                    results[r.rid].finished = now()
                    self.backend.release(h)
                    self.used -= nb
                    continue
                active.append(_Job(r, h, nb, r.iters, results[r.rid]))

        def arrivals():
            nonlocal nxt
            t = now()
            while nxt < len(reqs) and reqs[nxt].arrival <= t:
                pending.append(reqs[nxt])
                nxt += 1

        # ticks queued on the device and not yet seen to end: (token, jobs
        # whose last iterations they hold)
        inflight: deque = deque()

        def retire_done(block: bool):
            """Stamp the jobs of the ticks that have ended; with block, wait
            (taking arrivals meanwhile) until the oldest has ended."""
            while inflight:
                tok, jobs = inflight[0]
                if not self.backend.done(tok):
                    if not block:
                        return
                    arrivals()
                    admit()
                    self._sleep(self.poll_s)
                    continue
                inflight.popleft()
                t = now()
                for j in jobs:
                    j.result.finished = t
                block = False

        while True:
            arrivals()
            admit()
            retire_done(False)
            # cancelled active jobs leave at the tick boundary
            for j in [j for j in active if j.req.cancelled]:
                active.remove(j)
                self.backend.release(j.handle)
                self.used -= j.nbytes
                j.result.ok = False
                j.result.error = "cancelled"
                j.result.finished = now()
            if not active:
                if inflight:
                    retire_done(True)
                    continue
                if nxt >= len(reqs) and not pending:
                    break
                if pending and nxt >= len(reqs) and self.used == 0:
                    # nothing can ever free memory for the head request
                    r = pending.popleft()
                    results[r.rid].ok = False
                    results[r.rid].error = "cannot be admitted"
                    results[r.rid].finished = now()
                    continue
                if nxt < len(reqs):
                    self._sleep(max(0.0, min(reqs[nxt].arrival - now(), 0.01)))
                continue
            running = list(active)
            k = min(self.tick_iters, min(j.remaining for j in running))
            self.max_active_seen = max(self.max_active_seen, len(running))
            try:
                self.backend.step([j.handle for j in running], k)
            except Exception as e:
                # the whole tick failed: fail its blocks, keep the server alive
                for j in running:
                    self.backend.release(j.handle)
                    self.used -= j.nbytes
                    j.result.ok = False
                    j.result.error = f"step failed: {e}"
                    j.result.finished = now()
                active = [j for j in active if j not in running]
                continue
            self.ticks += 1
            # the iteration counts are known on the host: blocks whose last
            # iterations this tick holds are finished and released now (their
            # results and memory reuse are ordered after the tick on the
            # device); they count as done when the tick is seen to end
            ran = set(id(j) for j in running)
            keep, ended = [], []
            for j in active:
                if id(j) in ran:
                    j.remaining -= k
                if j.remaining <= 0:
                    j.result.output = self.backend.finish(j.handle)
                    self.backend.release(j.handle)
                    self.used -= j.nbytes
                    ended.append(j)
                else:
                    keep.append(j)
            active = keep
            inflight.append((self.backend.mark(), ended))
            # while the device works: take in and prepare new arrivals (they
            # join the next tick); wait only when `depth` ticks are queued
            arrivals()
            admit()
            retire_done(len(inflight) >= self.depth)
        retire_done(True)
        while inflight:
            retire_done(True)
        return [results[r.rid] for r in reqs]


def latency_stats(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results if r.ok])
    if lat.size == 0:
        return {"n_ok": 0, "n_failed": len(results)}
    return {"n_ok": int(lat.size), "n_failed": int(sum(1 for r in results if not r.ok)),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}


class GpuBackend:
    """Backend running block solves through libtgv.

    prepare() builds the block's histograms from resident pyramids and
    initialises its state on a side stream (overlapping the tick in flight
    on the main stream); step() issues one batched solve of k iterations of
    all given blocks on the main stream after waiting for their preparation
    and leaves the states open (the last iteration's primal half pending),
    so the next tick's first pass completes it fused with its own first
    dual half and a tick has no per-block opening or closing kernels;
    finish() closes the state and exports u; states live in torch-allocated
    memory, so retiring a block never synchronises the device."""

    def __init__(self, ctx, pyr, W: int, H: int, cams, bins=None, params=None, tile_z_of=None, keep_outputs=True):
        import torch
        import paper_2107_14790_amd as tgv
        self.torch = torch
        self.tgv = tgv
        self.ctx = ctx
        self.pyr = pyr
        self.W, self.H = W, H
        self.cams = tgv.cameras_from(cams)
        self.bins = bins or tgv.Bins()
        self.params = params or tgv.Params()
        self.tile_z_of = tile_z_of
        self.keep_outputs = keep_outputs
        self.main = torch.cuda.current_stream()
        self.side = torch.cuda.Stream()  # default priority

    def nbytes(self, grid) -> int:
        g = self.tgv.grid_from(grid)
        sb = self.tgv.state_bytes(g, self.params.storage)
        if sb < 0:
            raise ValueError(f"invalid grid {g.nx}x{g.ny}x{g.nz} halo {g.halo}")
        n = g.nx * g.ny * g.nz
        return sb + 16 * n + 4 * n

    def prepare(self, req):
        torch, tgv = self.torch, self.tgv
        g = tgv.grid_from(req.grid)
        n = g.nx * g.ny * g.nz
        with torch.cuda.stream(self.side):
            mem = torch.empty(tgv.state_bytes(g, self.params.storage) + 256, dtype=torch.uint8, device="cuda")
            off = (-mem.data_ptr()) % 256
            mem = mem[off:]
            hist = torch.empty((n, 8), dtype=torch.int16, device="cuda")
            self.ctx.build_histograms(self.pyr, self.W, self.H, self.cams, g, self.bins, out=hist, stream=self.side)
            u0 = torch.zeros(n, dtype=torch.float32, device="cuda")
            st = tgv.State(self.ctx, g, self.params.storage, memory=mem)
            st.reset(u0, stream=self.side)
            ev = torch.cuda.Event()
            ev.record(self.side)
        for t in (mem, hist, u0):
            t.record_stream(self.main)
        tz = self.tile_z_of(g) if self.tile_z_of else 0
        return {"state": st, "hist": hist, "u0": u0, "event": ev, "tile_z": tz, "grid": g}

    def step(self, handles, k: int):
        for h in handles:
            if h["event"] is not None:
                self.main.wait_event(h["event"])
                h["event"] = None
        p = dataclasses.replace(self.params, iters=int(k), flags=self.params.flags | self.tgv.FLAG_LEAVE_OPEN)
        self.ctx.solve_batch([h["state"] for h in handles], [h["hist"] for h in handles], p, self.bins,
                             tile_z=[h["tile_z"] or 32 for h in handles], stream=self.main)

    def mark(self):
        ev = self.torch.cuda.Event()
        ev.record(self.main)
        return ev

    def done(self, token) -> bool:
        return token is None or token.query()

    def finish(self, h):
        """Close the state (its last primal half) and export u; with
        keep_outputs False a float64 checksum of u (a device scalar)."""
        p = dataclasses.replace(self.params, iters=0)
        self.ctx.solve(h["grid"], h["hist"], None, p, self.bins, state=h["state"], stream=self.main)
        u = h["state"].export(stream=self.main, fields=("u",))["u"]
        if self.keep_outputs:
            return u
        with self.torch.cuda.stream(self.main):
            return u.double().sum()

    def release(self, h):
        h["state"].close()
        h["state"] = None
        h["hist"] = None
        h["u0"] = None


def poisson_arrivals(rate: float, count: int, seed: int = 5) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: exponential gaps of mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
