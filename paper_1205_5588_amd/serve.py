"""Serving loop: continuous batching of hysteresis and temperature-scan jobs.

Requests arrive over time, each with its own film (height map), seed,
temperature and schedule.  The server admits a waiting request as soon as a
slot is free and its device footprint (spin buffer + state buffer) fits the
memory budget, keeps every admitted film resident on the device, and
advances all admitted films together in chunks of sweeps (one batched launch
per sublattice, or one persistent launch per chunk).  While a chunk runs on
the GPU the host admits newly arrived requests (their films are built on
their own streams, so that work overlaps the chunk); after the chunk, films
whose schedules are finished are retired, their records read back and their
memory returned.  Latency is measured from arrival to retirement.

Because every random draw is keyed by (seed, replica, sweep, sublattice,
site), a request's result does not depend on what else is in the batch or on
the chunk boundaries: alone and in the mix give the same records bit for bit.

The scheduler is independent of the executor, so it can be driven on the CPU
with a fake executor and a fake clock.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Protocol, Sequence

import numpy as np


@dataclass
class Job:
    """What the server needs to know about a request."""
    rid: int
    arrival: float
    footprint: int            # device bytes while resident
    n_sweeps: int             # total sweeps of its schedule
    attempts: int = 0         # occupied sites x sweeps (filled in on admission)
    payload: object = None    # the request itself (handed to the executor)


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    records: np.ndarray
    attempts: int

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Executor(Protocol):
    def create(self, job: Job) -> object: ...
    def advance(self, handles: Sequence[object], max_sweeps: int) -> int: ...
    def wait(self) -> None: ...
    def remaining(self, handle: object) -> int: ...
    def records(self, handle: object) -> np.ndarray: ...
    def release(self, handle: object) -> None: ...
    def attempts_per_sweep(self, handle: object) -> int: ...


class Clock:
    """Wall clock; a fake clock with the same interface drives CPU tests."""

    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep_until(self, t: float) -> None:
        dt = t - self.now()
        if dt > 0:
            time.sleep(min(dt, 0.01))


@dataclass
class ServerStats:
    results: List[Result] = field(default_factory=list)
    max_active: int = 0
    max_bytes: int = 0
    chunks: int = 0
    refused_for_memory: int = 0   # admission attempts deferred because the budget was full

    def summary(self) -> dict:
        if not self.results:
            return {"requests": 0}
        lat = np.array([r.latency for r in self.results])
        t_first = min(r.arrival for r in self.results)
        t_last = max(r.finished for r in self.results)
        att = sum(r.attempts for r in self.results)
        # accepted flips in the records' kept sweeps (a T-scan step's discarded
        # sweeps are not counted)
        acc = sum(int(np.asarray(r.records)[:, 5].sum()) for r in self.results if len(r.records))
        return {
            "requests": len(self.results),
            "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()),
            "max_s": float(lat.max()),
            "attempts": int(att),
            "span_s": float(t_last - t_first),
            "attempts_per_s": float(att / max(t_last - t_first, 1e-9)),
            "accepted_kept": int(acc),
            "accepted_kept_per_s": float(acc / max(t_last - t_first, 1e-9)),
            "max_active": self.max_active,
            "max_bytes": self.max_bytes,
            "chunks": self.chunks,
        }


class Server:
    def __init__(self, executor: Executor, budget_bytes: int, max_slots: int, clock: Optional[Clock] = None,
                 target_chunk_s: float = 0.01, rate_estimate: float = 2e11, max_chunk: int = 256):
        if budget_bytes <= 0 or max_slots <= 0:
            raise ValueError("budget and slots must be positive")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.clock = clock or Clock()
        self.target_chunk_s = target_chunk_s
        self.rate = rate_estimate          # attempts/s, refined from measured chunks
        self.max_chunk = max_chunk

    def _chunk(self, active_attempts_per_sweep: int) -> int:
        if active_attempts_per_sweep <= 0:
            return 1
        n = int(self.target_chunk_s * self.rate / active_attempts_per_sweep)
        return max(1, min(self.max_chunk, n))

    def run(self, jobs: Sequence[Job], on_retire: Optional[Callable[[Result], None]] = None) -> ServerStats:
        for j in jobs:
            if j.footprint > self.budget:
                raise ValueError("request %d needs %d bytes, more than the whole budget" % (j.rid, j.footprint))
        waiting = sorted(jobs, key=lambda j: (j.arrival, j.rid))
        state = {"wi": 0, "used": 0}
        active: Dict[int, tuple] = {}   # rid -> (job, handle, admitted)
        stats = ServerStats()

        def admit() -> None:
            # arrived requests in arrival order, while a slot and the memory budget allow
            now = self.clock.now()
            while (state["wi"] < len(waiting) and waiting[state["wi"]].arrival <= now
                   and len(active) < self.max_slots):
                j = waiting[state["wi"]]
                if state["used"] + j.footprint > self.budget:
                    stats.refused_for_memory += 1
                    break
                h = self.ex.create(j)
                j.attempts = self.ex.attempts_per_sweep(h) * j.n_sweeps
                active[j.rid] = (j, h, self.clock.now())
                state["used"] += j.footprint
                state["wi"] += 1
            stats.max_active = max(stats.max_active, len(active))
            stats.max_bytes = max(stats.max_bytes, state["used"])

        while state["wi"] < len(waiting) or active:
            admit()
            if not active:
                if state["wi"] < len(waiting):
                    self.clock.sleep_until(waiting[state["wi"]].arrival)
                continue
            handles = [v[1] for v in active.values()]
            per_sweep = sum(self.ex.attempts_per_sweep(h) for h in handles if self.ex.remaining(h) > 0)
            chunk = self._chunk(per_sweep)
            t0 = self.clock.now()
            self.ex.advance(handles, chunk)
            admit()            # films of new arrivals are built while the chunk runs
            self.ex.wait()
            dt = self.clock.now() - t0
            stats.chunks += 1
            if dt > 0 and per_sweep > 0:
                # exponential average of the measured throughput sets the next chunk
                self.rate = 0.7 * self.rate + 0.3 * (per_sweep * chunk / dt)
            # retirement
            for rid in [r for r, v in active.items() if self.ex.remaining(v[1]) == 0]:
                j, h, adm = active.pop(rid)
                recs = self.ex.records(h)
                res = Result(rid, j.arrival, adm, self.clock.now(), recs, j.attempts)
                self.ex.release(h)
                state["used"] -= j.footprint
                stats.results.append(res)
                if on_retire:
                    on_retire(res)
        stats.results.sort(key=lambda r: r.rid)
        return stats


# --------------------------------------------------------------------------- GPU executor
def request_schedule(req) -> list:
    """(T, h_num, n_sweeps, n_discard) steps of a hysteresis or temperature-scan request."""
    if req.kind == "hysteresis":
        return [(req.T, h, req.sweeps_per_step, 0) for h in req.h_nums]
    return [(T, 0, req.sweeps_per_T, req.discard_per_T) for T in req.temps]


class GpuExecutor:
    """Runs admitted requests as resident films advanced by the batched kernels."""

    def __init__(self, max_slots: int, mode: int, tiling=None, fmt: int = 0, heights_of=None):
        import torch

        from .lattice import Batch

        self.batch = Batch(max_slots)
        self.mode = mode
        self.tiling = tiling
        self.fmt = fmt
        self.heights_of = heights_of or (lambda req: req.heights())
        self.torch = torch

    @staticmethod
    def footprint(req, fmt: int = 0) -> int:
        from .lattice import lattice_bytes

        s, a = lattice_bytes(req.X, req.Y, req.Z, fmt)
        return s + a

    def create(self, job: Job):
        from .lattice import Lattice

        req = job.payload
        lat = Lattice(self.heights_of(req), req.Z, req.seed, replica=0, init=req.init, fmt=self.fmt)
        if self.tiling:
            lat.set_tuning(*self.tiling)
        lat.schedule_load(request_schedule(req))
        lat._n_occ = lat.observables()["n_occ"]
        return lat

    def advance(self, handles, max_sweeps: int) -> int:
        return self.batch.advance(handles, max_sweeps, self.mode)

    def wait(self) -> None:
        self.batch.sync()

    def remaining(self, lat) -> int:
        return lat.remaining()

    def records(self, lat) -> np.ndarray:
        return lat.records()

    def release(self, lat) -> None:
        lat.close()

    def attempts_per_sweep(self, lat) -> int:
        return lat._n_occ
