"""The serving scheduler on the CPU: a fake executor runs the oracle, a fake
clock advances with the work done.  Checks admission by memory footprint,
continuous admission while others run, slot limits, retirement, latency
statistics, refusal of oversize requests, and that every result is the same
alone and in the mix."""

import numpy as np
import pytest

from oracle import cpu
from paper_1205_5588_amd.serve import Job, Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


class FakeExecutor:
    """Oracle films advanced sweep by sweep; simulated time grows with the work."""

    def __init__(self, clock, rate=1e6):
        self.clock = clock
        self.rate = rate
        self.created = []

    def create(self, job):
        req = job.payload
        f = cpu.Film(req["h"], req["Z"], req["seed"], 0, init=req["init"])
        st = {"film": f, "steps": list(req["steps"]), "i": 0, "done_in_step": 0, "acc": None, "recs": [],
              "left": sum(s[2] for s in req["steps"]), "rid": job.rid}
        self.created.append((job.rid, self.clock.now()))
        return st

    def _advance_one(self, st, n):
        while n > 0 and st["i"] < len(st["steps"]):
            T, h, ns, nd = st["steps"][st["i"]]
            a = st["done_in_step"]
            b = min(ns, a + n)
            disc = max(0, min(nd, b) - a)
            r = st["film"].run(T, h, b - a, disc)
            acc = st["acc"] or [0, 0, 0, 0]
            acc = [acc[0] + r.sum_M, acc[1] + r.sum_absM, acc[2] + r.sum_E, acc[3] + r.accepted]
            st["acc"] = acc
            n -= b - a
            st["left"] -= b - a
            st["done_in_step"] = b
            if b == ns:
                st["recs"].append([r.M, r.E] + acc)
                st["i"] += 1
                st["done_in_step"] = 0
                st["acc"] = None

    def advance(self, handles, max_sweeps):
        work = 0
        for st in handles:
            k = min(max_sweeps, st["left"])
            work += k * st["film"].state()[2]
            self._advance_one(st, k)
        self.clock.t += work / self.rate
        return max_sweeps

    def wait(self):
        pass

    def remaining(self, st):
        return st["left"]

    def records(self, st):
        return np.array(st["recs"], dtype=np.int64)

    def release(self, st):
        st["film"] = None

    def attempts_per_sweep(self, st):
        return st["film"].state()[2] if st["film"] is not None else 0


def _jobs(n=8, seed=0):
    rng = np.random.default_rng(seed)
    jobs = []
    t = 0.0
    for i in range(n):
        t += float(rng.exponential(0.02))
        Y, X, Z = int(rng.choice([8, 12, 16])), int(rng.choice([8, 16, 24])), int(rng.integers(1, 4))
        h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
        if rng.random() < 0.5:
            steps = [(2.5, int(v), int(rng.integers(3, 9)), 0) for v in (60, 20, -20, -60, 0)]
            init = 0
        else:
            steps = [(float(T), 0, 10, 3) for T in np.linspace(8.0, 2.0, 4)]
            init = 2
        payload = {"h": h, "Z": Z, "seed": int(rng.integers(1, 2**40)), "steps": steps, "init": init}
        jobs.append(Job(rid=i, arrival=t, footprint=X * Y * Z, n_sweeps=sum(s[2] for s in steps), payload=payload))
    return jobs


def _alone(payload):
    f = cpu.Film(payload["h"], payload["Z"], payload["seed"], 0, init=payload["init"])
    return np.array([f.run(*s).as_tuple() for s in payload["steps"]], dtype=np.int64)


def test_results_same_alone_and_in_mix(oracle_lib):
    clock = FakeClock()
    jobs = _jobs()
    srv = Server(FakeExecutor(clock, rate=2e5), budget_bytes=10**9, max_slots=4, clock=clock,
                 target_chunk_s=0.002, rate_estimate=2e5)
    stats = srv.run(jobs)
    assert len(stats.results) == len(jobs)
    for j, r in zip(sorted(jobs, key=lambda j: j.rid), stats.results):
        assert r.rid == j.rid
        np.testing.assert_array_equal(r.records, _alone(j.payload))
        assert r.finished >= r.admitted >= r.arrival
    assert stats.chunks > len(jobs)   # work really was interleaved in chunks


def test_admission_by_footprint_and_slots(oracle_lib):
    clock = FakeClock()
    jobs = _jobs(10, seed=1)
    budget = sorted(j.footprint for j in jobs)[-1] + sorted(j.footprint for j in jobs)[-2]
    srv = Server(FakeExecutor(clock, rate=1e5), budget_bytes=budget, max_slots=3, clock=clock,
                 target_chunk_s=0.001, rate_estimate=1e5)
    stats = srv.run(jobs)
    assert len(stats.results) == len(jobs)
    assert stats.max_bytes <= budget
    assert stats.max_active <= 3
    for j, r in zip(sorted(jobs, key=lambda j: j.rid), stats.results):
        np.testing.assert_array_equal(r.records, _alone(j.payload))


def test_continuous_admission(oracle_lib):
    """A request that arrives while others run is admitted before they finish."""
    clock = FakeClock()
    jobs = _jobs(6, seed=2)
    for k, j in enumerate(jobs):
        j.arrival = 0.001 * k
    srv = Server(FakeExecutor(clock, rate=5e4), budget_bytes=10**9, max_slots=16, clock=clock,
                 target_chunk_s=0.0005, rate_estimate=5e4)
    stats = srv.run(jobs)
    res = {r.rid: r for r in stats.results}
    first_finish = min(r.finished for r in stats.results)
    assert any(r.admitted < first_finish for r in stats.results if r.rid != min(res, key=lambda i: res[i].finished))
    assert stats.max_active >= 2


def test_latency_statistics(oracle_lib):
    clock = FakeClock()
    jobs = _jobs(7, seed=3)
    stats = Server(FakeExecutor(clock), budget_bytes=10**9, max_slots=2, clock=clock).run(jobs)
    s = stats.summary()
    lat = np.array([r.latency for r in stats.results])
    assert s["requests"] == 7
    assert s["p50_s"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_s"] == pytest.approx(np.percentile(lat, 99))
    assert s["attempts"] == sum(r.attempts for r in stats.results)


def test_oversize_request_refused():
    clock = FakeClock()
    jobs = _jobs(2, seed=4)
    with pytest.raises(ValueError):
        Server(FakeExecutor(clock), budget_bytes=min(j.footprint for j in jobs) - 1, max_slots=2,
               clock=clock).run(jobs)
    with pytest.raises(ValueError):
        Server(FakeExecutor(clock), budget_bytes=0, max_slots=2, clock=clock)
