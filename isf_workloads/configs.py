"""Workload definitions: seeds, film shapes, field ramps and temperature schedules.

Field values are carried as integers ``h_num`` with H = h_num / 20, so every
field the workloads use (multiples of 0.05) is exact.  Ramps go from +H down
to -H inclusive and back up, without repeating the turning point.

Seeds are fixed choices of this project (the paper gives none).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .heightmap import height_map

INIT_UP = 0
INIT_DOWN = 1
INIT_RANDOM = 2


def ramp_hnum(h_max_num: int, step_num: int) -> List[int]:
    """Field-reversal ramp +h_max -> -h_max -> +h_max in steps of ``step_num`` (units of 1/20)."""
    if h_max_num < 0 or step_num <= 0 or h_max_num % step_num:
        raise ValueError("ramp_hnum: h_max_num must be a non-negative multiple of step_num")
    down = list(range(h_max_num, -h_max_num - 1, -step_num))
    up = list(range(-h_max_num + step_num, h_max_num + 1, step_num))
    return down + up


def tscan_temperatures(t_hi: float, t_lo: float, step: float) -> List[float]:
    n = int(round((t_hi - t_lo) / step)) + 1
    return [t_hi - step * i for i in range(n)]


@dataclass
class PlainConfig:
    name: str
    X: int
    Y: int
    Z: int
    sigma: float
    height_seed: int
    mc_seed: int
    init: int
    # hysteresis: fixed T, list of h_num, sweeps per step
    T: Optional[float] = None
    h_nums: Optional[List[int]] = None
    sweeps_per_step: int = 0
    # temperature scan: list of T at H = 0, sweeps per T, discarded sweeps per T
    temps: Optional[List[float]] = None
    sweeps_per_T: int = 0
    discard_per_T: int = 0
    replica: int = 0

    def heights(self) -> np.ndarray:
        return height_map(self.X, self.Y, self.Z, self.sigma, self.height_seed)

    @property
    def n_sweeps(self) -> int:
        if self.h_nums is not None:
            return len(self.h_nums) * self.sweeps_per_step
        return len(self.temps) * self.sweeps_per_T


def config_plain_hysteresis_small() -> PlainConfig:
    """64x64x3 film, sigma 4 px, T = 3.0, H: +4 -> -4 -> +4 step 0.1, 100 sweeps per step."""
    return PlainConfig(
        name="plain_hysteresis_64x64x3",
        X=64, Y=64, Z=3, sigma=4.0, height_seed=1, mc_seed=101, init=INIT_UP,
        T=3.0, h_nums=ramp_hnum(80, 2), sweeps_per_step=100,
    )


def config_plain_tscan() -> PlainConfig:
    """512x512x5 film, sigma 8 px, H = 0, T 12.0 -> 1.0 step 0.25, 1000 sweeps per T (200 discarded)."""
    return PlainConfig(
        name="plain_tscan_512x512x5",
        X=512, Y=512, Z=5, sigma=8.0, height_seed=2, mc_seed=102, init=INIT_RANDOM,
        temps=tscan_temperatures(12.0, 1.0, 0.25), sweeps_per_T=1000, discard_per_T=200,
    )


def config_plain_hysteresis_large() -> PlainConfig:
    """2048x2048x8 film, sigma 16 px, T = 4.0, H: +6 -> -6 -> +6 step 0.05, 50 sweeps per step."""
    return PlainConfig(
        name="plain_hysteresis_2048x2048x8",
        X=2048, Y=2048, Z=8, sigma=16.0, height_seed=3, mc_seed=103, init=INIT_UP,
        T=4.0, h_nums=ramp_hnum(120, 1), sweeps_per_step=50,
    )


def _side_loguniform(rng: np.random.Generator, lo: int, hi: int) -> int:
    side = math.exp(rng.uniform(math.log(lo), math.log(hi)))
    return max(8, int(round(side / 8.0)) * 8)


@dataclass
class BatchedReplica:
    replica: int          # Philox replica index r = 16 f + j
    film: int             # film index f
    X: int
    Y: int
    Z: int
    sigma: float
    T: float
    height_seed: tuple
    heights_cache: Optional[np.ndarray] = field(default=None, repr=False)

    def heights(self) -> np.ndarray:
        if self.heights_cache is None:
            self.heights_cache = height_map(self.X, self.Y, self.Z, self.sigma, self.height_seed)
        return self.heights_cache


def batched_films(base_seed: int = 4, n_films: int = 16, n_temps: int = 16,
                  side_lo: int = 128, side_hi: int = 1024,
                  layers_lo: int = 2, layers_hi: int = 8):
    """Batched workload: ``n_films`` uneven films x ``n_temps`` shared temperatures.

    Returns (replicas, mc_seed, h_nums, sweeps_per_step).  All replicas start
    from all +1 and run the ramp +5 -> -5 -> +5 in steps of 0.1 with 20
    sweeps per step.  Films share one height map per film index; replica
    ``r = n_temps * f + j`` runs film f at temperature j.
    """
    rng = np.random.default_rng([base_seed, 0])
    films = []
    for f in range(n_films):
        side = _side_loguniform(rng, side_lo, side_hi)
        L = int(rng.integers(layers_lo, layers_hi + 1))
        sig = float(rng.uniform(2.0, 16.0))
        films.append((side, L, sig))
    temps = [float(t) for t in rng.uniform(1.0, 10.0, size=n_temps)]
    reps = []
    for f, (side, L, sig) in enumerate(films):
        for j, T in enumerate(temps):
            reps.append(BatchedReplica(replica=n_temps * f + j, film=f, X=side, Y=side, Z=L,
                                       sigma=sig, T=T, height_seed=(base_seed, f)))
    # replicas of one film share the height map
    cache = {}
    for r in reps:
        if r.film not in cache:
            cache[r.film] = r.heights()
        r.heights_cache = cache[r.film]
    return reps, base_seed, ramp_hnum(100, 2), 20


@dataclass
class ServeRequest:
    rid: int
    arrival: float        # seconds after the start of the run
    seed: int             # height-map seed and Monte Carlo key
    X: int
    Y: int
    Z: int
    sigma: float
    T: float
    kind: str             # "hysteresis" or "tscan"
    h_nums: Optional[List[int]] = None
    sweeps_per_step: int = 0
    temps: Optional[List[float]] = None
    sweeps_per_T: int = 0
    discard_per_T: int = 0

    def heights(self) -> np.ndarray:
        return height_map(self.X, self.Y, self.Z, self.sigma, self.seed)

    @property
    def init(self) -> int:
        return INIT_UP if self.kind == "hysteresis" else INIT_RANDOM

    @property
    def n_sweeps(self) -> int:
        if self.kind == "hysteresis":
            return len(self.h_nums) * self.sweeps_per_step
        return len(self.temps) * self.sweeps_per_T


def serving_requests(base_seed: int = 5, rate: float = 50.0, duration: float = 60.0,
                     side_lo: int = 64, side_hi: int = 2048,
                     layers_lo: int = 1, layers_hi: int = 10,
                     max_requests: Optional[int] = None) -> List[ServeRequest]:
    """Poisson arrivals at ``rate`` req/s over ``duration`` s with per-request films and jobs.

    Hysteresis jobs ramp +5 -> -5 -> +5 in steps of 0.1 with 10..100 sweeps
    per step; T-scan jobs visit 20 temperatures from 10.0 down to the
    request's T with 500 sweeps each (the first 100 of each discarded).
    """
    rng = np.random.default_rng([base_seed, 1])
    reqs: List[ServeRequest] = []
    t = 0.0
    rid = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        side = _side_loguniform(rng, side_lo, side_hi)
        L = int(rng.integers(layers_lo, layers_hi + 1))
        sig = float(rng.uniform(2.0, 16.0))
        T = float(rng.uniform(1.0, 9.0))
        kind = "hysteresis" if rng.random() < 0.5 else "tscan"
        seed = int(rng.integers(1, 2**62))
        spst = int(rng.integers(10, 101))
        req = ServeRequest(rid=rid, arrival=t, seed=seed, X=side, Y=side, Z=L, sigma=sig, T=T, kind=kind)
        if kind == "hysteresis":
            req.h_nums = ramp_hnum(100, 2)
            req.sweeps_per_step = spst
        else:
            req.temps = [float(v) for v in np.linspace(10.0, T, 20)]
            req.sweeps_per_T = 500
            req.discard_per_T = 100
        reqs.append(req)
        rid += 1
        if max_requests is not None and rid >= max_requests:
            break
    return reqs
