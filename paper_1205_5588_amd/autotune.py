"""Autotuner for the sweep kernels' launch shape.

Searches the tile shape (dwords or words along a row x rows across), the
rows handled per thread, graph replay vs plain launches, and for batches the
execution mode (one launch per sublattice vs one persistent launch).  Every
candidate runs the same schedule from the same start; a candidate whose
records or spins differ from the first one is rejected (all shapes must give
the identical trajectory, since draws are keyed by site and sweep only).

Results are cached in JSON keyed by the film shape class.
"""

from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from ._lib import (BATCH_PERSISTENT, BATCH_PHASE_LAUNCH, BATCH_PIPE, BATCH_WHOLE, FORMAT_BITPACK, FORMAT_INT8,
                   KERNEL_FILM, KERNEL_LIST, KERNEL_PIPE, KERNEL_SWEEP, KERNEL_TILES, IsfError)

TILINGS = {
    FORMAT_INT8: [(64, 4, 1), (64, 4, 2), (64, 4, 4), (32, 8, 1), (32, 8, 2), (32, 8, 4), (16, 16, 1), (16, 16, 2),
                  (16, 16, 4)],
    FORMAT_BITPACK: [(64, 4, 1), (64, 4, 2), (32, 8, 1), (32, 8, 2), (16, 16, 1), (16, 16, 2), (8, 32, 1), (8, 32, 2),
                     (8, 16, 1), (8, 8, 1)],
}

GRAPH_SWEEPS = 64  # sweeps per captured graph in the library

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def shape_key(X: int, Y: int, Z: int, fmt: int) -> str:
    return "%s:%dx%dx%d" % ("int8" if fmt == FORMAT_INT8 else "bitpack", X, Y, Z)


def default_tiling(X: int, fmt: int) -> Tuple[int, int, int]:
    """Heuristic sublattice-kernel shape for films not in the cache: widest tile that the row fills."""
    per_row = X // 8 if fmt == FORMAT_INT8 else (X // 2 + 31) // 32
    if per_row >= 64:
        return (64, 4, 2) if fmt == FORMAT_INT8 else (64, 4, 1)
    if per_row >= 32:
        return (32, 8, 2) if fmt == FORMAT_INT8 else (32, 8, 1)
    return (16, 16, 2) if fmt == FORMAT_INT8 else (16, 16, 1)


def film_resident(X: int, Y: int, Z: int) -> bool:
    """True where the film kernel runs in its resident form: no sublattice has more
    dwords than the kernel's 512 threads."""
    return (Z + 1) // 2 * (Y // 2) * (X // 8) <= 512


def default_tuning(X: int, Y: int, Z: int, fmt: int) -> tuple:
    """Heuristic (tile_x, tile_y, rows_or_waves, use_graph, kernel) for films not in the cache.

    Small INT8 films that the film kernel takes in its resident form run there
    (one block, many sweeps per launch: 2.6 us per sweep of 64 x 64 x 3 on
    MI355X, against 9.3 us for one launch per sweep).  Other INT8 films whose
    planes fit a whole-sweep kernel's LDS take one (the pipelined kernel with
    32 x 32 tiles on wide films such as 2048^2 x 8; the single-tile kernel with
    16 x 16 tiles on smaller films, where the pipelined kernel's 32 x 8 tiles
    win on some (512^2 x 5 at T up to 12) and lose on others (the batched
    workload's films, hot replicas among them), so the tuner decides); others
    take the sublattice tiles."""
    if fmt == FORMAT_INT8 and film_resident(X, Y, Z):
        return (512, 1, 1, False, KERNEL_FILM)
    if fmt == FORMAT_INT8 and Z <= 8:
        if X // 8 >= 256 and Y >= 512:
            return (32, 32, 16, True, KERNEL_PIPE)
        return (16, 16, 4, True, KERNEL_SWEEP)
    return default_tiling(X, fmt) + (True, KERNEL_TILES)


class TuningCache:
    def __init__(self, path: str = CACHE_PATH):
        self.path = path
        self.data: Dict[str, dict] = {}
        if os.path.exists(path):
            with open(path) as fh:
                self.data = json.load(fh)

    def get(self, key: str) -> Optional[dict]:
        return self.data.get(key)

    def put(self, key: str, value: dict) -> None:
        self.data[key] = value

    def save(self, path: Optional[str] = None) -> None:
        with open(path or self.path, "w") as fh:
            json.dump(self.data, fh, indent=1, sort_keys=True)


def lookup(X: int, Y: int, Z: int, fmt: int, cache: Optional[TuningCache] = None) -> tuple:
    cache = cache or TuningCache()
    hit = cache.get(shape_key(X, Y, Z, fmt))
    if hit:
        return tuple(hit["tiling"]) + (bool(hit["use_graph"]), int(hit.get("kernel", KERNEL_TILES)))
    return default_tuning(X, Y, Z, fmt)


LIST_CANDIDATES = [(64, 4, 1, KERNEL_LIST), (64, 4, 2, KERNEL_LIST)]
# whole-sweep kernel: (tile dwords, tile rows, waves per block); shapes whose LDS
# does not fit the film's Z are skipped
SWEEP_CANDIDATES = [(32, 16, 8, KERNEL_SWEEP), (16, 16, 4, KERNEL_SWEEP), (32, 8, 4, KERNEL_SWEEP),
                    (64, 8, 8, KERNEL_SWEEP), (32, 32, 8, KERNEL_SWEEP), (32, 32, 16, KERNEL_SWEEP)]
# pipelined whole-sweep kernel (one block per compute unit, double-buffered LDS)
PIPE_CANDIDATES = [(32, 16, 16, KERNEL_PIPE), (32, 16, 8, KERNEL_PIPE), (32, 32, 16, KERNEL_PIPE),
                   (64, 16, 16, KERNEL_PIPE), (32, 8, 8, KERNEL_PIPE)]
# the whole film in one block's LDS, many sweeps per launch (films that fit it)
FILM_CANDIDATES = [(512, 1, 1, KERNEL_FILM)]


def tune_lattice(make: Callable[[], "object"], fmt: int, T: float, h_num: int, sweeps: int = 64,
                 warmup: int = 8, candidates: Optional[Sequence[Tuple[int, ...]]] = None,
                 graphs: Sequence[bool] = (True, False), lists: bool = True) -> dict:
    """Time every launch shape on fresh copies of one film; returns the best and all timings.

    Candidates are (tile_x, tile_y, rows_per_thread[, kernel]); for INT8 films
    the occupied-dword list kernel (lists=True) and the whole-sweep kernel are
    tried too.  Shapes the library rejects for this film are skipped."""
    import torch

    cands = [tuple(c) + ((KERNEL_TILES,) if len(c) == 3 else ()) for c in (candidates or TILINGS[fmt])]
    if fmt == FORMAT_INT8 and candidates is None:
        cands += (LIST_CANDIDATES if lists else []) + SWEEP_CANDIDATES + PIPE_CANDIDATES + FILM_CANDIDATES
    ref_recs = ref_spins = None
    timings: List[dict] = []
    for tl in cands:
        for g in graphs:
            lat = make()
            if tl[3] == KERNEL_LIST:
                lat.attach_items()
            try:
                lat.set_tuning(tl[0], tl[1], tl[2], g, tl[3])
            except IsfError:
                lat.close()
                continue
            # warm up past one graph length (every candidate alike: the same trajectory)
            # so that a graph is built before the timed region
            lat.run_schedule([(T, h_num, warmup + GRAPH_SWEEPS, 0)])
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            ev0.record(lat.stream)
            recs = lat.run_schedule([(T, h_num, sweeps, 0)])
            ev1.record(lat.stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            spins = lat.spins()
            if ref_recs is None:
                ref_recs, ref_spins = recs, spins
            elif not (np.array_equal(recs, ref_recs) and np.array_equal(spins, ref_spins)):
                raise AssertionError("launch shape %s graph=%s changed the trajectory" % (tl, g))
            timings.append({"tiling": list(tl[:3]), "kernel": int(tl[3]), "use_graph": g, "ms_per_sweep": ms / sweeps})
            lat.close()
            del lat
    best = min(timings, key=lambda r: r["ms_per_sweep"])
    return {"tiling": best["tiling"], "kernel": best["kernel"], "use_graph": best["use_graph"],
            "ms_per_sweep": best["ms_per_sweep"], "all": timings}


# (tile_x, tile_y, rows or waves, batch mode); in the pipelined mode the shape is
# that of the films the pipelined kernel cannot take (sublattice launches)
# Sublattice shapes of both formats (a shape the format does not compile is
# refused and skipped): on batches of small films the narrow bit-packed tiles
# (8 or 16 words, 256 or 512 sites of a row per tile, one to four waves) and the int8 tiles with
# four rows per thread lead.
BATCH_CANDIDATES = [(64, 4, 2, BATCH_PHASE_LAUNCH), (64, 4, 4, BATCH_PHASE_LAUNCH), (32, 8, 2, BATCH_PHASE_LAUNCH),
                    (32, 8, 4, BATCH_PHASE_LAUNCH), (16, 16, 1, BATCH_PHASE_LAUNCH), (16, 16, 2, BATCH_PHASE_LAUNCH),
                    (8, 32, 1, BATCH_PHASE_LAUNCH), (8, 16, 1, BATCH_PHASE_LAUNCH), (8, 8, 1, BATCH_PHASE_LAUNCH),
                    (64, 4, 2, BATCH_PERSISTENT), (16, 16, 4, BATCH_WHOLE), (32, 8, 4, BATCH_WHOLE),
                    (32, 16, 8, BATCH_WHOLE), (64, 4, 2, BATCH_PIPE), (32, 8, 2, BATCH_PIPE)]


def tune_batch(make_lats: Callable[..., list], schedule_of: Callable[[int], list], fmt: int,
               sweeps: int = 8, candidates: Optional[Sequence[Tuple[int, int, int, int]]] = None,
               formats: Optional[Sequence[int]] = None) -> dict:
    """Time (tile_x, tile_y, rows_or_waves, batch mode) candidates on a batch of films
    (fresh copies per candidate, built by make_lats(fmt)), for each spin format in
    `formats` (default: fmt alone).  Whole-sweep and pipelined modes apply to INT8
    films only; a format the films cannot take and a candidate the library
    refuses or that reports a failed run are skipped.
    Every candidate must give every film the same records and spins."""
    import torch

    from .lattice import Batch

    timings = []
    skipped = []
    ref = None
    for f in (formats or [fmt]):
        cands = [c for c in (candidates or BATCH_CANDIDATES)
                 if f == FORMAT_INT8 or c[3] not in (BATCH_WHOLE, BATCH_PIPE)]
        for tx, ty, r, mode in cands:
            try:
                lats = make_lats(f)
            except (IsfError, ValueError) as e:
                skipped.append({"format": f, "reason": str(e)})
                break
            kernel = KERNEL_SWEEP if mode == BATCH_WHOLE else KERNEL_TILES
            b = None
            try:
                for i, l in enumerate(lats):
                    l.set_tuning(tx, ty, r, False, kernel)
                    l.schedule_load(schedule_of(i))
                b = Batch(len(lats))
                b.advance(lats, 2, mode)  # warm-up sweeps
                b.sync()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                b.advance(lats, sweeps, mode)
                b.sync()
                dt = time.perf_counter() - t0
            except IsfError as e:
                skipped.append({"format": f, "tiling": [tx, ty, r], "mode": mode, "reason": str(e)})
                for l in lats:
                    l.close()
                if b is not None:
                    b.close()
                continue
            state = [(tuple(l.observables().values()), hashlib.sha256(l.spins().tobytes()).hexdigest()) for l in lats]
            if ref is None:
                ref = state
            elif state != ref:
                raise AssertionError("batch shape %s mode %d format %d changed a trajectory" % ((tx, ty, r), mode, f))
            timings.append({"format": f, "tiling": [tx, ty, r], "mode": mode, "ms_per_sweep": dt * 1e3 / sweeps})
            b.close()
            for l in lats:
                l.close()
            del state
    best = min(timings, key=lambda r: r["ms_per_sweep"])
    return {"format": best["format"], "tiling": best["tiling"], "mode": best["mode"],
            "ms_per_sweep": best["ms_per_sweep"], "all": timings, "skipped": skipped}
