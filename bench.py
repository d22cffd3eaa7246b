"""Benchmark: spin-flip attempts/s and % of the HBM roofline on one MI355X.

The measured workload is the large plain hysteresis film (2048 x 2048 x 8
FCC film, sigma = 16 px height map, T = 4.0, field ramp +6 -> -6 -> +6 in
steps of 0.05, 50 sweeps per field step, int8 spins, all +1 at start).  One
bench "step" is one field step: 50 sweeps over the whole film (all four
sublattices, with the per-sweep observables and the step record).  Every
run sweeps the whole 481-step loop; the --steps timed steps are spread
evenly over it (both saturated ends, both field reversals), each bracketed
by HIP events on the film's stream, and the whole loop's rate is reported
beside them.  Inputs are resident in HBM before the timed region starts.

Beside the plain path the JSON line carries the same film in the bit-packed
format, the gated and anisotropic ramps, the batched workload (256 replicas
of uneven films) and the serving loop (p50/p99 latency), all on the same
GPU, plus the roofline of the dominant kernel, a draw-only ALU ceiling and
the CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_LIST, KERNEL_SWEEP, KERNEL_PIPE, KERNEL_FILM = 1, 2, 3, 4  # isf_tuning.kernel


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spread_steps(n_total, k):
    """k distinct field steps spread evenly over a ramp of n_total steps, both ends included."""
    if k >= n_total:
        return list(range(n_total))
    if k <= 1:
        return [n_total // 2]
    return sorted({int(i * (n_total - 1) / (k - 1) + 0.5) for i in range(k)})


def ramp_schedule(cfg, hs_num=0, an_num=0):
    return [(cfg.T, hv, cfg.sweeps_per_step, 0, hs_num, an_num) for hv in cfg.h_nums]


def bench_ramp(cfg, h, fmt, k, warmup, tuning=None, hs_num=0, an_num=0, aniso_ws=False):
    """The whole ramp on a fresh film, with k of its field steps timed.

    `warmup` untimed steps at the ramp's first field come first.  Then the
    ramp's 481 steps are enqueued as one schedule in chunks; HIP events on the
    film's stream bracket each of the k timed steps (spread over the loop) and
    the whole ramp.  Returns the lattice and the measurements."""
    import torch

    from paper_1205_5588_amd.lattice import Lattice

    lat = Lattice(h, cfg.Z, cfg.mc_seed, init=cfg.init, fmt=fmt)
    if aniso_ws:
        lat.attach_aniso_workspace()
    if tuning:
        if len(tuning) > 4 and tuning[4] == 1:
            lat.attach_items()
        lat.set_tuning(*tuning)
    n_occ = lat.observables()["n_occ"]
    sched = ramp_schedule(cfg, hs_num, an_num)
    sps = cfg.sweeps_per_step
    if warmup:
        lat.run_schedule([sched[0]] * warmup)
    sel = spread_steps(len(sched), k)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in sel]
    whole0, whole1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lat.schedule_load(sched)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    whole0.record(lat.stream)
    pos = 0
    for s, (a, b) in zip(sel, ev):
        if s > pos:
            lat.advance((s - pos) * sps)
        a.record(lat.stream)
        lat.advance(sps)
        b.record(lat.stream)
        pos = s + 1
    if pos < len(sched):
        lat.advance((len(sched) - pos) * sps)
    whole1.record(lat.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recs = lat.records()
    timed_ms = sum(a.elapsed_time(b) for a, b in ev)
    whole_ms = whole0.elapsed_time(whole1)
    sweeps = len(sel) * sps
    return {"lat": lat, "n_occ": n_occ, "steps": sel, "sweeps": sweeps, "timed_ms": timed_ms,
            "value": n_occ * sweeps / (timed_ms * 1e-3), "whole_ms": whole_ms, "wall_s": wall,
            "whole_value": n_occ * len(sched) * sps / (whole_ms * 1e-3), "records": recs}


def launch_durations(lat, cfg, steps, hs_num=0, an_num=0):
    """Mean duration of each launch of the film's sweep kernel over the given field
    steps of a second pass of the ramp: a pair of timing-only HIP events around every
    launch (isf_time_launches), untimed graph replay elsewhere.  Returns the mean
    milliseconds per launch of each of the four sublattices (whole-sweep kernels:
    entry 0 is the sweep)."""
    sched = ramp_schedule(cfg, hs_num, an_num)
    sps = cfg.sweeps_per_step
    lat.schedule_load(sched)
    tot = [0.0, 0.0, 0.0, 0.0]
    n = 0
    pos = 0
    for s in steps:
        if s > pos:
            lat.advance((s - pos) * sps)
        ms, got = lat.time_launches(sps)
        tot = [t + m * got for t, m in zip(tot, ms)]
        n += got
        pos = s + 1
    if pos < len(sched):
        lat.advance((len(sched) - pos) * sps)
    lat.records()
    return [t / max(n, 1) for t in tot]


def roofline_int8(lat, cfg, steps, region_ms_per_sweep):
    """Algorithmic bandwidth of the dominant kernel against the 8 TB/s HBM peak.

    Algorithmic bytes follow the four-phase schedule (N_c = X Y Z / 2 stored
    sites): each sublattice phase reads every stored byte and writes its active
    quarter, 1.25 N_c per phase and 5 N_c per sweep.  A whole-sweep launch is one
    sweep (5 N_c), a sublattice launch one phase (1.25 N_c).  The launch duration
    of a whole-sweep kernel (one launch per sweep) is the timed region's time
    per sweep, between HIP events on the film's stream; that of a sublattice
    launch is the mean over the timed field steps of a second pass of the ramp,
    from timing-only HIP events around every launch (reported for whole-sweep
    kernels too, where the events' own recording time makes it a little
    longer).  The film (16 MiB) sits in
    the 256 MB Infinity Cache and the whole-sweep kernels move about a third of
    the four-phase bytes (traffic), so the fraction is the schedule's figure of
    merit, not a measure of DRAM use: the kernel is bound by its integer VALU and
    LDS work and their latency (profiles/)."""
    ms = launch_durations(lat, cfg, steps)
    Nc = cfg.X * cfg.Y * cfg.Z // 2
    whole = lat.get_tuning()[4] in (KERNEL_SWEEP, KERNEL_PIPE)
    if whole:
        # one launch per sweep: the timed region's events give the launch duration
        # (the small gaps between graph-replayed launches included); the event
        # pairs around single launches add their own recording time
        mean_ms, bytes_per_launch, min_bytes = region_ms_per_sweep, 5.0 * Nc, 2.0 * Nc
    else:
        mean_ms, bytes_per_launch, min_bytes = sum(ms) / 4.0, 1.25 * Nc, 0.5 * Nc
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9
    kernel = lat_kernel_name(lat)
    trec = measured_traffic(kernel)
    traffic = int(trec["fetch_bytes_per_launch"] + trec["write_bytes_per_launch"]) if trec else None
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "kernel": kernel, "ms_per_launch": round(mean_ms, 5),
           "ms_per_launch_event_pairs" if whole else "ms_per_launch_by_sublattice":
               round(ms[0], 5) if whole else [round(v, 5) for v in ms],
           "ms_per_sweep_region": round(region_ms_per_sweep, 5),
           "bytes_per_launch": int(bytes_per_launch), "bytes_model": "four-phase schedule, 5 N_c per sweep",
           "frac_min_bytes": round(min_bytes / (mean_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "launches_timed": len(steps) * cfg.sweeps_per_step,
           "limiter": "integer VALU + LDS latency; film resident in the Infinity Cache"}
    if traffic:
        out["traffic_frac"] = round(traffic / (mean_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        out["traffic_window"] = trec.get("window")
    return out


def alu_ceiling(lat, cfg, n_sweeps=200):
    """Draw-only ceiling: the same film's stored dwords draw their attempts' Philox
    numbers (one 4x32-10 call per dword and sweep, vacant dwords included) and
    nothing else; attempts/s if a sweep cost only its draws."""
    lat.draw_xor(0, 4)
    _, ms = lat.draw_xor(1000, n_sweeps)
    n_occ = lat.observables()["n_occ"]
    Nc = cfg.X * cfg.Y * cfg.Z // 2
    return {"kind": "Philox4x32-10 draws only, one call per stored dword and sweep", "sweeps": n_sweeps,
            "us_per_sweep": round(ms * 1e3 / n_sweeps, 3),
            "draws_per_s": round(Nc * n_sweeps / (ms * 1e-3), 1),
            "attempts_per_s": round(n_occ * n_sweeps / (ms * 1e-3), 1)}


KERNEL_SOURCES = ("isf_sweep.hip", "isf_books.h", "isf_device.h", "isf_internal.h")


def measured_traffic(kernel):
    """The committed counter record of `kernel` (FETCH_SIZE and WRITE_SIZE bytes per
    launch, scaled by a copy of known size, and the launches they were taken over),
    or None when there is none or the kernel's sources changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(kernel)
    if not rec:
        return None
    csrc = os.path.join(ROOT, "paper_1205_5588_amd", "csrc")
    blob = b"".join(open(os.path.join(csrc, n), "rb").read() for n in KERNEL_SOURCES)
    if hashlib.sha256(blob).hexdigest() != rec["sources_sha256"]:
        return None
    return rec


def lat_kernel_name(lat):
    t = lat.get_tuning()
    return {KERNEL_LIST: "k_phase_i8_list", KERNEL_SWEEP: "k_sweep_i8_halo",
            KERNEL_PIPE: "k_sweep_i8_pipe", KERNEL_FILM: "k_sweep_i8_film"}.get(t[4], "k_phase_i8")


def bench_surface_image(lat, cfg, reps=20):
    """Simulated PMOKE image of the film (one [Y][X] int8 image per call), timed with
    HIP events on the film's stream."""
    import torch

    img = torch.empty(cfg.X * cfg.Y, dtype=torch.int8, device="cuda")
    lat.surface_image(out=img)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(lat.stream)
    for _ in range(reps):
        lat.surface_image(out=img)
    ev1.record(lat.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    return {"ms_per_image": round(ms, 5), "pixels_per_s": round(cfg.X * cfg.Y / (ms * 1e-3), 1)}


def tune_plain(cfg, h, fmt):
    from paper_1205_5588_amd.autotune import tune_lattice
    from paper_1205_5588_amd.lattice import Lattice

    res = tune_lattice(lambda: Lattice(h, cfg.Z, cfg.mc_seed, init=cfg.init, fmt=fmt), fmt, cfg.T, cfg.h_nums[0],
                       sweeps=128, warmup=4)
    return res


def bench_batched(args):
    """The batched workload: 16 uneven films x 16 temperatures = 256 replicas, each
    with its own ramp +5 -> -5 -> +5 (step 0.1, 20 sweeps per step)."""
    import torch

    from isf_workloads import batched_films
    from paper_1205_5588_amd.autotune import lookup, tune_batch
    from paper_1205_5588_amd.lattice import Batch, Lattice

    reps, seed, hnums, spst = batched_films()
    stream = torch.cuda.Stream()
    sched = [[(r.T, hv, spst, 0) for hv in hnums] for r in reps]

    heights = {}
    for r in reps:
        if r.film not in heights:
            heights[r.film] = r.heights()

    def make(fmt=0):
        return [Lattice(heights[r.film], r.Z, seed, replica=r.replica, init=0, fmt=fmt, stream=stream) for r in reps]

    t0 = time.perf_counter()
    tuned = tune_batch(make, lambda i: sched[i], 0, sweeps=6, formats=(0, 1))
    log("batch tuning %.1fs: best %s mode %d format %d (%.3f ms/sweep); skipped %s" % (
        time.perf_counter() - t0, tuned["tiling"], tuned["mode"], tuned["format"], tuned["ms_per_sweep"],
        tuned["skipped"]))
    kernel = KERNEL_SWEEP if tuned["mode"] == 2 else 0
    lats = make(tuned["format"])
    for l in lats:
        l.set_tuning(*tuned["tiling"], False, kernel)
    n_occ = [l.observables()["n_occ"] for l in lats]
    b = Batch(len(lats), stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = b.run(lats, sched, mode=tuned["mode"])
    dt = time.perf_counter() - t0
    attempts = sum(n * len(hnums) * spst for n in n_occ)
    out = {"value": round(attempts / dt, 1), "unit": "spin-flip attempts/s", "replicas": len(reps),
           "sweeps_per_replica": len(hnums) * spst, "attempts": attempts, "seconds": round(dt, 4),
           "mode": {0: "phase_launch", 1: "persistent", 2: "whole_sweep", 3: "pipelined"}[tuned["mode"]],
           "format": {0: "int8", 1: "bitpack"}[tuned["format"]], "tiling": tuned["tiling"],
           "tuning": tuned["all"], "tuning_skipped": tuned["skipped"],
           "graphs": "chunks of 64 sweeps replayed from a cached graph"}
    # the same replicas one after another through the plain path (a sample, shortened schedule)
    sample = list(range(0, len(reps), 16))
    short = 10
    plain_dt = 0.0   # run time only; film construction is excluded
    att = 0
    for i in sample:
        r = reps[i]
        l = Lattice(heights[r.film], r.Z, seed, replica=r.replica, init=0, stream=stream)
        l.set_tuning(*lookup(r.X, r.Y, r.Z, 0))  # the plain path's shape for this film
        torch.cuda.synchronize()
        ts = time.perf_counter()
        l.run_schedule(sched[i][:short])
        plain_dt += time.perf_counter() - ts
        att += n_occ[i] * short * spst
        l.close()
    out["plain_same_replicas"] = {"value": round(att / max(plain_dt, 1e-9), 1),
                                  "sample": "16 replicas (one per film), first %d field steps, run one after "
                                            "another through the plain path (its own launch shape per film, "
                                            "graph replay)" % short}
    del lats, b
    return out


def serving_inputs(args, rate=50.0, duration=None):
    """Requests and their height maps (the requests' payload, not server work),
    built in this process with a pool of threads (numpy's FFTs release the GIL)
    only when the serving measurement runs."""
    import concurrent.futures as cf

    from isf_workloads import height_map, serving_requests

    reqs = serving_requests(rate=rate, duration=duration or args.serve_duration)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        heights = list(ex.map(lambda q: height_map(q.X, q.Y, q.Z, q.sigma, q.seed), reqs))
    log("serving: %d requests, height maps %.1fs" % (len(reqs), time.perf_counter() - t0))
    return reqs, {q.rid: hh for q, hh in zip(reqs, heights)}


def bench_serving(args, reqs, hmap, rate=50.0, duration=None, shape=None):
    """Poisson arrivals (50 req/s for the configured duration) of hysteresis and
    temperature-scan jobs on films of 64^2..2048^2 x 1..10 layers.  shape: (format,
    sublattice tiling) for every request, e.g. the batch tuner's pick for the
    batched workload (default: int8 films in their own default shapes)."""
    duration = duration or args.serve_duration
    from paper_1205_5588_amd.serve import GpuExecutor, Job, Server

    fmt, tiling = shape if shape else (0, None)
    jobs = [Job(rid=q.rid, arrival=q.arrival, footprint=GpuExecutor.footprint(q, fmt), n_sweeps=q.n_sweeps,
                payload=q) for q in reqs]
    ex = GpuExecutor(max_slots=args.serve_slots, mode=args.serve_mode, heights_of=lambda q: hmap[q.rid],
                     tiling=tuple(tiling) + (False, 0) if tiling else None, fmt=fmt)
    srv = Server(ex, budget_bytes=int(args.serve_budget_gib * 2**30), max_slots=args.serve_slots,
                 target_chunk_s=0.02, rate_estimate=2e11, max_chunk=64)
    t0 = time.perf_counter()
    done = [0]

    def retired(_res):
        done[0] += 1
        if done[0] % 500 == 0:
            log("serving: %d of %d requests done after %.0f s" % (done[0], len(jobs), time.perf_counter() - t0))

    stats = srv.run(jobs, on_retire=retired)
    wall = time.perf_counter() - t0
    s = stats.summary()
    s["wall_s"] = round(wall, 2)
    s["offered_attempts_per_s"] = round(s["attempts"] / duration, 1)
    s["mode"] = {0: "phase_launch", 1: "persistent", 2: "whole_sweep", 3: "pipelined"}[args.serve_mode]
    s["format"] = {0: "int8", 1: "bitpack"}[fmt]
    s["tiling"] = list(tiling) if tiling else "each film's default"
    s["arrivals"] = "Poisson %g req/s for %g s" % (rate, duration)
    return s


def bench_small_configs(tune=True):
    """The two other plain workloads, whole, with HIP events around each: the small
    ramp (64x64x3, 161 field steps x 100 sweeps: a 6 KiB film that the film
    kernel sweeps from one compute unit's LDS, latency-bound, so no roofline) and the temperature scan (512x512x5, 45
    temperatures x 1000 sweeps, the first 200 of each discarded), each in the
    launch shape the tuner picks for it."""
    import torch

    from isf_workloads import config_plain_hysteresis_small, config_plain_tscan
    from paper_1205_5588_amd.autotune import lookup, tune_lattice
    from paper_1205_5588_amd.lattice import Lattice

    out = {}
    for name, cfg in (("small_ramp", config_plain_hysteresis_small()), ("temperature_scan", config_plain_tscan())):
        h = cfg.heights()
        T0, h0 = (cfg.T, cfg.h_nums[0]) if cfg.h_nums is not None else (cfg.temps[-1], 0)
        if tune:
            tb = tune_lattice(lambda: Lattice(h, cfg.Z, cfg.mc_seed, init=cfg.init), 0, T0, h0, sweeps=64,
                              warmup=4)
            tl = tuple(tb["tiling"]) + (tb["use_graph"], tb["kernel"])
        else:
            tl = lookup(cfg.X, cfg.Y, cfg.Z, 0)
        lat = Lattice(h, cfg.Z, cfg.mc_seed, init=cfg.init)
        lat.set_tuning(*tl)
        if cfg.h_nums is not None:
            sched = [(cfg.T, hv, cfg.sweeps_per_step, 0) for hv in cfg.h_nums]
        else:
            sched = [(T, 0, cfg.sweeps_per_T, cfg.discard_per_T) for T in cfg.temps]
        sweeps = sum(s[2] for s in sched)
        lat.run_schedule(sched[:1])  # warm-up: graphs and lists built
        lat.schedule_load(sched)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        while lat.advance(1 << 20):
            pass
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        n_occ = lat.observables()["n_occ"]
        out[name] = {"film": "%dx%dx%d" % (cfg.X, cfg.Y, cfg.Z), "sweeps": sweeps,
                     "attempts_per_s": round(n_occ * sweeps / (ms * 1e-3), 1),
                     "us_per_sweep": round(ms * 1e3 / sweeps, 3), "tuning": list(tl),
                     "hbm_frac_5Nc": None if name == "small_ramp" else
                     round(5 * (cfg.X * cfg.Y * cfg.Z // 2) / (ms * 1e-3 / sweeps) / 1e9 / HBM_PEAK_GBS, 4)}
        if name == "small_ramp":
            out[name]["roofline"] = "n/a: one compute unit, latency-bound"
        del lat
    return out


def cpu_baseline(cfg, h, budget_s=15.0):
    from oracle import cpu

    threads = min(16, os.cpu_count() or 1)
    cpu.set_threads(threads)
    f = cpu.Film(h, cfg.Z, cfg.mc_seed, init=cfg.init)
    n_occ = f.state()[2]
    t0 = time.perf_counter()
    f.run(cfg.T, cfg.h_nums[0], 1)
    one = time.perf_counter() - t0
    n = max(1, min(cfg.sweeps_per_step - 1, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    f.run(cfg.T, cfg.h_nums[0], n)
    dt = time.perf_counter() - t0
    used = cpu.threads()
    # the same oracle on one thread, two sweeps (its rate does not depend on the sweep)
    cpu.set_threads(1)
    t0 = time.perf_counter()
    f.run(cfg.T, cfg.h_nums[0], 2)
    dt1 = time.perf_counter() - t0
    cpu.set_threads(threads)
    return {"value": round(n_occ * n / dt, 1), "unit": "spin-flip attempts/s", "cores": used,
            "kind": "oracle",
            "sample": "%d sweeps (after 1 untimed) of the 2048x2048x8 film at T=4.0, H=+6.0, from all +1; "
                      "C oracle, gcc -O2, OpenMP over rows of one sublattice" % n,
            "single_thread_value": round(n_occ * 2 / dt1, 1)}


def copy_calibration(args):
    """Three plain device copies of --copy-mib MiB: what rocprofv3's byte counters read for
    them scales the counters of the kernels profiled in the same command."""
    if not args.copy_mib:
        return
    import torch

    n = args.copy_mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy calibration: 3 x %d bytes" % n)


def ramp_summary(r, cfg):
    """The JSON fields of one ramp measurement (bench_ramp)."""
    sps = cfg.sweeps_per_step
    return {"value": round(r["value"], 1), "unit": "spin-flip attempts/s", "steps_timed": len(r["steps"]),
            "ms_per_sweep": round(r["timed_ms"] / r["sweeps"], 5),
            "whole_ramp": {"steps": len(cfg.h_nums), "attempts_per_s": round(r["whole_value"], 1),
                           "ms_per_sweep": round(r["whole_ms"] / (len(cfg.h_nums) * sps), 5)}}


def bitpack_fields(r, cfg):
    """Bit-packed film: its rate and its fraction of HBM at the four-phase schedule's
    bytes for 1-bit spins and occupancy, 1.125 N_c per sweep."""
    out = ramp_summary(r, cfg)
    Nc = cfg.X * cfg.Y * cfg.Z // 2
    gbs = 1.125 * Nc / (out["ms_per_sweep"] * 1e-3) / 1e9
    out["hbm"] = {"bytes_per_sweep": int(1.125 * Nc), "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["tuning"] = list(r["lat"].get_tuning())
    return out


def run_only(args, cfg, h):
    """One extra measurement alone, as in the full run (same workloads and step counts)."""
    tl = tuple(int(v) for v in args.tiling.split(",")) if args.tiling else None
    kern = 0
    if tl is not None and len(tl) > 3:
        tl, kern = tl[:3], tl[3]
    if args.only == "batched":
        return bench_batched(args)
    if args.only == "plain":
        return run_plain_untimed(args, cfg, h)
    if args.only == "small":
        return bench_small_configs(tune=not args.no_tune)
    if args.only == "bitpack":
        if tl is None and not args.no_tune:
            tb = tune_plain(cfg, h, 1)
            tl = tuple(tb["tiling"])
            kern = tb["kernel"]
        tuning = None if tl is None else tl + (True, kern)
        return bitpack_fields(bench_ramp(cfg, h, 1, args.steps, 2, tuning), cfg)
    if tl is None:
        tl, kern = (32, 32, 16), KERNEL_PIPE
    return bench_aniso(cfg, h, args.steps, tl + (True, kern))


def run_plain_untimed(args, cfg, h):
    """The plain ramp's first --steps field steps (after one warm-up step) in the
    launch shape of --plain-tiling (default: the pipelined kernel, 32 x 32 tiles, graph
    replay), with no timing of any kind: the workload of the rocprofv3 counter passes."""
    import numpy as np

    from paper_1205_5588_amd.lattice import Lattice

    tl = (tuple(int(v) for v in args.plain_tiling.split(",")) if args.plain_tiling
          else (32, 32, 16, KERNEL_PIPE, 1))
    lat = Lattice(h, cfg.Z, cfg.mc_seed, init=cfg.init)
    lat.set_tuning(tl[0], tl[1], tl[2], bool(tl[4]), tl[3])
    sps = cfg.sweeps_per_step
    lat.run_schedule([(cfg.T, cfg.h_nums[0], sps, 0)])
    steps = [(cfg.T, hv, sps, 0) for hv in cfg.h_nums[: args.steps]]
    rec = lat.run_schedule(steps)
    out = {"kernel": lat_kernel_name(lat), "tiling": list(lat.get_tuning()), "sweeps": len(steps) * sps,
           "warmup_sweeps": sps, "accepted": int(np.asarray(rec)[:, 5].sum())}
    lat.close()
    return out


def bench_aniso(cfg, h, k, tuning):
    """The ramp with the anisotropy term of Eq. 7, h_an = 2 (an_num = 40).  On a whole-sweep
    kernel each field step runs at field h + h_an sign(M) from a copy of the spins and state,
    and again on the per-sublattice kernels (M frozen per phase) where the accepted flips do not
    rule out |M| < 2 at a phase start; on the per-sublattice kernels the term is applied phase
    by phase throughout."""
    whole = tuning[4] in (KERNEL_SWEEP, KERNEL_PIPE)
    r = bench_ramp(cfg, h, 0, k, 2, tuning, an_num=40, aniso_ws=whole)
    out = {**ramp_summary(r, cfg), "an_num": 40, "tiling": list(tuning[:3]),
           "kernel": {KERNEL_SWEEP: "k_sweep_i8_halo", KERNEL_PIPE: "k_sweep_i8_pipe"}.get(tuning[4], "k_phase_i8")}
    if whole:
        runs, redone = r["lat"].aniso_stats()
        out["step_parts_on_whole_kernel"] = runs
        out["run_again_per_sublattice"] = redone
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=481,
                    help="field steps timed, spread evenly over the 481-step loop (the whole loop always runs)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-duration", type=float, default=60.0)
    ap.add_argument("--serve-slots", type=int, default=512)
    ap.add_argument("--serve-mode", type=int, default=0)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (calibrates rocprofv3 byte counters)")
    ap.add_argument("--only", choices=["bitpack", "anisotropy", "batched", "plain", "small"], default=None,
                    help="run only this one of the extra measurements and print its result (for profiling); "
                         "plain: the first --steps field steps of the plain ramp and nothing else, untimed "
                         "(no events between launches), for counter passes; small: the small ramp and the "
                         "temperature scan")
    ap.add_argument("--plain-tiling", default=None,
                    help="the plain ramp's launch shape tx,ty,rows,kernel,graph instead of the tuner's (graph 0: "
                         "plain launches, e.g. for counter passes that need no graph replay)")
    ap.add_argument("--tiling", default=None,
                    help="with --only bitpack or anisotropy: the launch shape tx,ty,rows[,kernel] "
                         "(kernel 0: tiles, 1: occupied-dword lists; no tuning)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported "
              "(replicas and requests shard across GPUs without communication; see the design notes)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        print("bench.py: --steps must be at least 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from isf_workloads import config_plain_hysteresis_large

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = config_plain_hysteresis_large()
    t0 = time.perf_counter()
    h = cfg.heights()
    log("height map %.2fs" % (time.perf_counter() - t0))

    if args.only:
        res = run_only(args, cfg, h)
        copy_calibration(args)
        print(json.dumps({"only": args.only, **res}), flush=True)
        return

    from paper_1205_5588_amd.autotune import lookup

    tuning = lookup(cfg.X, cfg.Y, cfg.Z, 0)  # cached or heuristic shape, replaced by the tuner's pick
    tune_info = None
    if args.plain_tiling:
        v = [int(x) for x in args.plain_tiling.split(",")]
        if len(v) != 5:
            print("bench.py: --plain-tiling takes tx,ty,rows,kernel,graph", file=sys.stderr)
            sys.exit(2)
        tuning = (v[0], v[1], v[2], bool(v[4]), v[3])
    elif not args.no_tune:
        t0 = time.perf_counter()
        tune_info = tune_plain(cfg, h, 0)
        tuning = tuple(tune_info["tiling"]) + (tune_info["use_graph"], tune_info["kernel"])
        log("plain tuning %.1fs: %s" % (time.perf_counter() - t0, tune_info))
    r = bench_ramp(cfg, h, 0, args.steps, args.warmup, tuning)
    lat, n_occ, sweeps = r["lat"], r["n_occ"], r["sweeps"]
    log("plain int8: %d timed steps of %d, %d sweeps, %.3f ms timed, %.3e attempts/s; whole loop %.3f ms, "
        "%.3e attempts/s" % (len(r["steps"]), len(cfg.h_nums), sweeps, r["timed_ms"], r["value"], r["whole_ms"],
                            r["whole_value"]))
    lat_stats = lat.film_stats()
    roof = roofline_int8(lat, cfg, r["steps"], r["timed_ms"] / sweeps)
    log("roofline:", roof)
    ceiling = alu_ceiling(lat, cfg)
    log("draw-only ceiling:", ceiling)
    pmoke = bench_surface_image(lat, cfg)
    log("pmoke image:", pmoke)
    del lat

    small = bench_small_configs(tune=not args.no_tune)
    log("small configs:", small)
    extra = {"whole_ramp": ramp_summary(r, cfg)["whole_ramp"], "alu_ceiling": ceiling, "pmoke_image": pmoke,
             "other_plain_workloads": small,
             "film": lat_stats,
             "tuning": {"tiling": list(tuning[:3]), "use_graph": bool(tuning[3]), "kernel": int(tuning[4]),
                        "tuned": tune_info is not None,
                        "candidates": 0 if tune_info is None else len(tune_info["all"])}}
    if not args.no_extra:
        tb = None if args.no_tune else tune_plain(cfg, h, 1)
        tbt = lookup(cfg.X, cfg.Y, cfg.Z, 1) if tb is None else tuple(tb["tiling"]) + (tb["use_graph"], tb["kernel"])
        rb = bench_ramp(cfg, h, 1, args.steps, 2, tbt)
        extra["bitpack"] = bitpack_fields(rb, cfg)
        log("bitpack:", extra["bitpack"])
        del rb
        # the same ramp behind the switching-field gate of Eq. 9 with h_s = 2 (hs_num = 40)
        rg = bench_ramp(cfg, h, 0, args.steps, 2, tuning, hs_num=40)
        extra["gated"] = {**ramp_summary(rg, cfg), "hs_num": 40,
                          "accepted_per_attempt": round(float(rg["records"][:, 5].sum()) /
                                                        (rg["n_occ"] * len(cfg.h_nums) * cfg.sweeps_per_step), 5)}
        log("gated:", extra["gated"])
        del rg
        # the same ramp with the anisotropy term of Eq. 7, h_an = 2 (an_num = 40), on the
        # pipelined kernel (steps checked, and run again per sublattice near M = 0) and,
        # for comparison, on the per-sublattice kernels alone (M frozen per phase)
        extra["anisotropy"] = bench_aniso(cfg, h, args.steps, (32, 32, 16, True, KERNEL_PIPE))
        extra["anisotropy"]["per_sublattice_kernels"] = {
            k: v for k, v in bench_aniso(cfg, h, args.steps, (64, 4, 2, True, 0)).items()
            if k in ("value", "ms_per_sweep", "whole_ramp", "kernel")}
        log("anisotropy:", extra["anisotropy"])
        extra["batched"] = bench_batched(args)
        log("batched:", {k: v for k, v in extra["batched"].items() if k != "tuning"})
        if not args.no_serve:
            # requests take the format and sublattice shape the batch tuner picked for the
            # batched workload (films of the same kind) when both run one launch per sublattice
            bt = extra["batched"]
            shape = None
            if args.serve_mode == 0 and bt["mode"] == "phase_launch":
                shape = (0 if bt["format"] == "int8" else 1, bt["tiling"])
            extra["serving"] = bench_serving(args, *serving_inputs(args), shape=shape)
            log("serving:", extra["serving"])
            # the same request mix at 15 req/s for 30 s, below the GPU's capacity, where
            # the latency is service time rather than backlog
            d = min(30.0, args.serve_duration)
            extra["serving_below_capacity"] = bench_serving(args, *serving_inputs(args, 15.0, d), rate=15.0,
                                                            duration=d, shape=shape)
            log("serving below capacity:", extra["serving_below_capacity"])

    cpu_base = None
    if not args.no_cpu:
        cpu_base = cpu_baseline(cfg, h)
        log("cpu baseline:", cpu_base)

    copy_calibration(args)

    Nc = cfg.X * cfg.Y * cfg.Z // 2
    line = {
        "metric": "spin-flip attempts/s",
        "value": round(r["value"], 1),
        "unit": "spin-flip attempts/s",
        "n_gpus": 1,
        "steps": len(r["steps"]),
        "warmup": args.warmup,
        "ms_per_step": round(r["timed_ms"] / len(r["steps"]), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "plain hysteresis 2048x2048x8 FCC film, sigma=16 px, T=4.0, H +6->-6->+6 step 0.05, "
                               "50 sweeps per field step, int8 spins, 1 replica",
                   "n_occ": n_occ, "stored_sites": Nc, "sweeps_per_step": cfg.sweeps_per_step,
                   "timed_steps": "%d of the loop's %d field steps, spread evenly over it (both reversals "
                                  "included); the whole loop runs" % (len(r["steps"]), len(cfg.h_nums)),
                   "effective_GBps_4pass": round(5 * Nc * sweeps / (r["timed_ms"] * 1e-3) / 1e9, 1)},
        "roofline": roof,
        "cpu_baseline": cpu_base,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
