"""Benchmark: spin-flip attempts/s and % of the HBM roofline on one MI355X.

The measured workload is the large plain hysteresis film (2048 x 2048 x 8
FCC film, sigma = 16 px height map, T = 4.0, field ramp +6 -> -6 -> +6 in
steps of 0.05, 50 sweeps per field step, int8 spins, all +1 at start).  One
bench "step" is one field step: 50 sweeps over the whole film (all four
sublattices, with the per-sweep observables and the step record).  Inputs are
resident in HBM before the timed region starts.

Beside the plain path the JSON line carries the same film in the bit-packed
format, the batched workload (256 replicas of uneven films) and the serving
loop (p50/p99 latency), all on the same GPU, plus the roofline of the
dominant kernel and the CPU oracle timed on a bounded sample.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def plain_steps(cfg, first, count):
    hs = cfg.h_nums
    return [(cfg.T, hs[(first + i) % len(hs)], cfg.sweeps_per_step, 0) for i in range(count)]


def bench_plain(cfg, h, fmt, steps, warmup, tuning=None):
    import torch

    from paper_1205_5588_amd.lattice import Lattice

    lat = Lattice(h, cfg.Z, cfg.mc_seed, init=cfg.init, fmt=fmt)
    if tuning:
        lat.set_tuning(*tuning)
    n_occ = lat.observables()["n_occ"]
    if warmup:
        lat.run_schedule(plain_steps(cfg, 0, warmup))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(lat.stream)
    recs = lat.run_schedule(plain_steps(cfg, warmup, steps))
    ev1.record(lat.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    sweeps = steps * cfg.sweeps_per_step
    return lat, n_occ, sweeps, wall, gpu_ms, recs


def roofline_int8(lat, cfg, n_sweeps=40):
    """Mean duration of the sublattice kernel from HIP events around every launch."""
    lat.schedule_load([(cfg.T, cfg.h_nums[0], n_sweeps, 0)])
    ms, n = lat.time_launches(n_sweeps)
    mean_ms = sum(ms) / 4.0
    Nc = cfg.X * cfg.Y * cfg.Z // 2
    bytes_per_launch = 1.25 * Nc  # read all N_c site bytes once, write the active quarter
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_phase_i8", "ms_per_launch": [round(v, 5) for v in ms],
            "bytes_per_launch": int(bytes_per_launch)}


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
    return {"value": round(n_occ * n / dt, 1), "unit": "spin-flip attempts/s", "cores": cpu.threads(),
            "kind": "oracle",
            "sample": "%d sweeps (after 1 untimed) of the 2048x2048x8 film at T=4.0, H=+6.0, from all +1; "
                      "C oracle, gcc -O2, OpenMP over rows of one sublattice" % n}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=481)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported "
              "(replicas and requests shard across GPUs without communication; see the design notes)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from isf_workloads import config_plain_hysteresis_large

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = config_plain_hysteresis_large()
    t0 = time.perf_counter()
    h = cfg.heights()
    log("height map %.2fs" % (time.perf_counter() - t0))

    lat, n_occ, sweeps, wall, gpu_ms, recs = bench_plain(cfg, h, 0, args.steps, args.warmup)
    value = n_occ * sweeps / (gpu_ms * 1e-3)
    log("plain int8: %d steps, %d sweeps, %.3f s wall, %.3f ms gpu, %.3e attempts/s" %
        (args.steps, sweeps, wall, gpu_ms, value))
    roof = roofline_int8(lat, cfg)
    log("roofline:", roof)

    extra = {}
    if not args.no_extra:
        lat_b, n_occ_b, sw_b, wall_b, gpu_ms_b, recs_b = bench_plain(cfg, h, 1, min(args.steps, 40), 2)
        extra["bitpack"] = {"value": round(n_occ_b * sw_b / (gpu_ms_b * 1e-3), 1),
                            "unit": "spin-flip attempts/s", "steps": min(args.steps, 40)}
        log("bitpack:", extra["bitpack"])
        del lat_b

    cpu_base = None
    if not args.no_cpu:
        cpu_base = cpu_baseline(cfg, h)
        log("cpu baseline:", cpu_base)

    Nc = cfg.X * cfg.Y * cfg.Z // 2
    line = {
        "metric": "spin-flip attempts/s",
        "value": round(value, 1),
        "unit": "spin-flip attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(gpu_ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "plain hysteresis 2048x2048x8 FCC film, sigma=16 px, T=4.0, H +6->-6->+6 step 0.05, "
                               "50 sweeps per field step, int8 spins, 1 replica",
                   "n_occ": n_occ, "stored_sites": Nc, "sweeps_per_step": cfg.sweeps_per_step,
                   "effective_GBps_4pass": round(5 * Nc * sweeps / (gpu_ms * 1e-3) / 1e9, 1)},
        "roofline": roof,
        "cpu_baseline": cpu_base,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
