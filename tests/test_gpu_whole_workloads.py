"""GPU: the five workloads at their real length against the CPU oracle.

Each workload runs on the GPU the way the bench runs it (launch shapes from
the tuner's table, graph replay, batches, the serving loop).  The oracle then
repeats the same trajectory in segments: every segment starts from the GPU's
spins at its first sweep (restored into the oracle with the sweep counter, so
the oracle draws the same numbers) and must end with the GPU's records and
spins.  Since the oracle is deterministic, agreement on every segment of a run
is agreement on the whole run, and the segments can run side by side on the
host's cores.

  temperature scan 512 x 512 x 5: all 45 temperatures x 1000 sweeps (200
      discarded), every temperature a segment;
  large ramp 2048 x 2048 x 8: all 481 field steps in int8 (pipelined kernel)
      and bit-packed, equal record for record and spin for spin, and the
      oracle on 16 steps spread over the loop, the two field reversals among
      them; the same ramp with the anisotropy term on the pipelined kernel
      equal to the per-sublattice kernels;
  batched: all 256 replicas on the first three steps (pipelined batch mode,
      equal to the sublattice mode), and the whole 201-step ramp of the
      smallest, a median and the largest film in 16 segments;
  serving: a stratified sample of the Poisson request stream (largest sides,
      one and ten layers, both job kinds) on shortened schedules in a mix:
      alone == in the mix for all of them, the oracle for those it finishes in
      seconds and for a ten-layer film of about 1024^2.
"""

import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest

from oracle import cpu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def isf():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1205_5588_amd import lattice

    return lattice


def _workers():
    return max(1, min(16, os.cpu_count() or 1))


def _oracle_pool(tasks):
    """Run oracle checks (callables that raise on a mismatch) side by side, one film per
    host thread and one OpenMP thread per film (the oracle's calls release the GIL)."""
    cpu.lib()
    before = cpu.threads()

    def one(fn):
        cpu.set_threads(1)
        return fn()

    try:
        with cf.ThreadPoolExecutor(_workers()) as ex:
            for f in [ex.submit(one, t) for t in tasks]:
                f.result()
    finally:
        cpu.set_threads(before)


def _tuned(isf, lat):
    from paper_1205_5588_amd.autotune import lookup

    lat.set_tuning(*lookup(lat.X, lat.Y, lat.Z, lat.fmt))
    return lat


# ------------------------------------------------------------------ temperature scan
@pytest.mark.timeout(900)
def test_temperature_scan_whole_against_oracle(isf):
    from isf_workloads import config_plain_tscan

    c = config_plain_tscan()
    h = c.heights()
    sw, dc = c.sweeps_per_T, c.discard_per_T
    g = _tuned(isf, isf.Lattice(h, c.Z, c.mc_seed, init=c.init))
    _say("tscan: %d temperatures, tuning %s" % (len(c.temps), g.get_tuning()))
    snaps = [g.spins()]
    recs = []
    for T in c.temps:
        recs.append(g.temperature_scan([T], sw, dc)[0])
        snaps.append(g.spins())
    recs = np.array(recs)
    whole = _tuned(isf, isf.Lattice(h, c.Z, c.mc_seed, init=c.init))
    np.testing.assert_array_equal(whole.temperature_scan(c.temps, sw, dc), recs)
    np.testing.assert_array_equal(whole.spins(), snaps[-1])
    o = cpu.Film(h, c.Z, c.mc_seed, init=c.init)
    np.testing.assert_array_equal(o.spins(), snaps[0])
    n_occ = o.state()[2]
    _say("tscan: GPU done, oracle on %d segments" % len(c.temps))

    def segment(i, T):
        def run():
            f = cpu.Film(h, c.Z, c.mc_seed, init=c.init)
            f.set_spins(snaps[i], i * sw)
            r = f.run(T, 0, sw, dc).as_tuple()
            assert r == tuple(recs[i]), (i, T, r, recs[i])
            np.testing.assert_array_equal(f.spins(), snaps[i + 1], err_msg="T=%g" % T)
        return run

    _oracle_pool([segment(i, T) for i, T in enumerate(c.temps)])
    kept = sw - dc
    absm = [float(r[3]) / (float(kept) * float(n_occ)) for r in recs]
    assert absm[0] < 0.05   # disordered at T = 12


# ------------------------------------------------------------------ large ramp
@pytest.mark.timeout(900)
def test_large_ramp_whole_int8_bitpack_and_oracle(isf):
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    hs, sps = c.h_nums, c.sweeps_per_step
    n = len(hs)
    full = _tuned(isf, isf.Lattice(h, c.Z, c.mc_seed, init=c.init))
    _say("large ramp: %d steps, int8 tuning %s" % (n, full.get_tuning()))
    r_full = full.ramp_field(c.T, hs, sps)
    M = r_full[:, 0]
    down = int(np.argmax(M[: n // 2 + 1] < 0))
    up = n // 2 + int(np.argmax(M[n // 2:] > 0))
    assert M[down] < 0 < M[up], "the loop must reverse in both legs"
    chosen = sorted({0, n - 1, down, up} | set(range(20, n - 1, 40)))
    del full
    gi = _tuned(isf, isf.Lattice(h, c.Z, c.mc_seed, init=c.init))
    gb = _tuned(isf, isf.Lattice(h, c.Z, c.mc_seed, init=c.init, fmt=1))
    _say("large ramp: bit-packed tuning %s; oracle steps %s" % (gb.get_tuning(), chosen))
    ri, rb, seg = [], [], {}
    pos = 0
    for s in chosen + [n]:
        if s > pos:
            ri.append(gi.ramp_field(c.T, hs[pos:s], sps))
            rb.append(gb.ramp_field(c.T, hs[pos:s], sps))
            np.testing.assert_array_equal(gb.spins(), gi.spins(), err_msg="before step %d" % s)
        if s == n:
            break
        start = gi.spins()
        ri.append(gi.ramp_field(c.T, hs[s:s + 1], sps))
        rb.append(gb.ramp_field(c.T, hs[s:s + 1], sps))
        end = gi.spins()
        np.testing.assert_array_equal(gb.spins(), end, err_msg="after step %d" % s)
        seg[s] = (start, end)
        pos = s + 1
    ri, rb = np.concatenate(ri), np.concatenate(rb)
    np.testing.assert_array_equal(ri, r_full)
    np.testing.assert_array_equal(rb, r_full)
    _say("large ramp: GPU done (int8 == bit-packed on all %d steps), oracle on %d steps" % (n, len(seg)))

    def segment(s):
        def run():
            f = cpu.Film(h, c.Z, c.mc_seed, init=c.init)
            f.set_spins(seg[s][0], s * sps)
            r = f.run(c.T, hs[s], sps, 0).as_tuple()
            assert r == tuple(r_full[s]), (s, r, r_full[s])
            np.testing.assert_array_equal(f.spins(), seg[s][1], err_msg="step %d" % s)
        return run

    o = cpu.Film(h, c.Z, c.mc_seed, init=c.init)
    np.testing.assert_array_equal(o.spins(), seg[0][0])
    del o
    _oracle_pool([segment(s) for s in chosen])


# ------------------------------------------------------------------ batched
@pytest.mark.timeout(900)
def test_large_ramp_anisotropy_whole_kernel_equals_phase_kernels(isf):
    """The large ramp with the anisotropy term of Eq. 7 (h_an = 2), all 481 steps: on the
    pipelined whole-sweep kernel (steps at field h + h_an sign(M), run again per sublattice
    where |M| could have come below 2) and on the per-sublattice kernels, which apply the term
    phase by phase and are checked against the oracle elsewhere: equal record for record and
    spin for spin."""
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    steps = [(c.T, hn, c.sweeps_per_step, 0, 0, 40) for hn in c.h_nums]
    w = isf.Lattice(h, c.Z, c.mc_seed, init=c.init)
    w.attach_aniso_workspace()
    w.set_tuning(32, 32, 16, True, 3)
    _say("anisotropic ramp: whole-sweep kernel")
    rw = w.run_schedule(steps)
    runs, redone = w.aniso_stats()
    _say("anisotropic ramp: %d steps on the whole-sweep kernel, %d of them run again" % (runs, redone))
    p = isf.Lattice(h, c.Z, c.mc_seed, init=c.init)
    p.set_tuning(64, 4, 2, True, 0)
    _say("anisotropic ramp: per-sublattice kernels")
    rp = p.run_schedule(steps)
    np.testing.assert_array_equal(rw, rp)
    np.testing.assert_array_equal(w.spins(), p.spins())
    M = rp[:, 0]
    assert M.min() < 0 < M[-1], "the loop must reverse"
    assert 0 < redone < runs < len(steps) + 1
    # the oracle on the two steps where M changes sign (the per-sublattice kernels'
    # phases read M from many blocks there), each from the GPU's spins at its start
    n = len(steps)
    down = int(np.argmax(M < 0))
    up = n // 2 + int(np.argmax(M[n // 2:] > 0))
    cpu.set_threads(_workers())
    for s in (down, up):
        q = isf.Lattice(h, c.Z, c.mc_seed, init=c.init)
        q.set_tuning(64, 4, 2, True, 0)
        q.run_schedule(steps[:s])
        start = q.spins()
        np.testing.assert_array_equal(q.run_schedule(steps[s:s + 1])[0], rp[s])
        _say("anisotropic ramp: oracle on step %d (M %d -> %d)" % (s, M[s - 1], M[s]))
        f = cpu.Film(h, c.Z, c.mc_seed, init=c.init)
        f.set_spins(start, s * c.sweeps_per_step)
        assert f.run(*steps[s]).as_tuple() == tuple(rp[s]), s
        np.testing.assert_array_equal(f.spins(), q.spins())
        del q


@pytest.mark.timeout(900)
def test_batched_all_replicas_prefix_and_whole_ramps(isf):
    import torch

    from isf_workloads import batched_films

    reps, seed, hnums, spst = batched_films()
    stream = torch.cuda.Stream()
    n_pre = 3
    lats = [isf.Lattice(r.heights(), r.Z, seed, replica=r.replica, init=0, stream=stream) for r in reps]
    b = isf.Batch(len(lats), stream=stream)
    _say("batched: %d replicas, %d-step prefix" % (len(reps), n_pre))
    pre = b.run(lats, [[(r.T, hv, spst, 0) for hv in hnums[:n_pre]] for r in reps], mode=3)
    pre_spins = [l.spins() for l in lats]
    del lats, b
    # the sublattice mode gives the same trajectories
    lats = [isf.Lattice(r.heights(), r.Z, seed, replica=r.replica, init=0, stream=stream) for r in reps]
    b = isf.Batch(len(lats), stream=stream)
    pre0 = b.run(lats, [[(r.T, hv, spst, 0) for hv in hnums[:n_pre]] for r in reps], mode=0)
    for i, l in enumerate(lats):
        np.testing.assert_array_equal(pre0[i], pre[i], err_msg="replica %d, modes 0 and 3" % reps[i].replica)
        np.testing.assert_array_equal(l.spins(), pre_spins[i], err_msg="replica %d, modes 0 and 3" % reps[i].replica)
    del lats, b

    def prefix(i):
        def run():
            r = reps[i]
            f = cpu.Film(r.heights(), r.Z, seed, r.replica, init=0)
            got = np.array([f.run(r.T, hv, spst, 0).as_tuple() for hv in hnums[:n_pre]])
            np.testing.assert_array_equal(got, pre[i], err_msg="replica %d" % r.replica)
            np.testing.assert_array_equal(f.spins(), pre_spins[i], err_msg="replica %d" % r.replica)
        return run

    _oracle_pool([prefix(i) for i in range(len(reps))])
    del pre_spins

    # whole ramps of three films inside a batch of all 256 replicas, in 16 chunks
    size = [reps[16 * f].X * reps[16 * f].Y * reps[16 * f].Z for f in range(16)]
    order = sorted(range(16), key=lambda f: size[f])
    temp_rank = sorted(range(16), key=lambda j: reps[j].T)
    picks = [16 * order[0] + temp_rank[-1], 16 * order[8] + temp_rank[8], 16 * order[-1] + temp_rank[0]]
    lats = [isf.Lattice(r.heights(), r.Z, seed, replica=r.replica, init=0, stream=stream) for r in reps]
    b = isf.Batch(len(lats), stream=stream)
    bounds = [int(v) for v in np.linspace(0, len(hnums), 17)]
    _say("batched: whole ramps of replicas %s in %d chunks" % (picks, len(bounds) - 1))
    snaps = {p: [lats[p].spins()] for p in picks}
    recs = {p: [] for p in picks}
    for a, e in zip(bounds[:-1], bounds[1:]):
        out = b.run(lats, [[(r.T, hv, spst, 0) for hv in hnums[a:e]] for r in reps], mode=3)
        for p in picks:
            recs[p].append(out[p])
            snaps[p].append(lats[p].spins())
    del lats, b

    def chunk(p, k):
        def run():
            r = reps[p]
            f = cpu.Film(r.heights(), r.Z, seed, r.replica, init=0)
            f.set_spins(snaps[p][k], bounds[k] * spst)
            got = np.array([f.run(r.T, hv, spst, 0).as_tuple() for hv in hnums[bounds[k]:bounds[k + 1]]])
            np.testing.assert_array_equal(got, recs[p][k], err_msg="replica %d chunk %d" % (r.replica, k))
            np.testing.assert_array_equal(f.spins(), snaps[p][k + 1], err_msg="replica %d chunk %d" % (r.replica, k))
        return run

    # the largest film's chunks first: they take longest
    _oracle_pool([chunk(p, k) for p in reversed(picks) for k in range(len(bounds) - 1)])


# ------------------------------------------------------------------ serving
def _serving_sample():
    """A stratified sample of the serving stream: per job kind the largest film, a
    ten-layer film near 1024^2, a one-layer film and the smallest film; plus ten
    requests spread over the arrivals as the rest of the mix."""
    from isf_workloads import serving_requests

    reqs = serving_requests()
    picked = {}
    for kind in ("hysteresis", "tscan"):
        rs = [q for q in reqs if q.kind == kind]
        picked[max(rs, key=lambda q: q.X * q.Y * q.Z).rid] = "largest " + kind
        ten = [q for q in rs if q.Z == 10]
        picked[min(ten, key=lambda q: abs(q.X - 1024)).rid] = "10 layers ~1024 " + kind
        one = [q for q in rs if q.Z == 1]
        picked[max(one, key=lambda q: q.X).rid] = "1 layer " + kind
        picked[min(rs, key=lambda q: q.X * q.Y * q.Z).rid] = "smallest " + kind
    for q in reqs[:: len(reqs) // 10]:
        picked.setdefault(q.rid, "mix")
    sample = [q for q in reqs if q.rid in picked]
    t0 = sample[0].arrival
    for q in sample:
        # shortened schedules, same structure: two field steps at the request's sweeps per
        # step, or two temperatures of 50 sweeps with 10 discarded; arrivals compressed 100x
        q.arrival = (q.arrival - t0) / 100.0
        if q.kind == "hysteresis":
            q.h_nums = q.h_nums[:2]
        else:
            q.temps = q.temps[:2]
            q.sweeps_per_T, q.discard_per_T = 50, 10
    return sample, picked


@pytest.mark.timeout(900)
def test_serving_stratified_sample_in_mix(isf):
    from paper_1205_5588_amd.serve import GpuExecutor, Job, Server, request_schedule

    sample, picked = _serving_sample()
    jobs = [Job(rid=q.rid, arrival=q.arrival, footprint=GpuExecutor.footprint(q), n_sweeps=q.n_sweeps, payload=q)
            for q in sample]
    _say("serving sample: %s" % [(q.rid, q.X, q.Z, q.kind, picked[q.rid]) for q in sample])
    hmap = {q.rid: q.heights() for q in sample}
    srv = Server(GpuExecutor(max_slots=64, mode=0, heights_of=lambda q: hmap[q.rid]), budget_bytes=8 * 2**30,
                 max_slots=64, target_chunk_s=0.005, rate_estimate=2e11, max_chunk=32)
    stats = srv.run(jobs)
    assert len(stats.results) == len(sample)
    assert stats.max_active > 1 and stats.chunks > 1
    res = {r.rid: r.records for r in stats.results}
    spins = {}
    for q in sample:
        alone = isf.Lattice(hmap[q.rid], q.Z, q.seed, replica=0, init=q.init)
        np.testing.assert_array_equal(alone.run_schedule(request_schedule(q)), res[q.rid],
                                      err_msg="request %d" % q.rid)
        spins[q.rid] = alone.spins()
        alone.close()
    _say("serving sample: alone == in mix for all %d" % len(sample))

    def check(q):
        def run():
            f = cpu.Film(hmap[q.rid], q.Z, q.seed, 0, init=q.init)
            got = np.array([f.run(*s).as_tuple() for s in request_schedule(q)])
            np.testing.assert_array_equal(got, res[q.rid], err_msg="request %d" % q.rid)
            np.testing.assert_array_equal(f.spins(), spins[q.rid], err_msg="request %d" % q.rid)
        return run

    def attempts(q):
        return q.X * q.Y * q.Z // 4 * q.n_sweeps

    ten = [q for q in sample if picked[q.rid].startswith("10 layers")]
    checked = [q for q in sample if attempts(q) <= 3e8] + [min(ten, key=attempts)]
    checked = list({q.rid: q for q in checked}.values())
    _say("serving sample: oracle on %s" % [q.rid for q in checked])
    _oracle_pool([check(q) for q in sorted(checked, key=attempts, reverse=True)])
