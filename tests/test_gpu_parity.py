"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Spins and every integer record field (M, E_bond, sums, accepted flips) must be
identical; derived per-spin values are compared at tolerance 0 by computing
them the same way on both sides.  Cases cover several tiles and ragged tails,
both storage formats, every launch shape, graph and plain launches, the
degenerate films (one layer, empty, full), and the full-size workloads on a
prefix of their schedules.
"""

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


def _pair(isf, h, Z, seed, replica=0, init=0, fmt=0, tuning=None):
    g = isf.Lattice(h, Z, seed, replica=replica, init=init, fmt=fmt)
    if tuning is not None:
        g.set_tuning(*tuning)
    o = cpu.Film(h, Z, seed, replica, init=init)
    return g, o


def _rand_h(shape, Z, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, Z + 1, size=shape).astype(np.uint8)


def _assert_same(g, o, what=""):
    np.testing.assert_array_equal(g.spins(), o.spins(), err_msg="spins " + what)
    ob = g.observables()
    st = o.state()
    assert (ob["M"], ob["E"], ob["n_occ"], ob["n_bonds"], ob["sweeps"]) == st, (what, ob, st)


@pytest.mark.parametrize("fmt,X", [(0, 72), (1, 128), (1, 72)])
@pytest.mark.parametrize("init", [0, 1, 2])
def test_start_state(isf, fmt, X, init):
    h = _rand_h((38, X), 5, 1 + init)
    g, o = _pair(isf, h, 5, 0xDEADBEEF12345, replica=7, init=init, fmt=fmt)
    _say("start", fmt, init)
    _assert_same(g, o, "start")


SHAPES = [(72, 38, 5), (64, 64, 3), (136, 20, 4), (8, 4, 1), (264, 10, 2)]


@pytest.mark.parametrize("X,Y,Z", SHAPES)
def test_small_films_schedule(isf, X, Y, Z):
    h = _rand_h((Y, X), Z, X + Y + Z)
    steps = [(2.5, 30, 3, 0), (0.8, -45, 4, 1), (9.0, 0, 2, 0), (4.0, -7, 5, 2), (1e-3, 241, 1, 0)]
    g, o = _pair(isf, h, Z, 987654321, replica=3, init=2)
    _say("schedule", X, Y, Z)
    rg = g.run_schedule(steps)
    ro = np.array([o.run(*s).as_tuple() for s in steps], dtype=np.int64)
    np.testing.assert_array_equal(rg, ro)
    _assert_same(g, o)


TILINGS = [(64, 4, 1), (64, 4, 2), (64, 4, 4), (32, 8, 1), (32, 8, 2), (32, 8, 4), (16, 16, 1), (16, 16, 2),
           (16, 16, 4)]


@pytest.mark.parametrize("tiling", TILINGS)
def test_every_tiling_same_trajectory(isf, tiling):
    X, Y, Z = 328, 46, 6   # 41 dwords per row, 23 active rows: ragged in both tile directions
    h = _rand_h((Y, X), Z, 5)
    g, o = _pair(isf, h, Z, 42, replica=1, init=2, tuning=tiling + (False,))
    _say("tiling", tiling)
    hs = [60, 20, -20, -60, 0, 40]
    np.testing.assert_array_equal(g.ramp_field(3.0, hs, 6), cpu.hysteresis(o, 3.0, hs, 6))
    _assert_same(g, o)


@pytest.mark.parametrize("tiling", [(64, 4, 1), (32, 8, 2), (16, 16, 1), (8, 32, 2)])
def test_bitpack_matches_oracle(isf, tiling):
    X, Y, Z = 192, 22, 7   # 3 words per row
    h = _rand_h((Y, X), Z, 11)
    g, o = _pair(isf, h, Z, 5555, replica=2, init=2, fmt=1, tuning=tiling + (False,))
    _say("bitpack", tiling)
    steps = [(2.0, 25, 4, 0), (6.0, -13, 3, 1), (0.5, 0, 3, 0)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)


# bit-packed rows that end in a partly filled word (W = X/2 sites, W mod 32 = r):
# the periodic seam takes its column from bit r - 1 of the last word
BP_PARTIAL = [(8, 4, 2), (72, 10, 3), (88, 26, 4), (120, 12, 5), (1000, 6, 2)]


@pytest.mark.parametrize("tiling", [(64, 4, 1), (32, 8, 2), (16, 16, 1), (8, 32, 1), (8, 16, 1), (8, 8, 1)])
@pytest.mark.parametrize("X,Y,Z", BP_PARTIAL)
def test_bitpack_partial_words_match_oracle_and_int8(isf, tiling, X, Y, Z):
    h = _rand_h((Y, X), Z, 3 * X + Y)
    g, o = _pair(isf, h, Z, 8642, replica=5, init=2, fmt=1, tuning=tiling + (X % 16 == 8,))
    _say("bitpack partial words", X, Y, Z, tiling)
    steps = [(2.0, 25, 5, 0), (6.0, -13, 3, 1), (3.0, 30, 4, 0, 40), (0.5, 0, 3, 0)]
    rg = g.run_schedule(steps)
    np.testing.assert_array_equal(rg, np.array([o.run(*st).as_tuple() for st in steps]))
    _assert_same(g, o)
    i8 = isf.Lattice(h, Z, 8642, replica=5, init=2)
    np.testing.assert_array_equal(i8.run_schedule(steps), rg)
    np.testing.assert_array_equal(i8.spins(), g.spins())
    # a state written back and read again, then more sweeps from it
    cube = g.spins()
    cube[:, 0, :] = np.where(cube[:, 0, :] != 0, -cube[:, 0, :], 0)
    g.set_spins(cube, 100)
    o.set_spins(cube, 100)
    _assert_same(g, o, "written")
    np.testing.assert_array_equal(g.run_sweeps(4.0, -20, 3), o.run(4.0, -20, 3).as_tuple())
    _assert_same(g, o, "after writing")


def test_graph_replay_matches_plain(isf):
    X, Y, Z = 256, 64, 4
    h = _rand_h((Y, X), Z, 21)
    a = isf.Lattice(h, Z, 77, init=0)
    b = isf.Lattice(h, Z, 77, init=0)
    a.set_tuning(64, 4, 2, True)
    b.set_tuning(64, 4, 2, False)
    _say("graph")
    steps = [(3.5, 40, 150, 10), (3.5, -40, 130, 0), (2.0, 0, 64, 0)]
    ra = a.run_schedule(steps)
    rb = b.run_schedule(steps)
    np.testing.assert_array_equal(ra, rb)
    np.testing.assert_array_equal(a.spins(), b.spins())
    o = cpu.Film(h, Z, 77)
    np.testing.assert_array_equal(ra, np.array([o.run(*s).as_tuple() for s in steps]))


def test_degenerate_films(isf):
    _say("degenerate")
    # empty film: nothing occupied
    h = np.zeros((8, 16), dtype=np.uint8)
    g, o = _pair(isf, h, 3, 1, init=2)
    np.testing.assert_array_equal(g.run_sweeps(2.0, 10, 5), o.run(2.0, 10, 5).as_tuple())
    assert g.observables()["n_occ"] == 0
    # full film
    h = np.full((16, 32), 4, dtype=np.uint8)
    g, o = _pair(isf, h, 4, 2, init=1)
    np.testing.assert_array_equal(g.run_sweeps(7.0, -3, 9, 2), o.run(7.0, -3, 9, 2).as_tuple())
    _assert_same(g, o)
    # one layer (sublattices 2, 3 empty), square lattice
    h = np.ones((32, 64), dtype=np.uint8)
    g, o = _pair(isf, h, 1, 3, init=2)
    np.testing.assert_array_equal(g.run_sweeps(2.2, 0, 20), o.run(2.2, 0, 20).as_tuple())
    _assert_same(g, o)
    # zero sweeps
    r = g.run_sweeps(2.2, 0, 0)
    assert r[0] == g.observables()["M"] and r[2] == 0


def test_extreme_parameters(isf):
    h = _rand_h((20, 40), 3, 9)
    g, o = _pair(isf, h, 3, 123, init=2)
    _say("extreme")
    steps = [(1e-3, 1, 3, 0), (1e6, 0, 3, 0), (1e-3, -241, 2, 0), (1.0, 200000, 1, 0), (1.0, -200000, 1, 0),
             (0.31, 17, 3, 3)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)


def test_invalid_arguments_raise(isf):
    from paper_1205_5588_amd import IsfError

    h = _rand_h((8, 16), 2, 3)
    g = isf.Lattice(h, 2, 1)
    for bad in [(0.0, 0, 1, 0), (float("nan"), 0, 1, 0), (1.0, 300000, 1, 0), (1.0, 0, 0, 0), (1.0, 0, 2, 3)]:
        with pytest.raises(IsfError):
            g.run_schedule([bad])
    with pytest.raises(IsfError):
        isf.Lattice(np.full((8, 16), 3, dtype=np.uint8), 2, 1)   # h > Z
    with pytest.raises(IsfError):
        isf.Lattice(np.ones((8, 12), dtype=np.uint8), 2, 1)      # X % 8 != 0
    with pytest.raises(IsfError):
        g.set_tuning(128, 2, 1, False)
    with pytest.raises(IsfError):
        g.set_tuning(64, 4, 1, False, 1)      # list kernel before lists are attached
    with pytest.raises(IsfError):
        g.set_spins(np.full((2, 8, 16), 5, dtype=np.int8), 0)


def test_incremental_equals_recount_and_resume(isf):
    X, Y, Z = 96, 48, 5
    h = _rand_h((Y, X), Z, 33)
    g = isf.Lattice(h, Z, 999, replica=4, init=2)
    _say("recount/resume")
    for hn in (50, -10, -50, 20):
        g.run_sweeps(3.0, hn, 7)
        ob = g.observables()
        assert g.recount() == (ob["M"], ob["E"])
    # checkpoint, restore into a new handle, continue == uninterrupted
    snap, t = g.spins(), g.observables()["sweeps"]
    r1 = g.run_schedule([(2.5, -30, 11, 0), (2.5, 30, 5, 1)])
    g2 = isf.Lattice(h, Z, 999, replica=4, init=0)
    g2.set_spins(snap, t)
    r2 = g2.run_schedule([(2.5, -30, 11, 0), (2.5, 30, 5, 1)])
    np.testing.assert_array_equal(r1, r2)
    np.testing.assert_array_equal(g.spins(), g2.spins())


def test_field_reversal_symmetry_gpu(isf):
    h = _rand_h((24, 64), 4, 44)
    a = isf.Lattice(h, 4, 31337, init=2)
    b = isf.Lattice(h, 4, 31337, init=0)
    b.set_spins(-a.spins(), 0)
    _say("symmetry")
    hs = [40, 10, -20, -60, 0, 33, -1]
    ra = a.ramp_field(2.5, hs, 3)
    rb = b.ramp_field(2.5, [-v for v in hs], 3)
    np.testing.assert_array_equal(b.spins(), -a.spins())
    np.testing.assert_array_equal(rb[:, [0, 2]], -ra[:, [0, 2]])
    np.testing.assert_array_equal(rb[:, [1, 3, 4, 5]], ra[:, [1, 3, 4, 5]])


# ------------------------------------------------------------------ full-size workloads
@pytest.mark.parametrize("tuning", [None, (512, 1, 1, False, 4)])
def test_config_plain_hysteresis_small_full(isf, tuning):
    """The whole 64 x 64 x 3 ramp (161 steps of 100 sweeps) on the default sublattice
    kernels and on the film kernel (its default and the tuner's pick)."""
    from isf_workloads import config_plain_hysteresis_small

    c = config_plain_hysteresis_small()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=c.init, tuning=tuning)
    _say("small ramp, whole", tuning)
    rg = g.ramp_field(c.T, c.h_nums, c.sweeps_per_step)
    ro = cpu.hysteresis(o, c.T, c.h_nums, c.sweeps_per_step)
    np.testing.assert_array_equal(rg, ro)
    _assert_same(g, o)
    # derived per-spin magnetisation, same arithmetic on both sides: tolerance 0
    n = g.observables()["n_occ"]
    assert [float(r[0]) / float(n) for r in rg] == [float(r[0]) / float(n) for r in ro]


def test_config_plain_tscan_prefix(isf):
    from isf_workloads import config_plain_tscan

    c = config_plain_tscan()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=c.init)
    _say("c2 first temperatures, full film")
    temps = c.temps[:2]
    sw, dc = 250, 50
    rg = g.temperature_scan(temps, sw, dc)
    ro = cpu.tscan(o, temps, sw, dc)
    np.testing.assert_array_equal(rg, ro)
    _assert_same(g, o)
    n = g.observables()["n_occ"]
    kept = sw - dc
    assert [float(r[3]) / (float(kept) * float(n)) for r in rg] == [float(r[3]) / (float(kept) * float(n)) for r in ro]


@pytest.mark.parametrize("fmt", [0, 1])
def test_config_plain_hysteresis_large_prefix(isf, fmt):
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=c.init, fmt=fmt)
    _say("c3 prefix fmt", fmt)
    hs = c.h_nums[:1]
    rg = g.ramp_field(c.T, hs, 12)
    ro = cpu.hysteresis(o, c.T, hs, 12)
    np.testing.assert_array_equal(rg, ro)
    _assert_same(g, o)


# ------------------------------------------------------------------ batches
def _batch_films(isf, fmt=0):
    rng = np.random.default_rng(77)
    films = []
    for i, (X, Y, Z) in enumerate([(64, 40, 3), (192, 64, 5), (128, 16, 2), (320, 24, 6), (64, 64, 1)]):
        h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
        T = float(rng.uniform(1.0, 9.0))
        n_steps = 3 + i
        hs = [int(v) for v in rng.integers(-60, 61, size=n_steps)]
        sched = [(T, hv, int(rng.integers(2, 7)), 0) for hv in hs]
        films.append((h, Z, 1000 + i, i, sched))
    return films


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("fmt", [0, 1])
def test_batched_equals_alone_and_oracle(isf, mode, fmt):
    if mode == 2 and fmt == 1:
        pytest.skip("whole-sweep batches take INT8 films (rejection tested separately)")
    films = _batch_films(isf)
    if fmt == 1:  # 8 columns narrower: bit-packed rows that end in a partly filled word
        films = [(h[:, : h.shape[1] - 8], Z, s, r, sc) for (h, Z, s, r, sc) in films]
    _say("batch mode", mode, "fmt", fmt)
    lats = [isf.Lattice(h, Z, s, replica=r, init=2, fmt=fmt) for (h, Z, s, r, sc) in films]
    b = isf.Batch(len(lats))
    recs = b.run(lats, [f[4] for f in films], mode=mode)
    for (h, Z, s, r, sc), lat, rec in zip(films, lats, recs):
        o = cpu.Film(h, Z, s, r, init=2)
        np.testing.assert_array_equal(rec, np.array([o.run(*st).as_tuple() for st in sc]))
        np.testing.assert_array_equal(lat.spins(), o.spins())


@pytest.mark.parametrize("mode", [0, 2])
def test_batched_incremental_chunks(isf, mode):
    films = _batch_films(isf)
    lats = [isf.Lattice(h, Z, s, replica=r, init=2) for (h, Z, s, r, sc) in films]
    _say("batch chunks", mode)
    for lat, f in zip(lats, films):
        lat.schedule_load(f[4])
    b = isf.Batch(len(lats))
    k = 0
    while any(l.remaining() for l in lats):
        # odd chunk lengths, and a film read between chunks, close and reopen whole-sweep runs
        b.advance(lats, 3 if k % 2 == 0 else 2, mode=mode)
        b.sync()
        if k == 1:
            lats[1].observables()
        k += 1
    b.sync()
    for (h, Z, s, r, sc), lat in zip(films, lats):
        o = cpu.Film(h, Z, s, r, init=2)
        np.testing.assert_array_equal(lat.records(), np.array([o.run(*st).as_tuple() for st in sc]))


# ------------------------------------------------------------------ occupied-dword list kernel
@pytest.mark.parametrize("X,Y,Z", [(72, 38, 5), (8, 4, 1), (264, 10, 2), (328, 46, 6)])
@pytest.mark.parametrize("ipt", [1, 2])
def test_list_kernel_matches_oracle(isf, X, Y, Z, ipt):
    h = _rand_h((Y, X), Z, 7 * X + Y + Z)
    g, o = _pair(isf, h, Z, 24680, replica=6, init=2)
    g.attach_items()
    g.set_tuning(64, 4, ipt, ipt == 1, 1)
    assert g.get_tuning()[4] == 1
    _say("list kernel", X, Y, Z, ipt)
    steps = [(2.5, 30, 70, 0), (0.8, -45, 4, 1), (9.0, 0, 66, 6), (4.0, -7, 5, 2), (1e-3, 241, 1, 0)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)


def test_list_kernel_empty_and_full_films(isf):
    _say("list kernel degenerate")
    for h, Z in ((np.zeros((8, 16), dtype=np.uint8), 3), (np.full((16, 32), 4, dtype=np.uint8), 4),
                 (np.ones((32, 64), dtype=np.uint8), 1)):
        g, o = _pair(isf, h, Z, 5, init=2)
        g.attach_items()
        np.testing.assert_array_equal(g.run_sweeps(2.2, 10, 9, 3), o.run(2.2, 10, 9, 3).as_tuple())
        _assert_same(g, o)


def test_list_kernel_large_prefix(isf):
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=c.init)
    g.attach_items()
    _say("list kernel, large film prefix")
    hs = c.h_nums[:1]
    np.testing.assert_array_equal(g.ramp_field(c.T, hs, 12), cpu.hysteresis(o, c.T, hs, 12))
    _assert_same(g, o)


# ------------------------------------------------------------------ whole-sweep kernel (tile + halo in LDS)
SWEEP_SHAPES = [(72, 38, 5), (8, 4, 1), (264, 10, 2), (328, 46, 6), (520, 70, 9), (40, 6, 4)]
SWEEP_TILINGS = [(32, 16, 4), (16, 16, 8), (64, 8, 4), (32, 32, 16), (32, 8, 4), (64, 16, 4)]


@pytest.mark.parametrize("X,Y,Z", SWEEP_SHAPES)
@pytest.mark.parametrize("tiling", SWEEP_TILINGS)
def test_sweep_kernel_matches_oracle(isf, X, Y, Z, tiling):
    h = _rand_h((Y, X), Z, 5 * X + 3 * Y + Z)
    g, o = _pair(isf, h, Z, 13579, replica=4, init=2)
    g.set_tuning(tiling[0], tiling[1], tiling[2], (X + Y) % 2 == 0, 2)
    assert g.get_tuning()[4] == 2
    _say("sweep kernel", X, Y, Z, tiling)
    steps = [(2.5, 30, 66, 0), (0.8, -45, 4, 1), (9.0, 0, 3, 1), (4.0, -7, 5, 2), (1e-3, 241, 1, 0)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)


def test_sweep_kernel_degenerate_films(isf):
    _say("sweep kernel degenerate")
    for h, Z in ((np.zeros((8, 16), dtype=np.uint8), 3), (np.full((16, 32), 4, dtype=np.uint8), 4),
                 (np.ones((32, 64), dtype=np.uint8), 1), (np.full((4, 8), 2, dtype=np.uint8), 2)):
        g, o = _pair(isf, h, Z, 5, init=2)
        g.set_tuning(32, 16, 4, False, 2)
        np.testing.assert_array_equal(g.run_sweeps(2.2, 10, 9, 3), o.run(2.2, 10, 9, 3).as_tuple())
        _assert_same(g, o)


def test_sweep_kernel_rejects_unsupported(isf):
    from paper_1205_5588_amd._lib import IsfError

    h = _rand_h((16, 128), 4, 1)
    g = isf.Lattice(h, 4, 1, fmt=1)
    with pytest.raises(IsfError):
        g.set_tuning(32, 16, 4, False, 2)  # bit-packed film
    g = isf.Lattice(h, 4, 1)
    for bad in ((32, 12, 4), (48, 16, 4), (32, 16, 2), (32, 16, 32)):
        with pytest.raises(IsfError):
            g.set_tuning(bad[0], bad[1], bad[2], False, 2)
    tall = isf.Lattice(np.full((16, 512), 64, dtype=np.uint8), 64, 1)
    with pytest.raises(IsfError):
        tall.set_tuning(64, 16, 4, False, 2)  # LDS of a 64-plane region exceeds the block limit
    assert g.get_tuning()[4] == 0  # rejected shapes leave the previous tuning


@pytest.mark.parametrize("fmt,kernel,tiling", [(0, 0, (64, 4, 2)), (0, 0, (16, 16, 1)),
                                               (1, 0, (64, 4, 1)), (1, 0, (16, 16, 2))])
def test_max_depth_film_matches_oracle(isf, fmt, kernel, tiling):
    """Films of the deepest allowed stack, Z = 64 layers (and a column height of 64 in
    places), on the kernels that take them, against the oracle.  The whole-sweep
    kernels hold the tile's whole column in LDS and refuse such films (even the
    16 x 16 tile needs about 178 KiB at Z = 64)."""
    from paper_1205_5588_amd._lib import IsfError

    X, Y, Z = 64, 16, 64
    h = _rand_h((Y, X), Z, 64)
    h[0, :] = Z
    g, o = _pair(isf, h, Z, 6464, replica=3, init=2, fmt=fmt)
    if fmt == 0:
        for shape in ((16, 16, 4, 2), (32, 8, 4, 2), (32, 16, 8, 3)):
            with pytest.raises(IsfError):
                g.set_tuning(shape[0], shape[1], shape[2], True, shape[3])
    g.set_tuning(tiling[0], tiling[1], tiling[2], True, kernel)
    _say("max depth film", fmt, kernel, tiling)
    steps = [(3.0, 20, 6, 1), (8.0, -30, 5, 0, 40), (1e-3, 0, 2, 0)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*st).as_tuple() for st in steps]))
    _assert_same(g, o)


def test_sweep_kernel_large_prefix(isf):
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=c.init)
    g.set_tuning(32, 16, 4, True, 2)
    _say("sweep kernel, large film prefix")
    hs = c.h_nums[:1]
    np.testing.assert_array_equal(g.ramp_field(c.T, hs, 12), cpu.hysteresis(o, c.T, hs, 12))
    _assert_same(g, o)


def test_sweep_kernel_equals_tiles_tscan_film(isf):
    """Random start, high temperature (many flips) on the 512 x 512 x 5 film: sweep kernel == tile kernel."""
    from isf_workloads import config_plain_tscan

    c = config_plain_tscan()
    h = c.heights()
    a = isf.Lattice(h, c.Z, c.mc_seed, init=c.init)
    b = isf.Lattice(h, c.Z, c.mc_seed, init=c.init)
    b.set_tuning(16, 16, 8, True, 2)
    _say("sweep kernel vs tiles, tscan film")
    steps = [(12.0, 0, 40, 10), (5.0, 0, 30, 0), (3.0, 15, 70, 20)]
    np.testing.assert_array_equal(a.run_schedule(steps), b.run_schedule(steps))
    np.testing.assert_array_equal(a.spins(), b.spins())
    # timed launches follow the same trajectory
    for lat in (a, b):
        lat.schedule_load([(2.0, -20, 6, 0)])
    a.advance(6)
    ms, n = b.time_launches(6)
    assert n == 6 and ms[0] > 0.0
    np.testing.assert_array_equal(a.records(), b.records())
    np.testing.assert_array_equal(a.spins(), b.spins())


def test_sweep_kernel_switches_and_reads_midway(isf):
    """Whole-sweep runs opened and closed at odd places: chunked advances, kernel
    switches inside a step, observables and spins read between chunks."""
    h = _rand_h((46, 328), 6, 99)
    steps = [(2.5, 30, 7, 2), (0.8, -45, 5, 1), (6.0, 5, 9, 3)]
    g, o = _pair(isf, h, 6, 4242, replica=2, init=2)
    g.set_tuning(32, 16, 8, False, 2)
    g.schedule_load(steps)
    _say("sweep kernel switching")
    done = 0
    for chunk, kernel in ((3, 2), (1, 2), (4, 0), (2, 2), (5, 2), (3, 0), (1, 2), (2, 2)):
        if kernel == 2:
            g.set_tuning(32, 16, 8, False, 2)
        else:
            g.set_tuning(64, 4, 2, False, 0)
        done += g.advance(chunk)
        assert g.observables()["sweeps"] == done
        if chunk == 4:
            g.spins()  # brings the spins back from the spare copy mid-run
    g.advance(100)
    ro = np.array([o.run(*s).as_tuple() for s in steps])
    np.testing.assert_array_equal(g.records(), ro)
    _assert_same(g, o)


# ------------------------------------------------------------------ pipelined whole-sweep kernel
# (film, shape): rows of whole 16-byte pieces (X a multiple of 32), at least one
# region (tile + 4 dwords / 4 rows a side) wide and high; ragged tiles in x and y;
# each shape at the deepest film its two LDS buffers hold (32 x 16: Z = 14,
# 32 x 32: Z = 8, 64 x 16: Z = 7), one of them on rows that are not whole pieces
PIPE_CASES = [((320, 24, 5), (32, 16, 16)), ((352, 42, 6), (32, 16, 8)), ((576, 40, 9), (32, 16, 16)),
              ((384, 64, 1), (32, 32, 16)), ((352, 72, 8), (32, 32, 8)), ((640, 50, 3), (64, 16, 16)),
              ((1280, 960, 3), (32, 16, 16)), ((320, 32, 14), (32, 16, 16)), ((328, 30, 14), (32, 16, 8)),
              ((576, 24, 7), (64, 16, 16)), ((320, 16, 5), (32, 8, 8)), ((344, 22, 9), (32, 8, 16))]


@pytest.mark.parametrize("film,tiling", PIPE_CASES)
def test_pipe_kernel_matches_oracle(isf, film, tiling):
    X, Y, Z = film
    h = _rand_h((Y, X), Z, 7 * X + 5 * Y + Z)
    g, o = _pair(isf, h, Z, 24680, replica=3, init=2)
    g.set_tuning(tiling[0], tiling[1], tiling[2], (X + Y) % 2 == 0, 3)
    assert g.get_tuning()[4] == 3
    _say("pipe kernel", X, Y, Z, tiling)
    steps = [(2.5, 30, 66, 0), (0.8, -45, 4, 1), (9.0, 0, 3, 1), (4.0, -7, 5, 2), (1e-3, 241, 1, 0)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)


# ------------------------------------------------------------------ the film kernel (one block, whole film in LDS)
# sublattices of at most 512 dwords (one per thread: 64 x 64 x 3, 8 x 4 x 1, 136 x 20 x 4, ...) and
# of more (the listed form: 72 x 38 x 5 with 513, 256 x 128 x 4, 40 x 70 x 13)
FILM_CASES = [(64, 64, 3), (8, 4, 1), (72, 38, 5), (136, 20, 4), (264, 10, 2), (24, 6, 9), (512, 12, 1),
              (256, 128, 4), (40, 70, 13), (64, 62, 3)]


@pytest.mark.parametrize("X,Y,Z", FILM_CASES)
def test_film_kernel_matches_oracle(isf, X, Y, Z):
    """Many sweeps per launch from LDS, the books kept in the kernel: records of every step
    (discards, a step of one sweep, a frozen one) and the spins equal the oracle's."""
    h = _rand_h((Y, X), Z, 3 * X + Y + 13 * Z)
    g, o = _pair(isf, h, Z, 0x5EED0F11, replica=5, init=2)
    g.set_tuning(512, 1, 1, True, 4)
    assert g.get_tuning()[4] == 4
    _say("film kernel", X, Y, Z)
    steps = [(2.5, 30, 66, 0), (0.8, -45, 4, 1), (9.0, 0, 3, 1), (4.0, -7, 5, 2), (1e-3, 241, 1, 0)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)


@pytest.mark.parametrize("X,Y,Z", [(64, 64, 3), (72, 38, 5)])
def test_film_kernel_across_launch_chunks(isf, X, Y, Z):
    """A step longer than one launch's sweeps (4096) and a schedule advanced in pieces that
    end inside steps: the state carried from launch to launch through memory (both forms:
    one dword of each sublattice per thread, and the lists of a sublattice of 513 dwords)."""
    h = _rand_h((Y, X), Z, 99)
    g, o = _pair(isf, h, Z, 4242, replica=1, init=0)
    g.set_tuning(512, 1, 1, False, 4)
    _say("film kernel, long step")
    steps = [(3.5, 20, 4100, 100), (4.5, -20, 5000, 4097), (2.0, 0, 7, 0)]
    np.testing.assert_array_equal(g.run_schedule(steps[:2]), np.array([o.run(*s).as_tuple() for s in steps[:2]]))
    _assert_same(g, o, "long steps")
    g2, o2 = _pair(isf, h, Z, 4242, replica=1, init=0)
    g2.set_tuning(512, 1, 1, False, 4)
    g2.schedule_load(steps)
    done = 0
    while g2.remaining():
        done += g2.advance(1013)
    assert done == sum(s[2] for s in steps)
    np.testing.assert_array_equal(g2.records(), np.array([o2.run(*s).as_tuple() for s in steps]))
    _assert_same(g2, o2, "advanced in pieces")


def test_film_kernel_degenerate_films(isf):
    _say("film kernel degenerate")
    for h, Z in ((np.zeros((24, 64), dtype=np.uint8), 3), (np.full((24, 64), 4, dtype=np.uint8), 4),
                 (np.ones((40, 32), dtype=np.uint8), 1)):
        g, o = _pair(isf, h, Z, 5, init=2)
        g.set_tuning(512, 1, 1, False, 4)
        np.testing.assert_array_equal(g.run_sweeps(2.2, 10, 9, 3), o.run(2.2, 10, 9, 3).as_tuple())
        _assert_same(g, o)


def test_film_kernel_refusals(isf):
    """Shapes and films the film kernel does not take are refused, and a refused tuning
    leaves the film's own tuning in place."""
    from paper_1205_5588_amd._lib import IsfError

    _say("film kernel refusals")
    g = isf.Lattice(_rand_h((128, 256), 5, 1), 5, 1)  # (Z + 2) Y X / 8 dwords and lists above the LDS
    before = g.get_tuning()
    with pytest.raises(IsfError):
        g.set_tuning(512, 1, 1, True, 4)
    assert g.get_tuning() == before
    big = isf.Lattice(_rand_h((256, 2048), 1, 1), 1, 1)  # 196608 dwords: beyond 16-bit indices
    with pytest.raises(IsfError):
        big.set_tuning(512, 1, 1, True, 4)
    small = isf.Lattice(_rand_h((16, 64), 2, 1), 2, 1)
    for bad in ((256, 1, 1), (512, 2, 1), (512, 1, 2)):
        with pytest.raises(IsfError):
            small.set_tuning(bad[0], bad[1], bad[2], True, 4)
    bp = isf.Lattice(_rand_h((16, 64), 2, 1), 2, 1, fmt=1)
    with pytest.raises(IsfError):
        bp.set_tuning(512, 1, 1, True, 4)
    small.set_tuning(512, 1, 1, True, 4)
    with pytest.raises(IsfError):  # the anisotropy term
        small.schedule_load([(2.0, 0, 3, 0, 0, 40)])
    small.schedule_load([(2.0, 0, 3, 0)])
    with pytest.raises(IsfError):  # many sweeps per launch: no per-launch timing
        small.time_launches(3)
    small.set_tuning(64, 4, 2, True, 0)
    small.schedule_load([(2.0, 0, 3, 0, 0, 40)])
    with pytest.raises(IsfError):
        small.set_tuning(512, 1, 1, True, 4)
    for lat in (g, big, small, bp):
        lat.close()


def test_pipe_kernel_more_tiles_than_blocks_hold(isf):
    """A film with more tiles than the blocks of one per compute unit may take
    (32 x 16 tiles, 9600 of them): the grid grows instead."""
    h = _rand_h((4800, 8192), 1, 77)
    g, o = _pair(isf, h, 1, 1234, init=2)
    g.set_tuning(32, 16, 16, False, 3)
    _say("pipe kernel, 8192 x 4800 x 1")
    np.testing.assert_array_equal(g.run_sweeps(1.5, -10, 3), o.run(1.5, -10, 3).as_tuple())
    _assert_same(g, o)


def test_pipe_kernel_degenerate_films(isf):
    _say("pipe kernel degenerate")
    for h, Z in ((np.zeros((24, 320), dtype=np.uint8), 3), (np.full((24, 320), 4, dtype=np.uint8), 4),
                 (np.ones((40, 384), dtype=np.uint8), 1)):
        g, o = _pair(isf, h, Z, 5, init=2)
        g.set_tuning(32, 16, 16, False, 3)
        np.testing.assert_array_equal(g.run_sweeps(2.2, 10, 9, 3), o.run(2.2, 10, 9, 3).as_tuple())
        _assert_same(g, o)


def test_pipe_kernel_rejects_unsupported(isf):
    from paper_1205_5588_amd._lib import IsfError

    h = _rand_h((64, 512), 4, 1)
    with pytest.raises(IsfError):
        isf.Lattice(h, 4, 1, fmt=1).set_tuning(32, 16, 16, False, 3)  # bit-packed film
    g = isf.Lattice(h, 4, 1)
    for bad in ((32, 8, 4), (16, 16, 16), (32, 16, 4), (32, 16, 32), (64, 8, 16)):
        with pytest.raises(IsfError):
            g.set_tuning(bad[0], bad[1], bad[2], False, 3)
    for hh, Z in ((_rand_h((64, 256), 4, 3), 4),  # narrower than one 32 x 16 region (40 dwords)
                  (_rand_h((16, 512), 4, 4), 4),  # lower than one region (24 rows)
                  (np.full((32, 512), 64, dtype=np.uint8), 64)):  # LDS of a 64-plane double buffer
        with pytest.raises(IsfError):
            isf.Lattice(hh, Z, 1).set_tuning(32, 16, 16, False, 3)
    with pytest.raises(IsfError):
        isf.Lattice(_rand_h((64, 512), 9, 5), 9, 1).set_tuning(32, 32, 16, False, 3)  # 32 x 32 at Z = 9
    with pytest.raises(IsfError):
        isf.Lattice(_rand_h((32, 320), 15, 6), 15, 1).set_tuning(32, 16, 16, False, 3)  # 32 x 16 at Z = 15
    with pytest.raises(IsfError):
        isf.Lattice(_rand_h((24, 576), 8, 7), 8, 1).set_tuning(64, 16, 16, False, 3)  # 64 x 16 at Z = 8
    assert g.get_tuning()[4] == 0  # rejected shapes leave the previous tuning


@pytest.mark.parametrize("tiling", [(32, 32, 16), (32, 16, 16)])
def test_pipe_kernel_large_prefix(isf, tiling):
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=c.init)
    g.set_tuning(tiling[0], tiling[1], tiling[2], True, 3)
    _say("pipe kernel, large film prefix", tiling)
    hs = c.h_nums[:1]
    np.testing.assert_array_equal(g.ramp_field(c.T, hs, 12), cpu.hysteresis(o, c.T, hs, 12))
    _assert_same(g, o)


def test_pipe_kernel_large_film_reversal(isf):
    """The bench's film and launch shape in the reversal regime: all spins up in a reversed
    field, so most tiles flip more dwords per sweep than their change lists hold and are
    written whole; then back to a saturating field, where the lists hold them again."""
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=0)
    g.set_tuning(32, 32, 16, True, 3)
    _say("pipe kernel, large film reversal")
    steps = [(c.T, -40, 3, 0), (c.T, -20, 2, 1), (c.T, 120, 3, 0)]
    rg = g.run_schedule(steps)
    np.testing.assert_array_equal(rg, np.array([o.run(*st).as_tuple() for st in steps]))
    _assert_same(g, o)
    assert rg[0][5] > 0.01 * 3 * o.state()[2]  # heavy flipping in the reversed field


def test_pipe_kernel_equals_sweep_kernel_tscan_film(isf):
    """Random start, high temperature on the 512 x 512 x 5 film: pipelined == single-tile whole sweep,
    through graphs of 64 sweeps and timed launches."""
    from isf_workloads import config_plain_tscan

    c = config_plain_tscan()
    h = c.heights()
    a = isf.Lattice(h, c.Z, c.mc_seed, init=c.init)
    b = isf.Lattice(h, c.Z, c.mc_seed, init=c.init)
    a.set_tuning(16, 16, 8, True, 2)
    b.set_tuning(32, 16, 16, True, 3)
    _say("pipe kernel vs sweep kernel, tscan film")
    steps = [(12.0, 0, 140, 10), (5.0, 0, 30, 0), (3.0, 15, 70, 20)]
    np.testing.assert_array_equal(a.run_schedule(steps), b.run_schedule(steps))
    np.testing.assert_array_equal(a.spins(), b.spins())
    for lat in (a, b):
        lat.schedule_load([(2.0, -20, 6, 0)])
    a.advance(6)
    ms, n = b.time_launches(6)
    assert n == 6 and ms[0] > 0.0
    np.testing.assert_array_equal(a.records(), b.records())
    np.testing.assert_array_equal(a.spins(), b.spins())


def test_pipe_kernel_switches_and_reads_midway(isf):
    """Runs of the pipelined kernel opened and closed at odd places, switching with the
    single-tile whole sweep (other lists) and the sublattice tiles inside steps."""
    h = _rand_h((46, 352), 6, 98)
    steps = [(2.5, 30, 7, 2), (0.8, -45, 5, 1, 40), (6.0, 5, 9, 3)]
    g, o = _pair(isf, h, 6, 4243, replica=5, init=2)
    g.schedule_load(steps)
    _say("pipe kernel switching")
    done = 0
    for chunk, kernel in ((3, 3), (1, 3), (4, 2), (2, 3), (5, 0), (3, 3), (1, 2), (2, 3)):
        if kernel == 3:
            g.set_tuning(32, 16, 16, False, 3)
        elif kernel == 2:
            g.set_tuning(32, 16, 8, False, 2)
        else:
            g.set_tuning(64, 4, 2, False, 0)
        done += g.advance(chunk)
        assert g.observables()["sweeps"] == done
        if chunk == 4:
            g.spins()
    g.advance(100)
    ro = np.array([o.run(*s).as_tuple() for s in steps])
    np.testing.assert_array_equal(g.records(), ro)
    _assert_same(g, o)


def test_batched_whole_mode_rejects_bitpack(isf):
    from paper_1205_5588_amd._lib import IsfError

    h = _rand_h((16, 128), 3, 5)
    lats = [isf.Lattice(h, 3, 1, fmt=1)]
    lats[0].schedule_load([(2.0, 0, 2, 0)])
    with pytest.raises(IsfError):
        isf.Batch(1).advance(lats, 2, mode=2)


# ------------------------------------------------------------------ switching-field gate (Eq. 9)
GATED_STEPS = [(2.5, 30, 7, 0, 40), (0.8, -45, 4, 1, 160), (9.0, 0, 5, 2, -20), (3.0, -7, 6, 0, 0),
               (1e-3, 241, 2, 0, 20), (1.5, 60, 66, 3, 7)]


@pytest.mark.parametrize("kernel,tiling", [(0, (64, 4, 2)), (0, (16, 16, 1)), (1, (64, 4, 1)), (2, (32, 16, 8)),
                                           (2, (16, 16, 4)), (3, (32, 16, 16)), (4, (512, 1, 1))])
@pytest.mark.parametrize("X,Y,Z", [(72, 38, 5), (328, 46, 6), (8, 4, 1), (352, 46, 6)])
def test_gated_schedule_matches_oracle(isf, kernel, tiling, X, Y, Z):
    if kernel == 3 and (X // 8 < tiling[0] + 8 or Y < tiling[1] + 8):
        pytest.skip("film outside the pipelined kernel's shapes")
    h = _rand_h((Y, X), Z, 11 * X + Y + Z)
    g, o = _pair(isf, h, Z, 97531, replica=8, init=2)
    if kernel == 1:
        g.attach_items()
    g.set_tuning(tiling[0], tiling[1], tiling[2], X % 2 == 0, kernel)
    _say("gated schedule", kernel, tiling, X, Y, Z)
    np.testing.assert_array_equal(g.run_schedule(GATED_STEPS), np.array([o.run(*s).as_tuple() for s in GATED_STEPS]))
    _assert_same(g, o)


def test_gated_large_film_prefix(isf):
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=c.init)
    g.set_tuning(32, 32, 16, True, 3)
    _say("gated large film prefix")
    steps = [(c.T, hn, 5, 0, 40) for hn in (120, 60, 0, -60)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)


@pytest.mark.parametrize("mode", [0, 2])
def test_gated_batch_equals_oracle(isf, mode):
    films = _batch_films(isf)
    films = [(h, Z, s, r, [st + ((40 * (i + 1)) % 170,) for st in sc])
             for i, (h, Z, s, r, sc) in enumerate(films)]
    lats = [isf.Lattice(h, Z, s, replica=r, init=2) for (h, Z, s, r, sc) in films]
    _say("gated batch", mode)
    recs = isf.Batch(len(lats)).run(lats, [f[4] for f in films], mode=mode)
    for (h, Z, s, r, sc), lat, rec in zip(films, lats, recs):
        o = cpu.Film(h, Z, s, r, init=2)
        np.testing.assert_array_equal(rec, np.array([o.run(*st).as_tuple() for st in sc]))
        np.testing.assert_array_equal(lat.spins(), o.spins())


@pytest.mark.parametrize("tiling", [(64, 4, 1), (32, 8, 1), (16, 16, 2)])
@pytest.mark.parametrize("X,Y,Z", [(128, 16, 3), (256, 46, 5), (64, 4, 1)])
def test_gated_bitpacked_matches_oracle_and_int8(isf, tiling, X, Y, Z):
    """The gate on the bit-packed kernel: each group of four sites draws its gate numbers
    where a Metropolis test passed; the same trajectory as the oracle and the INT8 film."""
    h = _rand_h((Y, X), Z, 5 * X + Y + Z)
    g, o = _pair(isf, h, Z, 97531, replica=8, init=2, fmt=1)
    g.set_tuning(tiling[0], tiling[1], tiling[2], True, 0)
    _say("gated bit-packed", tiling, X, Y, Z)
    rg = g.run_schedule(GATED_STEPS)
    np.testing.assert_array_equal(rg, np.array([o.run(*s).as_tuple() for s in GATED_STEPS]))
    _assert_same(g, o)
    i8 = isf.Lattice(h, Z, 97531, replica=8, init=2)
    np.testing.assert_array_equal(i8.run_schedule(GATED_STEPS), rg)
    np.testing.assert_array_equal(i8.spins(), g.spins())


@pytest.mark.parametrize("mode", [0, 1])
def test_gated_bitpacked_batch_equals_oracle(isf, mode):
    rng = np.random.default_rng(5)
    films = []
    for i, (X, Y, Z) in enumerate([(64, 40, 3), (192, 64, 5), (128, 16, 2)]):
        h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
        sched = [(float(rng.uniform(1.0, 6.0)), int(hv), 3, 0, 40 * (i + 1)) for hv in rng.integers(-60, 61, size=4)]
        films.append((h, Z, 700 + i, i, sched))
    lats = [isf.Lattice(h, Z, s, replica=r, init=2, fmt=1) for (h, Z, s, r, sc) in films]
    _say("gated bit-packed batch", mode)
    recs = isf.Batch(len(lats)).run(lats, [f[4] for f in films], mode=mode)
    for (h, Z, s, r, sc), lat, rec in zip(films, lats, recs):
        o = cpu.Film(h, Z, s, r, init=2)
        np.testing.assert_array_equal(rec, np.array([o.run(*st).as_tuple() for st in sc]))
        np.testing.assert_array_equal(lat.spins(), o.spins())


# ------------------------------------------------------------------ PMOKE image and film statistics
@pytest.mark.parametrize("fmt,kernel,tiling", [(0, 0, (64, 4, 2)), (0, 2, (32, 16, 8)), (1, 0, (64, 4, 1)),
                                               (0, 3, (32, 16, 16)), (1, 0, (32, 8, 2))])
def test_surface_image_matches_oracle(isf, fmt, kernel, tiling):
    # the second bit-packed case has rows of 100 sites: three whole words and one of 4 sites
    X = (256 if tiling[0] == 64 else 200) if fmt else (352 if kernel == 3 else 200)
    h = _rand_h((58, X), 6, 40 + fmt + kernel)
    g, o = _pair(isf, h, 6, 1357, replica=2, init=2, fmt=fmt)
    g.set_tuning(tiling[0], tiling[1], tiling[2], False, kernel)
    _say("surface image", fmt, kernel)
    np.testing.assert_array_equal(g.surface_image(), o.surface_image())
    for hn, n in ((40, 3), (-60, 5), (0, 1)):  # odd sweep counts leave whole-sweep spins in the spare copy
        g.run_sweeps(2.0, hn, n)
        o.run(2.0, hn, n)
        np.testing.assert_array_equal(g.surface_image(), o.surface_image(), err_msg=str(hn))
    st, so = g.film_stats(), o.film_stats()
    assert (st["n_occ"], st["n_bonds"]) == (so["n_occ"], so["n_bonds"])
    assert st["mean_coordination"] == so["mean_coordination"] and st["p_c"] == so["p_c"]


def test_surface_image_of_the_ramp_film(isf):
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=c.init)
    g.set_tuning(32, 32, 16, True, 2)
    _say("surface image, large film")
    g.ramp_field(c.T, [-120], 3)
    o.run(c.T, -120, 3)
    np.testing.assert_array_equal(g.surface_image(), o.surface_image())
    with pytest.raises(Exception):
        import torch

        small = torch.empty(10, dtype=torch.int8, device="cuda")
        g.surface_image(out=small)


# ------------------------------------------------------------------ anisotropy (Eq. 7)
# (T, h_num, n_sweeps, n_discard, hs_num, an_num); the last step has no anisotropy
ANISO_STEPS = [(2.5, 30, 7, 0, 0, 40), (3.5, -45, 6, 1, 0, 160), (4.5, 0, 9, 2, 0, 20), (3.0, -7, 6, 0, 40, 60),
               (1e-3, 241, 2, 0, 0, 20), (2.0, -20, 66, 3, 7, 30), (4.0, 0, 5, 0, 0, 0)]


@pytest.mark.parametrize("kernel,tiling,graph", [(0, (64, 4, 2), True), (0, (16, 16, 1), False),
                                                 (0, (32, 8, 4), True), (1, (64, 4, 1), True)])
@pytest.mark.parametrize("X,Y,Z", [(72, 38, 5), (328, 46, 6), (8, 4, 1), (16, 8, 2)])
def test_aniso_schedule_matches_oracle(isf, kernel, tiling, graph, X, Y, Z):
    h = _rand_h((Y, X), Z, 13 * X + Y + Z)
    g, o = _pair(isf, h, Z, 24680, replica=5, init=2)
    if kernel == 1:
        g.attach_items()
    g.set_tuning(tiling[0], tiling[1], tiling[2], graph, kernel)
    _say("aniso schedule", kernel, tiling, graph, X, Y, Z)
    np.testing.assert_array_equal(g.run_schedule(ANISO_STEPS), np.array([o.run(*s).as_tuple() for s in ANISO_STEPS]))
    _assert_same(g, o)


@pytest.mark.parametrize("X,Y,Z,hseed,T", [(8, 4, 1, 25, 6.0), (16, 8, 2, 1, 12.0)])
def test_aniso_through_small_magnetisation(isf, X, Y, Z, hseed, T):
    """Hot small films at H = 0 pass through M = 0 (even site count) or M = +-1 (odd), the cases
    where the term is not a field."""
    h = _rand_h((Y, X), Z, hseed)
    g, o = _pair(isf, h, Z, 1234567, replica=2, init=2)
    steps = [(T, 0, 1, 0, 0, 20)] * 120 + [(T - 1.0, 3, 1, 0, 30, 45)] * 80
    _say("aniso small M", X, Y, Z)
    rg = g.run_schedule(steps)
    np.testing.assert_array_equal(rg, np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)
    assert np.any(np.abs(rg[:, 0]) == o.state()[2] % 2)


def test_aniso_large_film_prefix(isf):
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=c.init)
    g.set_tuning(64, 4, 2, True, 0)
    _say("aniso large film prefix")
    steps = [(c.T, hn, 3, 0, 0, 40) for hn in (120, 0, -60)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)


@pytest.mark.parametrize("kernel,tiling", [(3, (32, 16, 16)), (3, (32, 32, 16)), (2, (16, 16, 4)), (2, (32, 8, 4))])
@pytest.mark.parametrize("X,Y,Z", [(328, 46, 6), (352, 48, 4)])
def test_aniso_whole_kernels_match_oracle(isf, kernel, tiling, X, Y, Z):
    """The term on the whole-sweep kernels (steps at field h + h_an sign(M), checked and run
    again per sublattice where |M| could have come below 2): the schedule with discarded
    sweeps, gated steps, T -> 0 and a step without the term, then the same again in
    advances of 5 sweeps (steps cut in parts)."""
    h = _rand_h((Y, X), Z, 7 * X + Y + Z)
    g, o = _pair(isf, h, Z, 24680, replica=5, init=2)
    g.attach_aniso_workspace()
    g.set_tuning(tiling[0], tiling[1], tiling[2], True, kernel)
    _say("aniso whole kernels", kernel, tiling, X, Y, Z)
    np.testing.assert_array_equal(g.run_schedule(ANISO_STEPS), np.array([o.run(*s).as_tuple() for s in ANISO_STEPS]))
    _assert_same(g, o)
    g.schedule_load(ANISO_STEPS)
    while g.advance(5):
        pass
    want = np.array([o.run(*s).as_tuple() for s in ANISO_STEPS])
    np.testing.assert_array_equal(g.records(), want)
    _assert_same(g, o)
    runs, redone = g.aniso_stats()
    assert runs > 0 and redone <= runs


def test_aniso_whole_kernel_through_reversal(isf):
    """A field ramp through M = 0 with the term: the speculative whole-sweep steps and the steps
    run again per sublattice together equal the oracle and the per-sublattice kernels."""
    X, Y, Z = 352, 48, 4
    h = _rand_h((Y, X), Z, 31)
    steps = [(3.0, hn, 20, 0, 0, 40) for hn in list(range(60, -121, -20)) + list(range(-100, 61, 20))]
    g, o = _pair(isf, h, Z, 97531, replica=1, init=0)
    g.attach_aniso_workspace()
    g.set_tuning(32, 16, 16, True, 3)
    _say("aniso whole kernel through the reversal")
    rg = g.run_schedule(steps)
    np.testing.assert_array_equal(rg, np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)
    runs, redone = g.aniso_stats()
    assert 0 < redone < runs, (runs, redone)
    p = isf.Lattice(h, Z, 97531, replica=1, init=0)
    p.set_tuning(64, 4, 2, True, 0)
    np.testing.assert_array_equal(p.run_schedule(steps), rg)
    np.testing.assert_array_equal(p.spins(), g.spins())


def test_aniso_whole_kernel_large_film_prefix(isf):
    from isf_workloads import config_plain_hysteresis_large

    c = config_plain_hysteresis_large()
    h = c.heights()
    g, o = _pair(isf, h, c.Z, c.mc_seed, init=c.init)
    g.attach_aniso_workspace()
    g.set_tuning(32, 32, 16, True, 3)
    _say("aniso whole kernel, large film prefix")
    steps = [(c.T, hn, 3, 0, 0, 40) for hn in (120, 0, -60)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*s).as_tuple() for s in steps]))
    _assert_same(g, o)


def test_aniso_rejected_where_unsupported(isf):
    from paper_1205_5588_amd._lib import IsfError

    bp = isf.Lattice(_rand_h((16, 128), 3, 4), 3, 1, fmt=1)
    with pytest.raises(IsfError):
        bp.run_schedule([(2.0, 0, 3, 0, 0, 40)])
    h = _rand_h((40, 352), 4, 9)
    g, o = _pair(isf, h, 4, 77, init=2)
    with pytest.raises(IsfError):
        g.run_schedule([(2.0, 0, 3, 0, 0, -1)])  # negative anisotropy field
    for kernel, tiling in ((2, (16, 16, 4)), (3, (32, 16, 16))):
        g.set_tuning(tiling[0], tiling[1], tiling[2], True, kernel)
        with pytest.raises(IsfError):
            g.schedule_load([(2.0, 0, 3, 0, 0, 40)])
    g.set_tuning(64, 4, 2, True, 0)
    g.schedule_load([(2.0, 0, 3, 0, 0, 40)])
    with pytest.raises(IsfError):
        g.set_tuning(32, 16, 16, True, 3)  # a whole-sweep kernel under a schedule with the term
    with pytest.raises(IsfError):
        isf.Batch(1).advance([g], 3, mode=0)
    assert g.advance(3) == 3
    o.run(2.0, 0, 3, 0, 0, 40)
    _assert_same(g, o)
    # without the term the whole-sweep kernels are available again
    g.schedule_load([(2.0, 10, 2, 0)])
    g.set_tuning(32, 16, 16, True, 3)
    assert g.advance(2) == 2
    o.run(2.0, 10, 2)
    # the workspace: refused for a bit-packed film, short or misaligned buffers
    import ctypes

    import torch

    from paper_1205_5588_amd import _lib

    nb = ctypes.c_uint64()
    assert _lib.load().isf_aniso_workspace_bytes(bp.handle, ctypes.byref(nb)) == _lib.ISF_EINVAL
    assert _lib.load().isf_aniso_workspace_bytes(g.handle, ctypes.byref(nb)) == 0
    buf = torch.empty(int(nb.value) + 512, dtype=torch.uint8, device="cuda")
    lib = _lib.load()
    assert lib.isf_attach_aniso_workspace(g.handle, buf.data_ptr(), int(nb.value) - 1) == _lib.ISF_ENOSPC
    assert lib.isf_attach_aniso_workspace(g.handle, buf.data_ptr() + 16, int(nb.value)) == _lib.ISF_EINVAL
    assert lib.isf_attach_aniso_workspace(g.handle, None, int(nb.value)) == _lib.ISF_EINVAL
    # with a workspace the whole-sweep kernels take the term too
    g.attach_aniso_workspace()
    g.schedule_load([(2.0, 0, 3, 0, 0, 40)])
    assert g.advance(3) == 3
    o.run(2.0, 0, 3, 0, 0, 40)
    _assert_same(g, o)


# ------------------------------------------------------------------ draw-only ceiling
@pytest.mark.parametrize("fmt", [0, 1])
def test_draw_ceiling_checksum_equals_oracle_generator(isf, fmt):
    """The draw-only kernel draws, for every stored dword and sweep, the numbers of that
    dword's attempt: its XOR checksum equals the oracle's Philox over the same counters."""
    X, Y, Z = (72, 10, 3) if fmt == 0 else (128, 6, 2)
    h = _rand_h((Y, X), Z, 3)
    seed, rep = 0x1234_5678_9ABC_DEF0, 9
    g = isf.Lattice(h, Z, seed, replica=rep, fmt=fmt)
    _say("draw ceiling fmt", fmt)
    x, ms = g.draw_xor(0xFFFFFFFE, 3)   # the sweep counter wraps in word 1 of the counter
    key = (seed & 0xFFFFFFFF, seed >> 32)
    want = 0
    for t in (0xFFFFFFFE, 0xFFFFFFFF, 0):
        for z in range(Z):
            for y in range(Y):
                sigma = (y & 1) + 2 * (z & 1)
                for d in range(X // 8):
                    for w in cpu.philox(((z * Y + y) * (X // 8) + d, t, rep, sigma), key):
                        want ^= w
    assert x == want and ms > 0
    np.testing.assert_array_equal(g.spins(), cpu.Film(h, Z, seed, rep).spins())  # the film is untouched


# ------------------------------------------------------------------ pipelined kernel on any row width
@pytest.mark.parametrize("X,Y,Z,tiling", [(328, 46, 6, (32, 32, 16)), (344, 48, 5, (32, 16, 16)),
                                          (344, 48, 5, (32, 32, 8)), (488, 40, 8, (32, 32, 16))])
def test_pipe_kernel_rows_not_whole_pieces(isf, X, Y, Z, tiling):
    """Rows of 41, 43 and 61 dwords: a 16-byte piece would straddle the periodic seam, so
    regions load dword by dword and whole tiles are written dword by dword (ragged tiles
    in both directions, through reversal sweeps that overflow the change lists)."""
    h = _rand_h((Y, X), Z, X + Y)
    g, o = _pair(isf, h, Z, 0xABCDEF12, replica=4, init=2, tuning=tiling + (True, 3))
    _say("pipe, odd rows", X, Y, Z, tiling)
    steps = [(2.5, 60, 70, 0), (3.0, -80, 66, 3), (1.5, 100, 3, 1), (4.0, -20, 21, 0)]
    np.testing.assert_array_equal(g.run_schedule(steps), np.array([o.run(*st).as_tuple() for st in steps]))
    _assert_same(g, o)


def test_batched_pipe_mode_equals_alone_and_oracle(isf):
    """The batched pipelined mode: films it takes (rows of 40 dwords or more, 41 and 43 among
    them, at least 40 rows, Z <= 8) share one launch per sweep; the others (too narrow, too
    few rows, nine planes) run in the sublattice mode in the same call.  Schedules of
    different lengths, so films sit out launches; advanced in chunks."""
    rng = np.random.default_rng(321)
    shapes = [(328, 46, 6), (344, 48, 8), (320, 56, 2), (512, 40, 3), (64, 40, 3), (336, 24, 4), (320, 48, 9)]
    films = []
    for i, (X, Y, Z) in enumerate(shapes):
        h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
        T = float(rng.uniform(1.0, 9.0))
        sched = [(T, int(hv), int(rng.integers(3, 30)), 0) for hv in rng.integers(-80, 81, size=2 + i % 3)]
        films.append((h, Z, 700 + i, i, sched))
    _say("batched pipe mode")
    lats = [isf.Lattice(h, Z, s, replica=r, init=2) for (h, Z, s, r, sc) in films]
    b = isf.Batch(len(lats))
    for lat, f in zip(lats, films):
        lat.schedule_load(f[4])
    while sum(l.remaining() for l in lats):
        b.advance(lats, 17, mode=3)
    b.sync()
    for (h, Z, s, r, sc), lat in zip(films, lats):
        rec = lat.records()
        o = cpu.Film(h, Z, s, r, init=2)
        np.testing.assert_array_equal(rec, np.array([o.run(*st).as_tuple() for st in sc]), err_msg="film %d" % r)
        np.testing.assert_array_equal(lat.spins(), o.spins(), err_msg="film %d" % r)
        alone = isf.Lattice(h, Z, s, replica=r, init=2)
        np.testing.assert_array_equal(alone.run_schedule(sc), rec, err_msg="film %d alone" % r)
