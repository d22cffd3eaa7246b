"""Pins of the CPU oracle against results that do not come from the oracle itself.

Each test names what it pins:
  - Philox4x32-10 against the header implementations shipped with PyTorch and
    rocRAND (library routines, compiled here from their header source);
  - thresholds of Eq. (8) against a 50-digit evaluation of exp;
  - Gibbs averages of Eqs. (4)-(5) by exact enumeration of all 2^N states;
  - the Markov chain of Eq. (6) as explicit transition matrices (detailed
    balance, stationarity, sampled one-sweep frequencies);
  - incremental energy/magnetisation bookkeeping against a full recount;
  - the H -> -H symmetry of Eq. (3);
  - the T -> 0 ground state argument of Section 5;
  - disorder at high T;
  - the square-lattice special case (Onsager/Yang closed forms);
  - an isolated spin (tanh(H/T));
  - independence of the order of sites inside a sublattice;
  - Eq. (2) against the printed Table 1.
"""

import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import cpu, physics, ref

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------- Philox
def _random_counters(n, seed=7):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, 2**32, size=(n, 6), dtype=np.uint64).tolist()
    rows += [[0] * 6, [0xFFFFFFFF] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0xFFFFFFFF, 0]]
    return rows


_TORCH_PROG = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    at::philox_engine e((uint64_t)k0 | ((uint64_t)k1 << 32), (uint64_t)c2 | ((uint64_t)c3 << 32), 0);
    e.set_offset((uint64_t)c0 | ((uint64_t)c1 << 32));
    unsigned a = e(), b = e(), c = e(), d = e();
    printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
}
"""

_ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct probe : rocrand_device::philox4x32_10_engine {
  uint4 raw(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  probe p;
  while (scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = p.raw(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
}
"""


def _run_prog(exe, rows):
    inp = "".join("%x %x %x %x %x %x\n" % tuple(r) for r in rows)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]


def _check_against(rows, got):
    assert len(got) == len(rows)
    for r, g in zip(rows, got):
        ctr, key = r[:4], r[4:]
        assert cpu.philox(ctr, key) == g, r
        assert ref.philox4x32_10(ctr, key) == g, r


def test_philox_matches_torch_header(oracle_lib, tmp_path):
    import torch

    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    src = tmp_path / "p.cpp"
    src.write_text(_TORCH_PROG)
    exe = str(tmp_path / "p")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I" + inc, str(src), "-o", exe], check=True)
    rows = _random_counters(300)
    _check_against(rows, _run_prog(exe, rows))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_header(oracle_lib, tmp_path):
    src = tmp_path / "r.cpp"
    src.write_text(_ROCRAND_PROG)
    exe = str(tmp_path / "r")
    subprocess.run(["hipcc", "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950", str(src), "-o", exe],
                   check=True, capture_output=True)
    rows = _random_counters(300, seed=11)
    _check_against(rows, _run_prog(exe, rows))


# --------------------------------------------------------------------------- thresholds
def test_thresholds_against_high_precision_exp(oracle_lib):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    for T in (1e-3, 0.5, 1.0, 2.269, 3.0, 4.0, 7.3, 12.0, 1e6):
        for h_num in (-241, -120, -7, 0, 1, 55, 100, 120, 241):
            tab = cpu.threshold_table(T, h_num)
            for si, s in enumerate((-1, 1)):
                for n in range(-12, 13):
                    q = s * (20 * n + h_num)
                    thr = int(tab[si, n + 12])
                    if q <= 0:
                        assert thr == 0xFFFFFFFF
                        continue
                    exact = mpmath.exp(-mpmath.mpf(q) / 10 / T) * 2**32
                    # floor of a double within 1 ulp of exact: off by at most one count
                    assert abs(thr - int(mpmath.floor(exact))) <= 1, (T, h_num, s, n)
                    assert thr <= 2**32 - 430
    # monotone in q at fixed T
    vals = [cpu.lib().orc_threshold(q, 2.5) for q in range(1, 500)]
    assert all(a >= b for a, b in zip(vals, vals[1:]))
    # T -> 0: every uphill move is rejected
    assert all(cpu.lib().orc_threshold(q, 1e-3) == 0 for q in range(1, 200))


# --------------------------------------------------------------------------- exact enumeration
def _tiny_films():
    h8 = np.ones((4, 4), dtype=np.uint8)                    # square lattice, 8 sites
    h16 = np.full((4, 4), 2, dtype=np.uint8)                # two layers, 16 sites
    rng = np.random.default_rng(3)
    while True:                                             # three layers, <= 20 sites
        h20 = rng.integers(0, 4, size=(4, 4)).astype(np.uint8)
        n = ref.TinyFilm(h20, 3).N
        if 14 <= n <= 20:
            break
    return [(h8, 1), (h16, 2), (h20, 3)]


# h_num is kept off multiples of 20: then q = s (20 n + h_num) is never 0, no
# move is accepted deterministically at dE = 0, and the sweep chain is ergodic
# (checked on the 8-site film by its spectral gap below).  Temperatures and
# fields are chosen so that the chain tunnels between +M and -M often enough
# for block means to see both (the 16-site film has coordination 8).
@pytest.mark.parametrize("T,h_num", [(3.0, 45), (6.0, 5), (9.0, -25)])
def test_exact_enumeration(oracle_lib, T, h_num):
    for h, Z in _tiny_films():
        tf = ref.TinyFilm(h, Z)
        if tf.N <= 8:
            w = np.sort(np.abs(np.linalg.eigvals(ref.sweep_matrix(tf, T, h_num))))[::-1]
            assert w[0] == pytest.approx(1.0) and w[1] < 0.95
        ex = ref.enumerate_exact(tf, T, h_num)
        f = cpu.Film(h, Z, seed=0xC0FFEE + Z, replica=Z)
        f.run(T, h_num, 2000)
        nblk, blk = 40, 10000
        m, am, e = [], [], []
        for _ in range(nblk):
            r = f.run(T, h_num, blk)
            m.append(r.sum_M / blk)
            am.append(r.sum_absM / blk)
            e.append(r.sum_E / blk)
        for est, key in ((m, "M"), (am, "absM"), (e, "E_bond")):
            mean = float(np.mean(est))
            se = float(np.std(est, ddof=1) / math.sqrt(nblk))
            assert abs(mean - ex[key]) <= 5.0 * se + 1e-3, (key, Z, T, h_num, mean, ex[key], se)


def test_zero_field_tiny_film_is_not_ergodic():
    """At H = 0 a move with dE = 0 is always taken (Eq. 8 accepts E2 <= E1), which
    on the 8-site torus (every site of sublattice 0 bonded to every site of
    sublattice 1) leaves several unit eigenvalues in the sweep matrix: time
    averages there depend on the start, so exact-enumeration pins avoid H = 0."""
    tf = ref.TinyFilm(np.ones((4, 4), dtype=np.uint8), 1)
    w = np.sort(np.abs(np.linalg.eigvals(ref.sweep_matrix(tf, 2.5, 0))))[::-1]
    assert w[1] == pytest.approx(1.0)


# --------------------------------------------------------------------------- transition matrices
def _pair_and_triangle():
    pair = np.zeros((4, 4), dtype=np.uint8)
    pair[0, 0] = 1
    pair[1, 1] = 1
    tri = pair.copy()
    tri[0, 1] = 2              # h(x=1, y=0) = 2 -> site (1, 0, 1)
    return [(pair, 1), (tri, 2)]


def test_transition_matrix_structure():
    films = _pair_and_triangle()
    pf = ref.TinyFilm(*films[0])
    tf = ref.TinyFilm(*films[1])
    assert pf.N == 2 and len(pf.bonds) == 1 and sorted(pf.sub) == [0, 1]
    assert tf.N == 3 and len(tf.bonds) == 3 and sorted(tf.sub) == [0, 1, 2]
    for (h, Z) in films:
        film = ref.TinyFilm(h, Z)
        for T, hn in ((1.5, 10), (3.0, -40), (0.7, 0)):
            states, pi = ref.boltzmann(film, T, hn)
            for sigma in range(4):
                for quant, tol in ((False, 1e-15), (True, 2.0**-31)):
                    P = ref.phase_matrix(film, T, hn, sigma, quantised=quant)
                    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-15)
                    flow = pi[:, None] * P
                    assert np.max(np.abs(flow - flow.T)) <= tol
            S = ref.sweep_matrix(film, T, hn, quantised=False)
            assert np.max(np.abs(pi @ S - pi)) <= 1e-14


def test_transition_frequencies_sampled(oracle_lib):
    """One-sweep transition frequencies of the C oracle against the quantised sweep matrix."""
    h, Z = _pair_and_triangle()[1]
    film = ref.TinyFilm(h, Z)
    T, hn = 1.5, 10
    S = ref.sweep_matrix(film, T, hn, quantised=True)
    states = [tuple(s) for s in __import__("itertools").product((-1, 1), repeat=film.N)]
    idx = {s: a for a, s in enumerate(states)}
    start = (1, -1, 1)
    f = cpu.Film(h, Z, seed=99, replica=5)
    cube = np.zeros((Z, 4, 4), dtype=np.int8)
    for i, (x, y, z) in enumerate(film.sites):
        cube[z, y, x] = start[i]
    nsamp = 60000
    counts = np.zeros(len(states))
    for t in range(nsamp):
        f.set_spins(cube, t)
        f.run(T, hn, 1)
        sp = f.spins()
        counts[idx[tuple(int(sp[z, y, x]) for (x, y, z) in film.sites)]] += 1
    p = S[idx[start]]
    exp = nsamp * p
    sd = np.sqrt(nsamp * p * (1 - p)) + 1e-9
    assert np.all(np.abs(counts - exp) <= 5 * sd + 1), (counts, exp)
    assert counts[p == 0].sum() == 0


# --------------------------------------------------------------------------- bookkeeping / symmetry
def test_incremental_equals_recount(oracle_lib):
    from isf_workloads import config_plain_hysteresis_small

    c = config_plain_hysteresis_small()
    h = c.heights()
    f = cpu.Film(h, c.Z, c.mc_seed, init=cpu.INIT_RANDOM)
    assert f.state()[:2] == f.recount()
    for hn in c.h_nums[::7]:
        f.run(c.T, hn, 5)
        assert f.state()[:2] == f.recount()
    # the second implementation counts bonds independently
    tf = ref.TinyFilm(h, c.Z)
    sp = f.spins()
    tf.s = [int(sp[z, y, x]) for (x, y, z) in tf.sites]
    assert f.state()[0] == tf.magnetisation()
    assert f.state()[1] == tf.bond_energy()
    assert f.state()[3] == len(tf.bonds)
    assert f.state()[2] == tf.N


@pytest.mark.parametrize("init", [cpu.INIT_UP, cpu.INIT_RANDOM])
def test_field_reversal_symmetry(oracle_lib, init):
    rng = np.random.default_rng(5)
    h = rng.integers(0, 5, size=(24, 16)).astype(np.uint8)
    a = cpu.Film(h, 4, seed=777, replica=2, init=init)
    b = cpu.Film(h, 4, seed=777, replica=2, init=cpu.INIT_DOWN)
    b.set_spins(-a.spins(), 0)
    ramp = [40, 10, -20, -60, 0, 33, -1]
    for hn in ramp:
        ra = a.run(2.5, hn, 3).as_tuple()
        rb = b.run(2.5, -hn, 3).as_tuple()
        assert np.array_equal(b.spins(), -a.spins())
        assert rb == (-ra[0], ra[1], -ra[2], ra[3], ra[4], ra[5])


def test_zero_temperature_ground_state(oracle_lib):
    rng = np.random.default_rng(8)
    h = rng.integers(0, 5, size=(32, 32)).astype(np.uint8)
    f = cpu.Film(h, 4, seed=1, init=cpu.INIT_UP)
    n_occ, n_bonds = f.state()[2], f.state()[3]
    for _ in range(3):
        r = f.run(1e-3, 1, 10)
        assert r.M == n_occ and r.E == -n_bonds and r.accepted == 0
    for sign in (1, -1):
        g = cpu.Film(h, 4, seed=2, init=cpu.INIT_RANDOM)
        assert abs(g.state()[0]) < n_occ
        r = g.run(1e-3, 241 * sign, 1)
        assert r.M == sign * n_occ and r.E == -n_bonds
        r = g.run(1e-3, 241 * sign, 5)
        assert r.M == sign * n_occ and r.accepted == 0


def test_high_temperature_disorder(oracle_lib):
    rng = np.random.default_rng(9)
    h = rng.integers(0, 5, size=(64, 64)).astype(np.uint8)
    f = cpu.Film(h, 4, seed=3, init=cpu.INIT_UP)
    N = f.state()[2]
    f.run(50.0, 0, 50)
    r = f.run(50.0, 0, 1000)
    assert abs(r.sum_M / 1000 / N) <= 5 / math.sqrt(N)
    assert r.sum_absM / 1000 / N <= 3 / math.sqrt(N)


def test_square_lattice_onsager(oracle_lib):
    """Z = 1, h = 1 is the square lattice (offsets (+-1, +-1, 0)); T = 2 < Tc = 2.269."""
    X = Y = 256
    h = np.ones((Y, X), dtype=np.uint8)
    T = 2.0
    f = cpu.Film(h, 1, seed=2024, init=cpu.INIT_UP)
    N = f.state()[2]
    assert N == X * Y // 2 and f.state()[3] == 2 * N
    f.run(T, 0, 300)
    n = 2000
    r = f.run(T, 0, n)
    m = r.sum_absM / n / N
    u = r.sum_E / n / N
    assert abs(m - physics.square_lattice_magnetisation(T)) < 3e-3, m
    assert abs(u - physics.square_lattice_energy(T)) < 3e-3, u
    assert abs(physics.square_lattice_magnetisation(T) - 0.91132) < 1e-5
    assert abs(physics.square_lattice_energy(T) - (-1.74556)) < 1e-5


def test_isolated_spin(oracle_lib):
    h = np.zeros((4, 4), dtype=np.uint8)
    h[0, 0] = 1
    T, hn = 1.0, 10
    f = cpu.Film(h, 1, seed=17, init=cpu.INIT_UP)
    assert f.state()[2] == 1 and f.state()[3] == 0
    # exact two-state chain with the quantised threshold
    p = cpu.lib().orc_threshold(hn, T) / 2.0**32
    m_chain = (1 - p) / (1 + p)
    assert abs(m_chain - physics.single_spin_magnetisation(hn / 20, T)) < 1e-9
    nblk, blk = 50, 20000
    ms = [f.run(T, hn, blk).sum_M / blk for _ in range(nblk)]
    se = np.std(ms, ddof=1) / math.sqrt(nblk)
    assert abs(np.mean(ms) - m_chain) <= 5 * se + 1e-4


def test_site_order_independence(oracle_lib):
    rng = np.random.default_rng(12)
    h = rng.integers(0, 6, size=(38, 40)).astype(np.uint8)
    films = []
    for order in (0, 1, 2):
        f = cpu.Film(h, 5, seed=31337, replica=9, init=cpu.INIT_RANDOM)
        f.set_order(order)
        films.append(f)
    for hn in (0, 30, -45, 7):
        recs = [f.run(3.3, hn, 4).as_tuple() for f in films]
        assert recs[0] == recs[1] == recs[2]
        assert np.array_equal(films[0].spins(), films[1].spins())
        assert np.array_equal(films[0].spins(), films[2].spins())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c_oracle_matches_python_oracle(oracle_lib, seed):
    rng = np.random.default_rng(100 + seed)
    Y, X, Z = [(8, 8, 3), (6, 10, 4), (4, 12, 2)][seed]
    h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
    key = int(rng.integers(0, 2**63))
    rep = int(rng.integers(0, 1000))
    tf = ref.TinyFilm(h, Z, seed=key, replica=rep)
    tf.init_random()
    cf = cpu.Film(h, Z, key, rep, init=cpu.INIT_RANDOM)
    for T, hn in ((2.5, 20), (1.1, -7), (6.0, 0), (0.9, 55)):
        acc = sum(tf.sweep(T, hn) for _ in range(4))
        r = cf.run(T, hn, 4)
        sp = cf.spins()
        assert all(sp[z, y, x] == tf.s[i] for i, (x, y, z) in enumerate(tf.sites))
        assert r.M == tf.magnetisation() and r.E == tf.bond_energy() and r.accepted == acc


def test_table1_critical_concentration():
    rows = []
    with open(os.path.join(HERE, "golden", "table1.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    assert len(rows) == 4
    for ml, z, tc, p, pc in rows:
        assert round(physics.critical_concentration(z), 2) == pytest.approx(pc, abs=1e-9)
        # single bond counting: mean-field Tc = z J lies above the printed Tc in every row
        assert tc < z


# --------------------------------------------------------------------------- switching-field gate (Eq. 9)
# The gate's probability exp(-|S_i h_s|/T) does not depend on the spin, so it
# multiplies every flip probability by the same factor g: detailed balance and
# the Boltzmann stationary law of Eq. (3) are unchanged, only the dynamics slow
# down.  These pins check that, the gate thresholds, and the gate's own draw.
def test_gate_thresholds_against_high_precision_exp(oracle_lib):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    for T in (1e-3, 0.5, 1.0, 3.0, 7.3, 12.0, 1e6):
        assert cpu.gate_threshold(T, 0) == 0xFFFFFFFF == ref.gate_threshold(0, T)
        for hs in (1, 7, 40, 80, 160, 4000):
            thr = cpu.gate_threshold(T, hs)
            assert thr == cpu.gate_threshold(T, -hs) == ref.gate_threshold(hs, T)
            exact = mpmath.exp(-mpmath.mpf(hs) / 20 / T) * 2**32
            assert abs(thr - int(mpmath.floor(exact))) <= 1, (T, hs)
            assert thr <= 2**32 - 215  # never the sentinel
    assert cpu.gate_threshold(1e-3, 1) == 0


def test_gated_transition_matrices():
    for (h, Z) in _pair_and_triangle():
        film = ref.TinyFilm(h, Z)
        for T, hn, hs in ((1.5, 10, 30), (3.0, -40, 160), (0.7, 5, 7)):
            states, pi = ref.boltzmann(film, T, hn)
            g = ref.gate_probability(hs, T, quantised=False)
            for sigma in range(4):
                for quant, tol in ((False, 1e-15), (True, 2.0**-31)):
                    P = ref.phase_matrix(film, T, hn, sigma, quantised=quant, hs_num=hs)
                    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-15)
                    flow = pi[:, None] * P
                    assert np.max(np.abs(flow - flow.T)) <= tol
                # off-diagonal single flips are the ungated ones times g
                P0 = ref.phase_matrix(film, T, hn, sigma, quantised=False)
                P1 = ref.phase_matrix(film, T, hn, sigma, quantised=False, hs_num=hs)
                n_members = sum(1 for s in film.sub if s == sigma)
                if n_members == 1:
                    off = ~np.eye(len(states), dtype=bool)
                    assert np.allclose(P1[off], g * P0[off], atol=1e-15)
            S = ref.sweep_matrix(film, T, hn, quantised=False, hs_num=hs)
            assert np.max(np.abs(pi @ S - pi)) <= 1e-14


def test_gated_transition_frequencies_sampled(oracle_lib):
    """One-sweep frequencies of the gated C oracle against the gated quantised sweep matrix."""
    h, Z = _pair_and_triangle()[1]
    film = ref.TinyFilm(h, Z)
    T, hn, hs = 1.5, 10, 30
    S = ref.sweep_matrix(film, T, hn, quantised=True, hs_num=hs)
    S0 = ref.sweep_matrix(film, T, hn, quantised=True)
    states = [tuple(s) for s in __import__("itertools").product((-1, 1), repeat=film.N)]
    idx = {s: a for a, s in enumerate(states)}
    start = (1, -1, 1)
    assert np.max(np.abs(S[idx[start]] - S0[idx[start]])) > 0.05  # the gate changes this row
    f = cpu.Film(h, Z, seed=4242, replica=3)
    cube = np.zeros((Z, 4, 4), dtype=np.int8)
    for i, (x, y, z) in enumerate(film.sites):
        cube[z, y, x] = start[i]
    nsamp = 60000
    counts = np.zeros(len(states))
    for t in range(nsamp):
        f.set_spins(cube, t)
        f.run(T, hn, 1, 0, hs)
        sp = f.spins()
        counts[idx[tuple(int(sp[z, y, x]) for (x, y, z) in film.sites)]] += 1
    p = S[idx[start]]
    sd = np.sqrt(nsamp * p * (1 - p)) + 1e-9
    assert np.all(np.abs(counts - nsamp * p) <= 5 * sd + 1), (counts, nsamp * p)
    assert counts[p == 0].sum() == 0


def test_gated_isolated_spin(oracle_lib):
    """Two-state chain: up->down with g p, down->up with g (dE < 0 moves are gated
    too); m = tanh(H/T) as without the gate, flip rate g 2p/(1+p) per sweep."""
    h = np.zeros((4, 4), dtype=np.uint8)
    h[0, 0] = 1
    T, hn, hs = 1.0, 10, 12
    p = cpu.lib().orc_threshold(hn, T) / 2.0**32
    g = cpu.gate_threshold(T, hs) / 2.0**32
    f = cpu.Film(h, 1, seed=23, init=cpu.INIT_UP)
    nblk, blk = 40, 20000
    ms, rates = [], []
    for _ in range(nblk):
        r = f.run(T, hn, blk, 0, hs)
        ms.append(r.sum_M / blk)
        rates.append(r.accepted / blk)
    m_chain = (1 - p) / (1 + p)
    assert abs(np.mean(ms) - m_chain) <= 5 * np.std(ms, ddof=1) / math.sqrt(nblk) + 1e-4
    rate = g * 2 * p / (1 + p)
    assert abs(np.mean(rates) - rate) <= 5 * np.std(rates, ddof=1) / math.sqrt(nblk) + 1e-4


def test_gate_blocks_downhill_moves_at_low_temperature(oracle_lib):
    """T -> 0 with h_s > 0: the gate's probability is 0, so not even the moves
    that lower the energy happen (steps 4-5 come before steps 1-3)."""
    rng = np.random.default_rng(5)
    h = rng.integers(0, 4, size=(16, 16)).astype(np.uint8)
    f = cpu.Film(h, 3, seed=9, init=cpu.INIT_RANDOM)
    start = f.spins()
    r = f.run(1e-3, 241, 5, 0, 20)
    assert r.accepted == 0 and np.array_equal(f.spins(), start)
    r = f.run(1e-3, 241, 1, 0, 0)  # without the gate every down spin flips
    assert r.M == f.state()[2]


@pytest.mark.parametrize("seed", [0, 1])
def test_gated_c_oracle_matches_python_oracle(oracle_lib, seed):
    rng = np.random.default_rng(300 + seed)
    Y, X, Z = [(8, 8, 3), (6, 10, 4)][seed]
    h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
    key = int(rng.integers(0, 2**63))
    tf = ref.TinyFilm(h, Z, seed=key, replica=seed)
    tf.init_random()
    cf = cpu.Film(h, Z, key, seed, init=cpu.INIT_RANDOM)
    for T, hn, hs in ((2.5, 20, 40), (1.1, -7, 160), (6.0, 0, -80), (0.9, 55, 3)):
        acc = sum(tf.sweep(T, hn, hs) for _ in range(4))
        r = cf.run(T, hn, 4, 0, hs)
        sp = cf.spins()
        assert all(sp[z, y, x] == tf.s[i] for i, (x, y, z) in enumerate(tf.sites))
        assert r.M == tf.magnetisation() and r.E == tf.bond_energy() and r.accepted == acc


def test_gated_exact_enumeration(oracle_lib):
    """The gate leaves the Gibbs averages of Eqs. (4)-(5) unchanged (8-site film)."""
    h, Z = _tiny_films()[0]
    tf = ref.TinyFilm(h, Z)
    T, hn, hs = 3.0, 45, 40
    ex = ref.enumerate_exact(tf, T, hn)
    f = cpu.Film(h, Z, seed=0xBEEF, replica=1)
    f.run(T, hn, 2000, 0, hs)
    nblk, blk = 40, 10000
    m = [f.run(T, hn, blk, 0, hs).sum_M / blk for _ in range(nblk)]
    se = float(np.std(m, ddof=1) / math.sqrt(nblk))
    assert abs(float(np.mean(m)) - ex["M"]) <= 5.0 * se + 1e-3


# --------------------------------------------------------------------------- PMOKE image, mean coordination
def _columns_with_a_site(h):
    """Closed form: column (x, y) holds a site iff some z < h with z = x + y (mod 2), i.e.
    h >= 2, or h == 1 and x + y even."""
    Y, X = h.shape
    parity = (np.add.outer(np.arange(Y), np.arange(X)) % 2) == 0
    return (h >= 2) | ((h == 1) & parity)


def test_surface_image_closed_forms(oracle_lib):
    rng = np.random.default_rng(21)
    for L in (1, 2, 3, 5):
        h = np.full((12, 16), L, dtype=np.uint8)  # flat slab of L layers: full coordination 12 - 8/L
        f = cpu.Film(h, L, seed=1, init=cpu.INIT_UP)
        st = f.film_stats()
        assert st["mean_coordination"] == pytest.approx(12.0 - 8.0 / L, abs=1e-12)
        assert st["p_c"] == pytest.approx(2.0 / (12.0 - 8.0 / L), abs=1e-12)
        img = f.surface_image()
        # every column holds a site when L >= 2, the columns with x + y even when L == 1
        np.testing.assert_array_equal(img, _columns_with_a_site(h).astype(np.int8))
        assert (img != 0).mean() == (0.5 if L == 1 else 1.0)
    h = rng.integers(0, 5, size=(20, 24)).astype(np.uint8)
    for init in (cpu.INIT_UP, cpu.INIT_DOWN, cpu.INIT_RANDOM):
        f = cpu.Film(h, 4, seed=5, init=init)
        img = f.surface_image()
        np.testing.assert_array_equal(img != 0, _columns_with_a_site(h))
        if init == cpu.INIT_UP:
            assert set(np.unique(img)) <= {0, 1}
    # the image of the reversed state is the reversed image (H -> -H symmetry of the display)
    f = cpu.Film(h, 4, seed=5, init=cpu.INIT_RANDOM)
    f.run(2.5, 30, 3)
    g = cpu.Film(h, 4, seed=5, init=cpu.INIT_RANDOM)
    g.set_spins(-f.spins(), 3)
    np.testing.assert_array_equal(g.surface_image(), -f.surface_image())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_surface_image_c_matches_python(oracle_lib, seed):
    rng = np.random.default_rng(700 + seed)
    Y, X, Z = [(8, 8, 3), (6, 10, 4), (10, 12, 5)][seed]
    h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
    key = int(rng.integers(0, 2**63))
    tf = ref.TinyFilm(h, Z, seed=key, replica=1)
    tf.init_random()
    cf = cpu.Film(h, Z, key, 1, init=cpu.INIT_RANDOM)
    for T, hn in ((2.5, 20), (1.1, -7)):
        for _ in range(3):
            tf.sweep(T, hn)
        cf.run(T, hn, 3)
        np.testing.assert_array_equal(cf.surface_image(), tf.surface_image())
    assert cf.film_stats()["mean_coordination"] == pytest.approx(tf.mean_coordination(), abs=1e-12)


# --------------------------------------------------------------------------- anisotropy (Eq. 7)
# The anisotropy term -h_an |M| couples every site to the global M; the oracle
# freezes M at the start of each sublattice phase.  On films with at most one
# site per sublattice this is serial Metropolis on the Hamiltonian of Eq. (7),
# whose Gibbs measure is then stationary; that, closed forms and symmetries
# pin the term's sign and its cases (|M| >= 2, M = 0, M = +-1).
_ANISO_CASES = ((1.5, 10, 30), (3.0, -40, 15), (0.7, 0, 8), (2.0, 5, 50))


def test_anisotropy_q_cases():
    """|M| >= 2: a flip of s changes q by h_an sign(M) s (an extra field along M);
    a flip that raises |M| from 0 or 1 lowers q by an_num; one that lowers |M| from 1 leaves it."""
    for a in (0, 7, 40):
        for M in range(-9, 10):
            for s in (-1, 1):
                q = ref.anisotropy_q(M, s, a)
                if abs(M) >= 2:
                    assert q == a * s * (1 if M > 0 else -1)
                elif abs(M - 2 * s) > abs(M):
                    assert q == -a
                else:
                    assert q == 0


def test_anisotropy_transition_matrices():
    for (h, Z) in _pair_and_triangle():
        film = ref.TinyFilm(h, Z)
        for T, hn, an in _ANISO_CASES:
            states, pi = ref.boltzmann(film, T, hn, an)
            _, pi0 = ref.boltzmann(film, T, hn)
            assert np.max(np.abs(pi - pi0)) > 1e-3  # the term matters here
            for sigma in range(4):
                for quant, tol in ((False, 1e-15), (True, 2.0**-31)):
                    P = ref.phase_matrix(film, T, hn, sigma, quantised=quant, an_num=an)
                    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-15)
                    flow = pi[:, None] * P
                    assert np.max(np.abs(flow - flow.T)) <= tol
            S = ref.sweep_matrix(film, T, hn, quantised=False, an_num=an)
            assert np.max(np.abs(pi @ S - pi)) <= 1e-14


def test_anisotropy_transition_frequencies_sampled(oracle_lib):
    """One-sweep frequencies of the C oracle with anisotropy against the quantised sweep matrix."""
    h, Z = _pair_and_triangle()[1]
    film = ref.TinyFilm(h, Z)
    T, hn, an = 2.5, -5, 40
    S = ref.sweep_matrix(film, T, hn, quantised=True, an_num=an)
    S0 = ref.sweep_matrix(film, T, hn, quantised=True)
    states = [tuple(s) for s in __import__("itertools").product((-1, 1), repeat=film.N)]
    idx = {s: a for a, s in enumerate(states)}
    start = (1, -1, -1)  # M = -1 when the first phase starts
    assert np.max(np.abs(S[idx[start]] - S0[idx[start]])) > 0.2  # the term changes this row
    f = cpu.Film(h, Z, seed=5151, replica=7)
    cube = np.zeros((Z, 4, 4), dtype=np.int8)
    for i, (x, y, z) in enumerate(film.sites):
        cube[z, y, x] = start[i]
    nsamp = 60000
    counts = np.zeros(len(states))
    for t in range(nsamp):
        f.set_spins(cube, t)
        f.run(T, hn, 1, 0, 0, an)
        sp = f.spins()
        counts[idx[tuple(int(sp[z, y, x]) for (x, y, z) in film.sites)]] += 1
    p = S[idx[start]]
    sd = np.sqrt(nsamp * p * (1 - p)) + 1e-9
    assert np.all(np.abs(counts - nsamp * p) <= 5 * sd + 1), (counts, nsamp * p)
    assert counts[p == 0].sum() == 0


def test_anisotropy_two_free_spins_closed_form(oracle_lib):
    """Two unbonded spins in different sublattices: the C oracle's long-run <M> and <|M|>
    against the closed form of the Gibbs measure of Eq. (7)."""
    h = np.zeros((8, 8), dtype=np.uint8)
    h[0, 0] = 1   # (0, 0, 0), sublattice 0
    h[3, 3] = 1   # (3, 3, 0), sublattice 1, not a neighbour
    T, hn, an = 1.0, 5, 10
    f = cpu.Film(h, 1, seed=31, init=cpu.INIT_UP)
    assert f.state()[2] == 2 and f.state()[3] == 0
    m_ex, a_ex = physics.two_free_spins_with_anisotropy(hn / 20, an / 20, T)
    m_free, _ = physics.two_free_spins_with_anisotropy(hn / 20, 0.0, T)
    assert abs(m_ex - m_free) > 0.15
    nblk, blk = 40, 20000
    ms, As = [], []
    for _ in range(nblk):
        r = f.run(T, hn, blk, 0, 0, an)
        ms.append(r.sum_M / blk)
        As.append(r.sum_absM / blk)
    for vals, ex in ((ms, m_ex), (As, a_ex)):
        se = np.std(vals, ddof=1) / math.sqrt(nblk)
        assert abs(np.mean(vals) - ex) <= 5 * se + 1e-4, (np.mean(vals), ex)


def test_anisotropy_exact_enumeration(oracle_lib):
    """Triangle (one site per sublattice): time averages of the C oracle equal the Gibbs
    averages of the Hamiltonian of Eq. (7) by exact enumeration."""
    h, Z = _pair_and_triangle()[1]
    tf = ref.TinyFilm(h, Z)
    T, hn, an = 2.0, 6, 24
    ex = ref.enumerate_exact(tf, T, hn, an)
    ex0 = ref.enumerate_exact(tf, T, hn)
    assert abs(ex["absM"] - ex0["absM"]) > 0.1
    f = cpu.Film(h, Z, seed=0xA11, replica=2)
    f.run(T, hn, 1000, 0, 0, an)
    nblk, blk = 40, 10000
    ms, As = [], []
    for _ in range(nblk):
        r = f.run(T, hn, blk, 0, 0, an)
        ms.append(r.sum_M / blk)
        As.append(r.sum_absM / blk)
    for vals, key in ((ms, "M"), (As, "absM")):
        se = float(np.std(vals, ddof=1) / math.sqrt(nblk))
        assert abs(float(np.mean(vals)) - ex[key]) <= 5.0 * se + 1e-3, (key, np.mean(vals), ex[key])


@pytest.mark.parametrize("seed", [0, 1])
def test_anisotropy_c_oracle_matches_python_oracle(oracle_lib, seed):
    rng = np.random.default_rng(700 + seed)
    Y, X, Z = [(8, 8, 3), (6, 10, 4)][seed]
    h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
    key = int(rng.integers(0, 2**63))
    tf = ref.TinyFilm(h, Z, seed=key, replica=seed)
    tf.init_random()
    cf = cpu.Film(h, Z, key, seed, init=cpu.INIT_RANDOM)
    for T, hn, hs, an in ((2.5, 20, 0, 40), (1.1, -7, 160, 12), (6.0, 0, 0, 100), (0.9, 55, 3, 5),
                          (4.0, -30, 0, 60)):
        acc = sum(tf.sweep(T, hn, hs, an) for _ in range(4))
        r = cf.run(T, hn, 4, 0, hs, an)
        sp = cf.spins()
        assert all(sp[z, y, x] == tf.s[i] for i, (x, y, z) in enumerate(tf.sites))
        assert r.M == tf.magnetisation() and r.E == tf.bond_energy() and r.accepted == acc


@pytest.mark.parametrize("init", [cpu.INIT_UP, cpu.INIT_RANDOM])
def test_anisotropy_field_reversal_symmetry(oracle_lib, init):
    """The term is even in M, so H -> -H with all spins reversed mirrors the run bit for bit."""
    rng = np.random.default_rng(6)
    h = rng.integers(0, 5, size=(24, 16)).astype(np.uint8)
    a = cpu.Film(h, 4, seed=778, replica=3, init=init)
    b = cpu.Film(h, 4, seed=778, replica=3, init=cpu.INIT_DOWN)
    b.set_spins(-a.spins(), 0)
    for hn, an in ((40, 20), (10, 60), (-20, 5), (-60, 200), (0, 30), (33, 1)):
        ra = a.run(3.5, hn, 3, 0, 0, an).as_tuple()
        rb = b.run(3.5, -hn, 3, 0, 0, an).as_tuple()
        assert np.array_equal(b.spins(), -a.spins())
        assert rb == (-ra[0], ra[1], -ra[2], ra[3], ra[4], ra[5])


def test_anisotropy_is_a_field_shift_while_the_excess_lasts(oracle_lib):
    """With |M| >= 2 at every phase start the term acts as the field h_an sign(M): the run
    equals the run without it at h_num + an_num sign(M), bit for bit."""
    rng = np.random.default_rng(10)
    h = rng.integers(0, 5, size=(32, 32)).astype(np.uint8)
    for init, sign in ((cpu.INIT_UP, 1), (cpu.INIT_DOWN, -1)):
        a = cpu.Film(h, 4, seed=55, init=init)
        b = cpu.Film(h, 4, seed=55, init=init)
        N = a.state()[2]
        for _ in range(15):
            ra = a.run(2.0, 4 * sign, 1, 0, 0, 30)
            rb = b.run(2.0, 4 * sign + 30 * sign, 1)
            assert ra.as_tuple() == rb.as_tuple()
            assert np.array_equal(a.spins(), b.spins())
            # M far from 0: no phase can reach |M| < 2
            assert sign * ra.M > N // 2
        assert ra.accepted > 0


def test_anisotropy_supports_the_spin_excess_at_low_temperature(oracle_lib):
    """T -> 0, free spins magnetised up in a reversed field: with h_an > |H| the excess holds
    (the move costs 2 (h_an - |H|) > 0), without the term every spin flips in the first sweep."""
    h = np.zeros((8, 8), dtype=np.uint8)
    for (y, x) in ((0, 0), (3, 3), (4, 0), (0, 4), (6, 2), (3, 5)):
        h[y, x] = 1
    f = cpu.Film(h, 1, seed=3, init=cpu.INIT_UP)
    N, n_bonds = f.state()[2], f.state()[3]
    assert N == 6 and n_bonds == 0
    r = f.run(1e-3, -10, 5, 0, 0, 20)
    assert r.M == N and r.accepted == 0
    r = f.run(1e-3, -10, 1, 0, 0, 0)
    assert r.M == -N and r.accepted == N


# --------------------------------------------------------------------------- discarded sweeps
# A run of n sweeps at one (T, H) keeps the sums of M, |M|, E_bond and the accepted
# flips over its last n - d sweeps only: the first d are equilibration (Section 3:
# a fixed number of Monte Carlo steps per temperature or field step; the M(T)
# curve of Fig. 3 averages after it).  The pins below fix that window by its
# definition: one-sweep runs (d = 0, whose M and E_bond are the recount's) summed
# by hand over i >= d, a second implementation, and the split of a run at d.
WINDOWS = [(12, 0), (12, 1), (12, 5), (12, 11), (12, 12), (1, 0), (1, 1), (40, 8)]


@pytest.mark.parametrize("n,d", WINDOWS)
def test_discard_window_is_the_sum_over_the_later_sweeps(oracle_lib, n, d):
    rng = np.random.default_rng(31 + n + 100 * d)
    Y, X, Z = 24, 40, 4
    h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
    T, hn = 3.5, 7   # hot enough that M, E_bond and the accepted count change every sweep
    a = cpu.Film(h, Z, 0xABCDEF, 3, init=cpu.INIT_RANDOM)
    b = cpu.Film(h, Z, 0xABCDEF, 3, init=cpu.INIT_RANDOM)
    a.run(T, hn, 3)   # the window is relative to the call, not to the chain's start
    b.run(T, hn, 3)
    rec = a.run(T, hn, n, d).as_tuple()
    per = []
    for _ in range(n):
        r = b.run(T, hn, 1, 0)
        assert (r.M, r.E) == b.recount()
        assert (r.sum_M, r.sum_absM, r.sum_E) == (r.M, abs(r.M), r.E)
        per.append(r)
    kept = per[d:]
    want = (per[-1].M, per[-1].E, sum(r.M for r in kept), sum(abs(r.M) for r in kept), sum(r.E for r in kept),
            sum(r.accepted for r in kept))
    assert rec == want
    assert len({r.accepted for r in per}) > 1 or n == 1
    np.testing.assert_array_equal(a.spins(), b.spins())
    assert a.state() == b.state()


@pytest.mark.parametrize("n,d", [(6, 0), (6, 2), (6, 6), (5, 4)])
def test_discard_window_c_matches_python(oracle_lib, n, d):
    rng = np.random.default_rng(77 + d)
    Y, X, Z = 6, 10, 3
    h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
    key, rep = 0x1234_5678_9ABC, 5
    tf = ref.TinyFilm(h, Z, seed=key, replica=rep)
    tf.init_random()
    cf = cpu.Film(h, Z, key, rep, init=cpu.INIT_RANDOM)
    for T, hn, hs, an in ((2.0, 11, 0, 0), (5.0, -3, 40, 0), (1.5, 0, 0, 20)):
        rp = tf.run(T, hn, n, d, hs, an)
        rc = cf.run(T, hn, n, d, hs, an).as_tuple()
        assert rp == rc, (T, hn, hs, an)
    sp = cf.spins()
    assert all(sp[z, y, x] == tf.s[i] for i, (x, y, z) in enumerate(tf.sites))


def test_discard_window_splits_the_run(oracle_lib):
    """run(n, d) == run(d, d) followed by run(n - d, 0): the discarded sweeps advance
    the chain and contribute nothing; the kept ones are the whole second run.  Also
    the temperature-scan shape (discard per temperature, chain continued across)."""
    from isf_workloads import config_plain_tscan

    c = config_plain_tscan()
    rng = np.random.default_rng(5)
    Y, X, Z = 32, 32, c.Z
    h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
    a = cpu.Film(h, Z, c.mc_seed, init=cpu.INIT_RANDOM)
    b = cpu.Film(h, Z, c.mc_seed, init=cpu.INIT_RANDOM)
    n, d = 25, 5
    temps = c.temps[::11]
    got = cpu.tscan(a, temps, n, d)
    for i, T in enumerate(temps):
        head = b.run(T, 0, d, d).as_tuple()
        assert head[2:] == (0, 0, 0, 0)
        tail = b.run(T, 0, n - d, 0).as_tuple()
        assert tuple(got[i]) == tail, T
    np.testing.assert_array_equal(a.spins(), b.spins())
    assert a.state() == b.state()
