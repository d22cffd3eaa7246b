"""Second, pure-Python oracle for tiny films, plus exact results that pin the C oracle.

TEST INFRASTRUCTURE ONLY.  Written independently of isf_oracle.c (site
lists and explicit neighbour tables instead of a cube), so that the two can
check each other on small films.

Contents:
  philox4x32_10      -- Philox4x32-10 (Salmon et al., SC 2011) on Python ints
  threshold          -- Eq. (8) threshold floor(2^32 exp(-(q/10)/T)) via math.exp
  gate_threshold     -- Eq. (9) switching-field gate floor(2^32 exp(-|h_s|/T)), h_s = hs_num/20
  anisotropy_q       -- the change of the anisotropy energy -h_an |M| of Eq. (7)
                        for one flip, in tenths
  TinyFilm           -- the sweep of Section 5 (steps 1-3) on a site list, and a
                        run of sweeps at one (T, H) whose first sweeps are
                        discarded from the recorded sums
  enumerate_exact    -- partition function of Eq. (4) and Gibbs averages of
                        Eq. (5) by enumerating all 2^N configurations
  phase_matrix, sweep_matrix -- the Markov chain of Eq. (6) written as
                        transition matrices for 2-3 site systems
"""

from __future__ import annotations

import itertools
import math
from typing import Dict, List, Tuple

import numpy as np

M32 = 0xFFFFFFFF
_NB = [(dx, dy, 0) for dx in (1, -1) for dy in (1, -1)] + \
      [(dx, 0, dz) for dx in (1, -1) for dz in (1, -1)] + \
      [(0, dy, dz) for dy in (1, -1) for dz in (1, -1)]


def philox4x32_10(ctr, key):
    c = [int(v) & M32 for v in ctr]
    k0, k1 = int(key[0]) & M32, int(key[1]) & M32
    for _ in range(10):
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ c[3] ^ k1) & M32, p0 & M32]
        k0 = (k0 + 0x9E3779B9) & M32
        k1 = (k1 + 0xBB67AE85) & M32
    return c


def threshold(q: int, T: float) -> int:
    """32-bit acceptance threshold of a move with dE = q/10 (q <= 0: sentinel, always accepted)."""
    if q <= 0:
        return M32
    return int(math.floor(math.ldexp(math.exp(-(q / 10.0) / T), 32)))


def gate_threshold(hs_num: int, T: float) -> int:
    """32-bit threshold of the switching-field gate (hs_num = 0: sentinel, the gate always passes)."""
    if hs_num == 0:
        return M32
    return int(math.floor(math.ldexp(math.exp(-(abs(hs_num) / 20.0) / T), 32)))


def gate_probability(hs_num: int, T: float, quantised: bool = True) -> float:
    if hs_num == 0:
        return 1.0
    if quantised:
        return gate_threshold(hs_num, T) / 2.0**32
    return math.exp(-(abs(hs_num) / 20.0) / T)


def accept_probability(q: int, T: float, quantised: bool = True) -> float:
    """Probability that the rule accepts a move with dE = q/10."""
    if q <= 0:
        return 1.0
    if quantised:
        return threshold(q, T) / 2.0**32
    return math.exp(-(q / 10.0) / T)


def anisotropy_energy(M: int, an_num: int) -> float:
    """Anisotropy term of Eq. (7), -h_an |M| with h_an = an_num / 20."""
    return -(an_num / 20.0) * abs(M)


def anisotropy_q(M: int, s: int, an_num: int) -> int:
    """10 (E_an(M - 2s) - E_an(M)): the anisotropy part of q when spin s flips
    while the magnetisation is M.  |M - 2s| - |M| is even, so this is an integer."""
    return -(an_num * (abs(M - 2 * s) - abs(M))) // 2


class TinyFilm:
    """A film as an explicit list of occupied sites with neighbour lists."""

    def __init__(self, h: np.ndarray, Z: int, seed: int = 0, replica: int = 0):
        h = np.asarray(h)
        self.Y, self.X = h.shape
        self.Z = Z
        self.seed = int(seed)
        self.replica = int(replica)
        self.sites: List[Tuple[int, int, int]] = []
        for z in range(Z):
            for y in range(self.Y):
                for x in range(self.X):
                    if (x + y + z) % 2 == 0 and z < int(h[y, x]):
                        self.sites.append((x, y, z))
        index: Dict[Tuple[int, int, int], int] = {s: i for i, s in enumerate(self.sites)}
        self.nbrs: List[List[int]] = []
        for (x, y, z) in self.sites:
            lst = []
            for dx, dy, dz in _NB:
                zz = z + dz
                if not 0 <= zz < Z:
                    continue
                j = index.get(((x + dx) % self.X, (y + dy) % self.Y, zz))
                if j is not None:
                    lst.append(j)
            self.nbrs.append(lst)
        self.sub = [(y & 1) + 2 * (z & 1) for (x, y, z) in self.sites]
        self.bonds = sorted({(min(i, j), max(i, j)) for i in range(len(self.sites)) for j in self.nbrs[i]})
        self.s = [1] * len(self.sites)
        self.t = 0

    @property
    def N(self) -> int:
        return len(self.sites)

    def draw(self, i: int, t: int, tag: int) -> int:
        x, y, z = self.sites[i]
        k = (z * self.Y + y) * (self.X // 2) + x // 2
        ctr = (k >> 2, t & M32, self.replica, self.sub[i] + 4 * tag)
        key = (self.seed & M32, (self.seed >> 32) & M32)
        return philox4x32_10(ctr, key)[k & 3]

    def init_random(self) -> None:
        self.s = [1 if self.draw(i, 0, 1) < 0x80000000 else -1 for i in range(self.N)]
        self.t = 0

    def surface_image(self) -> np.ndarray:
        """PMOKE image from the site list: per column the site with the largest z."""
        img = np.zeros((self.Y, self.X), dtype=np.int8)
        top: Dict[Tuple[int, int], int] = {}
        for i, (x, y, z) in enumerate(self.sites):
            if (x, y) not in top or self.sites[top[(x, y)]][2] < z:
                top[(x, y)] = i
        for (x, y), i in top.items():
            img[y, x] = self.s[i]
        return img

    def mean_coordination(self) -> float:
        return 2.0 * len(self.bonds) / self.N if self.N else 0.0

    def magnetisation(self) -> int:
        return sum(self.s)

    def bond_energy(self) -> int:
        return -sum(self.s[i] * self.s[j] for i, j in self.bonds)

    def sweep(self, T: float, h_num: int, hs_num: int = 0, an_num: int = 0) -> int:
        """One sweep; with hs_num != 0 each attempt first passes the switching-field
        gate of Eq. (9) (steps 4-5 of Section 5) with its own draw (tag 2).  With
        an_num != 0 the anisotropy term of Eq. (7) enters with M frozen at its
        value when the sublattice's phase starts."""
        acc = 0
        g = gate_threshold(hs_num, T)
        for sigma in range(4):
            M = self.magnetisation()
            for i in range(self.N):
                if self.sub[i] != sigma:
                    continue
                if g != M32 and not self.draw(i, self.t, 2) < g:
                    continue
                n = sum(self.s[j] for j in self.nbrs[i])
                q = self.s[i] * (20 * n + h_num) + anisotropy_q(M, self.s[i], an_num)
                if q <= 0 or self.draw(i, self.t, 0) < threshold(q, T):
                    self.s[i] = -self.s[i]
                    acc += 1
        self.t += 1
        return acc

    def run(self, T: float, h_num: int, n_sweeps: int, n_discard: int = 0, hs_num: int = 0,
            an_num: int = 0) -> Tuple[int, int, int, int, int, int]:
        """n_sweeps sweeps at one (T, H); the first n_discard of them are equilibration
        (the fixed number of Monte Carlo steps per temperature or field step of
        Section 3, of which the M(T) curve of Fig. 3 keeps the later ones).  Returns
        (M, E_bond) after the last sweep and, over the kept sweeps only, the sums of M,
        |M| and E_bond taken after each sweep and the number of accepted flips."""
        if not 0 <= n_discard <= n_sweeps:
            raise ValueError("n_discard must lie in [0, n_sweeps]")
        kept_M = kept_absM = kept_E = kept_acc = 0
        for i in range(n_sweeps):
            acc = self.sweep(T, h_num, hs_num, an_num)
            if i < n_discard:
                continue
            m = self.magnetisation()
            kept_M += m
            kept_absM += abs(m)
            kept_E += self.bond_energy()
            kept_acc += acc
        return (self.magnetisation(), self.bond_energy(), kept_M, kept_absM, kept_E, kept_acc)


def enumerate_exact(film: TinyFilm, T: float, h_num: int, an_num: int = 0):
    """Exact Gibbs averages over all 2^N configurations (Eqs. 4-5 with J = k = 1, H = h_num/20,
    and the anisotropy term -h_an |M| of Eq. (7) with h_an = an_num/20).

    Returns dict with Z (partition function), <M>, <M^2>, <|M|>, <E_bond>, <E_total>.
    """
    N = film.N
    if N > 22:
        raise ValueError("enumerate_exact: too many sites")
    codes = np.arange(2**N, dtype=np.int64)
    spins = ((codes[:, None] >> np.arange(N)[None, :]) & 1).astype(np.int64) * 2 - 1
    M = spins.sum(axis=1)
    Eb = np.zeros(2**N, dtype=np.int64)
    for i, j in film.bonds:
        Eb -= spins[:, i] * spins[:, j]
    H = h_num / 20.0
    E = Eb - H * M - (an_num / 20.0) * np.abs(M)
    w = np.exp(-(E - E.min()) / T)
    Zp = w.sum()
    p = w / Zp
    return {
        "Z": float(Zp * math.exp(-E.min() / T)),
        "M": float((p * M).sum()),
        "M2": float((p * M * M).sum()),
        "absM": float((p * np.abs(M)).sum()),
        "E_bond": float((p * Eb).sum()),
        "E": float((p * E).sum()),
    }


def boltzmann(film: TinyFilm, T: float, h_num: int, an_num: int = 0) -> Tuple[List[Tuple[int, ...]], np.ndarray]:
    states = list(itertools.product((-1, 1), repeat=film.N))
    H = h_num / 20.0
    E = []
    for st in states:
        eb = -sum(st[i] * st[j] for i, j in film.bonds)
        E.append(eb - H * sum(st) + anisotropy_energy(sum(st), an_num))
    E = np.array(E)
    w = np.exp(-(E - E.min()) / T)
    return states, w / w.sum()


def phase_matrix(film: TinyFilm, T: float, h_num: int, sigma: int, quantised: bool = True,
                 hs_num: int = 0, an_num: int = 0) -> np.ndarray:
    """Transition matrix of one sublattice phase: its sites are updated independently;
    a site flips if its switching-field gate (probability g) and the Metropolis test pass.
    The anisotropy term sees the magnetisation of the state the phase starts from."""
    g = gate_probability(hs_num, T, quantised)
    states = list(itertools.product((-1, 1), repeat=film.N))
    idx = {st: a for a, st in enumerate(states)}
    P = np.zeros((len(states), len(states)))
    members = [i for i in range(film.N) if film.sub[i] == sigma]
    for a, st in enumerate(states):
        # each member flips independently with its own acceptance probability
        probs = []
        M = sum(st)
        for i in members:
            n = sum(st[j] for j in film.nbrs[i])
            q = st[i] * (20 * n + h_num) + anisotropy_q(M, st[i], an_num)
            probs.append(g * accept_probability(q, T, quantised))
        for flips in itertools.product((0, 1), repeat=len(members)):
            pr = 1.0
            new = list(st)
            for f, i, pi in zip(flips, members, probs):
                pr *= pi if f else (1.0 - pi)
                if f:
                    new[i] = -new[i]
            P[a, idx[tuple(new)]] += pr
    return P


def sweep_matrix(film: TinyFilm, T: float, h_num: int, quantised: bool = True, hs_num: int = 0,
                 an_num: int = 0) -> np.ndarray:
    P = np.eye(2**film.N)
    for sigma in range(4):
        P = P @ phase_matrix(film, T, h_num, sigma, quantised, hs_num, an_num)
    return P
