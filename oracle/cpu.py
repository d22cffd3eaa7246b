"""ctypes wrapper of the plain C oracle (test infrastructure only).

Drives the dynamics the way the paper's experiments do: a field-reversal
hysteresis ramp at fixed T (Fig. 5, Section 6) or a temperature scan at
H = 0 (Fig. 3, Section 4), with a finite number of sweeps per field or
temperature step (Section 3).
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

from .build import build_oracle, oracle_lib_path

INIT_UP, INIT_DOWN, INIT_RANDOM = 0, 1, 2

_lib = None


class Record(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("E", ctypes.c_int64), ("sum_M", ctypes.c_int64),
                ("sum_absM", ctypes.c_int64), ("sum_E", ctypes.c_int64), ("accepted", ctypes.c_int64)]

    def as_tuple(self):
        return (self.M, self.E, self.sum_M, self.sum_absM, self.sum_E, self.accepted)


def lib():
    global _lib
    if _lib is None:
        path = oracle_lib_path()
        src = os.path.join(os.path.dirname(path), "isf_oracle.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            build_oracle()
        L = ctypes.CDLL(path)
        L.orc_film_new.restype = ctypes.c_void_p
        L.orc_film_new.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_uint64, ctypes.c_uint32]
        L.orc_film_free.argtypes = [ctypes.c_void_p]
        L.orc_init.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_set_order.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_run.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_uint32,
                              ctypes.c_uint32, ctypes.POINTER(Record)]
        L.orc_run.restype = ctypes.c_int
        L.orc_run_gated.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
        L.orc_run_gated.restype = ctypes.c_int
        L.orc_run_full.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
        L.orc_run_full.restype = ctypes.c_int
        L.orc_gate_threshold.argtypes = [ctypes.c_int32, ctypes.c_double]
        L.orc_gate_threshold.restype = ctypes.c_uint32
        L.orc_surface_image.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_get_spins.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_set_spins.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]
        L.orc_set_spins.restype = ctypes.c_int
        L.orc_state.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_recount.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.orc_threshold_table.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.c_void_p]
        L.orc_threshold.argtypes = [ctypes.c_int32, ctypes.c_double]
        L.orc_threshold.restype = ctypes.c_uint32
        L.orc_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def philox(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def threshold_table(T: float, h_num: int) -> np.ndarray:
    """uint32 array [2][25]: [s > 0][n + 12] -> threshold of q = s (20 n + h_num)."""
    out = np.zeros((2, 25), dtype=np.uint32)
    lib().orc_threshold_table(float(T), int(h_num), out.ctypes.data)
    return out


def gate_threshold(T: float, hs_num: int) -> int:
    return int(lib().orc_gate_threshold(int(hs_num), float(T)))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def threads() -> int:
    return int(lib().orc_threads())


class Film:
    """One film (one replica) in the oracle."""

    def __init__(self, h: np.ndarray, Z: int, seed: int, replica: int = 0, init: int = INIT_UP):
        h = np.ascontiguousarray(h, dtype=np.uint8)
        self.Y, self.X = h.shape
        self.Z = int(Z)
        self._h = h
        self._p = lib().orc_film_new(self.X, self.Y, self.Z, h.ctypes.data, int(seed) & (2**64 - 1),
                                     int(replica))
        if not self._p:
            raise ValueError("oracle: invalid film (X, Y must be even and >= 4, Z >= 1)")
        lib().orc_init(self._p, int(init))

    def __del__(self):
        p = getattr(self, "_p", None)
        if p:
            lib().orc_film_free(p)
            self._p = None

    def set_order(self, order: int) -> None:
        lib().orc_set_order(self._p, int(order))

    def run(self, T: float, h_num: int, n_sweeps: int, n_discard: int = 0, hs_num: int = 0,
            an_num: int = 0) -> Record:
        """n_sweeps sweeps at (T, H = h_num/20), behind the switching-field gate of h_s = hs_num/20,
        with the anisotropy field h_an = an_num/20 of Eq. (7) (M frozen per sublattice phase)."""
        r = Record()
        rc = lib().orc_run_full(self._p, float(T), int(h_num), int(hs_num), int(an_num), int(n_sweeps),
                                int(n_discard), ctypes.byref(r))
        if rc != 0:
            raise ValueError("oracle: invalid run arguments")
        return r

    def spins(self) -> np.ndarray:
        out = np.zeros((self.Z, self.Y, self.X), dtype=np.int8)
        lib().orc_get_spins(self._p, out.ctypes.data)
        return out

    def set_spins(self, cube: np.ndarray, t: int) -> None:
        cube = np.ascontiguousarray(cube, dtype=np.int8)
        if cube.shape != (self.Z, self.Y, self.X):
            raise ValueError("oracle: cube shape mismatch")
        if lib().orc_set_spins(self._p, cube.ctypes.data, int(t)) != 0:
            raise ValueError("oracle: occupied sites must hold +-1")

    def surface_image(self) -> np.ndarray:
        """Simulated PMOKE image [Y][X]: +1 / -1 = spin of the column's top occupied site, 0 = none."""
        out = np.zeros((self.Y, self.X), dtype=np.int8)
        lib().orc_surface_image(self._p, out.ctypes.data)
        return out

    def film_stats(self) -> dict:
        """Mean coordination z = 2 N_bonds / N_occ and the critical concentration p_c = 2/z of Eq. (2)."""
        _, _, n_occ, n_bonds, _ = self.state()
        z = 2.0 * n_bonds / n_occ if n_occ else 0.0
        return {"n_occ": n_occ, "n_bonds": n_bonds, "mean_coordination": z, "p_c": 2.0 / z if z else float("inf")}

    def state(self):
        """(M, E_bond, N_occ, N_bonds, sweeps done)."""
        out = np.zeros(5, dtype=np.int64)
        lib().orc_state(self._p, out.ctypes.data)
        return tuple(int(v) for v in out)

    def recount(self):
        M = ctypes.c_int64()
        E = ctypes.c_int64()
        lib().orc_recount(self._p, ctypes.byref(M), ctypes.byref(E))
        return int(M.value), int(E.value)


def hysteresis(film: Film, T: float, h_nums: Sequence[int], sweeps_per_step: int,
               n_steps: Optional[int] = None) -> np.ndarray:
    """Field ramp: per step (M, E, sum_M, sum_absM, sum_E, accepted) after the step's sweeps."""
    steps = list(h_nums)[: n_steps] if n_steps is not None else list(h_nums)
    out = np.zeros((len(steps), 6), dtype=np.int64)
    for i, hn in enumerate(steps):
        out[i] = film.run(T, hn, sweeps_per_step, 0).as_tuple()
    return out


def tscan(film: Film, temps: Sequence[float], sweeps_per_T: int, discard_per_T: int,
          n_temps: Optional[int] = None) -> np.ndarray:
    """Temperature scan at H = 0: per T (M, E, sum_M, sum_absM, sum_E, accepted) over kept sweeps."""
    ts = list(temps)[: n_temps] if n_temps is not None else list(temps)
    out = np.zeros((len(ts), 6), dtype=np.int64)
    for i, T in enumerate(ts):
        out[i] = film.run(T, 0, sweeps_per_T, discard_per_T).as_tuple()
    return out
