"""ctypes declarations of the C ABI in include/isf.h.

Argument marshalling only.  Loading fails loudly if libisf.so has not been
built: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libisf.so")

ISF_OK, ISF_EINVAL, ISF_ENOSPC, ISF_EHIP, ISF_ESTATE = 0, -1, -2, -3, -4
FORMAT_INT8, FORMAT_BITPACK = 0, 1
INIT_UP, INIT_DOWN, INIT_RANDOM = 0, 1, 2
BATCH_PHASE_LAUNCH, BATCH_PERSISTENT, BATCH_WHOLE, BATCH_PIPE = 0, 1, 2, 3
MAX_STEPS = 1024


class IsfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("isf error %d: %s" % (code, msg))
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("X", ctypes.c_uint32), ("Y", ctypes.c_uint32), ("Z", ctypes.c_uint32),
                ("replica", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("format", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class Record(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("E", ctypes.c_int64), ("sum_M", ctypes.c_int64),
                ("sum_absM", ctypes.c_int64), ("sum_E", ctypes.c_int64), ("accepted", ctypes.c_int64)]


class Step(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("h_num", ctypes.c_int32), ("n_sweeps", ctypes.c_uint32),
                ("n_discard", ctypes.c_uint32), ("hs_num", ctypes.c_int32), ("an_num", ctypes.c_int32)]


class FilmStats(ctypes.Structure):
    _fields_ = [("n_occ", ctypes.c_int64), ("n_bonds", ctypes.c_int64), ("mean_coordination", ctypes.c_double),
                ("p_c", ctypes.c_double), ("concentration", ctypes.c_double)]


class Obs(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("E", ctypes.c_int64), ("n_occ", ctypes.c_int64),
                ("n_bonds", ctypes.c_int64), ("sweeps", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_uint32), ("tile_y", ctypes.c_uint32), ("rows_per_thread", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("kernel", ctypes.c_uint32)]


KERNEL_TILES, KERNEL_LIST, KERNEL_SWEEP, KERNEL_PIPE, KERNEL_FILM = 0, 1, 2, 3, 4


EXPORTS = {
    "isf_abi_version": (ctypes.c_int32, []),
    "isf_last_error": (ctypes.c_char_p, []),
    "isf_lattice_bytes": (ctypes.c_int32, [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_uint64)]),
    "isf_lattice_create": (ctypes.c_int32, [ctypes.POINTER(Desc), ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_void_p)]),
    "isf_lattice_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "isf_run_schedule": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Step), ctypes.c_uint32,
                                          ctypes.POINTER(Record)]),
    "isf_run_sweeps": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.POINTER(Record)]),
    "isf_ramp_field": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(Record)]),
    "isf_temperature_scan": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_uint32,
                                              ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32,
                                              ctypes.POINTER(Record)]),
    "isf_read_observables": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Obs)]),
    "isf_read_spins": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "isf_write_spins": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]),
    "isf_threshold_table": (ctypes.c_int32, [ctypes.c_double, ctypes.c_int32, ctypes.c_void_p]),
    "isf_gate_threshold": (ctypes.c_int32, [ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint32)]),
    "isf_surface_image": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]),
    "isf_film_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "isf_set_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "isf_get_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "isf_schedule_load": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Step), ctypes.c_uint32]),
    "isf_advance": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]),
    "isf_schedule_remaining": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "isf_schedule_records": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Record), ctypes.c_uint32]),
    "isf_batch_workspace_bytes": (ctypes.c_int32, [ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]),
    "isf_batch_create": (ctypes.c_int32, [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "isf_batch_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "isf_batch_advance": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32,
                                           ctypes.c_uint32, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "isf_batch_sync": (ctypes.c_int32, [ctypes.c_void_p]),
    "isf_batch_run": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32,
                                       ctypes.POINTER(ctypes.POINTER(Step)), ctypes.POINTER(ctypes.c_uint32),
                                       ctypes.POINTER(ctypes.POINTER(Record)), ctypes.c_int32]),
    "isf_recount_films": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "isf_draw_xor": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_float)]),
    "isf_time_launches": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_uint32)]),
    "isf_aniso_workspace_bytes": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "isf_attach_aniso_workspace": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]),
    "isf_aniso_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "isf_items_bytes": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "isf_attach_items": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]),
    "isf_recount": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64)]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libisf.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libisf.so is not built (%s); run paper_1205_5588_amd/build.py" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc: int) -> None:
    if rc != ISF_OK:
        raise IsfError(rc, load().isf_last_error().decode("utf-8", "replace"))
