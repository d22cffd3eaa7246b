"""Python binding: films on the GPU, with PyTorch owning device memory and streams.

Every Monte Carlo step runs in the HIP library (libisf.so); this module only
allocates torch tensors for the library's buffers, converts arguments and
results, and keeps the buffers alive as long as the handles.
"""

from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import (BATCH_PERSISTENT, BATCH_PHASE_LAUNCH, FORMAT_BITPACK, FORMAT_INT8, INIT_DOWN, INIT_RANDOM,
                   INIT_UP, KERNEL_LIST, KERNEL_TILES, MAX_STEPS, Desc, Obs, Record, Step, Tuning, check)

RECORD_FIELDS = ("M", "E", "sum_M", "sum_absM", "sum_E", "accepted")


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the isf library needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _records_array(recs) -> np.ndarray:
    return np.array([[r.M, r.E, r.sum_M, r.sum_absM, r.sum_E, r.accepted] for r in recs], dtype=np.int64).reshape(
        -1, 6)


def threshold_table(T: float, h_num: int) -> np.ndarray:
    """The library's acceptance thresholds [2][25] (computed on the host, no GPU needed)."""
    out = np.zeros((2, 25), dtype=np.uint32)
    check(_lib.load().isf_threshold_table(float(T), int(h_num), out.ctypes.data))
    return out


def lattice_bytes(X: int, Y: int, Z: int, fmt: int = FORMAT_INT8) -> Tuple[int, int]:
    d = Desc(X, Y, Z, 0, 0, fmt, 0)
    s = ctypes.c_uint64()
    a = ctypes.c_uint64()
    check(_lib.load().isf_lattice_bytes(ctypes.byref(d), ctypes.byref(s), ctypes.byref(a)))
    return int(s.value), int(a.value)


def make_steps(steps: Sequence[Tuple]):
    """steps: (T, h_num, n_sweeps, n_discard[, hs_num[, an_num]]) each; hs_num = 0 (no switching-field
    gate) and an_num = 0 (no anisotropy) if absent."""
    arr = (Step * max(1, len(steps)))()
    for i, st in enumerate(steps):
        T, h, n, nd = st[:4]
        hs = st[4] if len(st) > 4 else 0
        an = st[5] if len(st) > 5 else 0
        arr[i] = Step(float(T), int(h), int(n), int(nd), int(hs), int(an))
    return arr


class Lattice:
    """One film (one replica) resident on a GPU.

    heights: uint8 array [Y][X] with values in [0, Z]; occupied sites are
    (x, y, z) with x+y+z even and z < heights[y][x].
    """

    def __init__(self, heights: np.ndarray, Z: int, seed: int, replica: int = 0, init: int = INIT_UP,
                 fmt: int = FORMAT_INT8, device: Optional[str] = None, stream=None,
                 spin_buf=None, aux_buf=None, items: bool = False):
        torch = _torch()
        h = np.ascontiguousarray(heights, dtype=np.uint8)
        self.Y, self.X = h.shape
        self.Z = int(Z)
        self.fmt = int(fmt)
        self.seed = int(seed) & (2**64 - 1)
        self.replica = int(replica)
        self.device = torch.device(device or "cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._desc = Desc(self.X, self.Y, self.Z, self.replica, self.seed, self.fmt, 0)
        sb, ab = lattice_bytes(self.X, self.Y, self.Z, self.fmt)
        self.spin_bytes, self.aux_bytes = sb, ab
        # buffers may come from a caller's arena (serving); else allocate here
        self.spin_buf = spin_buf if spin_buf is not None else torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.aux_buf = aux_buf if aux_buf is not None else torch.empty(ab, dtype=torch.uint8, device=self.device)
        if self.spin_buf.numel() < sb or self.aux_buf.numel() < ab:
            raise ValueError("lattice buffers too small")
        # the buffers were allocated on torch's current stream; order the library's stream after it
        # (no device-wide synchronisation: other films may be running)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(_lib.load().isf_lattice_create(ctypes.byref(self._desc), h.ctypes.data, int(init),
                                                 self.spin_buf.data_ptr(), sb, self.aux_buf.data_ptr(), ab,
                                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)))
        self._h = handle
        self._n_loaded = 0
        self.items_buf = None
        if items and self.fmt == FORMAT_INT8:
            self.attach_items()

    def attach_items(self) -> None:
        """Build the film's occupied-dword lists on the device and select the list kernel."""
        torch = _torch()
        nb = ctypes.c_uint64()
        check(_lib.load().isf_items_bytes(self.handle, ctypes.byref(nb)))
        self.items_buf = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        check(_lib.load().isf_attach_items(self.handle, self.items_buf.data_ptr(), int(nb.value)))

    def attach_aniso_workspace(self) -> None:
        """Device workspace that lets the whole-sweep kernels run schedules with the
        anisotropy term of Eq. 7 (steps run at field h + h_an sign(M) while |M| >= 2
        is certain, otherwise again on the per-sublattice kernels)."""
        torch = _torch()
        nb = ctypes.c_uint64()
        check(_lib.load().isf_aniso_workspace_bytes(self.handle, ctypes.byref(nb)))
        self.aniso_ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        check(_lib.load().isf_attach_aniso_workspace(self.handle, self.aniso_ws.data_ptr(), int(nb.value)))

    def aniso_stats(self) -> Tuple[int, int]:
        """(step parts run on the whole-sweep kernel, those of them run again per sublattice)."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        check(_lib.load().isf_aniso_stats(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    # ------------------------------------------------------------------ lifecycle
    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.load().isf_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("lattice closed")
        return self._h

    # ------------------------------------------------------------------ tuning
    def set_tuning(self, tile_x: int = 64, tile_y: int = 4, rows_per_thread: int = 2, use_graph: bool = True,
                   kernel: int = KERNEL_TILES):
        t = Tuning(tile_x, tile_y, rows_per_thread, 1 if use_graph else 0, int(kernel))
        check(_lib.load().isf_set_tuning(self.handle, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        check(_lib.load().isf_get_tuning(self.handle, ctypes.byref(t)))
        return (t.tile_x, t.tile_y, t.rows_per_thread, bool(t.use_graph), int(t.kernel))

    # ------------------------------------------------------------------ runs
    def run_schedule(self, steps: Sequence[Tuple[float, int, int, int]]) -> np.ndarray:
        """steps: (T, h_num, n_sweeps, n_discard[, hs_num[, an_num]]) each; returns int64 [n, 6] records."""
        n = len(steps)
        arr = make_steps(steps)
        out = (Record * max(1, n))()
        check(_lib.load().isf_run_schedule(self.handle, arr, n, out))
        return _records_array(out[:n])

    def run_sweeps(self, T: float, h_num: int, n_sweeps: int, n_discard: int = 0) -> np.ndarray:
        r = Record()
        check(_lib.load().isf_run_sweeps(self.handle, float(T), int(h_num), int(n_sweeps), int(n_discard),
                                         ctypes.byref(r)))
        return _records_array([r])[0]

    def ramp_field(self, T: float, h_nums: Sequence[int], sweeps_per_step: int) -> np.ndarray:
        n = len(h_nums)
        hs = (ctypes.c_int32 * max(1, n))(*[int(v) for v in h_nums])
        out = (Record * max(1, n))()
        check(_lib.load().isf_ramp_field(self.handle, float(T), hs, n, int(sweeps_per_step), out))
        return _records_array(out[:n])

    def temperature_scan(self, temps: Sequence[float], sweeps_per_T: int, discard_per_T: int,
                         h_num: int = 0) -> np.ndarray:
        n = len(temps)
        ts = (ctypes.c_double * max(1, n))(*[float(v) for v in temps])
        out = (Record * max(1, n))()
        check(_lib.load().isf_temperature_scan(self.handle, ts, n, int(h_num), int(sweeps_per_T),
                                               int(discard_per_T), out))
        return _records_array(out[:n])

    # incremental
    def schedule_load(self, steps: Sequence[Tuple[float, int, int, int]]) -> None:
        arr = make_steps(steps)
        check(_lib.load().isf_schedule_load(self.handle, arr, len(steps)))
        self._n_loaded = len(steps)

    def advance(self, max_sweeps: int) -> int:
        got = ctypes.c_uint64()
        check(_lib.load().isf_advance(self.handle, int(max_sweeps), ctypes.byref(got)))
        return int(got.value)

    def remaining(self) -> int:
        r = ctypes.c_uint64()
        check(_lib.load().isf_schedule_remaining(self.handle, ctypes.byref(r)))
        return int(r.value)

    def records(self, n: Optional[int] = None) -> np.ndarray:
        n = self._n_loaded if n is None else int(n)
        out = (Record * max(1, n))()
        check(_lib.load().isf_schedule_records(self.handle, out, n))
        return _records_array(out[:n])

    def time_launches(self, n_sweeps: int) -> Tuple[List[float], int]:
        """Run up to n_sweeps sweeps of the loaded schedule with HIP events around
        every sublattice launch; returns (mean ms per launch for each sublattice, sweeps run)."""
        ms = (ctypes.c_double * 4)()
        n = ctypes.c_uint32()
        check(_lib.load().isf_time_launches(self.handle, int(n_sweeps), ms, ctypes.byref(n)))
        return [float(v) for v in ms], int(n.value)

    def draw_xor(self, t0: int, n_sweeps: int) -> Tuple[int, float]:
        """Draw-only ceiling: every stored dword draws its attempt's Philox numbers for
        sweeps t0 .. t0 + n_sweeps - 1 and nothing else; returns (XOR of all words drawn,
        milliseconds of the launch).  The film is not changed."""
        torch = _torch()
        out = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        ms = ctypes.c_float()
        check(_lib.load().isf_draw_xor(self.handle, int(t0) & 0xFFFFFFFF, int(n_sweeps), out.data_ptr(),
                                       ctypes.byref(ms)))
        return int(out.cpu().item()) & 0xFFFFFFFF, float(ms.value)

    # ------------------------------------------------------------------ state
    def observables(self) -> dict:
        o = Obs()
        check(_lib.load().isf_read_observables(self.handle, ctypes.byref(o)))
        return {"M": o.M, "E": o.E, "n_occ": o.n_occ, "n_bonds": o.n_bonds, "sweeps": o.sweeps}

    def recount(self) -> Tuple[int, int]:
        M = ctypes.c_int64()
        E = ctypes.c_int64()
        check(_lib.load().isf_recount(self.handle, ctypes.byref(M), ctypes.byref(E)))
        return int(M.value), int(E.value)

    def surface_image(self, out=None) -> np.ndarray:
        """Simulated PMOKE image [Y][X] int8 (+1 / -1 surface spin, 0 background) after the
        sweeps enqueued so far.  out: optional int8 CUDA tensor of X*Y elements to fill."""
        import torch

        img = out if out is not None else torch.empty(self.Y * self.X, dtype=torch.int8, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))  # the buffer's allocation
        check(_lib.load().isf_surface_image(self.handle, img.data_ptr(), img.numel()))
        if out is not None:
            return out
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return img.view(self.Y, self.X).cpu().numpy()

    def film_stats(self) -> dict:
        """Mean coordination 2 N_bonds / N_occ, p_c = 2/z (Eq. 2) and the occupied fraction."""
        st = _lib.FilmStats()
        check(_lib.load().isf_film_stats(self.handle, ctypes.byref(st)))
        return {"n_occ": st.n_occ, "n_bonds": st.n_bonds, "mean_coordination": st.mean_coordination,
                "p_c": st.p_c, "concentration": st.concentration}

    def spins(self) -> np.ndarray:
        out = np.zeros((self.Z, self.Y, self.X), dtype=np.int8)
        check(_lib.load().isf_read_spins(self.handle, out.ctypes.data))
        return out

    def set_spins(self, cube: np.ndarray, sweeps: int) -> None:
        cube = np.ascontiguousarray(cube, dtype=np.int8)
        if cube.shape != (self.Z, self.Y, self.X):
            raise ValueError("cube shape mismatch")
        check(_lib.load().isf_write_spins(self.handle, cube.ctypes.data, int(sweeps)))


class Batch:
    """Advance many lattices together (one launch per sublattice, or one persistent launch)."""

    def __init__(self, max_lats: int, device: Optional[str] = None, stream=None):
        torch = _torch()
        self.device = torch.device(device or "cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        nb = ctypes.c_uint64()
        check(_lib.load().isf_batch_workspace_bytes(int(max_lats), ctypes.byref(nb)))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(_lib.load().isf_batch_create(int(max_lats), self.ws.data_ptr(), int(nb.value),
                                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.max_lats = int(max_lats)

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().isf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def advance(self, lats: Sequence[Lattice], max_sweeps: int, mode: int = BATCH_PHASE_LAUNCH) -> int:
        arr = (ctypes.c_void_p * max(1, len(lats)))(*[l.handle for l in lats])
        got = ctypes.c_uint64()
        check(_lib.load().isf_batch_advance(self._h, arr, len(lats), int(max_sweeps), int(mode), ctypes.byref(got)))
        return int(got.value)

    def sync(self) -> None:
        check(_lib.load().isf_batch_sync(self._h))

    def run(self, lats: Sequence[Lattice], schedules: Sequence[Sequence[Tuple[float, int, int, int]]],
            mode: int = BATCH_PHASE_LAUNCH) -> List[np.ndarray]:
        n = len(lats)
        arr = (ctypes.c_void_p * max(1, n))(*[l.handle for l in lats])
        step_arrs = [make_steps(s) for s in schedules]
        outs = [(Record * max(1, len(s)))() for s in schedules]
        sp = (ctypes.POINTER(Step) * max(1, n))(*[ctypes.cast(a, ctypes.POINTER(Step)) for a in step_arrs])
        op = (ctypes.POINTER(Record) * max(1, n))(*[ctypes.cast(o, ctypes.POINTER(Record)) for o in outs])
        ns = (ctypes.c_uint32 * max(1, n))(*[len(s) for s in schedules])
        check(_lib.load().isf_batch_run(self._h, arr, n, sp, ns, op, int(mode)))
        for l, s in zip(lats, schedules):
            l._n_loaded = len(s)
        return [_records_array(o[:len(s)]) for o, s in zip(outs, schedules)]
