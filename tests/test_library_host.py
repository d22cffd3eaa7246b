"""Host-side checks of the HIP library (no GPU needed): it loads, exports
every symbol include/isf.h declares, validates descriptions, and its
threshold tables equal the oracle's for every (T, h_num) the workloads use."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import cpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1205_5588_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_1205_5588_amd.build import build

        build()
    return _lib.load()


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "isf.h")).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)  # declarations only, not the comments
    return sorted(set(re.findall(r"\b(isf_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    syms = _declared_symbols()
    assert len(syms) >= 25
    for s in syms:
        assert hasattr(lib, s), s
    from paper_1205_5588_amd import _lib

    assert set(syms) == set(_lib.EXPORTS), set(syms) ^ set(_lib.EXPORTS)
    assert lib.isf_abi_version() == 2


def _bytes(lib, X, Y, Z, fmt=0, reserved=0):
    from paper_1205_5588_amd._lib import Desc

    d = Desc(X, Y, Z, 0, 0, fmt, reserved)
    s = ctypes.c_uint64()
    a = ctypes.c_uint64()
    rc = lib.isf_lattice_bytes(ctypes.byref(d), ctypes.byref(s), ctypes.byref(a))
    return rc, s.value, a.value


def test_descriptor_validation(lib):
    rc, s, a = _bytes(lib, 2048, 2048, 8)
    assert rc == 0 and s == 10 * 2048 * 1024 and a > 0
    rc, s, _ = _bytes(lib, 2048, 2048, 8, fmt=1)
    assert rc == 0 and s == 10 * 2048 * 2 * 32 * 4
    for bad in [(4, 8, 2), (12, 8, 2), (16, 6, 0), (16, 7, 2), (16, 2, 2), (16, 8, 65)]:
        assert _bytes(lib, *bad)[0] == -1, bad
    assert _bytes(lib, 12, 8, 2, fmt=1)[0] == -1      # BITPACK too needs X % 8 == 0
    # BITPACK rows of W = X/2 sites take ceil(W/32) words per bit plane: X = 72 -> 36 sites -> 2 words
    rc, s, _ = _bytes(lib, 72, 8, 2, fmt=1)
    assert rc == 0 and s == 4 * 8 * 2 * 2 * 4
    assert _bytes(lib, 64, 8, 2, fmt=2)[0] == -1      # unknown format
    assert _bytes(lib, 64, 8, 2, reserved=1)[0] == -1
    assert b"Z=65" in lib.isf_last_error() or b"reserved" in lib.isf_last_error()


def test_threshold_validation(lib):
    out = np.zeros((2, 25), dtype=np.uint32)
    for T in (0.0, -1.0, float("inf"), float("nan"), 2e6):
        assert lib.isf_threshold_table(T, 0, out.ctypes.data) == -1
    assert lib.isf_threshold_table(1.0, 200001, out.ctypes.data) == -1
    assert lib.isf_threshold_table(1.0, 200000, out.ctypes.data) == 0


def _workload_pairs():
    from isf_workloads import (batched_films, config_plain_hysteresis_large, config_plain_hysteresis_small,
                               config_plain_tscan, serving_requests)

    pairs = set()
    for c in (config_plain_hysteresis_small(), config_plain_hysteresis_large()):
        pairs |= {(c.T, h) for h in c.h_nums}
    pairs |= {(T, 0) for T in config_plain_tscan().temps}
    reps, _, hn, _ = batched_films()
    for r in reps[::16]:
        pairs |= {(r.T, h) for h in hn}
    for q in serving_requests(max_requests=40):
        if q.kind == "hysteresis":
            pairs |= {(q.T, h) for h in q.h_nums[::10]}
        else:
            pairs |= {(T, 0) for T in q.temps}
    pairs |= {(1e-3, 1), (1e-3, 241), (50.0, 0), (1e6, -200000)}
    return sorted(pairs)


def test_threshold_tables_equal_oracle(lib, oracle_lib):
    pairs = _workload_pairs()
    assert len(pairs) > 1000
    out = np.zeros((2, 25), dtype=np.uint32)
    for T, h in pairs:
        assert lib.isf_threshold_table(float(T), int(h), out.ctypes.data) == 0
        np.testing.assert_array_equal(out, cpu.threshold_table(T, h), err_msg=str((T, h)))


def test_gate_thresholds_equal_oracle(lib, oracle_lib):
    """Switching-field gate thresholds (Eq. 9) of the library against the oracle's."""
    import ctypes

    out = ctypes.c_uint32()
    for T in (1e-3, 0.5, 1.0, 2.0, 3.0, 4.0, 9.0, 12.0, 1e6):
        for hs in (0, 1, -1, 7, 40, 80, 160, -160, 200000):
            assert lib.isf_gate_threshold(float(T), int(hs), ctypes.byref(out)) == 0
            assert out.value == cpu.gate_threshold(T, hs), (T, hs)
    assert lib.isf_gate_threshold(1.0, 200001, ctypes.byref(out)) == -1
    assert lib.isf_gate_threshold(0.0, 40, ctypes.byref(out)) == -1
    assert lib.isf_gate_threshold(1.0, 40, None) == -1


def test_default_tuning_takes_the_film_kernel_where_resident():
    """Small INT8 films run on the film kernel by default only where every sublattice
    fits one dword per thread (the kernel's 512 threads); bit-packed films never."""
    from paper_1205_5588_amd._lib import FORMAT_BITPACK, FORMAT_INT8, KERNEL_FILM
    from paper_1205_5588_amd.autotune import default_tuning, film_resident

    assert film_resident(64, 64, 3)  # 2 planes x 32 rows x 8 dwords = 512
    assert not film_resident(64, 66, 3)
    assert not film_resident(72, 38, 5)  # 3 x 19 x 9 = 513
    assert film_resident(512, 12, 1) and film_resident(8, 4, 1)
    assert default_tuning(64, 64, 3, FORMAT_INT8) == (512, 1, 1, False, KERNEL_FILM)
    assert default_tuning(64, 64, 3, FORMAT_BITPACK)[4] != KERNEL_FILM
    assert default_tuning(2048, 2048, 8, FORMAT_INT8)[4] != KERNEL_FILM
    assert default_tuning(72, 38, 5, FORMAT_INT8)[4] != KERNEL_FILM
