"""GPU: the allocation-free recount (isf_recount_films, for callers that cannot
allocate) equals isf_recount film by film, called through the C ABI: two calls
in a row, the second on fewer films after more sweeps, so counters left by the
first call would show."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def isf():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1205_5588_amd import lattice

    return lattice


def _films(isf):
    rng = np.random.default_rng(2024)
    out = []
    for i, (X, Y, Z, fmt, tuning) in enumerate([(72, 38, 5, 0, None), (352, 48, 4, 0, (32, 32, 16, True, 3)),
                                               (136, 20, 4, 0, (16, 16, 4, True, 2)), (128, 22, 7, 1, None),
                                               (64, 64, 1, 0, None), (192, 10, 3, 1, None)]):
        h = rng.integers(0, Z + 1, size=(Y, X)).astype(np.uint8)
        lat = isf.Lattice(h, Z, 1000 + i, replica=i, init=2, fmt=fmt)
        if tuning:
            lat.set_tuning(*tuning)
        out.append(lat)
    return out


def _recount_films(lats):
    from paper_1205_5588_amd import _lib

    n = len(lats)
    descs = (_lib.Desc * n)(*[_lib.Desc(l.X, l.Y, l.Z, l.replica, l.seed, l.fmt, 0) for l in lats])
    ptrs = (ctypes.c_void_p * n)(*[l.spin_buf.data_ptr() for l in lats])
    out = np.zeros((n, 4), dtype=np.int64)
    _lib.check(_lib.load().isf_recount_films(descs, ptrs, n, None, out.ctypes.data))
    return out


def _expected(lat):
    M, E = lat.recount()   # isf_recount: also leaves the current spins in the main buffer
    ob = lat.observables()
    return [M, E, ob["n_occ"], ob["n_bonds"]]


def test_recount_films_equals_recount_on_two_calls(isf):
    lats = _films(isf)
    for l in lats:
        l.run_schedule([(2.5, 20, 6, 0), (7.0, -35, 5, 2)])
    want = np.array([_expected(l) for l in lats], dtype=np.int64)
    got = _recount_films(lats)
    np.testing.assert_array_equal(got, want)
    assert (want[:, 2] > 0).all()
    # second call: fewer films, after more sweeps (their M and E change)
    sub = [lats[4], lats[1], lats[3]]
    for l in sub:
        l.run_schedule([(9.0, 0, 4, 0)])
    want2 = np.array([_expected(l) for l in sub], dtype=np.int64)
    got2 = _recount_films(sub)
    np.testing.assert_array_equal(got2, want2)
    assert not np.array_equal(got2, got[[4, 1, 3]])


def test_recount_films_refuses_more_than_its_counters_hold(isf):
    from paper_1205_5588_amd import _lib

    lat = _films(isf)[0]
    n = 1025
    descs = (_lib.Desc * n)(*[_lib.Desc(lat.X, lat.Y, lat.Z, 0, 0, 0, 0)] * n)
    ptrs = (ctypes.c_void_p * n)(*[lat.spin_buf.data_ptr()] * n)
    out = np.zeros((n, 4), dtype=np.int64)
    with pytest.raises(_lib.IsfError) as ei:
        _lib.check(_lib.load().isf_recount_films(descs, ptrs, n, None, out.ctypes.data))
    assert ei.value.code == _lib.ISF_ENOSPC
    assert _lib.load().isf_recount_films(None, None, 0, None, None) == 0
