"""Synthetic surface-topography height maps.

The paper turns each pixel of an STM/AFM image into a column of atomic
layers of the film (Sections 2-3: rows = image height, columns = image
width, depth = number of Co layers).  Here a seeded random surface stands in
for the image:

1. per-pixel N(0, 1) noise from ``numpy.random.default_rng(seed)``;
2. a periodic Gaussian blur of width ``sigma`` pixels, applied in Fourier
   space with transfer function ``exp(-2 pi^2 sigma^2 (fx^2 + fy^2))``;
3. normalisation to zero mean and unit variance (population std);
4. ``h = clamp(floor(L/2 + (L/2) g + 1/2), 0, L)`` (round half up), which
   is ``round(1.5 + 1.5 g)`` for L = 3.

A lattice site (x, y, z) is then occupied iff z < h[y][x].
"""

from __future__ import annotations

import numpy as np


def _rng(seed):
    if isinstance(seed, (tuple, list)):
        return np.random.default_rng([int(s) for s in seed])
    return np.random.default_rng(int(seed))


def height_map(X: int, Y: int, L: int, sigma: float, seed) -> np.ndarray:
    """Return a uint8 height map of shape (Y, X) with values in [0, L]."""
    if X <= 0 or Y <= 0 or L < 0:
        raise ValueError("height_map: X, Y must be positive and L >= 0")
    rng = _rng(seed)
    g = rng.standard_normal((Y, X))
    fy = np.fft.fftfreq(Y)
    fx = np.fft.fftfreq(X)
    transfer = np.exp(-2.0 * np.pi**2 * float(sigma) ** 2 * (fy[:, None] ** 2 + fx[None, :] ** 2))
    g = np.fft.ifft2(np.fft.fft2(g) * transfer).real
    g = g - g.mean()
    sd = g.std()
    if sd > 0:
        g = g / sd
    h = np.floor(L / 2.0 + (L / 2.0) * g + 0.5)
    return np.clip(h, 0, L).astype(np.uint8)


def occupancy_count(h: np.ndarray) -> int:
    """Number of occupied FCC sites for height map ``h`` (sites with x+y+z even, z < h).

    Pure counting of the input, used to size workloads; it is not part of the
    dynamics.
    """
    h = np.asarray(h, dtype=np.int64)
    Y, X = h.shape
    par = (np.arange(Y)[:, None] + np.arange(X)[None, :]) & 1
    # z ranges over [0, h); z with z + x + y even: count = ceil((h - par)/2) for h > par
    return int(np.maximum((h - par + 1) // 2, 0).sum())
