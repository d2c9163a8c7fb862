"""The oracle's own discrete Fourier transform: dense per-axis DFT matrices.

No FFT is used: each axis is transformed by an explicit n x n matrix
F[j, m] = exp(sign * 2 pi i (j m mod n) / n), with the exponent reduced
exactly in integers before the trigonometric call.  The 3D transform is the
product of the three axis transforms.

Conventions (the pair that defines the local-potential operator):
* inverse (G -> r): f(r_j) = sum_m c_m exp(+2 pi i m.j / N), unnormalised;
* forward (r -> G): c_m = (1/N) sum_j f(r_j) exp(-2 pi i m.j / N).
Boxes are stored as (N3, N2, N1) arrays, x fastest.
"""

from __future__ import annotations

import functools

import numpy as np


@functools.lru_cache(maxsize=32)
def dft_matrix(n: int, sign: int) -> np.ndarray:
    j = np.arange(n)
    e = np.outer(j, j) % n
    return np.exp(sign * 2j * np.pi * e / n)


def dft_axis(f: np.ndarray, axis: int, sign: int) -> np.ndarray:
    """Unnormalised DFT of ``f`` along ``axis`` with exp(sign 2 pi i j m / n)."""
    n = f.shape[axis]
    fm = dft_matrix(n, sign)
    g = np.moveaxis(f, axis, -1)
    out = g @ fm          # fm is symmetric
    return np.moveaxis(out, -1, axis)


def inv3(c: np.ndarray) -> np.ndarray:
    """G-space box (N3, N2, N1) -> real-space values, +i, unnormalised."""
    f = dft_axis(c, 2, +1)
    f = dft_axis(f, 1, +1)
    return dft_axis(f, 0, +1)


def fwd3(f: np.ndarray) -> np.ndarray:
    """Real-space box -> G-space coefficients, -i, scaled by 1/N."""
    c = dft_axis(f, 2, -1)
    c = dft_axis(c, 1, -1)
    c = dft_axis(c, 0, -1)
    return c / f.size
