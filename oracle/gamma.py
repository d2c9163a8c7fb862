"""Gamma-point (k = 0) real wavefunctions in the oracle's terms (the
"real-valued wavefunctions, k = 0 only sampling" case of section "Evolution of
the GPU-enabled version").

TEST INFRASTRUCTURE ONLY: used by the tests, never by the library.

A real function psi(r) has psi(-G) = conj(psi(G)).  At k = 0 the sphere is
symmetric under G -> -G, and in lexicographic Miller order entry i0 + h and
entry i0 - h are G and -G (i0 = the index of (0,0,0)); a half-sphere vector of
nh = i0 + 1 values holds G = 0 (real) and the G after it.  The oracle keeps
working on full-sphere complex vectors: ``expand`` rebuilds one from the stored
half, ``restrict`` reads the stored half back.  H is real in real space at
k = 0, so H maps such vectors to such vectors and its eigenvalues are those of
the complex problem (each has a real eigenvector).
"""

from __future__ import annotations

import numpy as np


def expand(psi_half: np.ndarray) -> np.ndarray:
    """(nb, nh) half-sphere coefficients -> (nb, 2 nh - 1) full sphere:
    [conj(psi[nh-1]), ..., conj(psi[1]), Re psi[0], psi[1], ..., psi[nh-1]]."""
    p = np.atleast_2d(np.asarray(psi_half, dtype=np.complex128))
    nh = p.shape[1]
    out = np.empty((p.shape[0], 2 * nh - 1), dtype=np.complex128)
    out[:, nh - 1:] = p
    out[:, nh - 1] = p[:, 0].real
    out[:, :nh - 1] = np.conj(p[:, :0:-1])
    return out


def restrict(psi_full: np.ndarray) -> np.ndarray:
    """(nb, 2 nh - 1) full-sphere coefficients -> the stored half (nb, nh)."""
    p = np.atleast_2d(psi_full)
    nh = (p.shape[1] + 1) // 2
    return np.ascontiguousarray(p[:, nh - 1:])
