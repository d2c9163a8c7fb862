"""FP64 oracle of the electronic charge density of a block of bands.

The paper lists charge density generation among the kernels ported to the GPU
(section "Evolution of the GPU-enabled version"); it is the step that follows
the iterative diagonalisation in the self-consistency cycle named in the same
section.  The paper prints no formula; the standard plane-wave form is used:

    rho(r) = (1 / Omega) sum_i f_i |psi_i(r)|^2,
    psi_i(r) = sum_G c_i(G) exp(i (k + G) . r),

on the points r = (x / N1) a1 + (y / N2) a2 + (z / N3) a3 of the FFT grid,
with Omega the cell volume, f_i the occupation weights and c_i the plane-wave
coefficients (one band per row of psi).  The Bloch phase exp(i k . r) has unit
modulus and drops out of |psi|^2.  With sum_G |c_i(G)|^2 = 1 the grid
quadrature (Omega / N) sum_r rho(r) equals sum_i f_i (Parseval).

Array layout of the result: (N3, N2, N1), x fastest.
"""

from __future__ import annotations

import numpy as np

from .dft import inv3


def cell_volume(cell) -> float:
    """Omega = |det(a1, a2, a3)| (bohr^3)."""
    return float(abs(np.linalg.det(np.asarray(cell.lattice, dtype=np.float64))))


def psi_real_space(cell, psi_row: np.ndarray) -> np.ndarray:
    """One band on the grid, sum_G c(G) exp(i G . r) (the k phase left out):
    the sphere placed in the box and the oracle's inverse 3D DFT."""
    n1, n2, n3 = cell.fft
    m = cell.miller
    box = np.zeros((n3, n2, n1), dtype=np.complex128)
    box[m[:, 2] % n3, m[:, 1] % n2, m[:, 0] % n1] = psi_row
    return inv3(box)


def density(cell, psi: np.ndarray, occ) -> np.ndarray:
    """rho(r) = (1/Omega) sum_i occ_i |psi_i(r)|^2 on the (N3, N2, N1) grid."""
    psi = np.atleast_2d(psi)
    occ = np.asarray(occ, dtype=np.float64).reshape(-1)
    if occ.shape[0] != psi.shape[0]:
        raise ValueError("one occupation per band")
    n1, n2, n3 = cell.fft
    rho = np.zeros((n3, n2, n1), dtype=np.float64)
    for i in range(psi.shape[0]):
        f = psi_real_space(cell, psi[i])
        rho += occ[i] * (f.real ** 2 + f.imag ** 2)
    return rho / cell_volume(cell)


def density_direct(cell, psi: np.ndarray, occ) -> np.ndarray:
    """The same density by direct summation of the plane waves at every grid
    point, exp(2 pi i (h x / N1 + k y / N2 + l z / N3)), without any transform.
    Cost O(nb npw N): tiny cells only (a brute-force check of ``density``)."""
    psi = np.atleast_2d(psi)
    occ = np.asarray(occ, dtype=np.float64).reshape(-1)
    n1, n2, n3 = cell.fft
    z, y, x = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    frac = np.stack([x.ravel() / n1, y.ravel() / n2, z.ravel() / n3], axis=1)   # (N, 3)
    phase = np.exp(2j * np.pi * (frac @ cell.miller.T.astype(np.float64)))      # (N, npw)
    rho = np.zeros(n1 * n2 * n3)
    for i in range(psi.shape[0]):
        f = phase @ psi[i]
        rho += occ[i] * np.abs(f) ** 2
    return rho.reshape(n3, n2, n1) / cell_volume(cell)
