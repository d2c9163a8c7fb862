"""FP64 oracle of the Kohn-Sham Hamiltonian applied to a block of bands.

H = T + V_loc + V_NL in the plane-wave basis {|k+G>, G in the sphere}, the
operator whose GPU kernels the paper lists as "local-potential,
pseudopotential, kinetic-energy contributions to the Hamiltonian" (section
"Evolution of the GPU-enabled version").  Rydberg units.

* T_G = |k+G|^2 (kinetic contribution).
* (V_loc psi)_G = sum_G' Vt[(m_G - m_G') mod N] psi_G', with Vt the forward
  transform of V(r) on the grid: computed the FFT way (place the sphere in the
  box, inverse 3D transform, multiply by V(r), forward transform, read the
  sphere back) through the oracle's dense DFT; ``dense_h`` writes the same
  operator out as a matrix.
* V_NL psi = beta (D (beta^H psi)) with beta the (nkb, npw) projector table
  and D block-diagonal per atom (pseudopotential contribution).

Arrays: psi is (nb, npw) complex128, one band per row.
"""

from __future__ import annotations

import numpy as np

from .dft import fwd3, inv3


def _recip(lattice):
    return 2.0 * np.pi * np.linalg.inv(np.asarray(lattice, dtype=np.float64)).T


def kinetic(cell) -> np.ndarray:
    """|k+G|^2 for every G of the sphere (Ry)."""
    q = cell.miller.astype(np.float64) @ _recip(cell.lattice) + np.asarray(cell.kpt)[None, :]
    return np.einsum("ij,ij->i", q, q)


def _box_index(cell):
    n1, n2, n3 = cell.fft
    m = cell.miller
    return m[:, 2] % n3, m[:, 1] % n2, m[:, 0] % n1


def vloc_psi(cell, psi: np.ndarray) -> np.ndarray:
    """Local-potential term, FFT route (scatter, inverse 3D DFT, x V, forward, gather)."""
    n1, n2, n3 = cell.fft
    iz, iy, ix = _box_index(cell)
    psi = np.atleast_2d(psi)
    out = np.empty_like(psi, dtype=np.complex128)
    for b in range(psi.shape[0]):
        box = np.zeros((n3, n2, n1), dtype=np.complex128)
        box[iz, iy, ix] = psi[b]
        f = inv3(box) * cell.vloc
        c = fwd3(f)
        out[b] = c[iz, iy, ix]
    return out


def _d_blocks(cell):
    """Yield (row offset, nproj, D block) per atom."""
    off = 0
    doff = 0
    for n in cell.nproj:
        n = int(n)
        blk = np.asarray(cell.dmat[doff:doff + n * n]).reshape(n, n)
        yield off, n, blk
        off += n
        doff += n * n


def vnl_psi(cell, psi: np.ndarray) -> np.ndarray:
    """Nonlocal term: becp = beta^H psi, ps = D becp, out = beta ps."""
    psi = np.atleast_2d(psi)
    if cell.nkb == 0:
        return np.zeros_like(psi, dtype=np.complex128)
    becp = np.conj(cell.beta) @ psi.T          # (nkb, nb)
    ps = np.empty_like(becp)
    for off, n, blk in _d_blocks(cell):
        ps[off:off + n] = blk @ becp[off:off + n]
    return (cell.beta.T @ ps).T


def apply_h(cell, psi: np.ndarray) -> np.ndarray:
    psi = np.atleast_2d(psi)
    return kinetic(cell)[None, :] * psi + vloc_psi(cell, psi) + vnl_psi(cell, psi)


def vloc_coeffs(cell) -> np.ndarray:
    """Vt = forward transform of V(r) (box of Fourier coefficients)."""
    return fwd3(np.asarray(cell.vloc, dtype=np.complex128))


def dense_h(cell) -> np.ndarray:
    """H[G, G'] = delta T_G + Vt[(m_G - m_G') mod N] + sum_ij beta_i(G) D_ij conj(beta_j(G'))."""
    n1, n2, n3 = cell.fft
    vt = vloc_coeffs(cell)
    m = cell.miller
    d = m[:, None, :] - m[None, :, :]
    h = vt[d[..., 2] % n3, d[..., 1] % n2, d[..., 0] % n1]
    h[np.diag_indices_from(h)] += kinetic(cell)
    if cell.nkb:
        for off, n, blk in _d_blocks(cell):
            bb = cell.beta[off:off + n]
            h += bb.T @ blk @ np.conj(bb)
    return h


def dense_eigs(cell, nb: int) -> np.ndarray:
    """The nb lowest eigenvalues of the dense H of ``dense_h`` (ascending), by
    LAPACK's Hermitian eigensolver (a library step: the definition written out
    for cells small enough to hold H)."""
    import scipy.linalg as sla
    return sla.eigh(dense_h(cell), eigvals_only=True, subset_by_index=[0, nb - 1])


def hdiag(cell) -> np.ndarray:
    """Diagonal of H (real): T_G + Vt[0] + sum_ij beta_i(G) D_ij conj(beta_j(G))."""
    v0 = float(np.mean(cell.vloc))
    d = kinetic(cell) + v0
    if cell.nkb:
        for off, n, blk in _d_blocks(cell):
            bb = cell.beta[off:off + n]
            d = d + np.real(np.einsum("ig,ij,jg->g", bb, blk, np.conj(bb)))
    return d
