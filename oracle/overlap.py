"""FP64 oracle of the overlap operator and the generalized block Davidson.

The paper lists the overlap operator among the kernels of the GPU port
(section "Evolution of the GPU-enabled version"); with ultrasoft and PAW
pseudopotentials the Kohn-Sham problem becomes H psi = eps S psi.  It gives no
formula; this is the standard separable form

    S = 1 + sum_a sum_ij |beta_i^a> q_ij^a <beta_j^a|,

with the projectors of the nonlocal term and per-atom Hermitian q blocks (the
layout of D), and the textbook generalized block Davidson: the steps of
``oracle.davidson`` with the overlap carried along,

1. V = psi0, W = H V, U = S V; Hr = V^H W, Sr = V^H U (Hermitised).
2. Rayleigh-Ritz on (Hr, Sr): Cholesky of Sr, the standard problem, y.
3. psi = V y, H psi = W y, S psi = U y; r = H psi - eps S psi; converged when
   ||r||_2 <= rtol.
4. t = P(eps) r with P_G = 1 / sqrt(1 + (h_G - eps)^2), normalised.
5. Restart when full: V = psi, W = H psi, U = S psi, Hr = diag(eps), Sr = I
   (the Ritz vectors are S-orthonormal).
6. Append t, H t, S t; extend Hr, Sr.
The output psi is S-orthonormal: psi^H S psi = I.

Arrays hold one vector per row: V is (nbase, npw).
"""

from __future__ import annotations

import numpy as np

from .davidson import CholeskyError, rayleigh_ritz
from .hamiltonian import dense_h


def _q_blocks(cell):
    off = 0
    qoff = 0
    for n in cell.nproj:
        n = int(n)
        yield off, n, np.asarray(cell.qmat[qoff:qoff + n * n]).reshape(n, n)
        off += n
        qoff += n * n


def apply_s(cell, psi: np.ndarray) -> np.ndarray:
    """S psi = psi + beta (q (beta^H psi)); psi (nb, npw)."""
    psi = np.atleast_2d(np.asarray(psi, dtype=np.complex128))
    if getattr(cell, "qmat", None) is None or cell.nkb == 0:
        return psi.copy()
    becp = np.conj(cell.beta) @ psi.T
    qs = np.empty_like(becp)
    for off, n, blk in _q_blocks(cell):
        qs[off:off + n] = blk @ becp[off:off + n]
    return psi + (cell.beta.T @ qs).T


def dense_s(cell) -> np.ndarray:
    """S[G, G'] = delta + sum_ij beta_i(G) q_ij conj(beta_j(G'))."""
    s = np.eye(cell.npw, dtype=np.complex128)
    if getattr(cell, "qmat", None) is not None and cell.nkb:
        for off, n, blk in _q_blocks(cell):
            bb = cell.beta[off:off + n]
            s += bb.T @ blk @ np.conj(bb)
    return s


def dense_eigs_gen(cell, nb: int) -> np.ndarray:
    """The nb lowest eigenvalues of H y = eps S y from the dense matrices, by
    LAPACK's generalized Hermitian eigensolver (a library step)."""
    import scipy.linalg as sla
    return sla.eigh(dense_h(cell), dense_s(cell), eigvals_only=True,
                    subset_by_index=[0, nb - 1])


def davidson_gen(apply_h, apply_s_fn, psi0: np.ndarray, hdiag: np.ndarray, *,
                 nvecx: int | None = None, rtol: float = 1e-8, maxiter: int = 200):
    """Generalized block Davidson for the nb lowest pairs of H psi = eps S psi."""
    psi0 = np.atleast_2d(np.asarray(psi0, dtype=np.complex128))
    nb, npw = psi0.shape
    nvecx = 2 * nb if nvecx is None else nvecx
    if nvecx < 2 * nb:
        raise ValueError("nvecx must be >= 2 nb")
    v = np.zeros((nvecx, npw), dtype=np.complex128)
    w = np.zeros_like(v)
    u = np.zeros_like(v)
    hr = np.zeros((nvecx, nvecx), dtype=np.complex128)
    sr = np.zeros_like(hr)
    v[:nb] = psi0
    w[:nb] = apply_h(psi0)
    u[:nb] = apply_s_fn(psi0)
    nbase = nb
    hr[:nb, :nb] = v[:nb].conj() @ w[:nb].T
    sr[:nb, :nb] = v[:nb].conj() @ u[:nb].T
    band_applies = nb
    chol_fail_prev = False
    y = None
    it = 0
    while True:
        it += 1
        try:
            eps, y = rayleigh_ritz(hr[:nbase, :nbase], sr[:nbase, :nbase], nb)
            chol_fail_prev = False
        except CholeskyError:
            if chol_fail_prev or y is None:
                raise
            chol_fail_prev = True
            psi, hpsi, spsi = y.T @ v[:y.shape[0]], y.T @ w[:y.shape[0]], y.T @ u[:y.shape[0]]
            v[:nb], w[:nb], u[:nb] = psi, hpsi, spsi
            nbase = nb
            hr[:nb, :nb] = v[:nb].conj() @ w[:nb].T
            sr[:nb, :nb] = v[:nb].conj() @ u[:nb].T
            continue
        psi = y.T @ v[:nbase]
        hpsi = y.T @ w[:nbase]
        spsi = y.T @ u[:nbase]
        r = hpsi - eps[:, None] * spsi
        rn = np.linalg.norm(r, axis=1)
        conv = rn <= rtol
        if conv.all() or it >= maxiter:
            break
        idx = np.nonzero(~conv)[0]
        nc = idx.size
        t = r[idx] / np.sqrt(1.0 + (hdiag[None, :] - eps[idx, None]) ** 2)
        t /= np.linalg.norm(t, axis=1, keepdims=True)
        if nbase + nc > nvecx:
            v[:nb], w[:nb], u[:nb] = psi, hpsi, spsi
            nbase = nb
            hr[:nb, :nb] = np.diag(eps)
            sr[:nb, :nb] = np.eye(nb)
        v[nbase:nbase + nc] = t
        w[nbase:nbase + nc] = apply_h(t)
        u[nbase:nbase + nc] = apply_s_fn(t)
        band_applies += nc
        new = slice(nbase, nbase + nc)
        hr[:nbase + nc, new] = v[:nbase + nc].conj() @ w[new].T
        sr[:nbase + nc, new] = v[:nbase + nc].conj() @ u[new].T
        hr[new, :nbase] = hr[:nbase, new].conj().T
        sr[new, :nbase] = sr[:nbase, new].conj().T
        nbase += nc
    info = dict(iters=it, converged=bool(conv.all()), resid=rn, band_applies=band_applies,
                notconv=int((~conv).sum()))
    return eps, psi, info
