"""FP64 oracle of the block Davidson iterative diagonalisation.

The paper names the Davidson method as one of the iterative solvers of the
Kohn-Sham problem (section "Evolution of the GPU-enabled version"), calls the
Hamiltonian builder as an external routine (section "Domain-specific
mathematical libraries") and solves the small dense generalized eigenproblem
with a dense-solver library.  It gives no algorithm; this is the textbook
block Davidson with a diagonal preconditioner, in these steps:

1. basis V = psi0 (nb vectors), W = H V; reduced matrices Hr = V^H W and
   Sr = V^H V, both Hermitised.
2. Rayleigh-Ritz: Cholesky Sr = L L^H, standard problem L^-1 Hr L^-H z = eps z,
   y = L^-H z; keep the nb lowest (eps ascending, Y).
3. Ritz vectors psi_i = V y_i, residuals r_i = W y_i - eps_i V y_i; band i is
   converged when ||r_i||_2 <= rtol.
4. For each unconverged band, t_i = P(eps_i) r_i with
   P_G = 1 / sqrt(1 + (h_G - eps_i)^2), h_G = diag(H)_G; t_i normalised.
5. If the basis would exceed nvecx: restart with V <- V Y, W <- W Y,
   Hr <- diag(eps), Sr <- I.
6. Append the t_i to V, their H t_i to W, extend Hr and Sr; go to 2.
A failed Cholesky restarts from the Ritz vectors once; a second failure in a
row is an error.

Arrays hold one vector per row: V is (nbase, npw).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class CholeskyError(RuntimeError):
    pass


def rayleigh_ritz(hr: np.ndarray, sr: np.ndarray, nb: int):
    """Lowest nb solutions of hr y = eps sr y (Cholesky + standard eigh)."""
    hr = 0.5 * (hr + hr.conj().T)
    sr = 0.5 * (sr + sr.conj().T)
    try:
        lo = sla.cholesky(sr, lower=True)
    except np.linalg.LinAlgError as e:  # not positive definite
        raise CholeskyError(str(e)) from e
    x = sla.solve_triangular(lo, hr, lower=True)                 # L^-1 Hr
    a = sla.solve_triangular(lo, x.conj().T, lower=True)         # L^-1 Hr L^-H
    a = 0.5 * (a + a.conj().T)
    w, z = np.linalg.eigh(a)
    y = sla.solve_triangular(lo.conj().T, z[:, :nb], lower=False)
    return w[:nb], y


def davidson(apply_h, psi0: np.ndarray, hdiag: np.ndarray, *, nvecx: int | None = None,
             rtol: float = 1e-8, maxiter: int = 200, history: bool = False):
    """Block Davidson for the nb lowest eigenpairs; returns (eps, psi, info)."""
    psi0 = np.atleast_2d(np.asarray(psi0, dtype=np.complex128))
    nb, npw = psi0.shape
    nvecx = 2 * nb if nvecx is None else nvecx
    if nvecx < 2 * nb:
        raise ValueError("nvecx must be >= 2 nb")
    v = np.zeros((nvecx, npw), dtype=np.complex128)
    w = np.zeros_like(v)
    hr = np.zeros((nvecx, nvecx), dtype=np.complex128)
    sr = np.zeros_like(hr)
    v[:nb] = psi0
    w[:nb] = apply_h(psi0)
    nbase = nb
    hr[:nb, :nb] = v[:nb].conj() @ w[:nb].T
    sr[:nb, :nb] = v[:nb].conj() @ v[:nb].T
    band_applies = nb
    hist = []
    restarts = 0
    chol_fail_prev = False
    eps = y = None
    it = 0
    conv = np.zeros(nb, dtype=bool)
    rn = np.full(nb, np.inf)
    while True:
        it += 1
        try:
            eps, y = rayleigh_ritz(hr[:nbase, :nbase], sr[:nbase, :nbase], nb)
            chol_fail_prev = False
        except CholeskyError:
            if chol_fail_prev or y is None:
                raise
            chol_fail_prev = True
            # restart from the last Ritz vectors (orthonormal)
            psi = y.T @ v[:y.shape[0]]
            hpsi = y.T @ w[:y.shape[0]]
            v[:nb], w[:nb] = psi, hpsi
            nbase = nb
            hr[:nb, :nb] = v[:nb].conj() @ w[:nb].T
            sr[:nb, :nb] = v[:nb].conj() @ v[:nb].T
            restarts += 1
            continue
        if history:
            hist.append(eps.copy())
        psi = y.T @ v[:nbase]
        hpsi = y.T @ w[:nbase]
        r = hpsi - eps[:, None] * psi
        rn = np.linalg.norm(r, axis=1)
        conv = rn <= rtol
        if conv.all() or it >= maxiter:
            break
        idx = np.nonzero(~conv)[0]
        nc = idx.size
        t = r[idx] / np.sqrt(1.0 + (hdiag[None, :] - eps[idx, None]) ** 2)
        t /= np.linalg.norm(t, axis=1, keepdims=True)
        if nbase + nc > nvecx:
            v[:nb], w[:nb] = psi, hpsi
            nbase = nb
            hr[:nb, :nb] = np.diag(eps)
            sr[:nb, :nb] = np.eye(nb)
            restarts += 1
        v[nbase:nbase + nc] = t
        w[nbase:nbase + nc] = apply_h(t)
        band_applies += nc
        new = slice(nbase, nbase + nc)
        hr[:nbase + nc, new] = v[:nbase + nc].conj() @ w[new].T
        sr[:nbase + nc, new] = v[:nbase + nc].conj() @ v[new].T
        hr[new, :nbase] = hr[:nbase, new].conj().T
        sr[new, :nbase] = sr[:nbase, new].conj().T
        nbase += nc
    info = dict(iters=it, converged=bool(conv.all()), resid=rn, band_applies=band_applies,
                restarts=restarts, notconv=int((~conv).sum()))
    if history:
        info["history"] = np.array(hist)
    return eps, psi, info
