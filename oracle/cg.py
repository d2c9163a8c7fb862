"""FP64 oracle of the band-by-band conjugate-gradient eigensolver.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper names the conjugate-gradient method beside Davidson as the two
iterative solvers of the Kohn-Sham problem (section "Evolution of the
GPU-enabled version") and gives no algorithm.  This is the textbook
preconditioned band-by-band CG on the Rayleigh quotient, in these steps
(vectors are rows; <a|b> = sum_G conj(a_G) b_G):

1. X = psi0, HX = H X; Rayleigh-Ritz on the block (the Davidson oracle's
   ``rayleigh_ritz`` on X^H HX, X^H X): X <- Y^T X, HX <- Y^T HX, so the
   block starts orthonormal and ordered.
2. For band m = 0, 1, ...: x = X_m made orthogonal to the (already updated)
   bands j < m and normalised, hx = H x, lam = <x|hx>.  Then repeat:
   a. r = hx - lam x; stop if ||r|| <= rtol (or after maxiter iterations);
   b. g = P(lam) r with P_G = 1 / sqrt(1 + (h_G - lam)^2), h_G = diag(H)_G
      (the Davidson preconditioner);
   c. g <- g - sum_{j<m} X_j <X_j|g> - x <x|g>  (kept orthogonal to the
      lower bands and to x);
   d. gamma = Re <g|r>; d = g on the first iteration, else
      d = g + beta d with the Polak-Ribiere factor
      beta = max(0, (gamma - Re <g_prev|r>) / gamma_prev) (restarting along g
      when it turns negative; the Fletcher-Reeves factor gamma / gamma_prev
      stalls here, the operator's shift lam changing every iteration);
   e. d <- d - x <x|d>; dn = d / ||d||; hd = H dn;
   f. exact minimisation of the Rayleigh quotient over span{x, dn} (an
      orthonormal pair): the lower eigenpair (mu, (c0, c1)) of the 2 x 2
      Hermitian matrix [[lam, <x|hd>], [<dn|hx>, <dn|hd>]], with c0 >= 0;
      x <- c0 x + c1 dn, hx <- c0 hx + c1 hd, lam <- mu.
   X_m = x, HX_m = hx.
3. A final Rayleigh-Ritz of the converged block orders the bands and returns
   eigenvectors of the block's projection.

Step f includes x itself (c = (1, 0)), so lam never increases (a pin).
"""

from __future__ import annotations

import numpy as np

from .davidson import rayleigh_ritz


def lower_eigpair_2x2(a: float, b: complex, c: float):
    """Lower eigenvalue and unit eigenvector (c0 >= 0) of [[a, b], [conj(b), c]]."""
    h = 0.5 * (a - c)
    mu = 0.5 * (a + c) - np.hypot(h, abs(b))
    # (M - mu) v = 0 with v = (c - mu, -conj(b)) or (b, mu - a): take the longer
    v1 = np.array([c - mu, -np.conj(b)], dtype=np.complex128)
    v2 = np.array([b, mu - a], dtype=np.complex128)
    v = v1 if np.linalg.norm(v1) >= np.linalg.norm(v2) else v2
    n = np.linalg.norm(v)
    if n == 0.0:
        return mu, 1.0 + 0j, 0j
    v = v / n
    # make c0 real and >= 0 (a common phase does not change the eigenvector)
    a0 = abs(v[0])
    if a0 > 0:
        return mu, complex(a0, 0.0), v[1] * (np.conj(v[0]) / a0)
    return mu, 0j, v[1] / abs(v[1])


def _rotate(x, hx):
    eps, y = rayleigh_ritz(x.conj() @ hx.T, x.conj() @ x.T, x.shape[0])
    return eps, y.T @ x, y.T @ hx


def cg(apply_h, psi0: np.ndarray, hdiag: np.ndarray, *, rtol: float = 1e-8,
       maxiter: int = 100, history: bool = False):
    """Lowest nb eigenpairs by band-by-band PCG; returns (eps, psi, info)."""
    x0 = np.atleast_2d(np.asarray(psi0, dtype=np.complex128))
    nb, npw = x0.shape
    hx0 = apply_h(x0)
    applies = nb
    _, X, HX = _rotate(x0, hx0)
    X = X.copy()
    HX = HX.copy()
    eps = np.zeros(nb)
    resid = np.zeros(nb)
    iters = np.zeros(nb, dtype=int)
    hist = []
    for m in range(nb):
        x = X[m].copy()
        if m > 0:
            x = x - X[:m].T @ (X[:m].conj() @ x)
        x /= np.linalg.norm(x)
        hx = apply_h(x[None, :])[0]
        applies += 1
        lam = float(np.vdot(x, hx).real)
        d = None
        gam_prev = None
        g_prev = None
        lams = [lam]
        rn = np.inf
        it = 0
        while True:
            r = hx - lam * x
            rn = float(np.linalg.norm(r))
            if rn <= rtol or it >= maxiter:
                break
            it += 1
            g = r / np.sqrt(1.0 + (hdiag - lam) ** 2)
            if m > 0:
                g = g - X[:m].T @ (X[:m].conj() @ g)
            g = g - x * np.vdot(x, g)
            gam = float(np.vdot(g, r).real)
            if d is None:
                d = g.copy()
            else:
                beta = max(0.0, (gam - float(np.vdot(g_prev, r).real)) / gam_prev)
                d = g + beta * d
            gam_prev = gam
            g_prev = g
            d = d - x * np.vdot(x, d)
            dnorm = float(np.linalg.norm(d))
            if dnorm == 0.0:
                break
            dn = d / dnorm
            hd = apply_h(dn[None, :])[0]
            applies += 1
            mu, c0, c1 = lower_eigpair_2x2(lam, np.vdot(x, hd), float(np.vdot(dn, hd).real))
            x = c0 * x + c1 * dn
            hx = c0 * hx + c1 * hd
            lam = float(mu)
            lams.append(lam)
        X[m], HX[m] = x, hx
        eps[m], resid[m], iters[m] = lam, rn, it
        if history:
            hist.append(np.array(lams))
    eps, X, HX = _rotate(X, HX)
    r = HX - eps[:, None] * X
    info = dict(iters=iters, band_applies=applies, resid=np.linalg.norm(r, axis=1),
                resid_bandwise=resid, notconv=int((resid > rtol).sum()))
    if history:
        info["history"] = hist
    return eps, X, info
