"""FP64 oracle of the nonlocal projectors beta_i(k+G) built from their radial
functions (the "calculation of pseudopotential terms" among the quantum-engine
modules, section "Quantum-engine modules"; the pseudopotential contribution is
one of the GPU-ported Hamiltonian kernels, section "Evolution of the
GPU-enabled version").

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's CPU baseline,
never by the library.

The paper prints no formula; the form is the standard separable projector of
a norm-conserving pseudopotential.  For projector i = (atom a of species s,
radial channel c of s with angular momentum l, real harmonic m):

  beta_i(q) = (4 pi / sqrt(Omega)) (-i)^l F_c(|q|) Y_lm(q / |q|) exp(-i q . tau_a),
  F_c(q)    = int_0^inf r^2 beta_c(r) j_l(q r) dr,          q = k + G.

Here the radial functions are the synthetic ones of the cell generator,
beta_c(r) = r^l exp(-r^2 / sigma_c).  The oracle evaluates F_c by direct
quadrature of that integral at every |q| (no table, no closed form), the
spherical Bessel functions j_l from their elementary expressions, and the real
harmonics from their Cartesian expressions on the unit vector.

Projector order: atoms in order; within an atom its species' channels in order;
within a channel m in the order
  l = 0: 1;   l = 1: x, y, z;   l = 2: xy, yz, zx, 3z^2 - 1, x^2 - y^2.
"""

from __future__ import annotations

import math

import numpy as np


def spherical_bessel(l: int, x: np.ndarray) -> np.ndarray:
    """j_l(x) for l = 0, 1, 2: elementary forms for x >= 1, the power series
    x^l / (2l+1)!! * sum_k (-x^2/2)^k / (k! (2l+3)(2l+5)...(2l+2k+1)) below,
    where the elementary forms lose digits to cancellation."""
    if l not in (0, 1, 2):
        raise ValueError("l > 2 not supported")
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    small = np.abs(x) < 1.0
    xs = x[small]
    xl = x[~small]
    h = -0.5 * xs * xs
    term = np.ones_like(xs)
    acc = np.ones_like(xs)
    for k in range(1, 18):
        term = term * h / (k * (2 * l + 2 * k + 1))
        acc = acc + term
    dfact = {0: 1.0, 1: 3.0, 2: 15.0}[l]
    out[small] = xs ** l / dfact * acc
    if l == 0:
        out[~small] = np.sin(xl) / xl
    elif l == 1:
        out[~small] = np.sin(xl) / xl ** 2 - np.cos(xl) / xl
    else:
        out[~small] = (3.0 / xl ** 3 - 1.0 / xl) * np.sin(xl) - 3.0 * np.cos(xl) / xl ** 2
    return out


def radial_transform(l: int, sigma: float, q: np.ndarray, nr: int = 4001,
                     rmax_sigmas: float = 12.0, chunk: int = 2048) -> np.ndarray:
    """F(q) = int_0^inf r^2 * r^l exp(-r^2/sigma) * j_l(q r) dr by composite
    Simpson quadrature on [0, rmax_sigmas * sqrt(sigma)] (the integrand there is
    below exp(-rmax_sigmas^2) of its scale)."""
    q = np.asarray(q, dtype=np.float64).ravel()
    rmax = rmax_sigmas * math.sqrt(sigma)
    if nr % 2 == 0:
        nr += 1
    r = np.linspace(0.0, rmax, nr)
    h = r[1] - r[0]
    w = np.ones(nr)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    w *= h / 3.0
    radial = w * r ** (2 + l) * np.exp(-r * r / sigma)
    out = np.empty_like(q)
    for i in range(0, q.size, chunk):
        qq = q[i:i + chunk]
        out[i:i + chunk] = spherical_bessel(l, np.outer(qq, r)) @ radial
    return out


def real_harmonics(l: int, u: np.ndarray) -> np.ndarray:
    """Y_lm(u) for unit vectors u (n, 3), shape (2l+1, n); rows with u = 0
    (q = 0) give the value of the Cartesian expression at 0."""
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    if l == 0:
        return np.full((1, u.shape[0]), 1.0 / math.sqrt(4.0 * math.pi))
    if l == 1:
        return math.sqrt(3.0 / (4.0 * math.pi)) * np.stack([x, y, z])
    if l == 2:
        a = math.sqrt(15.0 / (4.0 * math.pi))
        b = math.sqrt(5.0 / (16.0 * math.pi))
        c = math.sqrt(15.0 / (16.0 * math.pi))
        return np.stack([a * x * y, a * y * z, a * z * x, b * (3.0 * z * z - 1.0),
                         c * (x * x - y * y)])
    raise ValueError("l > 2 not supported")


def qvectors(lattice, kpt, miller) -> np.ndarray:
    """q = k + G (cartesian, bohr^-1) for every Miller triple, (npw, 3)."""
    b = 2.0 * np.pi * np.linalg.inv(np.asarray(lattice, dtype=np.float64)).T
    return np.asarray(miller, dtype=np.float64) @ b + np.asarray(kpt, dtype=np.float64)[None, :]


def beta_projectors(lattice, kpt, miller, positions, ityp, species) -> np.ndarray:
    """beta_i(k+G), (nkb, npw) complex128.

    positions (nat, 3) cartesian bohr; ityp (nat,) species index;
    species: list over species of lists of (l, sigma) radial channels."""
    lattice = np.asarray(lattice, dtype=np.float64)
    omega = abs(np.linalg.det(lattice))
    q = qvectors(lattice, kpt, miller)
    qn = np.sqrt(np.einsum("ij,ij->i", q, q))
    u = np.zeros_like(q)
    nz = qn > 0.0
    u[nz] = q[nz] / qn[nz, None]
    pref = 4.0 * math.pi / math.sqrt(omega)
    radial = {}
    for chans in species:
        for (l, sig) in chans:
            if (l, sig) not in radial:
                radial[(l, sig)] = radial_transform(l, sig, qn)
    ylm = {l: real_harmonics(l, u) for l in {l for chans in species for (l, _) in chans}}
    ityp = np.asarray(ityp, dtype=np.int64)
    nkb = sum(sum(2 * l + 1 for (l, _) in species[s]) for s in ityp)
    out = np.empty((nkb, q.shape[0]), dtype=np.complex128)
    i = 0
    for a, tau in enumerate(np.asarray(positions, dtype=np.float64)):
        phase = np.exp(-1j * (q @ tau))
        for (l, sig) in species[ityp[a]]:
            base = pref * (-1j) ** l * radial[(l, sig)] * phase
            for m in range(2 * l + 1):
                out[i] = base * ylm[l][m]
                i += 1
    return out
