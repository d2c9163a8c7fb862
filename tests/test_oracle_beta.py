"""Pins of the projector oracle (CPU).  Each names the plausible mistake it
catches; none re-evaluates the oracle's own expressions."""

import math

import numpy as np
import pytest
import scipy.special as sp

import cellgen
from oracle import beta as ob


@pytest.mark.parametrize("l", [0, 1, 2])
def test_bessel_matches_library(l):
    # elementary forms and their small-argument series against the library
    # routine (a wrong series coefficient or a sign in the cosine term fails)
    x = np.concatenate([np.linspace(0.0, 1.2, 241), np.linspace(1.2, 80.0, 4001)])
    assert np.abs(ob.spherical_bessel(l, x) - sp.spherical_jn(l, x)).max() < 2e-15


@pytest.mark.parametrize("l", [0, 1, 2])
@pytest.mark.parametrize("sigma", [1.5, 0.75])
def test_radial_transform_closed_form(l, sigma):
    # int r^2 r^l exp(-r^2/s) j_l(q r) dr = sqrt(pi) s^(l+3/2) / 2^(l+2) q^l exp(-s q^2/4)
    # (Gaussian integral; a dropped r^2 or a wrong power of r fails)
    q = np.linspace(0.0, 9.0, 91)
    ref = math.sqrt(math.pi) * sigma ** (l + 1.5) / 2.0 ** (l + 2) * q ** l \
        * np.exp(-sigma * q * q / 4.0)
    got = ob.radial_transform(l, sigma, q)
    scale = math.sqrt(math.pi) * sigma ** (l + 1.5) / 2.0 ** (l + 2)
    assert np.abs(got - ref).max() < 1e-12 * scale


def _sphere_rule(nt=24, nph=48):
    # Gauss-Legendre in cos(theta) x uniform phi: exact for the degree-4
    # products of harmonics integrated here
    t, wt = np.polynomial.legendre.leggauss(nt)
    ph = np.arange(nph) * 2.0 * np.pi / nph
    T, P = np.meshgrid(t, ph, indexing="ij")
    st = np.sqrt(1.0 - T * T)
    u = np.stack([st * np.cos(P), st * np.sin(P), T], axis=-1).reshape(-1, 3)
    w = (wt[:, None] * np.full(nph, 2.0 * np.pi / nph)[None, :]).ravel()
    return u, w


def test_real_harmonics_orthonormal():
    # a wrong normalisation constant or a repeated component fails
    u, w = _sphere_rule()
    Y = np.concatenate([ob.real_harmonics(l, u) for l in (0, 1, 2)])
    G = (Y * w[None, :]) @ Y.T
    assert np.abs(G - np.eye(9)).max() < 1e-13


def test_real_harmonics_addition_theorem():
    # sum_m Y_lm(u) Y_lm(v) = (2l+1)/(4 pi) P_l(u . v): a sign or index slip in
    # one component fails (orthonormality alone does not see a sign)
    rng = np.random.default_rng(7)
    u = rng.normal(size=(50, 3))
    v = rng.normal(size=(50, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    c = np.einsum("ij,ij->i", u, v)
    for l in (0, 1, 2):
        s = np.einsum("mi,mi->i", ob.real_harmonics(l, u), ob.real_harmonics(l, v))
        ref = (2 * l + 1) / (4 * math.pi) * sp.eval_legendre(l, c)
        assert np.abs(s - ref).max() < 1e-14


def _species(proj):
    return [cellgen.cells.PROJ_SETS[proj]]


@pytest.mark.parametrize("name,over", [("c1", {}),
                                        ("t", dict(lattice=np.array([[7.0, 0.4, 0.0],
                                                                     [0.0, 8.0, 0.3],
                                                                     [0.5, 0.0, 9.0]]),
                                                   frac=np.array([[0.1, 0.2, 0.3],
                                                                  [0.6, 0.5, 0.9]]),
                                                   kpt=(0.13, -0.05, 0.21), ecutwfc=12.0,
                                                   fft=(15, 16, 18), proj="s2pd",
                                                   dfixed=True, nbnd=4))])
def test_matches_generator_closed_form(name, over):
    # the generator builds beta from the closed-form radial transform and
    # polynomial harmonics q^l Y_lm; the oracle from quadrature and unit-vector
    # harmonics.  A wrong (-i)^l, structure-factor sign or projector order fails.
    c = cellgen.make_cell(name, **over)
    b = ob.beta_projectors(c.lattice, c.kpt, c.miller, c.positions,
                           np.zeros(c.nat, dtype=int), _species(c.proj_set))
    assert b.shape == c.beta.shape
    assert np.abs(b - c.beta).max() < 1e-11 * np.abs(c.beta).max()


def test_parseval_norm():
    # sum over G of |beta_i(k+G)|^2 = int |beta_c(r) Y_lm|^2 d^3r
    #   = int r^(2l+2) exp(-2 r^2/s) dr = Gamma(l+3/2)/2 (s/2)^(l+3/2)
    # for an isolated projector inside a large sphere: a missing 4 pi or
    # 1/sqrt(Omega) fails by orders of magnitude, a wrong harmonic norm by O(1)
    a = 14.0
    lat = np.diag([a, a, a])
    c = cellgen.make_cell("t", lattice=lat, frac=np.array([[0.3, 0.4, 0.5]]),
                          kpt=(0.07, 0.02, -0.04), ecutwfc=60.0, fft=(80, 80, 80),
                          proj="s2pd", dfixed=True, nbnd=4, with_beta=False)
    b = ob.beta_projectors(c.lattice, c.kpt, c.miller, c.positions, [0], _species("s2pd"))
    got = np.sum(np.abs(b) ** 2, axis=1)
    i = 0
    for (l, s) in cellgen.cells.PROJ_SETS["s2pd"]:
        ref = math.gamma(l + 1.5) / 2.0 * (s / 2.0) ** (l + 1.5)
        for m in range(2 * l + 1):
            assert abs(got[i] - ref) < 1e-7 * ref, (l, s, m, got[i], ref)
            i += 1


def test_lattice_translation_phase():
    # moving an atom by a lattice vector R multiplies its projectors by
    # exp(-i k . R): using G instead of k + G in the structure factor fails
    c = cellgen.make_cell("c1")
    sp_ = _species(c.proj_set)
    b0 = ob.beta_projectors(c.lattice, c.kpt, c.miller, c.positions, [0, 0], sp_)
    R = c.lattice[0] - 2.0 * c.lattice[2]
    pos = c.positions.copy()
    pos[1] += R
    b1 = ob.beta_projectors(c.lattice, c.kpt, c.miller, pos, [0, 0], sp_)
    n0 = b0.shape[0] // 2
    assert np.abs(b1[:n0] - b0[:n0]).max() == 0.0
    ph = np.exp(-1j * np.dot(c.kpt, R))
    assert np.abs(b1[n0:] - ph * b0[n0:]).max() < 1e-13 * np.abs(b0).max()
