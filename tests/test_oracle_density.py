"""Pins of the charge density oracle (CPU): quadrature, closed forms, brute
force, translation, linearity.  Each names the plausible mistake it catches."""

import numpy as np
import pytest

import cellgen
import oracle


def _tiny_cell():
    # anisotropic box with odd and even sizes, general k, small sphere
    return cellgen.make_cell("t", lattice=np.array([[6.0, 0.3, 0.0], [0.0, 7.0, 0.4],
                                                    [0.2, 0.0, 8.0]]),
                             frac=np.array([[0.1, 0.2, 0.3]]), kpt=(0.11, -0.07, 0.23),
                             ecutwfc=6.0, fft=(9, 10, 12), proj="sp", dfixed=True, nbnd=4)


def test_quadrature_equals_occupation_sum():
    # integral of rho over the cell = sum of occupations (drops of 1/Omega,
    # of the |.|^2 or of bands fail this)
    c = cellgen.make_cell("c1")
    psi = cellgen.make_psi0(c.npw, 6, seed=71)
    occ = np.array([2.0, 2.0, 1.5, 1.0, 0.25, 0.0])
    rho = oracle.density(c, psi, occ)
    n = np.prod(c.fft)
    assert abs(oracle.cell_volume(c) / n * rho.sum() - occ.sum()) < 1e-12


def test_single_plane_wave_is_uniform():
    c = cellgen.make_cell("c1")
    psi = np.zeros((1, c.npw), dtype=np.complex128)
    psi[0, 17] = np.exp(0.3j)
    rho = oracle.density(c, psi, [2.0])
    assert np.allclose(rho, 2.0 / oracle.cell_volume(c), rtol=0, atol=1e-14)


def test_two_plane_waves_closed_form():
    # |a e^{iG1.r} + b e^{iG2.r}|^2 = |a|^2 + |b|^2 + 2 Re(a conj(b) e^{i(G1-G2).r}),
    # written with explicit cosines on the grid points (an axis swap or a
    # transposed box fails it: G1 - G2 is anisotropic)
    c = _tiny_cell()
    m = c.miller
    i1 = int(np.flatnonzero((m == [1, 0, 0]).all(1))[0])
    i2 = int(np.flatnonzero((m == [0, -1, 1]).all(1))[0])
    a, b = 0.6 - 0.2j, -0.3 + 0.7j
    psi = np.zeros((1, c.npw), dtype=np.complex128)
    psi[0, i1], psi[0, i2] = a, b
    rho = oracle.density(c, psi, [1.0])
    n1, n2, n3 = c.fft
    z, y, x = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    d = m[i1] - m[i2]
    th = 2 * np.pi * (d[0] * x / n1 + d[1] * y / n2 + d[2] * z / n3)
    ab = a * np.conj(b)
    ref = abs(a) ** 2 + abs(b) ** 2 + 2 * (ab.real * np.cos(th) - ab.imag * np.sin(th))
    assert np.abs(rho - ref / oracle.cell_volume(c)).max() < 1e-14


def test_brute_force_tiny_cell():
    c = _tiny_cell()
    psi = cellgen.make_psi0(c.npw, 3, seed=72)
    occ = [2.0, 1.0, 0.5]
    assert np.abs(oracle.density(c, psi, occ) - oracle.density_direct(c, psi, occ)).max() \
        < 1e-13


def test_grid_translation_rolls_density():
    # psi(r - t) for t one grid step along a1: c(G) -> c(G) exp(-2 pi i h / N1);
    # rho rolls by +1 along x (a flipped transform sign rolls it the other way)
    c = _tiny_cell()
    psi = cellgen.make_psi0(c.npw, 2, seed=73)
    n1 = c.fft[0]
    shifted = psi * np.exp(-2j * np.pi * c.miller[:, 0] / n1)[None, :]
    r0 = oracle.density(c, psi, [1.0, 1.0])
    r1 = oracle.density(c, shifted, [1.0, 1.0])
    assert np.abs(r1 - np.roll(r0, 1, axis=2)).max() < 1e-14


def test_linear_in_occupations_and_nonnegative():
    c = cellgen.make_cell("c1")
    psi = cellgen.make_psi0(c.npw, 3, seed=74)
    f1, f2 = np.array([1.0, 0.0, 2.0]), np.array([0.5, 1.5, 0.0])
    r = oracle.density(c, psi, f1 + f2)
    assert np.abs(r - oracle.density(c, psi, f1) - oracle.density(c, psi, f2)).max() < 1e-13
    assert r.min() >= 0.0


def test_rejects_mismatched_occupations():
    c = cellgen.make_cell("c1")
    with pytest.raises(ValueError):
        oracle.density(c, cellgen.make_psi0(c.npw, 2, seed=1), [1.0])
