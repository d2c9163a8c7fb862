"""The seeded input generator: workload shapes and the model pseudopotential.

* plane-wave / stick / x-extent counts of the named cells are fixed integers
  (enumerated once and written here);
* P8: the closed-form radial transform of r^l exp(-r^2/sigma) equals numerical
  quadrature with spherical Bessel functions;
* P9: the Fourier-series local potential equals the direct real-space image
  sum of the Gaussians.
"""

import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import spherical_jn

import cellgen
from cellgen import cells as C


@pytest.mark.parametrize("name,npw,nst,ext,box", [
    ("c1", 1503, 161, 15, (30, 30, 30)),
    ("c2", 23976, 1007, 36, (72, 72, 72)),
    ("c3", 148093, 3389, 65, (135, 135, 135)),
    ("c5", 186449, 3809, 69, (160, 160, 168)),
])
def test_workload_shapes(name, npw, nst, ext, box):
    sp = C._spec(name)
    lat = np.asarray(sp["lattice"], float)
    k = np.asarray(sp["kfrac"]) * (2 * np.pi / lat[0, 0])
    m = C.sphere_miller(lat, k, sp["ecutwfc"])
    assert m.shape[0] == npw
    assert len(np.unique(m[:, :2], axis=0)) == nst
    assert m[:, 0].max() - m[:, 0].min() + 1 == ext
    assert tuple(sp["fft"]) == box
    # every |m_i| fits the box without aliasing
    assert (2 * np.abs(m).max(0) + 1 <= np.array(box)).all()


def test_miller_lexicographic_sticks_contiguous():
    cell = cellgen.make_cell("c1")
    m = cell.miller.astype(np.int64)
    key = (m[:, 0] * 1000 + m[:, 1]) * 1000 + m[:, 2]
    assert (np.diff(key) > 0).all()
    same = (m[1:, 0] == m[:-1, 0]) & (m[1:, 1] == m[:-1, 1])
    assert (m[1:, 2][same] - m[:-1, 2][same] == 1).all()


def test_minimal_box_served():
    lat = np.diag([5.43, 5.43, 5.43])
    assert C.fft_box_min(lat, 80.0) == (15, 15, 15)
    assert C.fft_box_min(np.diag([40.0, 40.0, 42.0]), 120.0) == (144, 144, 150)


@pytest.mark.parametrize("l,sigma", [(0, 1.5), (1, 1.5), (1, 0.75), (2, 1.5)])
def test_p8_radial_closed_form_vs_quadrature(l, sigma):
    for q in [0.0, 0.3, 1.7, 4.2]:
        val, _ = quad(lambda r: r * r * r ** l * math.exp(-r * r / sigma) * spherical_jn(l, q * r),
                      0, 40, limit=400, epsabs=1e-14, epsrel=1e-12)
        ref = C.radial_ft_closed(l, sigma, np.array(q))
        assert abs(val - ref) < 1e-10


def test_p9_vloc_fourier_equals_image_sum():
    lat = np.diag([10.0, 10.0, 10.0])
    pos = np.array([[0, 0, 0], [5.0, 5.0, 5.0]])
    v1 = C.vloc_fourier(lat, (30, 30, 30), pos)
    v2 = C.vloc_image_sum(lat, (30, 30, 30), pos)
    assert np.abs(v1 - v2).max() < 1e-13


def test_p9_vloc_orthorhombic():
    lat = np.diag([6.0, 7.0, 8.0])
    pos = np.array([[0.3, 1.2, 7.7], [4.0, 0.2, 2.0]])
    v1 = C.vloc_fourier(lat, (24, 25, 30), pos)
    v2 = C.vloc_image_sum(lat, (24, 25, 30), pos)
    assert np.abs(v1 - v2).max() < 1e-12


def test_beta_is_harmonic_times_radial():
    # |beta_s(q)|^2 summed over m of the p-triplet = (3/4pi) q^2 F_1(q)^2 / q^2 * (4pi)^2/Omega
    cell = cellgen.make_cell("c1")
    b = 2 * np.pi / 10.0
    q = np.linalg.norm(cell.miller * b, axis=1)
    p = cell.beta[1:4]
    lhs = (np.abs(p) ** 2).sum(0)
    rhs = (4 * np.pi) ** 2 / 1000.0 * 3 / (4 * np.pi) * C.radial_ft_closed(1, 1.5, q) ** 2
    assert np.abs(lhs - rhs).max() < 1e-14


def test_psi0_seeded_normalised():
    a = cellgen.make_psi0(100, 5, seed=3)
    b = cellgen.make_psi0(100, 5, seed=3)
    assert np.array_equal(a, b)
    assert np.allclose(np.linalg.norm(a, axis=1), 1.0, atol=1e-15)


def test_served_trace_shape():
    tr = cellgen.served_trace(200)
    t = np.array([r["t_arrive"] for r in tr])
    assert (np.diff(t) > 0).all()
    assert 5 < 200 / t[-1] < 40          # rate ~ 20 / s
    assert all(8 <= r["nat"] <= 128 and 1 <= r["nk"] <= 4 for r in tr)
    cell = cellgen.random_served_cell(8, 20.0, 0, seed=9)
    assert cell.nbnd == 16 and cell.fft == (15, 15, 15)
