"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test is chosen so that a plausible mistake somewhere in the oracle (a
dropped term, a wrong sign or index, a transposed axis, a missing conjugate,
a wrong normalisation) fails at least one of them:

* P1  free electrons: eigenvalues are the closed-form lattice shells
      (2 pi / a)^2 |f + m|^2, written here as literals.
* P2  constant potential: H psi - H0 psi = c psi exactly.
* P3  Hermiticity of apply_h.
* P4  the oracle DFT: Parseval, round trip, and agreement with numpy.fft.
* P5  brute force: the FFT route equals the operator written as a dense
      matrix (Fourier coefficients from numpy.fft, not the oracle's DFT),
      and Davidson equals LAPACK's dense eigensolver.
* P6  a single cosine potential couples G only to G +- n0 with amplitude
      v exp(+-i phi): fixes the sign convention and the axis order.
* P7  rank-1 nonlocal operator: eigenvalue from the secular equation.
* P10 O_h symmetry of the first cell: exact degeneracies.
* P11 translation of all atoms by a grid vector leaves the spectrum unchanged.
* P13 linearity.
* P14 k -> k + b1 with the sphere re-centred leaves the spectrum unchanged.
* P15 Ritz values never increase from one Davidson iteration to the next.
"""

import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.optimize import brentq

import cellgen
import oracle

TWO_PI = 2 * math.pi


def _c1(**kw):
    return cellgen.make_cell("c1", **kw)


def _dense_ref(cell):
    """Dense H from its definition with numpy.fft for the Fourier coefficients."""
    n1, n2, n3 = cell.fft
    vt = np.fft.fftn(cell.vloc) / cell.vloc.size
    m = cell.miller
    d = m[:, None, :] - m[None, :, :]
    h = vt[d[..., 2] % n3, d[..., 1] % n2, d[..., 0] % n1]
    b = 2 * np.pi * np.linalg.inv(cell.lattice).T
    q = m @ b + cell.kpt
    h[np.diag_indices_from(h)] += (q * q).sum(1)
    off = doff = 0
    for n in cell.nproj:
        blk = cell.dmat[doff:doff + n * n].reshape(n, n)
        bb = cell.beta[off:off + n]
        h += bb.T @ blk @ bb.conj()
        off += n
        doff += n * n
    return h


# ---------------------------------------------------------------- P4 DFT

@pytest.mark.parametrize("shape", [(5, 6, 7), (15, 10, 6), (9, 8, 1)])
def test_p4_dft_parseval_roundtrip_numpy(shape):
    rng = np.random.default_rng(1)
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    c = oracle.fwd3(f)
    assert np.allclose(np.sum(np.abs(c) ** 2) * f.size, np.sum(np.abs(f) ** 2), rtol=1e-13)
    assert np.abs(oracle.inv3(c) - f).max() < 1e-13
    assert np.abs(c - np.fft.fftn(f) / f.size).max() < 1e-14
    assert np.abs(oracle.inv3(f) - np.fft.ifftn(f) * f.size).max() < 1e-12


def test_p4_dft_axis_order():
    # a delta at (z, y, x) = (1, 2, 3) transforms to exp(-2 pi i (m3 + 2 m2 / N2 ...)).
    shape = (4, 5, 6)
    f = np.zeros(shape, complex)
    f[1, 2, 3] = 1.0
    c = oracle.fwd3(f)
    m3, m2, m1 = np.meshgrid(range(4), range(5), range(6), indexing="ij")
    ref = np.exp(-2j * np.pi * (m3 * 1 / 4 + m2 * 2 / 5 + m1 * 3 / 6)) / f.size
    assert np.abs(c - ref).max() < 1e-15


# ---------------------------------------------------------------- P1 free electrons

def test_p1_free_electron_gamma_c1():
    cell = _c1(vzero=True, nobeta=True)
    psi0 = cellgen.make_psi0(cell.npw, 16, seed=10502)
    eps, psi, info = oracle.davidson(lambda x: oracle.apply_h(cell, x), psi0,
                                     oracle.hdiag(cell), rtol=1e-9, nvecx=64)
    s = 0.39478417604357434   # (2 pi / 10)^2
    ref = np.array([0.0] + [s] * 6 + [2 * s] * 9)
    assert info["converged"]
    assert np.abs(eps - ref).max() < 1e-10


def test_p1_dense_eigs_free_electron_shells():
    # the dense route at V = 0, no projectors: the lowest |k+G|^2 shells of C1
    cell = _c1(vzero=True, nobeta=True)
    s = 0.39478417604357434
    ref = np.array([0.0] + [s] * 6 + [2 * s] * 9)
    assert np.abs(oracle.dense_eigs(cell, 16) - ref).max() < 1e-12


def test_p1_free_electron_kpoint_c2_shells():
    # k = (1/4,1/4,1/4) 2pi/a, a = 20.52: |f+m|^2 = 3/16, 11/16 (x3), 19/16 (x3),
    # 27/16 (x1), 35/16 (x3) ... in units of (2 pi / a)^2.
    cell = cellgen.make_cell("c2", vzero=True, nobeta=True, ecutwfc=2.0, fft=(16, 16, 16))
    u = (TWO_PI / 20.52) ** 2
    ref = u * np.array([3, 11, 11, 11, 19, 19, 19, 27]) / 16.0
    eps, _, info = oracle.davidson(lambda x: oracle.apply_h(cell, x),
                                   cellgen.make_psi0(cell.npw, 8), oracle.hdiag(cell),
                                   rtol=1e-10, nvecx=24)
    assert abs(ref[0] - 0.017579) < 1e-6 and abs(ref[1] - 0.064458) < 1e-6
    assert np.abs(eps - ref).max() < 1e-11


# ---------------------------------------------------------------- P2 constant V

def test_p2_constant_potential_shift():
    c = 0.731
    cell = _c1()
    cell0 = _c1(vzero=True)
    cellc = _c1(vloc=np.full((30, 30, 30), c))
    psi = cellgen.make_psi0(cell.npw, 3, seed=7)
    d = oracle.apply_h(cellc, psi) - oracle.apply_h(cell0, psi)
    assert np.abs(d - c * psi).max() < 1e-13


# ---------------------------------------------------------------- P3 / P13

def test_p3_hermiticity_and_p13_linearity():
    cell = _c1()
    rng = np.random.default_rng(3)
    phi = cellgen.make_psi0(cell.npw, 1, seed=1)[0]
    psi = cellgen.make_psi0(cell.npw, 1, seed=2)[0]
    hp = oracle.apply_h(cell, psi)[0]
    hf = oracle.apply_h(cell, phi)[0]
    assert abs(np.vdot(phi, hp) - np.conj(np.vdot(psi, hf))) < 1e-13
    a, b = 0.3 - 1.1j, -2.0 + 0.25j
    lhs = oracle.apply_h(cell, a * psi + b * phi)[0]
    assert np.abs(lhs - (a * hp + b * hf)).max() < 1e-13 * np.abs(lhs).max() * 10
    del rng


# ---------------------------------------------------------------- P5 brute force

def test_p5_fft_route_equals_dense_c1():
    cell = _c1()
    h = _dense_ref(cell)
    psi = cellgen.make_psi0(cell.npw, 4, seed=11)
    hp = oracle.apply_h(cell, psi)
    assert np.abs(psi @ h.T - hp).max() < 1e-12
    assert np.abs(oracle.dense_h(cell) - h).max() < 1e-13


def test_p5_fft_route_equals_dense_anisotropic_kpoint():
    # orthorhombic cell, non-cubic box and a general k: catches axis mix-ups
    cell = cellgen.make_cell("t", lattice=np.diag([7.0, 8.0, 9.5]), frac=np.array(
        [[0.1, 0.2, 0.3], [0.6, 0.5, 0.9], [0.3, 0.8, 0.55]]), kpt=(0.11, -0.07, 0.23),
        ecutwfc=12.0, ecutrho=48.0, fft=None, proj="s2pd", dfixed=False, nbnd=8)
    assert len(set(cell.fft)) == 3
    h = _dense_ref(cell)
    assert np.abs(h - h.conj().T).max() < 1e-13
    psi = cellgen.make_psi0(cell.npw, 3, seed=12)
    assert np.abs(psi @ h.T - oracle.apply_h(cell, psi)).max() < 1e-12


def test_p5_davidson_equals_lapack_c1():
    cell = _c1()
    h = oracle.dense_h(cell)
    ref = sla.eigh(h, eigvals_only=True, subset_by_index=[0, 15])
    eps, psi, info = oracle.davidson(lambda x: x @ h.T, cellgen.make_psi0(cell.npw, 16),
                                     oracle.hdiag(cell), rtol=1e-9)
    assert info["converged"]
    assert np.abs(eps - ref).max() < 1e-10
    # Ritz vectors orthonormal and residuals small
    assert np.abs(psi.conj() @ psi.T - np.eye(16)).max() < 1e-10
    assert np.abs(psi @ h.T - eps[:, None] * psi).max() < 1e-8


def test_p5_davidson_equals_lapack_served_cell():
    cell = cellgen.random_served_cell(nat=8, ecutwfc=20.0, kidx=1, seed=5)
    h = _dense_ref(cell)
    nb = cell.nbnd
    ref = sla.eigh(h, eigvals_only=True, subset_by_index=[0, nb - 1])
    eps, _, info = oracle.davidson(lambda x: oracle.apply_h(cell, x),
                                   cellgen.make_psi0(cell.npw, nb), oracle.hdiag(cell),
                                   rtol=1e-9, nvecx=4 * nb)
    assert info["converged"]
    assert np.abs(eps - ref).max() < 1e-10


# ---------------------------------------------------------------- P6 single cosine

def test_p6_single_cosine_couples_g_plus_minus_n0():
    cell = cellgen.make_cell("t", lattice=np.diag([6.0, 7.0, 8.0]), frac=np.zeros((1, 3)),
                             ecutwfc=10.0, fft=(12, 15, 16), proj="sp", nbnd=4, nobeta=True)
    n1, n2, n3 = cell.fft
    n0 = np.array([1, 2, -3])
    v, phi = 0.37, 0.61
    j3, j2, j1 = np.meshgrid(range(n3), range(n2), range(n1), indexing="ij")
    arg = 2 * np.pi * (n0[0] * j1 / n1 + n0[1] * j2 / n2 + n0[2] * j3 / n3) + phi
    cell.vloc = 2 * v * np.cos(arg)
    m = cell.miller
    ig = int(np.nonzero((m == [0, 0, 0]).all(1))[0][0])
    e = np.zeros((1, cell.npw), complex)
    e[0, ig] = 1.0
    out = oracle.vloc_psi(cell, e)[0]
    ip = int(np.nonzero((m == n0).all(1))[0][0])
    im = int(np.nonzero((m == -n0).all(1))[0][0])
    ref = np.zeros(cell.npw, complex)
    ref[ip] = v * np.exp(1j * phi)
    ref[im] = v * np.exp(-1j * phi)
    assert np.abs(out - ref).max() < 1e-14


# ---------------------------------------------------------------- P7 rank-1 nonlocal

def test_p7_rank1_nonlocal_secular_equation():
    cell = _c1(vzero=True)
    cell.beta = cell.beta[:1].copy()        # the s projector of atom 0 only
    cell.nproj = np.array([1], dtype=np.int32)
    dval = -3.0
    cell.dmat = np.array([dval], dtype=complex)
    kin = (TWO_PI / 10.0) ** 2 * (cell.miller ** 2).sum(1)
    b2 = np.abs(cell.beta[0]) ** 2

    def f(lam):
        return 1.0 - dval * np.sum(b2 / (lam - kin))

    lam0 = brentq(f, -1e3, -1e-12, xtol=1e-15, rtol=1e-15)
    eps, _, info = oracle.davidson(lambda x: oracle.apply_h(cell, x),
                                   cellgen.make_psi0(cell.npw, 4), oracle.hdiag(cell),
                                   rtol=1e-10, nvecx=16)
    assert lam0 < 0
    assert abs(eps[0] - lam0) < 1e-10


# ---------------------------------------------------------------- P10, P11, P14, P15

def _lowest(cell, nb, nvecx=None):
    h = oracle.dense_h(cell)
    return sla.eigh(h, eigvals_only=True, subset_by_index=[0, nb - 1])


def test_p10_oh_degeneracies_c1():
    eps = _lowest(_c1(), 16)
    groups = [(0, 1), (1, 2), (2, 3), (3, 6), (6, 8), (8, 11), (11, 14), (14, 16)]
    for lo, hi in groups:
        assert np.ptp(eps[lo:hi]) < 1e-12
    for (lo1, hi1), (lo2, _) in zip(groups[:-1], groups[1:]):
        assert eps[lo2] - eps[hi1 - 1] > 1e-3


def test_p11_translation_by_grid_vector():
    base = _lowest(_c1(), 16)
    shift = np.array([3, -7, 11]) / 30.0 * 10.0
    moved = _c1(frac=np.array([[0, 0, 0], [.5, .5, .5]]) + shift / 10.0)
    assert np.abs(_lowest(moved, 16) - base).max() < 1e-12


def test_p14_k_shift_by_reciprocal_vector():
    kw = dict(lattice=np.diag([6.0, 6.5, 7.0]), frac=np.array([[0, 0, 0], [.4, .3, .6]]),
              ecutwfc=10.0, ecutrho=40.0, fft=(12, 12, 15), proj="2s2p", dfixed=False,
              nbnd=6)
    k = np.array([0.05, 0.1, -0.02])
    b1 = 2 * np.pi / 6.0 * np.array([1.0, 0, 0])
    c0 = cellgen.make_cell("t", kpt=k, **kw)
    c1 = cellgen.make_cell("t", kpt=k + b1, **kw)
    assert c0.npw == c1.npw
    assert np.abs(_lowest(c0, 6) - _lowest(c1, 6)).max() < 1e-12


def test_p15_ritz_values_monotone():
    cell = _c1()
    h = oracle.dense_h(cell)
    eps, _, info = oracle.davidson(lambda x: x @ h.T, cellgen.make_psi0(cell.npw, 16),
                                   oracle.hdiag(cell), rtol=1e-9, history=True)
    hist = info["history"]
    assert info["restarts"] > 0
    assert (np.diff(hist, axis=0) <= 1e-12).all()


def test_hdiag_equals_dense_diagonal():
    cell = cellgen.make_cell("c1", proj="s2pd", dfixed=False)
    h = _dense_ref(cell)
    assert np.abs(oracle.hdiag(cell) - np.real(np.diag(h))).max() < 1e-13
