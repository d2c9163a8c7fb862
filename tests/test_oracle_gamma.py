"""Pins of the Gamma-point representation used by the oracle (CPU): the
half-sphere storage and its expansion describe real functions, H maps them to
real functions, and the real eigenproblem has the complex problem's
eigenvalues.  Each names the plausible mistake it catches."""

import numpy as np
import scipy.linalg as sla

import cellgen
import oracle
from oracle import gamma


def _c1():
    return cellgen.make_cell("c1")


def test_sphere_is_mirror_symmetric_in_lexicographic_order():
    # entry i0 - h is -G of entry i0 + h: the index arithmetic expand relies on
    c = _c1()
    m = c.miller
    i0 = int(np.flatnonzero((m == 0).all(1))[0])
    assert m.shape[0] == 2 * i0 + 1
    assert (m[i0 - np.arange(i0 + 1)] == -m[i0 + np.arange(i0 + 1)]).all()
    h = cellgen.gamma_half(c)
    assert h.miller.shape[0] == i0 + 1 and (h.miller[0] == 0).all()


def test_expanded_vectors_are_real_in_real_space():
    # a wrong mirror index or a missing conjugate gives a complex psi(r)
    c = _c1()
    n1, n2, n3 = c.fft
    ph = gamma.expand(cellgen.make_psi0((c.npw + 1) // 2, 3, seed=5))
    for b in range(3):
        box = np.zeros((n3, n2, n1), dtype=np.complex128)
        box[c.miller[:, 2] % n3, c.miller[:, 1] % n2, c.miller[:, 0] % n1] = ph[b]
        f = oracle.inv3(box)
        assert np.abs(f.imag).max() < 1e-13 * np.abs(f.real).max()
    assert np.array_equal(gamma.restrict(ph)[:, 1:], cellgen.make_psi0((c.npw + 1) // 2, 3,
                                                                        seed=5)[:, 1:])


def test_h_keeps_gamma_symmetry_and_inner_product_form():
    # H is real in real space at k = 0: H psi of a symmetric vector is
    # symmetric; and the half-sphere inner product 2 Re sum - a0 b0 equals the
    # full one (a dropped factor 2 or a doubled G = 0 term fails)
    c = _c1()
    nh = (c.npw + 1) // 2
    a = gamma.expand(cellgen.make_psi0(nh, 2, seed=6))
    hp = oracle.apply_h(c, a)
    back = gamma.expand(gamma.restrict(hp))
    assert np.abs(back - hp).max() < 1e-12 * np.abs(hp).max()
    x, y = gamma.restrict(a)[0], gamma.restrict(hp)[1]
    half = 2 * np.vdot(x, y).real - x[0].real * y[0].real
    assert abs(half - np.vdot(a[0], hp[1])) < 1e-12 * abs(np.vdot(a[0], hp[1]))


def test_real_eigenproblem_has_the_complex_eigenvalues():
    # the lowest eigenvalues of H restricted to real functions (a real
    # symmetric matrix in the basis cos/sin of the half sphere) equal those of
    # the complex problem, multiplicities included
    c = cellgen.make_cell("c1")
    H = oracle.dense_h(c)
    n = c.npw
    i0 = n // 2
    # orthonormal real basis of symmetric vectors: e_0, (e_G + e_-G)/sqrt2, i(e_G - e_-G)/sqrt2
    B = np.zeros((n, n), dtype=np.complex128)
    B[i0, 0] = 1.0
    for h in range(1, i0 + 1):
        B[i0 + h, 2 * h - 1] = B[i0 - h, 2 * h - 1] = 1 / np.sqrt(2)
        B[i0 + h, 2 * h] = 1j / np.sqrt(2)
        B[i0 - h, 2 * h] = -1j / np.sqrt(2)
    Hr = B.conj().T @ H @ B
    assert np.abs(Hr.imag).max() < 1e-12 * np.abs(Hr).max()
    er = sla.eigh(Hr.real, eigvals_only=True, subset_by_index=[0, c.nbnd - 1])
    ec = sla.eigh(H, eigvals_only=True, subset_by_index=[0, c.nbnd - 1])
    assert np.abs(er - ec).max() < 1e-10
