"""Pins of the overlap operator and the generalized Davidson oracle
(oracle/overlap.py), without the GPU:

* with q = 0, S is the identity and the generalized solver gives the standard
  Davidson's eigenvalues;
* S is Hermitian and, with q >= 0, bounded below by the identity; its dense
  form applied to bands equals apply_s;
* rank-1 secular equation: with V = 0, D = 0 and one projector of weight q,
  H y = eps S y has its lowest eigenvalue at the root of
  1 = eps q sum_G |beta(G)|^2 / (T_G - eps) in (0, min T) (k != 0), found by
  bracketing, against both the dense generalized eigensolve and the Davidson;
* the Davidson output is S-orthonormal with small generalized residuals and
  matches the dense generalized eigenvalues on a small cell.
"""

import numpy as np
import scipy.optimize as so

import cellgen
import oracle
from oracle import overlap


def _small(**kw):
    return cellgen.make_cell("c1", ecutwfc=8.0, fft=(18, 18, 18), nbnd=8,
                             kfrac=(0.25, 0.1, -0.15), **kw)


def test_q_zero_is_the_standard_problem():
    c = _small()
    assert c.qmat is None
    psi = cellgen.make_psi0(c.npw, 3, seed=3)
    assert np.array_equal(overlap.apply_s(c, psi), psi)
    cz = _small(overlap=True)
    cz.qmat = np.zeros_like(cz.qmat)
    psi0 = cellgen.make_psi0(c.npw, 8)
    e1, _, _ = oracle.davidson(lambda x: oracle.apply_h(c, x), psi0, oracle.hdiag(c), rtol=1e-10,
                               nvecx=24)
    e2, _, _ = overlap.davidson_gen(lambda x: oracle.apply_h(cz, x),
                                    lambda x: overlap.apply_s(cz, x), psi0, oracle.hdiag(cz),
                                    rtol=1e-10, nvecx=24)
    assert np.abs(e1 - e2).max() < 1e-11


def test_s_hermitian_positive_and_dense_form():
    c = _small(overlap=True)
    rng = np.random.default_rng(4)
    a = cellgen.make_psi0(c.npw, 2, seed=5)
    sa = overlap.apply_s(c, a)
    assert abs(np.vdot(a[0], sa[1]) - np.conj(np.vdot(a[1], sa[0]))) < 1e-13
    assert np.all(np.real(np.einsum("bg,bg->b", a.conj(), sa)) >= 1.0 - 1e-14)
    assert np.real(np.einsum("bg,bg->b", a.conj(), sa)).max() > 1.0 + 1e-6   # q acts
    ds = overlap.dense_s(c)
    assert np.abs(ds - ds.conj().T).max() < 1e-14
    assert np.abs((ds @ a.T).T - sa).max() < 1e-13
    del rng


def test_rank1_secular_equation():
    # V = 0, D = 0, one atom with one s projector of weight q
    c = _small(vzero=True, overlap=True, frac=np.array([[0.1, 0.2, 0.3]]))
    keep = 1
    c.beta = c.beta[:keep]
    c.nproj = np.array([keep], dtype=np.int32)
    c.dmat = np.zeros(1, dtype=np.complex128)
    q = 0.7
    c.qmat = np.array([q], dtype=np.complex128)
    t = oracle.kinetic(c)
    w = np.abs(c.beta[0]) ** 2
    assert t.min() > 0
    f = lambda e: e * q * np.sum(w / (t - e)) - 1.0
    root = so.brentq(f, 1e-12, t.min() * (1 - 1e-12), xtol=1e-15, rtol=1e-15)
    e_dense = overlap.dense_eigs_gen(c, 2)
    assert abs(e_dense[0] - root) < 1e-12
    e_dav, _, info = overlap.davidson_gen(lambda x: oracle.apply_h(c, x),
                                          lambda x: overlap.apply_s(c, x),
                                          cellgen.make_psi0(c.npw, 4), oracle.hdiag(c),
                                          rtol=1e-11, nvecx=16)
    assert info["converged"] and abs(e_dav[0] - root) < 1e-11


def test_davidson_gen_matches_dense_and_is_s_orthonormal():
    c = _small(overlap=True)
    e_ref = overlap.dense_eigs_gen(c, 8)
    eps, psi, info = overlap.davidson_gen(lambda x: oracle.apply_h(c, x),
                                          lambda x: overlap.apply_s(c, x),
                                          cellgen.make_psi0(c.npw, 8), oracle.hdiag(c),
                                          rtol=1e-10, nvecx=32)
    assert info["converged"]
    assert np.abs(eps - e_ref).max() < 1e-10
    g = psi.conj() @ overlap.apply_s(c, psi).T
    assert np.abs(g - np.eye(8)).max() < 1e-10
    r = oracle.apply_h(c, psi) - eps[:, None] * overlap.apply_s(c, psi)
    assert np.linalg.norm(r, axis=1).max() <= 1e-10
    # S != I matters: the standard problem's eigenvalues differ
    assert np.abs(eps - oracle.dense_eigs(c, 8)).max() > 1e-3
