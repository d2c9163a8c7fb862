"""Pins of the CG oracle (oracle/cg.py) against LAPACK, closed forms and its
own invariants; CPU only."""

import numpy as np
import pytest
import scipy.linalg as sla

import cellgen
import oracle
from oracle.cg import lower_eigpair_2x2


def test_2x2_lower_eigenpair_against_eigh():
    rng = np.random.default_rng(5)
    cases = [(0.3, 0.0 + 0.0j, 1.2), (1.2, 0.0j, 0.3), (0.5, 0.0j, 0.5), (-1.0, 1e-14 + 0j, 2.0)]
    for _ in range(50):
        cases.append((rng.normal(), complex(rng.normal(), rng.normal()), rng.normal()))
    for a, b, c in cases:
        m = np.array([[a, b], [np.conj(b), c]])
        w, _ = np.linalg.eigh(m)
        mu, c0, c1 = lower_eigpair_2x2(a, b, c)
        v = np.array([c0, c1])
        assert abs(mu - w[0]) < 1e-14 * max(1.0, abs(w).max())
        assert abs(np.linalg.norm(v) - 1.0) < 1e-14
        assert np.linalg.norm(m @ v - mu * v) < 1e-13 * max(1.0, abs(w).max())
        assert abs(c0.imag) == 0.0 and c0.real >= 0.0


def _c1():
    c = cellgen.make_cell("c1")
    return c, lambda x: oracle.apply_h(c, x), oracle.hdiag(c)


def test_cg_c1_matches_lapack_and_is_monotone():
    c, ah, hd = _c1()
    nb = 10
    ref = sla.eigh(oracle.dense_h(c), eigvals_only=True, subset_by_index=[0, nb - 1])
    psi0 = cellgen.make_psi0(c.npw, nb, seed=7)
    eps, psi, info = oracle.cg(ah, psi0, hd, rtol=1e-9, maxiter=300, history=True)
    assert info["notconv"] == 0
    assert np.abs(eps - ref).max() < 1e-10, np.abs(eps - ref).max()
    assert np.abs(psi.conj() @ psi.T - np.eye(nb)).max() < 1e-12
    assert info["resid"].max() < 1e-8
    # the Rayleigh quotient of each band never rises
    for lams in info["history"]:
        assert np.all(np.diff(lams) <= 1e-12 * max(1.0, abs(lams).max()))
    # and it agrees with the Davidson oracle
    e_dav, _, _ = oracle.davidson(ah, psi0, hd, rtol=1e-9, nvecx=4 * nb)
    assert np.abs(eps - e_dav).max() < 1e-10


def test_cg_free_electron_shells():
    # V = 0, no projectors: eigenvalues |k + G|^2, shells of 1, 6 and 12 at k = 0
    c = cellgen.make_cell("c1", vzero=True, nobeta=True)
    s = 0.39478417604357434   # (2 pi / 10)^2
    ref = np.array([0.0] + [s] * 6 + [2 * s] * 9)
    psi0 = cellgen.make_psi0(c.npw, 16, seed=8)
    eps, _, info = oracle.cg(lambda x: oracle.apply_h(c, x), psi0, oracle.hdiag(c),
                             rtol=1e-10, maxiter=300)
    assert np.abs(eps - ref).max() < 1e-10


def test_cg_maxiter_reports_unconverged():
    c, ah, hd = _c1()
    psi0 = cellgen.make_psi0(c.npw, 4, seed=9)
    eps, psi, info = oracle.cg(ah, psi0, hd, rtol=1e-14, maxiter=2)
    assert info["notconv"] > 0 and np.all(info["iters"] <= 2)
    assert np.abs(psi.conj() @ psi.T - np.eye(4)).max() < 1e-12
