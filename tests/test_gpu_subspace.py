"""The library's own dense solver of the Rayleigh-Ritz step (qeh_subspace_eigh
and qeh_davidson's own subspace path) against LAPACK: random Hermitian pencils,
exact multiplets (which Householder reduction does not split), near
multiplets, a real symmetric pencil of the Gamma path, a window that cuts a
multiplet, bitwise repeatability, the error returns, and Davidson solves on it
against the dense oracle Hamiltonian."""

import os
import sys

import numpy as np
import pytest
import scipy.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import cellgen  # noqa: E402
import oracle   # noqa: E402

pytestmark = pytest.mark.gpu


def _q():
    import paper_2104_10502_amd as q
    return q


def _herm(rng, n, real=False):
    x = rng.standard_normal((n, n)) + (0 if real else 1j) * rng.standard_normal((n, n))
    return (x + x.conj().T) / 2


def _spd(rng, n, real=False):
    x = rng.standard_normal((n, n)) + (0 if real else 1j) * rng.standard_normal((n, n))
    return np.eye(n) + 0.3 * (x @ x.conj().T) / n


def _solve(h, s, nb):
    import torch
    q = _q()
    ht = torch.from_numpy(np.ascontiguousarray(h, dtype=np.complex128)).cuda()
    st = torch.from_numpy(np.ascontiguousarray(s, dtype=np.complex128)).cuda()
    e, y = q.subspace_eigh(ht, st, nb)
    torch.cuda.synchronize()
    return e.cpu().numpy(), y.cpu().numpy()


def _check(h, s, nb, tol=1e-12, label=""):
    e, y = _solve(h, s, nb)
    ref = sla.eigh(h, s, eigvals_only=True, subset_by_index=[0, nb - 1])
    scale = max(1.0, np.abs(sla.eigh(h, s, eigvals_only=True)).max())
    assert np.all(np.diff(e) >= -1e-14 * scale), label
    err = np.abs(e - ref).max() / scale
    res = np.linalg.norm(h @ y - (s @ y) * e[None, :], axis=0).max() / scale
    orth = np.abs(y.conj().T @ s @ y - np.eye(nb)).max()
    print("%s n=%d nb=%d: eig %.1e resid %.1e orth %.1e" % (label, len(h), nb, err, res, orth),
          flush=True)
    assert err < tol, (label, err)
    assert res < 10 * tol, (label, res)
    assert orth < 1e-10, (label, orth)
    return e, y


@pytest.mark.parametrize("n,nb", [(1, 1), (2, 1), (17, 9), (64, 32), (200, 100), (256, 256),
                                  (512, 256), (700, 350), (1024, 512), (2048, 1024)])
def test_random_pencil(n, nb):
    rng = np.random.default_rng(n)
    _check(_herm(rng, n), _spd(rng, n), nb, label="random")


@pytest.mark.parametrize("mult", [2, 6, 12])
@pytest.mark.parametrize("n", [64, 300])
def test_exact_multiplets(n, mult):
    # H = L A L^H, S = L L^H: the pencil's eigenvalues are A's, each `mult` times
    rng = np.random.default_rng(100 + n + mult)
    u, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.repeat(rng.standard_normal(n // mult + 1), mult)[:n]
    a = (u * lam) @ u.conj().T
    s = _spd(rng, n)
    lo = np.linalg.cholesky(s)
    _check(lo @ a @ lo.conj().T, s, n // 2, label="multiplets x%d" % mult)


@pytest.mark.parametrize("gap", [1e-9, 1e-13])
def test_near_multiplets(gap):
    rng = np.random.default_rng(7)
    n = 160
    u, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.sort(rng.standard_normal(n))
    lam[1::2] = lam[0::2] + gap * (1 + np.abs(lam[0::2]))
    _check((u * lam) @ u.conj().T, np.eye(n), n // 2, label="pairs %g apart" % gap)


def test_window_cuts_a_multiplet():
    rng = np.random.default_rng(9)
    n = 96
    u, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.sort(rng.standard_normal(n))
    lam[40:56] = lam[40]          # 16-fold, window ends at 48
    _check((u * lam) @ u.conj().T, np.eye(n), 48, label="cut multiplet")


@pytest.mark.parametrize("n", [64, 128, 256, 1000])
def test_real_symmetric_pencil(n):
    # the Gamma path's reduced pair: complex storage, imaginary parts zero
    rng = np.random.default_rng(n + 5)
    h, s = _herm(rng, n, real=True), _spd(rng, n, real=True)
    e, y = _check(h.astype(np.complex128), s.astype(np.complex128), n // 2, label="real")
    assert np.abs(y.imag).max() == 0.0


@pytest.mark.parametrize("n", [48, 100, 300])
def test_bitwise_repeatable(n):
    # (repeats: a workgroup race would show as a rare bitwise difference;
    # n = 48 runs the LDS-resident reduction alone, 100 and 300 the step
    # kernel, the blocked Cholesky and the multi-workgroup bisection too)
    rng = np.random.default_rng(11)
    h, s = _herm(rng, n), _spd(rng, n)
    e1, y1 = _solve(h, s, n // 2)
    for _ in range(6):
        e2, y2 = _solve(h, s, n // 2)
        assert np.array_equal(e1, e2) and np.array_equal(y1, y2)


def test_error_returns():
    import torch
    q = _q()
    rng = np.random.default_rng(3)
    h = _herm(rng, 32)
    bad_s = np.diag(np.r_[np.ones(20), -1.0, np.ones(11)]).astype(np.complex128)
    with pytest.raises(q.QehError) as ei:
        _solve(h, bad_s, 8)
    assert ei.value.status == q.QEH_ERR_CHOLESKY
    hn = h.copy()
    hn[3, 5] = np.nan
    hn[5, 3] = np.nan
    with pytest.raises(q.QehError) as ei:
        _solve(hn, np.eye(32), 8)
    assert ei.value.status == q.QEH_ERR_NUMERIC
    # the same two failures at an order that takes the multi-workgroup
    # Cholesky and Householder paths
    h2 = _herm(rng, 200)
    bad_s2 = np.diag(np.r_[np.ones(150), -1.0, np.ones(49)]).astype(np.complex128)
    with pytest.raises(q.QehError) as ei:
        _solve(h2, bad_s2, 8)
    assert ei.value.status == q.QEH_ERR_CHOLESKY
    h2[77, 140] = np.nan
    h2[140, 77] = np.nan
    with pytest.raises(q.QehError) as ei:
        _solve(h2, np.eye(200), 8)
    assert ei.value.status == q.QEH_ERR_NUMERIC
    big = torch.zeros((2049, 2049), dtype=torch.complex128, device="cuda")
    with pytest.raises(q.QehError) as ei:
        q.subspace_eigh(big, big, 4)
    assert ei.value.status == q.QEH_ERR_INVALID


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-6)])
def test_davidson_own_solver_c1(prec, tol):
    # C1 (O_h symmetric: exact multiplets, a 12-fold shell cut by the window)
    import torch
    q = _q()
    c = cellgen.make_cell("c1")
    ref = sla.eigh(oracle.dense_h(c), eigvals_only=True, subset_by_index=[0, 15])
    res = {}
    for sub in (q.QEH_SUBSPACE_OWN, q.QEH_SUBSPACE_ROCSOLVER):
        ctx = q.Context.from_cell(c, precision=prec, block=16)
        p = torch.from_numpy(cellgen.make_psi0(c.npw, 16)).cuda()
        eig, info = ctx.davidson(p, rtol=1e-8, subspace=sub)
        assert info["status"] == 0
        res[sub] = np.sort(eig)
        # orthonormal Ritz vectors
        g = (p.conj() @ p.T).cpu().numpy()
        assert np.abs(g - np.eye(16)).max() < 1e-10
        ctx.close()
    print("own vs LAPACK %.2e, rocSOLVER vs LAPACK %.2e" % (
        np.abs(res[1] - ref).max(), np.abs(res[2] - ref).max()), flush=True)
    assert np.abs(res[q.QEH_SUBSPACE_OWN] - ref).max() < tol


def test_davidson_own_solver_gamma_64_bands_and_repeatable():
    import torch
    q = _q()
    c = cellgen.make_cell("c1")
    h = cellgen.gamma_half(c)
    ref = sla.eigh(oracle.dense_h(c), eigvals_only=True, subset_by_index=[0, 63])
    out = []
    for _ in range(2):
        ctx = q.Context.from_cell(h, precision=0, block=32)
        p = torch.from_numpy(cellgen.make_psi0(h.npw, 64, seed=5)).cuda()
        eig, info = ctx.davidson(p, rtol=1e-8, subspace=q.QEH_SUBSPACE_OWN)
        assert info["status"] == 0
        out.append((eig.copy(), p.cpu().numpy()))
        ctx.close()
    assert np.abs(np.sort(out[0][0]) - ref).max() < 1e-9
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_davidson_own_solver_served_cell():
    # a served-trace-sized cell (64 atoms, 30 Ry, 40^3 box, 128 bands, n up to
    # 256) in the mixed form against LAPACK on the dense oracle H
    import torch
    q = _q()
    c = cellgen.random_served_cell(64, 30.0, 0, seed=21)
    ref = sla.eigh(oracle.dense_h(c), eigvals_only=True, subset_by_index=[0, c.nbnd - 1])
    for prec, tol in ((0, 1e-9), (1, 1e-5)):
        ctx = q.Context.from_cell(c, precision=prec, block=c.nbnd)
        p = torch.from_numpy(cellgen.make_psi0(c.npw, c.nbnd)).cuda()
        eig, info = ctx.davidson(p, rtol=1e-8, subspace=q.QEH_SUBSPACE_OWN)
        err = np.abs(np.sort(eig) - ref).max()
        print("served cell prec %d: %d iterations, max |eps - LAPACK| %.2e" %
              (prec, info["iters"], err), flush=True)
        assert info["status"] == 0 and err < tol
        ctx.close()
