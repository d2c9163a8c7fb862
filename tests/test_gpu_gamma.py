"""GPU parity of the Gamma-point path (real wavefunctions at k = 0 stored over
half the sphere, two bands per complex FFT) against the FP64 oracle, which
works on the full sphere (``oracle.gamma.expand`` / ``restrict``).

Bars as for general k: H|psi> FP64 per-band relative L2 <= 1e-12 and
element-wise <= 1e-12 max|H psi|, mixed relative L2 <= 1e-5; eigenvalues
against LAPACK on the full dense H (the real problem has the complex
problem's eigenvalues): FP64 1e-9 Ry, mixed 1e-6 Ry.
"""

import time

import numpy as np
import pytest
import scipy.linalg as sla

import cellgen
import oracle
from oracle import gamma

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _q():
    import paper_2104_10502_amd as q
    return q


def _rel_l2(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _psi_half(nh, nb, seed):
    p = cellgen.make_psi0(nh, nb, seed=seed)
    p[:, 0] = p[:, 0].real   # psi(G = 0) real
    return p


def _apply(h, psi, prec, block, part=None, **kw):
    q = _q()
    ctx = q.Context.from_cell(h, precision=prec, block=block, **kw)
    out = ctx.apply_h(torch.from_numpy(psi).cuda(), part=part).cpu().numpy()
    return out, ctx


def _check(got, ref, prec):
    err = _rel_l2(got, ref).max()
    if prec == 0:
        assert err < 1e-12, err
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    else:
        assert err < 1e-5, err


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nb,block", [(16, 16), (15, 6)])
def test_gamma_apply_h_c1(prec, nb, block):
    # 15 bands in blocks of 6: two full blocks of three pairs, a tail of three
    # bands (one pair and a band without a partner)
    c = cellgen.make_cell("c1")
    h = cellgen.gamma_half(c)
    psi = _psi_half(h.npw, nb, 21)
    print("case gamma apply c1 prec", prec, "nb", nb, "block", block, flush=True)
    got, ctx = _apply(h, psi, prec, block)
    ref = gamma.restrict(oracle.apply_h(c, gamma.expand(psi)))
    assert got.shape == (nb, h.npw)
    _check(got, ref, prec)
    # H psi(G = 0) is real
    assert np.abs(got[:, 0].imag).max() <= 1e-12 * np.abs(got).max()


@pytest.mark.parametrize("prec", [0, 1])
def test_gamma_apply_h_parts(prec):
    c = cellgen.make_cell("c1")
    h = cellgen.gamma_half(c)
    psi = _psi_half(h.npw, 5, 22)
    full = gamma.expand(psi)
    loc, _ = _apply(h, psi, prec, 4, part=0)
    nl, _ = _apply(h, psi, prec, 4, part=1)
    ref_loc = gamma.restrict(oracle.kinetic(c)[None, :] * full + oracle.vloc_psi(c, full))
    ref_nl = gamma.restrict(oracle.vnl_psi(c, full))
    _check(loc, ref_loc, prec)
    _check(nl, ref_nl, prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_gamma_register_kernels(prec):
    # a 32^3 box: the lane-pair plane and stick kernels (mixed) and the
    # lane-quad plane kernel (FP64) run on the packed pairs
    c = cellgen.make_cell("c1", fft=(32, 32, 32))
    h = cellgen.gamma_half(c)
    psi = _psi_half(h.npw, 12, 23)
    got, ctx = _apply(h, psi, prec, 12)
    info = ctx.info()
    assert info["plane_path"] == (4 if prec == 0 else 2)
    ref = gamma.restrict(oracle.apply_h(c, gamma.expand(psi)))
    _check(got, ref, prec)


def test_gamma_device_projectors():
    # projectors built on the device over the half sphere
    c = cellgen.make_cell("c1")
    h = cellgen.gamma_half(c)
    pg = cellgen.projgen_tables(c)
    psi = _psi_half(h.npw, 8, 24)
    got, _ = _apply(h, psi, 0, 8, projgen=pg)
    co = cellgen.make_cell("c1")
    co.beta = oracle.beta_projectors(c.lattice, c.kpt, c.miller, c.positions,
                                     np.zeros(c.nat, dtype=int), [cellgen.PROJ_SETS[c.proj_set]])
    ref = gamma.restrict(oracle.apply_h(co, gamma.expand(psi)))
    # the projectors' interpolation error (<= ~1e-9 of the channel scale)
    # enters beta D beta^H twice
    assert _rel_l2(got, ref).max() < 1e-8


@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 1e-6)])
def test_gamma_davidson_c1_vs_lapack(prec, tol):
    q = _q()
    c = cellgen.make_cell("c1")
    h = cellgen.gamma_half(c)
    ref = sla.eigh(oracle.dense_h(c), eigvals_only=True, subset_by_index=[0, c.nbnd - 1])
    ctx = q.Context.from_cell(h, precision=prec, block=c.nbnd)
    # the mixed form finishes with FP64 H applications on an FP64 Gamma context
    c64 = q.Context.from_cell(h, precision=0, block=c.nbnd) if prec == 1 else None
    p = torch.from_numpy(cellgen.make_psi0(h.npw, c.nbnd)).cuda()   # Im psi(0) != 0: zeroed
    eig, info = ctx.davidson(p, rtol=1e-8, refine=c64)
    assert info["status"] == 0
    assert np.abs(np.sort(eig) - ref).max() < tol, np.abs(np.sort(eig) - ref).max()
    # Ritz vectors: real functions, orthonormal in the full-sphere product,
    # eigenvectors of the oracle's H
    ph = p.cpu().numpy()
    assert np.abs(ph[:, 0].imag).max() <= 1e-12
    full = gamma.expand(ph)
    gram = full.conj() @ full.T
    assert np.abs(gram - np.eye(c.nbnd)).max() < (1e-10 if prec == 0 else 1e-8)
    r = oracle.apply_h(c, full) - eig[:, None] * full
    if prec == 0:
        assert np.linalg.norm(r, axis=1).max() < 1e-8
    else:
        assert info["resid_max"] < 2e-4


def test_gamma_davidson_restarts_odd_blocks():
    # 11 bands in blocks of 4 and a small basis: restarts, odd pair counts
    q = _q()
    c = cellgen.make_cell("c1")
    h = cellgen.gamma_half(c)
    ref = sla.eigh(oracle.dense_h(c), eigvals_only=True, subset_by_index=[0, 10])
    ctx = q.Context.from_cell(h, precision=0, block=4)
    p = torch.from_numpy(cellgen.make_psi0(h.npw, 11, seed=3)).cuda()
    eig, info = ctx.davidson(p, nvecx=22, rtol=1e-8)
    assert info["restarts"] > 0
    assert np.abs(np.sort(eig) - ref).max() < 1e-9


def test_gamma_served_request():
    q = _q()
    c = cellgen.make_cell("c1")
    h = cellgen.gamma_half(c)
    ref = sla.eigh(oracle.dense_h(c), eigvals_only=True, subset_by_index=[0, c.nbnd - 1])
    srv = q.Server(1 << 30, max_slots=2)
    t = srv.submit([h], [cellgen.make_psi0(h.npw, c.nbnd)], c.nbnd, precision=q.QEH_FP64)
    t0 = time.time()
    r = None
    while r is None and time.time() - t0 < 60:
        r = srv.poll(t)
        time.sleep(0.01)
    srv.close()
    assert r is not None and r["status"] == 0, r
    assert np.abs(r["eig"][0] - ref).max() < 1e-9


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("block", [16, 3])
def test_gamma_density(prec, block):
    # occupations with runs of equal values (bands paired in one transform)
    # and isolated values (bands alone), in blocks of 16 and of 3 transforms
    q = _q()
    c = cellgen.make_cell("c1")
    h = cellgen.gamma_half(c)
    occ = np.array([2.0, 2.0, 2.0, 1.5, 1.5, 0.3, 2.0, 2.0, 1.0, 0.0, 0.0])
    psi = _psi_half(h.npw, occ.size, 25)
    ctx = q.Context.from_cell(h, precision=prec, block=block)
    got = ctx.density(torch.from_numpy(psi).cuda(), occ).cpu().numpy()
    ref = oracle.density(c, gamma.expand(psi), occ)
    tol = 1e-12 if prec == 0 else 1e-5
    assert np.abs(got - ref).max() < tol * np.abs(ref).max()


@pytest.mark.parametrize("prec", [0, 1])
def test_gamma_c2_bench_launch(prec):
    # the benchmark's Gamma leg: the 64-atom cell at k = 0, 128 bands in one
    # block (64 packed pairs); sampled bands (both members of a pair, and a
    # band from another pair) against the oracle on the full sphere
    c = cellgen.make_cell("c2", kfrac=(0.0, 0.0, 0.0))
    h = cellgen.gamma_half(c)
    psi = _psi_half(h.npw, 128, 10502)
    print("case gamma c2 bench launch prec", prec, flush=True)
    got, _ = _apply(h, psi, prec, 128)
    idx = [0, 1, 77]
    ref = gamma.restrict(oracle.apply_h(c, gamma.expand(psi[idx])))
    err = _rel_l2(got[idx], ref)
    assert err.max() < (1e-12 if prec == 0 else 1e-5), err


@pytest.mark.parametrize("prec", [0, 1])
def test_gamma_single_band_and_empty(prec):
    # one band (a pair with no partner), and zero bands (nothing launched)
    q = _q()
    c = cellgen.make_cell("c1")
    h = cellgen.gamma_half(c)
    psi = _psi_half(h.npw, 1, 26)
    got, ctx = _apply(h, psi, prec, 8)
    ref = gamma.restrict(oracle.apply_h(c, gamma.expand(psi)))
    _check(got, ref, prec)
    empty = torch.zeros((0, h.npw), dtype=torch.complex128, device="cuda")
    assert ctx.apply_h(empty).shape == (0, h.npw)


@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 1e-6)])
def test_gamma_davidson_64_bands(prec, tol):
    # 64 bands: reduced problems up to n = 128 (the real symmetric subspace
    # step; the complex eigensolver gave non-finite vectors for such input)
    q = _q()
    c = cellgen.make_cell("c1")
    h = cellgen.gamma_half(c)
    ref = sla.eigh(oracle.dense_h(c), eigvals_only=True, subset_by_index=[0, 63])
    ctx = q.Context.from_cell(h, precision=prec, block=32)
    c64 = q.Context.from_cell(h, precision=0, block=32) if prec == 1 else None
    p = torch.from_numpy(cellgen.make_psi0(h.npw, 64, seed=5)).cuda()
    eig, info = ctx.davidson(p, rtol=1e-8, refine=c64)
    assert info["status"] == 0
    # sorted eigenvalues are unique even where the window cuts a degenerate
    # shell: all 64 are compared
    assert np.abs(np.sort(eig) - ref).max() < tol
