"""The overlap operator S = 1 + sum |beta> q <beta| on the GPU (qeh_apply_s) and
the generalized Davidson (qeh_davidson on a context with q blocks) against
the oracle (oracle/overlap.py): S psi element-wise on general-k and Gamma
cells in both forms; eigenvalues against LAPACK's dense generalized solver,
S-orthonormal Ritz vectors, generalized residuals recomputed by the oracle;
the mixed form refined in FP64; a served request carrying q blocks."""

import numpy as np
import pytest

import cellgen
import oracle
from oracle import gamma, overlap

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _q():
    import paper_2104_10502_amd as q
    return q


def _rel(a, b):
    return (np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)).max()


@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 1e-6)])
def test_apply_s_general_k_and_gamma(prec, tol):
    q = _q()
    c = cellgen.make_cell("c1", kfrac=(0.25, 0.25, 0.25), overlap=True)
    psi = cellgen.make_psi0(c.npw, 20, seed=31)
    ref = overlap.apply_s(c, psi)
    ctx = q.Context.from_cell(c, precision=prec, block=8)   # ragged: 8 + 8 + 4
    got = ctx.apply_s(torch.from_numpy(psi).cuda()).cpu().numpy()
    assert _rel(got, ref) < tol
    assert np.abs(got - psi).max() > 1e-4                   # q acts
    ctx.close()
    cg = cellgen.make_cell("c1", overlap=True)
    h = cellgen.gamma_half(cg)
    ph = cellgen.make_psi0(h.npw, 9, seed=32)
    ph[:, 0] = ph[:, 0].real
    ref = gamma.restrict(overlap.apply_s(cg, gamma.expand(ph)))
    ctx = q.Context.from_cell(h, precision=prec, block=4)
    got = ctx.apply_s(torch.from_numpy(ph).cuda()).cpu().numpy()
    assert _rel(got, ref) < tol
    ctx.close()
    # no q blocks: S is the identity
    c0 = cellgen.make_cell("c1")
    p0 = cellgen.make_psi0(c0.npw, 3, seed=33)
    ctx = q.Context.from_cell(c0, precision=prec, block=8)
    got = ctx.apply_s(torch.from_numpy(p0).cuda()).cpu().numpy()
    assert np.array_equal(got, p0)
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 1e-6)])
@pytest.mark.parametrize("kind", ["general_k", "gamma"])
def test_generalized_davidson_vs_lapack(prec, tol, kind):
    q = _q()
    if kind == "gamma":
        full = cellgen.make_cell("c1", overlap=True)
        cell = cellgen.gamma_half(full)
    else:
        full = cell = cellgen.make_cell("c1", kfrac=(0.25, 0.25, 0.25), overlap=True)
    nb = 16
    ref = overlap.dense_eigs_gen(full, nb)
    ref_std = oracle.dense_eigs(full, nb)
    ctx = q.Context.from_cell(cell, precision=prec, block=nb)
    c64 = q.Context.from_cell(cell, precision=0, block=nb)
    p = torch.from_numpy(cellgen.make_psi0(cell.npw, nb, seed=5)).cuda()
    eig, info = ctx.davidson(p, rtol=1e-8, refine=c64 if prec == 1 else None)
    err = np.abs(np.sort(eig) - ref).max()
    print("%s prec %d: %d iterations (%d FP64), resid %.1e, |eps - LAPACK| %.2e, "
          "S != 1 moves eps by %.2e" % (kind, prec, info["iters"], info["refine_iters"],
                                       info["resid_max"], err, np.abs(ref - ref_std).max()),
          flush=True)
    assert info["status"] == 0 and err < tol
    # S-orthonormal Ritz vectors, generalized residuals by the oracle
    ph = p.cpu().numpy()
    vecs = gamma.expand(ph) if kind == "gamma" else ph
    sv = overlap.apply_s(full, vecs)
    g = vecs.conj() @ sv.T
    assert np.abs(g - np.eye(nb)).max() < 1e-9
    r = oracle.apply_h(full, vecs) - eig[:, None] * sv
    assert np.linalg.norm(r, axis=1).max() < (1e-8 if prec == 0 else 1.01e-5)
    ctx.close()
    c64.close()


def test_served_request_with_overlap():
    q = _q()
    c = cellgen.make_cell("c1", kfrac=(0.25, -0.25, 0.25), overlap=True)
    nb = c.nbnd
    ref = overlap.dense_eigs_gen(c, nb)
    srv = q.Server(2 << 30, max_slots=2)
    ts = [srv.submit([c], [cellgen.make_psi0(c.npw, nb, seed=9)], nb, precision=p, rtol=1e-9)
          for p in (q.QEH_FP64, q.QEH_MIXED)]
    import time
    out = {}
    t0 = time.time()
    while len(out) < 2 and time.time() - t0 < 120:
        for t in ts:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.005)
    srv.close()
    for t, tol in zip(ts, (1e-9, 1e-6)):
        r = out[t]
        assert r["status"] == 0, r["error"]
        assert np.abs(np.sort(r["eig"][0]) - ref).max() < tol
