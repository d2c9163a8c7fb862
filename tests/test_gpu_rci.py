"""Reverse-communication Davidson (qeh_dav_rci_*): the solver hands each
H|psi> product to the caller.

* Served with qeh_apply_h on the same context, the run is qeh_davidson's bit
  for bit (same enqueue order, same kernels): eigenvalues, Ritz vectors and
  counters compared exactly, for the general, Gamma and overlap (S != 1)
  paths.
* Served by the CPU oracle's H (the external Hamiltonian builder case), the
  eigenvalues match LAPACK on the oracle's dense H.
* A shifted operator H + sigma shifts every eigenvalue by sigma.
"""

import numpy as np
import pytest
import scipy.linalg as sla

import cellgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _q():
    import paper_2104_10502_amd as q
    return q


def _psi0(cell, nb, seed=10502):
    return torch.from_numpy(cellgen.make_psi0(cell.npw, nb, seed=seed)).cuda()


def _cells():
    return {
        "c1": cellgen.make_cell("c1"),
        "gamma": cellgen.gamma_half(cellgen.make_cell("c1")),
        "overlap": cellgen.make_cell("c1", overlap=True),
    }


@pytest.mark.parametrize("which", ["c1", "gamma", "overlap"])
@pytest.mark.parametrize("prec", [0, 1])
def test_rci_with_library_h_is_davidson_bitwise(which, prec):
    q = _q()
    cell = _cells()[which]
    nb = 12
    ctx = q.Context.from_cell(cell, precision=prec, block=8)
    p_ref = _psi0(cell, nb)
    eig_ref, info_ref = ctx.davidson(p_ref, nvecx=36, rtol=1e-9)
    calls = []

    def apply(x, y):
        calls.append(x.shape[0])
        ctx.apply_h(x, out=y)

    p = _psi0(cell, nb)
    eig, info = ctx.davidson_rci(p, apply, nvecx=36, rtol=1e-9)
    torch.cuda.synchronize()
    print(which, prec, info["iters"], info["restarts"], len(calls), flush=True)
    assert info["status"] == info_ref["status"]
    if prec == 0:
        assert info["status"] == 0
    assert np.array_equal(eig, eig_ref)
    assert torch.equal(p, p_ref)
    for k in ("iters", "restarts", "band_applies", "notconv"):
        assert info[k] == info_ref[k], k
    assert info["resid_max"] == info_ref["resid_max"]
    assert sum(calls) == info["band_applies"] and calls[0] == nb
    assert info["t_hpsi"] == 0.0


def test_rci_with_oracle_h_matches_lapack():
    # the caller's Hamiltonian builder is the CPU oracle (FP64): every request
    # is copied to the host, applied there, and copied back
    q = _q()
    cell = cellgen.make_cell("c1")
    nb = 10
    ref = sla.eigh(oracle.dense_h(cell), eigvals_only=True, subset_by_index=[0, nb - 1])
    ctx = q.Context.from_cell(cell, precision=q.QEH_FP64, block=16)

    def apply(x, y):
        h = oracle.apply_h(cell, x.cpu().numpy())
        y.copy_(torch.from_numpy(np.ascontiguousarray(h)).to(y.device))

    p = _psi0(cell, nb)
    eig, info = ctx.davidson_rci(p, apply, nvecx=40, rtol=1e-9)
    assert info["status"] == 0
    assert np.abs(eig - ref).max() < 1e-9, np.abs(eig - ref).max()
    # returned vectors: orthonormal eigenvectors of the oracle's H
    psi = p.cpu().numpy()
    assert np.abs(psi.conj() @ psi.T - np.eye(nb)).max() < 1e-10
    r = oracle.apply_h(cell, psi) - eig[:, None] * psi
    assert np.linalg.norm(r, axis=1).max() < 1e-8


def test_rci_shifted_operator_shifts_eigenvalues():
    q = _q()
    cell = cellgen.make_cell("c1")
    nb = 10
    sigma = 0.75
    ref = sla.eigh(oracle.dense_h(cell), eigvals_only=True, subset_by_index=[0, nb - 1])
    ctx = q.Context.from_cell(cell, precision=q.QEH_FP64, block=16)

    def apply(x, y):
        ctx.apply_h(x, out=y)
        y.add_(x, alpha=sigma)

    p = _psi0(cell, nb)
    eig, info = ctx.davidson_rci(p, apply, nvecx=40, rtol=1e-9)
    assert info["status"] == 0
    assert np.abs(eig - (ref + sigma)).max() < 1e-9


def test_rci_maxiter_and_repeated_step():
    q = _q()
    cell = cellgen.make_cell("c1")
    nb = 8
    ctx = q.Context.from_cell(cell, precision=q.QEH_FP64, block=8)
    p = _psi0(cell, nb)
    eig, info = ctx.davidson_rci(p, lambda x, y: ctx.apply_h(x, out=y), nvecx=24, rtol=1e-12,
                                 maxiter=2, allow_notconv=True)
    assert info["status"] == q.QEH_ERR_NOT_CONVERGED and info["iters"] == 2
    assert np.all(np.isfinite(eig)) and np.all(np.diff(eig) >= 0)
    # the raw handle: after the end every step returns the final status
    import ctypes
    work = torch.empty(ctx.davidson_plan(nb, 24), dtype=torch.uint8, device="cuda")
    p = _psi0(cell, nb)
    e = np.zeros(nb)
    o = q.DavOpts(24, 1e-12, 2, 0, None)
    h = ctypes.c_void_p()
    assert q._lib.qeh_dav_rci_create(ctx._h, nb, ctypes.c_void_p(p.data_ptr()), p.stride(0),
                                     e.ctypes.data_as(q._c_dbl_p), ctypes.byref(o),
                                     ctypes.c_void_p(work.data_ptr()), work.numel(),
                                     ctypes.byref(h)) == 0
    req = q.RciRequest()
    n_req = 0
    while True:
        st = q._lib.qeh_dav_rci_step(h, ctypes.byref(req))
        if st != q.QEH_RCI_APPLY_H:
            break
        n_req += 1
        assert req.ld == ctx.npw and 0 < req.n <= nb
        assert q._lib.qeh_apply_h(ctx._h, req.n, ctypes.c_void_p(req.x), req.ld,
                                  ctypes.c_void_p(req.y), req.ld) == 0
    # the starting block and the corrections of the first iteration
    assert st == q.QEH_ERR_NOT_CONVERGED and n_req == 2
    assert q._lib.qeh_dav_rci_step(h, ctypes.byref(req)) == st and req.n == 0
    info = q.DavInfo()
    assert q._lib.qeh_dav_rci_destroy(h, ctypes.byref(info)) == 0
    assert info.iters == 2


def test_rci_rejects_refine_context():
    q = _q()
    cell = cellgen.make_cell("c1")
    ctx = q.Context.from_cell(cell, precision=q.QEH_MIXED, block=8)
    c64 = q.Context.from_cell(cell, precision=q.QEH_FP64, block=8)
    import ctypes
    nb = 4
    work = torch.empty(ctx.davidson_plan(nb, 16), dtype=torch.uint8, device="cuda")
    p = _psi0(cell, nb)
    e = np.zeros(nb)
    o = q.DavOpts(16, 1e-8, 0, 0, c64._h)
    h = ctypes.c_void_p()
    st = q._lib.qeh_dav_rci_create(ctx._h, nb, ctypes.c_void_p(p.data_ptr()), p.stride(0),
                                   e.ctypes.data_as(q._c_dbl_p), ctypes.byref(o),
                                   ctypes.c_void_p(work.data_ptr()), work.numel(),
                                   ctypes.byref(h))
    assert st == q.QEH_ERR_INVALID and h.value is None
    assert b"refine" in q._lib.qeh_last_error()
