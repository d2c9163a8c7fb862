"""The C-ABI library without a GPU: it loads, exports every function that
include/qeh.h declares, the binding's structs match the header's layout (a
gcc-compiled probe prints sizeof/offsetof), and host-side validation in
qeh_ctx_plan (which makes no device call) rejects malformed cells with the
documented status codes.
"""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import cellgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qeh.h")


def _q():
    import paper_2104_10502_amd as q
    return q


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qeh_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    q = _q()
    names = declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(q.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(q.exported_symbols())


def test_struct_layout_matches_header(tmp_path):
    q = _q()
    probe = tmp_path / "probe.c"
    probe.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "qeh.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(qeh_cell),
         offsetof(qeh_cell, npw), offsetof(qeh_cell, miller), offsetof(qeh_cell, beta),
         offsetof(qeh_cell, block), sizeof(qeh_dav_opts), sizeof(qeh_dav_info),
         offsetof(qeh_cell, projgen), sizeof(qeh_projgen), offsetof(qeh_projgen, dq),
         offsetof(qeh_projgen, tab), sizeof(qeh_rci_request), offsetof(qeh_rci_request, n),
         sizeof(qeh_cg_opts));
  return 0;
}
''')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(probe), "-o", str(exe)],
                   check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    C = q.QehCell
    P = q.QehProjgen
    assert vals == [ctypes.sizeof(C), C.npw.offset, C.miller.offset, C.beta.offset,
                    C.block.offset, ctypes.sizeof(q.DavOpts), ctypes.sizeof(q.DavInfo),
                    C.projgen.offset, ctypes.sizeof(P), P.dq.offset, P.tab.offset,
                    ctypes.sizeof(q.RciRequest), q.RciRequest.n.offset, ctypes.sizeof(q.CgOpts)]


def _plan(cell, **kw):
    q = _q()
    if "projgen" in kw:
        # beta built on the device: marshalled by the binding's own helper
        keep = []
        c = q._cell_struct(cell.lattice, kw.get("fft", cell.fft), cell.kpt, cell.miller,
                           cell.vloc, kw.get("nproj", cell.nproj), None, cell.dmat,
                           kw.get("precision", 0), kw.get("block", 16), keep,
                           projgen=kw["projgen"])
        n = ctypes.c_size_t()
        st = q._lib.qeh_ctx_plan(ctypes.byref(c), ctypes.byref(n))
        nb = ctypes.c_size_t()
        stb = q._lib.qeh_beta_plan(ctypes.byref(c), ctypes.byref(nb))
        assert stb == st
        return st, n.value, q._lib.qeh_last_error().decode()
    miller = np.ascontiguousarray(kw.get("miller", cell.miller), dtype=np.int32)
    vloc = np.ascontiguousarray(kw.get("vloc", cell.vloc), dtype=np.float64)
    nproj = np.ascontiguousarray(cell.nproj, dtype=np.int32)
    beta = np.ascontiguousarray(cell.beta, dtype=np.complex128)
    dmat = np.ascontiguousarray(cell.dmat, dtype=np.complex128)
    c = q.QehCell()
    c.lattice[:] = list(np.asarray(cell.lattice).ravel())
    c.fft[:] = list(kw.get("fft", cell.fft))
    c.kpt[:] = list(cell.kpt)
    c.npw = miller.shape[0]
    c.miller = miller.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    c.vloc = vloc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.nat = nproj.shape[0]
    c.nproj = nproj.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    c.beta = beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.dmat = dmat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.precision = kw.get("precision", 0)
    c.block = kw.get("block", 16)
    n = ctypes.c_size_t()
    st = q._lib.qeh_ctx_plan(ctypes.byref(c), ctypes.byref(n))
    return st, n.value, q._lib.qeh_last_error().decode()


@pytest.fixture(scope="module")
def c1():
    return cellgen.make_cell("c1")


def test_plan_ok(c1):
    st, n, _ = _plan(c1)
    assert st == 0 and n > 16 * c1.npw * c1.nkb
    st32, n32, _ = _plan(c1, precision=1)
    assert st32 == 0 and n32 < n


def test_plan_rejects_unsorted_miller(c1):
    m = c1.miller.copy()
    m[[3, 4]] = m[[4, 3]]
    st, _, msg = _plan(c1, miller=m)
    assert st == -1 and "lexicographic" in msg


def test_plan_rejects_gap_in_stick(c1):
    m = c1.miller
    # an element whose neighbours on both sides belong to the same (h, k) stick
    same = (m[1:-1, :2] == m[:-2, :2]).all(1) & (m[1:-1, :2] == m[2:, :2]).all(1)
    g = 1 + int(np.nonzero(same)[0][0])
    m = np.delete(m, g, axis=0)
    st, _, msg = _plan(c1, miller=m)
    assert st == -1 and "contiguous" in msg


def test_plan_rejects_box_too_small(c1):
    st, _, msg = _plan(c1, fft=(12, 30, 30), vloc=np.zeros((30, 30, 12)))
    assert st == -1 and "box" in msg


def test_plan_rejects_prime_11(c1):
    st, _, msg = _plan(c1, fft=(33, 30, 30), vloc=np.zeros((30, 30, 33)))
    assert st == -1 and "prime" in msg


def test_plan_rejects_nonfinite_vloc(c1):
    v = c1.vloc.copy()
    v[1, 2, 3] = np.nan
    st, _, msg = _plan(c1, vloc=v)
    assert st == -3


def test_plan_rejects_bad_block_and_precision(c1):
    assert _plan(c1, block=0)[0] == -1
    assert _plan(c1, precision=7)[0] == -1


def test_null_context_arguments():
    # argument checks that return before any device call
    q = _q()
    assert q._lib.qeh_ctx_hdiag(None, None) == -1
    assert b"null" in q._lib.qeh_last_error()


def test_reverse_communication_null_arguments():
    # argument checks of the reverse-communication handle, before any device call
    q = _q()
    req = q.RciRequest()
    assert q._lib.qeh_dav_rci_step(None, ctypes.byref(req)) == q.QEH_ERR_INVALID
    assert q._lib.qeh_dav_rci_destroy(None, None) == q.QEH_ERR_INVALID
    out = ctypes.c_void_p(1)
    st = q._lib.qeh_dav_rci_create(None, 4, None, 0, None, None, None, 0, ctypes.byref(out))
    assert st == q.QEH_ERR_INVALID and out.value is None
    assert q._lib.qeh_dav_rci_create(None, 4, None, 0, None, None, None, 0, None) == \
        q.QEH_ERR_INVALID


def test_cg_null_arguments():
    # argument checks of the CG entry points, before any device call
    q = _q()
    n = ctypes.c_size_t()
    assert q._lib.qeh_cg_plan(None, 4, ctypes.byref(n)) == q.QEH_ERR_INVALID
    assert q._lib.qeh_cg(None, 4, None, 0, None, None, None, 0, None) == q.QEH_ERR_INVALID


def test_status_strings():
    q = _q()
    for s in range(-8, 2):
        assert q._lib.qeh_status_str(s) != b"unknown status"


def test_plan_with_device_projectors(c1):
    # beta built on the device: the plan adds the generator's staging area
    st, n, _ = _plan(c1)
    stg, ng, msg = _plan(c1, projgen=cellgen.projgen_tables(c1))
    assert st == 0 and stg == 0, msg
    assert ng > n


def test_plan_rejects_bad_projgen(c1):
    pg = cellgen.projgen_tables(c1)
    # table ends before the sphere does
    short = dict(pg, tab=pg["tab"][:, :100])
    st, _, msg = _plan(c1, projgen=short)
    assert st == -1 and "table" in msg
    # projector count of an atom does not match its species' channels
    st, _, msg = _plan(c1, projgen=pg, nproj=np.array([4, 3]))
    assert st == -1 and "nproj" in msg
    # l out of range
    st, _, msg = _plan(c1, projgen=dict(pg, lchan=np.array([0, 3])))
    assert st == -1 and "l must" in msg
    # species index out of range
    st, _, msg = _plan(c1, projgen=dict(pg, ityp=np.array([0, 1])))
    assert st == -1 and "ityp" in msg
    # nq < 4 and dq <= 0
    st, _, _ = _plan(c1, projgen=dict(pg, tab=pg["tab"][:, :3]))
    assert st == -1
    st, _, _ = _plan(c1, projgen=dict(pg, dq=0.0))
    assert st == -1
    # non-finite table value and position
    bad = pg["tab"].copy()
    bad[1, 7] = np.inf
    assert _plan(c1, projgen=dict(pg, tab=bad))[0] == -3
    tau = pg["tau"].copy()
    tau[0, 1] = np.nan
    assert _plan(c1, projgen=dict(pg, tau=tau))[0] == -3


def test_plan_rejects_no_beta_no_projgen(c1):
    q = _q()
    keep = []
    c = q._cell_struct(c1.lattice, c1.fft, c1.kpt, c1.miller, c1.vloc, c1.nproj, None,
                       c1.dmat, 0, 16, keep)
    n = ctypes.c_size_t()
    assert q._lib.qeh_ctx_plan(ctypes.byref(c), ctypes.byref(n)) == -1
    assert "projgen" in q._lib.qeh_last_error().decode()


def _plan_gamma(cell, miller=None, kpt=None, dmat=None, beta="keep"):
    q = _q()
    keep = []
    c = q._cell_struct(cell.lattice, cell.fft, cell.kpt if kpt is None else kpt,
                       cell.miller if miller is None else miller, cell.vloc, cell.nproj,
                       cell.beta if isinstance(beta, str) else beta,
                       cell.dmat if dmat is None else dmat, 0, 16, keep, gamma=True)
    n = ctypes.c_size_t()
    st = q._lib.qeh_ctx_plan(ctypes.byref(c), ctypes.byref(n))
    return st, n.value, q._lib.qeh_last_error().decode()


def test_plan_gamma(c1):
    # the half-sphere cell plans; its arena holds the packed band pairs
    h = cellgen.gamma_half(c1)
    st, n, msg = _plan_gamma(h)
    assert st == 0, msg
    assert n > 16 * (16 // 2) * c1.npw
    # k != 0, a list not starting at (0,0,0), a G before (0,0,0), complex D,
    # complex beta(G = 0): rejected
    assert _plan_gamma(h, kpt=np.array([0.0, 0.0, 0.01]))[0] == -1
    assert _plan_gamma(h, miller=h.miller[1:])[0] == -1
    bad = h.miller.copy()
    bad[5] = -bad[5]
    assert _plan_gamma(h, miller=bad)[0] == -1
    d = h.dmat.copy()
    d[0] += 0.1j
    assert _plan_gamma(h, dmat=d)[0] == -1
    b = h.beta.copy()
    b[0, 0] += 1e-3j
    assert _plan_gamma(h, beta=b)[0] == -1
