"""Python binding of the qeh HIP library (plane-wave H|psi> and block Davidson
on one MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libqeh.so``.  PyTorch provides device memory (the arena and the
band arrays) and the HIP stream.  Importing this module loads the library and
raises if it has not been built; there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqeh.so")

QEH_OK = 0
QEH_ERR_INVALID = -1
QEH_ERR_NOMEM = -2
QEH_ERR_NUMERIC = -3
QEH_ERR_CHOLESKY = -4
QEH_ERR_NOT_CONVERGED = -5
QEH_ERR_REJECTED = -6
QEH_ERR_DEVICE = -7
QEH_ERR_BUSY = -8
QEH_RCI_APPLY_H = 1
QEH_FP64 = 0
QEH_MIXED = 1
NSTAGES = 9
STAGE_NAMES = ["k1_scatter_zinv", "k2_plane", "k3_zfwd_gather", "calbec_gemm", "dscale",
               "addnl_gemm", "density_columns", "density_rows", "density_reduce"]

if not os.path.exists(LIB_PATH):
    raise ImportError("libqeh.so is not built: run `python -m paper_2104_10502_amd.build` "
                      "(or __graft_entry__.build()) first; there is no non-GPU fallback")
# PyTorch's HIP runtime is loaded before the library, so that the library binds
# to the same runtime instance whichever module a process imports first (two
# runtimes in one process do not share devices).
import torch as _torch_runtime  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_dbl_p = ctypes.POINTER(ctypes.c_double)


class QehProjgen(ctypes.Structure):
    _fields_ = [("tau", _c_dbl_p), ("ityp", _c_int_p), ("nsp", ctypes.c_int),
                ("nchan", _c_int_p), ("lchan", _c_int_p), ("nq", ctypes.c_int),
                ("dq", ctypes.c_double), ("tab", _c_dbl_p)]


class QehCell(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_double * 9), ("fft", ctypes.c_int * 3),
                ("kpt", ctypes.c_double * 3), ("npw", ctypes.c_int),
                ("miller", _c_int_p), ("vloc", _c_dbl_p), ("nat", ctypes.c_int),
                ("nproj", _c_int_p), ("beta", _c_dbl_p), ("dmat", _c_dbl_p),
                ("precision", ctypes.c_int), ("block", ctypes.c_int),
                ("projgen", ctypes.POINTER(QehProjgen)), ("gamma", ctypes.c_int),
                ("qmat", _c_dbl_p)]


class DavOpts(ctypes.Structure):
    _fields_ = [("nvecx", ctypes.c_int), ("rtol", ctypes.c_double), ("maxiter", ctypes.c_int),
                ("subspace", ctypes.c_int), ("refine", ctypes.c_void_p)]


class CgOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("maxiter", ctypes.c_int)]


class RciRequest(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("n", ctypes.c_int),
                ("ld", ctypes.c_int)]


class DavInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("notconv", ctypes.c_int), ("restarts", ctypes.c_int),
                ("band_applies", ctypes.c_long), ("resid_max", ctypes.c_double),
                ("t_total", ctypes.c_double), ("t_hpsi", ctypes.c_double),
                ("t_subspace", ctypes.c_double), ("refine_iters", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_sz_p = ctypes.POINTER(ctypes.c_size_t)
_SIGS = {
    "qeh_ctx_plan": ([ctypes.POINTER(QehCell), _sz_p], ctypes.c_int),
    "qeh_ctx_create": ([ctypes.POINTER(QehCell), _vp, ctypes.c_size_t, _vp,
                        ctypes.POINTER(_vp)], ctypes.c_int),
    "qeh_ctx_destroy": ([_vp], ctypes.c_int),
    "qeh_apply_h": ([_vp, ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int], ctypes.c_int),
    "qeh_apply_s": ([_vp, ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int], ctypes.c_int),
    "qeh_apply_h_part": ([_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp,
                          ctypes.c_int], ctypes.c_int),
    "qeh_davidson_plan": ([_vp, ctypes.c_int, ctypes.POINTER(DavOpts), _sz_p], ctypes.c_int),
    "qeh_davidson": ([_vp, ctypes.c_int, _vp, ctypes.c_int, _c_dbl_p, ctypes.POINTER(DavOpts),
                      _vp, ctypes.c_size_t, ctypes.POINTER(DavInfo)], ctypes.c_int),
    "qeh_cg_plan": ([_vp, ctypes.c_int, _sz_p], ctypes.c_int),
    "qeh_cg": ([_vp, ctypes.c_int, _vp, ctypes.c_int, _c_dbl_p, ctypes.POINTER(CgOpts), _vp,
                ctypes.c_size_t, ctypes.POINTER(DavInfo)], ctypes.c_int),
    "qeh_dav_rci_create": ([_vp, ctypes.c_int, _vp, ctypes.c_int, _c_dbl_p,
                            ctypes.POINTER(DavOpts), _vp, ctypes.c_size_t, ctypes.POINTER(_vp)],
                           ctypes.c_int),
    "qeh_dav_rci_step": ([_vp, ctypes.POINTER(RciRequest)], ctypes.c_int),
    "qeh_dav_rci_destroy": ([_vp, ctypes.POINTER(DavInfo)], ctypes.c_int),
    "qeh_density_plan": ([_vp, _sz_p], ctypes.c_int),
    "qeh_subspace_plan": ([ctypes.c_int, ctypes.c_int, _sz_p], ctypes.c_int),
    "qeh_subspace_eigh": ([ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp, _vp,
                           ctypes.c_int, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "qeh_beta_plan": ([ctypes.POINTER(QehCell), _sz_p], ctypes.c_int),
    "qeh_beta_generate": ([ctypes.POINTER(QehCell), ctypes.c_int, _vp, ctypes.c_long, _vp,
                           ctypes.c_size_t, _vp], ctypes.c_int),
    "qeh_beta_generate_static": ([ctypes.POINTER(QehCell), ctypes.c_int, _vp, ctypes.c_long,
                                  _vp], ctypes.c_int),
    "qeh_density": ([_vp, ctypes.c_int, _vp, ctypes.c_int, _c_dbl_p, _vp, _vp, ctypes.c_size_t],
                    ctypes.c_int),
    "qeh_ctx_profile": ([_vp, ctypes.c_int], ctypes.c_int),
    "qeh_ctx_stage_times": ([_vp, _c_dbl_p, ctypes.POINTER(ctypes.c_long), ctypes.c_int],
                            ctypes.c_int),
    "qeh_ctx_info": ([_vp, ctypes.POINTER(ctypes.c_long), ctypes.c_int], ctypes.c_int),
    "qeh_ctx_hdiag": ([_vp, _vp], ctypes.c_int),
    "qeh_server_create": ([_vp, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_vp)],
                          ctypes.c_int),
    "qeh_submit": ([_vp, ctypes.POINTER(QehCell), ctypes.c_int, ctypes.c_int, _c_dbl_p,
                    ctypes.POINTER(DavOpts), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "qeh_poll": ([_vp, ctypes.c_uint64, _c_dbl_p, ctypes.POINTER(DavInfo), _c_dbl_p],
                 ctypes.c_int),
    "qeh_cancel": ([_vp, ctypes.c_uint64], ctypes.c_int),
    "qeh_server_stats": ([_vp, _c_dbl_p, ctypes.c_int], ctypes.c_int),
    "qeh_server_destroy": ([_vp], ctypes.c_int),
    "qeh_status_str": ([ctypes.c_int], ctypes.c_char_p),
    "qeh_last_error": ([], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class QehError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.qeh_last_error().decode(errors="replace")
        super().__init__("%s: %s (%d): %s" % (where, _lib.qeh_status_str(status).decode(),
                                              status, msg))


def _check(st, where, allow=()):
    if st != QEH_OK and st not in allow:
        raise QehError(st, where)
    return st


def exported_symbols():
    """Names the library exports (for load checks)."""
    return sorted(_SIGS)


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def _projgen_struct(pg, keep):
    """QehProjgen from a dict with tau (nat,3), ityp (nat,), nchan (nsp,),
    lchan (sum nchan,), dq and tab (sum nchan, nq); ``keep`` holds the arrays."""
    k = dict(tau=np.ascontiguousarray(pg["tau"], dtype=np.float64),
             ityp=np.ascontiguousarray(pg["ityp"], dtype=np.int32),
             nchan=np.ascontiguousarray(pg["nchan"], dtype=np.int32),
             lchan=np.ascontiguousarray(pg["lchan"], dtype=np.int32),
             tab=np.ascontiguousarray(pg["tab"], dtype=np.float64))
    if k["tab"].ndim != 2:
        raise ValueError("projgen tab must be (channels, nq)")
    keep.append(k)
    p = QehProjgen()
    p.tau = k["tau"].ctypes.data_as(_c_dbl_p)
    p.ityp = k["ityp"].ctypes.data_as(_c_int_p)
    p.nsp = int(k["nchan"].shape[0])
    p.nchan = k["nchan"].ctypes.data_as(_c_int_p)
    p.lchan = k["lchan"].ctypes.data_as(_c_int_p)
    p.nq = int(k["tab"].shape[1])
    p.dq = float(pg["dq"])
    p.tab = k["tab"].ctypes.data_as(_c_dbl_p)
    keep.append(p)
    return p


def _cell_struct(lattice, fft, kpt, miller, vloc, nproj, beta, dmat, precision, block, keep,
                 projgen=None, gamma=False, qmat=None):
    """Fill a QehCell from host arrays; ``keep`` collects the arrays it points to.
    With beta None and a projgen dict, the library builds beta on the device."""
    k = dict(miller=np.ascontiguousarray(miller, dtype=np.int32),
             vloc=np.ascontiguousarray(vloc, dtype=np.float64),
             nproj=np.ascontiguousarray(nproj, dtype=np.int32),
             beta=None if beta is None else np.ascontiguousarray(beta, dtype=np.complex128),
             dmat=np.ascontiguousarray(dmat, dtype=np.complex128))
    keep.append(k)
    c = QehCell()
    c.lattice[:] = [float(x) for x in np.asarray(lattice, dtype=np.float64).ravel()]
    c.fft[:] = [int(x) for x in fft]
    c.kpt[:] = [float(x) for x in np.asarray(kpt, dtype=np.float64).ravel()]
    c.npw = int(k["miller"].shape[0])
    c.miller = k["miller"].ctypes.data_as(_c_int_p)
    c.vloc = k["vloc"].ctypes.data_as(_c_dbl_p)
    c.nat = int(k["nproj"].shape[0])
    c.nproj = k["nproj"].ctypes.data_as(_c_int_p)
    c.beta = k["beta"].ctypes.data_as(_c_dbl_p) if k["beta"] is not None else None
    c.dmat = k["dmat"].ctypes.data_as(_c_dbl_p)
    c.precision = int(precision)
    c.block = int(block)
    if beta is None and projgen is not None:
        c.projgen = ctypes.pointer(_projgen_struct(projgen, keep))
    c.gamma = 1 if gamma else 0
    if qmat is not None:
        k["qmat"] = np.ascontiguousarray(qmat, dtype=np.complex128)
        c.qmat = k["qmat"].ctypes.data_as(_c_dbl_p)
    return c


def generate_beta(lattice, kpt, miller, nproj, projgen, precision=QEH_FP64, device=None,
                  stream=None):
    """Projectors of ``projgen`` on the sphere ``miller`` built on the device:
    (nkb, npw) complex128 (QEH_FP64) or complex64 (QEH_MIXED) CUDA tensor."""
    torch = _torch()
    dev = torch.device(device if device is not None else "cuda")
    keep = []
    miller = np.ascontiguousarray(miller, dtype=np.int32)
    nproj = np.ascontiguousarray(nproj, dtype=np.int32)
    c = _cell_struct(lattice, (1, 1, 1), kpt, miller, np.zeros(1), nproj, None,
                     np.zeros(0, dtype=np.complex128), precision, 1, keep, projgen=projgen)
    n = ctypes.c_size_t()
    _check(_lib.qeh_beta_plan(ctypes.byref(c), ctypes.byref(n)), "qeh_beta_plan")
    work = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device=dev)
    nkb, npw = int(nproj.sum()), int(miller.shape[0])
    out = torch.empty((nkb, npw), dtype=torch.complex128 if precision == QEH_FP64
                      else torch.complex64, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(_lib.qeh_beta_generate(ctypes.byref(c), int(precision), _vp(out.data_ptr()), npw,
                                  _vp(work.data_ptr()), int(work.numel()), _stream_ptr(st)),
           "qeh_beta_generate")
    return out


QEH_SUBSPACE_AUTO, QEH_SUBSPACE_OWN, QEH_SUBSPACE_ROCSOLVER = 0, 1, 2


def subspace_eigh(h, s, nb, stream=None):
    """qeh_subspace_eigh: the nb lowest eigenpairs of h y = eps s y for n x n
    complex128 CUDA tensors (Hermitian h, positive definite s, n <= 2048);
    returns (eig float64 CUDA tensor (nb,), Y complex128 CUDA tensor (n, nb)),
    Y column j the eigenvector of eig[j]."""
    torch = _torch()
    n = h.shape[0]
    if h.shape != (n, n) or s.shape != (n, n) or h.dtype != torch.complex128 or \
            s.dtype != torch.complex128 or h.device.type != "cuda" or s.device != h.device:
        raise ValueError("h, s must be n x n complex128 CUDA tensors on one device")
    # column-major storage: the transposes' rows are the matrices' columns
    hc = h.t().contiguous()
    sc = s.t().contiguous()
    need = ctypes.c_size_t()
    _check(_lib.qeh_subspace_plan(int(n), int(nb), ctypes.byref(need)), "qeh_subspace_plan")
    work = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=h.device)
    eig = torch.empty(nb, dtype=torch.float64, device=h.device)
    yc = torch.empty((nb, n), dtype=torch.complex128, device=h.device)   # column-major n x nb
    st = stream if stream is not None else torch.cuda.current_stream(h.device)
    _check(_lib.qeh_subspace_eigh(int(n), int(nb), _vp(hc.data_ptr()), _vp(sc.data_ptr()), int(n),
                                  _vp(eig.data_ptr()), _vp(yc.data_ptr()), int(n),
                                  _vp(work.data_ptr()), int(work.numel()), _stream_ptr(st)),
           "qeh_subspace_eigh")
    return eig, yc.t()


BETA_STATIC_BYTES = 8 << 20   # QEH_BETA_STATIC_BYTES


def generate_beta_static(lattice, kpt, miller, nproj, projgen, precision=QEH_FP64,
                         out=None, device=None, stream=None):
    """qeh_beta_generate_static: the projectors of ``projgen`` written into
    ``out`` (an existing (nkb, >= npw) complex128 / complex64 CUDA tensor, or a
    new one) with the library's static staging array instead of a workspace."""
    torch = _torch()
    dev = torch.device(device if device is not None else "cuda")
    keep = []
    miller = np.ascontiguousarray(miller, dtype=np.int32)
    nproj = np.ascontiguousarray(nproj, dtype=np.int32)
    c = _cell_struct(lattice, (1, 1, 1), kpt, miller, np.zeros(1), nproj, None,
                     np.zeros(0, dtype=np.complex128), precision, 1, keep, projgen=projgen)
    nkb, npw = int(nproj.sum()), int(miller.shape[0])
    dt = torch.complex128 if precision == QEH_FP64 else torch.complex64
    if out is None:
        out = torch.empty((nkb, npw), dtype=dt, device=dev)
    if out.dtype != dt or out.dim() != 2 or out.shape[0] != nkb or out.shape[1] < npw or \
            out.stride(1) != 1:
        raise ValueError("out must be (nkb, >= npw) %s with unit stride" % dt)
    st = stream if stream is not None else torch.cuda.current_stream(out.device)
    _check(_lib.qeh_beta_generate_static(ctypes.byref(c), int(precision), _vp(out.data_ptr()),
                                         out.stride(0), _stream_ptr(st)),
           "qeh_beta_generate_static")
    return out


class Server:
    """Continuous-batching Davidson server over a device arena of ``arena_bytes``."""

    def __init__(self, arena_bytes, max_slots=8, device=None):
        torch = _torch()
        self.device = torch.device(device if device is not None else "cuda")
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = _vp()
        _check(_lib.qeh_server_create(_vp(self.arena.data_ptr()), int(arena_bytes),
                                      int(max_slots), ctypes.byref(h)), "qeh_server_create")
        self._h = h
        self._nk = {}

    def submit(self, cells, psi0s, nb, precision=QEH_MIXED, block=None, nvecx=0, rtol=1e-8,
               maxiter=0, subspace=0):
        """cells: list of cell-like objects (one per k-point); psi0s: list of (nb, npw)."""
        if len(psi0s) != len(cells):
            raise ValueError("submit: %d cells but %d start-vector blocks" % (len(cells), len(psi0s)))
        for k, (c, p) in enumerate(zip(cells, psi0s)):
            if np.shape(p) != (int(nb), int(len(c.miller))):
                raise ValueError("submit: k-point %d start vectors have shape %s, expected (%d, %d)"
                                 % (k, np.shape(p), int(nb), len(c.miller)))
        keep = []
        arr = (QehCell * len(cells))()
        for i, c in enumerate(cells):
            pg = getattr(c, "projgen", None)
            arr[i] = _cell_struct(c.lattice, c.fft, c.kpt, c.miller, c.vloc, c.nproj,
                                  None if pg is not None else c.beta, c.dmat, precision,
                                  block or nb, keep, projgen=pg,
                                  gamma=getattr(c, "gamma", False),
                                  qmat=getattr(c, "qmat", None))
        psi = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.complex128).ravel()
                                                   for p in psi0s]))
        o = DavOpts(int(nvecx), float(rtol), int(maxiter), int(subspace))
        t = ctypes.c_uint64()
        _check(_lib.qeh_submit(self._h, arr, len(cells), int(nb), psi.ctypes.data_as(_c_dbl_p),
                               ctypes.byref(o), ctypes.byref(t)), "qeh_submit")
        self._nk[t.value] = (len(cells), int(nb))
        return t.value

    def poll(self, ticket):
        """None while busy; else dict(status, eig (nk, nb), info list, stamps)."""
        nk, nb = self._nk[ticket]
        eig = np.zeros(nk * nb)
        info = (DavInfo * nk)()
        ts = (ctypes.c_double * 4)()
        st = _lib.qeh_poll(self._h, ticket, eig.ctypes.data_as(_c_dbl_p), info, ts)
        if st == QEH_ERR_BUSY:
            return None
        del self._nk[ticket]
        err = _lib.qeh_last_error().decode(errors="replace") if st != QEH_OK else ""
        return dict(status=st, error=err, eig=eig.reshape(nk, nb),
                    info=[info[i].as_dict() for i in range(nk)], stamps=list(ts))

    def cancel(self, ticket):
        return _lib.qeh_cancel(self._h, ticket)

    def stats(self):
        out = (ctypes.c_double * 8)()
        _check(_lib.qeh_server_stats(self._h, out, 8), "qeh_server_stats")
        keys = ["queued", "running", "finished", "bytes_in_use", "arena_bytes", "peak_running",
                "busy_s", "uptime_s"]
        return dict(zip(keys, list(out)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.qeh_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A cell at one k-point, resident on the device.

    Inputs are plain host arrays: lattice (3,3) rows a_i, fft (N1,N2,N3), kpt (3,),
    miller (npw,3) int, vloc (N3,N2,N1) float64, nproj (nat,) int,
    beta (nkb,npw) complex128, dmat (sum nproj^2,) complex128, optional qmat (same
    layout as dmat: the overlap's q blocks, S != 1).  With beta None,
    ``projgen`` (a dict: tau, ityp, nchan, lchan, dq, tab) describes the radial
    tables from which the library builds beta on the device.  ``gamma=True``:
    real wavefunctions at k = 0, miller (and psi, beta) over the half sphere.
    """

    def __init__(self, lattice, fft, kpt, miller, vloc, nproj, beta, dmat, *,
                 precision=QEH_FP64, block=64, device=None, stream=None, projgen=None,
                 gamma=False, qmat=None):
        torch = _torch()
        self.device = torch.device(device if device is not None else "cuda")
        keep = []
        c = _cell_struct(lattice, fft, kpt, miller, vloc, nproj, beta, dmat, precision, block,
                         keep, projgen=projgen, gamma=gamma, qmat=qmat)
        self._keep = keep
        self._cell = c
        nbytes = ctypes.c_size_t()
        _check(_lib.qeh_ctx_plan(ctypes.byref(c), ctypes.byref(nbytes)), "qeh_ctx_plan")
        self.arena_bytes = int(nbytes.value)
        self.arena = torch.empty(max(self.arena_bytes, 256), dtype=torch.uint8,
                                 device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _vp()
        _check(_lib.qeh_ctx_create(ctypes.byref(c), _vp(self.arena.data_ptr()),
                                   self.arena_bytes, _stream_ptr(self.stream), ctypes.byref(h)),
               "qeh_ctx_create")
        self._h = h
        self.npw = c.npw
        self.precision = int(precision)
        self.block = int(block)
        # the host copies are no longer needed after create
        self._keep = None
        self._cell = None

    @classmethod
    def from_cell(cls, cell, **kw):
        pg = kw.get("projgen")
        kw.setdefault("gamma", getattr(cell, "gamma", False))
        kw.setdefault("qmat", getattr(cell, "qmat", None))
        return cls(cell.lattice, cell.fft, cell.kpt, cell.miller, cell.vloc, cell.nproj,
                   None if pg is not None else cell.beta, cell.dmat, **kw)

    # ---------------------------------------------------------------- H|psi>
    def _bands(self, psi):
        torch = _torch()
        if psi.dtype != torch.complex128 or psi.device.type != "cuda":
            raise TypeError("psi must be a complex128 CUDA tensor")
        if psi.dim() != 2 or psi.shape[1] < self.npw or psi.stride(1) != 1:
            raise ValueError("psi must be (nb, >= npw) with unit stride along G")
        return psi

    def apply_s(self, psi, out=None):
        """S psi (the overlap; a copy of psi without q blocks)."""
        torch = _torch()
        psi = self._bands(psi)
        nb = psi.shape[0]
        if out is None:
            out = torch.empty((nb, self.npw), dtype=torch.complex128, device=psi.device)
        _check(_lib.qeh_apply_s(self._h, nb, _vp(psi.data_ptr()), psi.stride(0),
                                _vp(out.data_ptr()), out.stride(0)), "qeh_apply_s")
        return out

    def apply_h(self, psi, out=None, part=None):
        torch = _torch()
        psi = self._bands(psi)
        nb = psi.shape[0]
        if out is None:
            out = torch.empty((nb, self.npw), dtype=torch.complex128, device=psi.device)
        ld_in, ld_out = psi.stride(0), out.stride(0)
        if part is None:
            st = _lib.qeh_apply_h(self._h, nb, _vp(psi.data_ptr()), ld_in, _vp(out.data_ptr()),
                                  ld_out)
        else:
            st = _lib.qeh_apply_h_part(self._h, int(part), nb, _vp(psi.data_ptr()), ld_in,
                                       _vp(out.data_ptr()), ld_out)
        _check(st, "qeh_apply_h")
        return out

    # ---------------------------------------------------------------- density
    def density_plan(self):
        n = ctypes.c_size_t()
        _check(_lib.qeh_density_plan(self._h, ctypes.byref(n)), "qeh_density_plan")
        return int(n.value)

    def density(self, psi, occ, out=None, work=None):
        """rho(r) = (1/Omega) sum_b occ[b] |psi_b(r)|^2 as a (N3, N2, N1) float64 CUDA tensor."""
        torch = _torch()
        psi = self._bands(psi)
        nb = psi.shape[0]
        occ = np.ascontiguousarray(np.asarray(occ, dtype=np.float64).reshape(-1))
        if occ.shape[0] != nb:
            raise ValueError("one occupation per band")
        shape = (self.info()["n3"], self.info()["n2"], self.info()["n1"])
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=psi.device)
        if tuple(out.shape) != shape or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of shape %s" % (shape,))
        need = self.density_plan()
        if work is None or work.numel() < need:
            work = torch.empty(max(need, 256), dtype=torch.uint8, device=psi.device)
        _check(_lib.qeh_density(self._h, nb, _vp(psi.data_ptr()), psi.stride(0),
                                occ.ctypes.data_as(_c_dbl_p), _vp(out.data_ptr()),
                                _vp(work.data_ptr()), int(work.numel())), "qeh_density")
        return out

    # ---------------------------------------------------------------- Davidson
    def davidson_plan(self, nb, nvecx=0, rtol=1e-8, maxiter=0, subspace=0):
        o = DavOpts(int(nvecx), float(rtol), int(maxiter), int(subspace))
        n = ctypes.c_size_t()
        _check(_lib.qeh_davidson_plan(self._h, int(nb), ctypes.byref(o), ctypes.byref(n)),
               "qeh_davidson_plan")
        return int(n.value)

    def davidson(self, psi, nvecx=0, rtol=1e-8, maxiter=0, work=None, allow_notconv=False,
                 subspace=0, refine=None):
        """In-place Davidson on psi (nb, npw) complex128; returns (eig ndarray, info dict).
        subspace: QEH_SUBSPACE_AUTO / _OWN / _ROCSOLVER (reduced-problem solver);
        refine: an FP64 Context of the same cell on the same stream, for the
        mixed form's FP64 refinement phase."""
        torch = _torch()
        psi = self._bands(psi)
        nb = psi.shape[0]
        o = DavOpts(int(nvecx), float(rtol), int(maxiter), int(subspace),
                    refine._h if refine is not None else None)
        need = self.davidson_plan(nb, nvecx, rtol, maxiter, subspace)
        if work is None or work.numel() < need:
            work = torch.empty(max(need, 256), dtype=torch.uint8, device=psi.device)
        eig = np.zeros(nb, dtype=np.float64)
        info = DavInfo()
        st = _lib.qeh_davidson(self._h, nb, _vp(psi.data_ptr()), psi.stride(0),
                               eig.ctypes.data_as(_c_dbl_p), ctypes.byref(o),
                               _vp(work.data_ptr()), int(work.numel()), ctypes.byref(info))
        _check(st, "qeh_davidson", allow=(QEH_ERR_NOT_CONVERGED,) if allow_notconv else ())
        d = info.as_dict()
        d["status"] = st
        return eig, d

    def cg_plan(self, nb):
        n = ctypes.c_size_t()
        _check(_lib.qeh_cg_plan(self._h, int(nb), ctypes.byref(n)), "qeh_cg_plan")
        return int(n.value)

    def cg(self, psi, rtol=1e-8, maxiter=0, work=None, allow_notconv=False):
        """In-place band-by-band conjugate gradient on psi (nb, npw) complex128;
        returns (eig ndarray, info dict) like davidson()."""
        torch = _torch()
        psi = self._bands(psi)
        nb = psi.shape[0]
        need = self.cg_plan(nb)
        if work is None or work.numel() < need:
            work = torch.empty(max(need, 256), dtype=torch.uint8, device=psi.device)
        o = CgOpts(float(rtol), int(maxiter))
        eig = np.zeros(nb, dtype=np.float64)
        info = DavInfo()
        st = _lib.qeh_cg(self._h, nb, _vp(psi.data_ptr()), psi.stride(0),
                         eig.ctypes.data_as(_c_dbl_p), ctypes.byref(o), _vp(work.data_ptr()),
                         int(work.numel()), ctypes.byref(info))
        _check(st, "qeh_cg", allow=(QEH_ERR_NOT_CONVERGED,) if allow_notconv else ())
        d = info.as_dict()
        d["status"] = st
        return eig, d

    def davidson_rci(self, psi, apply, nvecx=0, rtol=1e-8, maxiter=0, work=None,
                     allow_notconv=False, subspace=0):
        """Davidson with H supplied by the caller (reverse communication).
        apply(x, y) receives two complex128 (n, npw) views of the solver's work
        area and must write H x into y on this context's stream.  Returns
        (eig ndarray, info dict) like davidson()."""
        torch = _torch()
        psi = self._bands(psi)
        nb = psi.shape[0]
        o = DavOpts(int(nvecx), float(rtol), int(maxiter), int(subspace), None)
        need = self.davidson_plan(nb, nvecx, rtol, maxiter, subspace)
        if work is None or work.numel() < need:
            work = torch.empty(max(need, 256), dtype=torch.uint8, device=psi.device)
        eig = np.zeros(nb, dtype=np.float64)
        h = _vp()
        _check(_lib.qeh_dav_rci_create(self._h, nb, _vp(psi.data_ptr()), psi.stride(0),
                                       eig.ctypes.data_as(_c_dbl_p), ctypes.byref(o),
                                       _vp(work.data_ptr()), int(work.numel()),
                                       ctypes.byref(h)), "qeh_dav_rci_create")
        base, size = work.data_ptr(), work.numel()

        def view(ptr, n, ld):
            off = ptr - base
            nbytes = 16 * n * ld
            if off < 0 or off % 16 or off + nbytes > size:
                raise RuntimeError("request outside the work area")
            return work[off:off + nbytes].view(torch.complex128).view(n, ld)

        req = RciRequest()
        info = DavInfo()
        try:
            while True:
                st = _lib.qeh_dav_rci_step(h, ctypes.byref(req))
                if st != QEH_RCI_APPLY_H:
                    break
                apply(view(req.x, req.n, req.ld), view(req.y, req.n, req.ld))
        finally:
            dst = _lib.qeh_dav_rci_destroy(h, ctypes.byref(info))
        _check(st, "qeh_dav_rci_step", allow=(QEH_ERR_NOT_CONVERGED,) if allow_notconv else ())
        _check(dst, "qeh_dav_rci_destroy")
        d = info.as_dict()
        d["status"] = st
        return eig, d

    # ---------------------------------------------------------------- profiling
    def profile(self, enable=True):
        _check(_lib.qeh_ctx_profile(self._h, 1 if enable else 0), "qeh_ctx_profile")

    def stage_times(self):
        ms = (ctypes.c_double * NSTAGES)()
        n = (ctypes.c_long * NSTAGES)()
        _check(_lib.qeh_ctx_stage_times(self._h, ms, n, NSTAGES), "qeh_ctx_stage_times")
        return {STAGE_NAMES[i]: (ms[i], n[i]) for i in range(NSTAGES)}

    def hdiag(self):
        """diag(H) over the plane waves (float64 device tensor, npw values),
        the preconditioner's diagonal; copied on the context stream."""
        torch = _torch()
        out = torch.empty(self.npw, dtype=torch.float64, device=self.device)
        _check(_lib.qeh_ctx_hdiag(self._h, ctypes.c_void_p(out.data_ptr())), "qeh_ctx_hdiag")
        return out

    def info(self):
        out = (ctypes.c_long * 12)()
        _check(_lib.qeh_ctx_info(self._h, out, 12), "qeh_ctx_info")
        keys = ["npw", "nst", "nkb", "n1", "n2", "n3", "ext", "block", "precision", "plane_path",
                "stick_path", "wide_tiles"]
        return dict(zip(keys, list(out)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.qeh_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
