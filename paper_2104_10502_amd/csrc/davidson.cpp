// Block Davidson eigensolver on one GPU.
//
// The paper names the Davidson method among the GPU-accelerated iterative
// solvers, solves the small dense generalized eigenproblem with a GPU dense
// solver, and keeps the iterative solver separate from the Hamiltonian
// builder it calls (sections "Evolution of the GPU-enabled version" and
// "Domain-specific mathematical libraries").  It gives no algorithm; this is
// the textbook block Davidson:
//
//   V = psi0, W = H V, Hr = V^H W, Sr = V^H V
//   loop: Hr y = eps Sr y (Cholesky of Sr, lowest nb) ->
//         Ritz vectors P = V Y, Q = W Y, residual norms ||Q - eps P|| ->
//         (one device->host copy of nb eigenvalues + norms per iteration) ->
//         corrections t = (Q - eps P) / sqrt(1 + (diag H - eps)^2), normalised,
//         for the unconverged bands -> restart (V = P, W = Q) if the basis is
//         full -> W_new = H t -> new columns of Hr, Sr.
//
// Everything runs on the context stream.  The reductions and rotations are
// the library's MFMA complex GEMMs in FP64.  The dense Hermitian generalized
// eigensolve of the reduced pair (the paper's dense GPU solver step) runs on
// the library's own kernels for bases up to 512 vectors (eigh_kernels.hip:
// deterministic, about ten launches per iteration, no library handle) and on
// rocSOLVER above that, with its workspace taken from the caller's work area
// so the library allocates no device memory.  Small pinned host buffers hold
// the per-iteration readback.
#include "davidson.h"

#include <new>

#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>

namespace qeh {
qeh_status apply_h_impl(qeh_ctx *c, int part, int nb, const double *psi, int ldpsi,
                        double *hpsi, int ldh);
qeh_status apply_s_impl(qeh_ctx *c, int nb, const double *psi, int ldpsi, double *spsi,
                        int ldsp);

namespace {

constexpr int kMaxSplit = kReduceMaxSplit;

size_t bump2(size_t *cur, size_t bytes) {
  const size_t o = *cur;
  *cur += (bytes + kAlign - 1) / kAlign * kAlign;
  return o;
}

qeh_status solver_bytes(int n, bool real, size_t *out) {
  // the answer depends on n and the routine set only: cache it; the query
  // needs a handle, made once (creating one per query cost more than the
  // query itself)
  static std::mutex mu;
  static std::map<std::pair<int, bool>, size_t> cache;
  static rocblas_handle h = nullptr;
  std::lock_guard<std::mutex> lk(mu);
  const std::pair<int, bool> key(n, real);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *out = it->second;
    return QEH_OK;
  }
  if (!h && rocblas_create_handle(&h) != rocblas_status_success) {
    h = nullptr;
    set_error("rocblas_create_handle failed");
    return QEH_ERR_DEVICE;
  }
  rocblas_start_device_memory_size_query(h);
  rocsolver_zpotrf(h, rocblas_fill_lower, n, nullptr, n, nullptr);
  rocsolver_ztrtri(h, rocblas_fill_lower, rocblas_diagonal_non_unit, n, nullptr, n, nullptr);
  rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, n, nullptr, n, nullptr, nullptr,
                   nullptr);
  if (real) {
    // the real routines of the Gamma-point path (queried for Gamma contexts
    // only: general-k solves run the complex set alone)
    rocsolver_dpotrf(h, rocblas_fill_lower, n, nullptr, n, nullptr);
    rocsolver_dtrtri(h, rocblas_fill_lower, rocblas_diagonal_non_unit, n, nullptr, n, nullptr);
    rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, nullptr, n, nullptr,
                     nullptr, nullptr);
  }
  size_t sz = 0;
  rocblas_stop_device_memory_size_query(h, &sz);
  *out = sz;
  cache[key] = sz;
  return QEH_OK;
}

}  // namespace

// out(i, j) = sum_G conj(X_i[G]) Y_j[G] for i < nrow, j < ncol; out col-major
// with ld.  K = npw is long: split into fixed chunks whose partial products
// go to `part` and are summed in double in a fixed order.
hipError_t reduce_cols(const qeh_ctx *c, const double2 *X, int nrow, const double2 *Y, int ncol,
                       double2 *out, int ld, double2 *part) {
  const int tiles = ((ncol + 63) / 64) * ((nrow + 63) / 64);
  int ns = std::max(1, (512 + tiles - 1) / tiles);
  ns = std::min(ns, std::max(1, c->npw / 256));
  ns = std::min(ns, kMaxSplit);
  int kc = (c->npw + ns - 1) / ns;
  kc = (kc + 7) / 8 * 8;
  ns = (c->npw + kc - 1) / kc;
  GemmDesc g{};
  g.A = Y;
  g.lda = c->npw;
  g.ta = T_D2;
  g.B = X;
  g.ldb = c->npw;
  g.tb = T_D2;
  g.bmode = 0;
  g.conjB = 1;
  g.tc = T_D2;
  g.M = ncol;
  g.N = nrow;
  g.K = c->npw;
  g.prec = G_F64;
  hipError_t e;
  if (ns == 1) {
    g.C = out;
    g.ldc = ld;
    g.nsplit = 1;
    g.kchunk = c->npw;
    e = launch_cgemm(g, c->stream);
  } else {
    g.C = part;
    g.ldc = nrow;
    g.nsplit = ns;
    g.kchunk = kc;
    g.split_stride = (long)ncol * nrow;
    e = launch_cgemm(g, c->stream);
    if (e == hipSuccess)
      e = launch_splitk_reduce(part, T_D2, (long)ncol * nrow, ns, ncol, nrow, nrow, out, ld, 0,
                               c->stream);
  }
  // Gamma: half-sphere sums -> real inner products of the full-sphere vectors
  if (e == hipSuccess && c->gamma)
    e = launch_gamma_inner(out, ld, nrow, ncol, X, Y, c->npw, c->stream);
  return e;
}

// Column-major products of n x n matrices (ld): out = P Q with P given by
// its columns: out(i,j) = sum_k P(i,k) Q(k,j).  In the GEMM's row-major view
// out^T[j][i] = sum_k Q^T[j][k] P^T... -> A = Q (element (j,k) at Q[j*ld+k]),
// B(k,i) = P(i,k) at P[k*ld+i].
hipError_t square_product(const qeh_ctx *c, const double2 *Qm, const double2 *Pm, double2 *out,
                          int n, int ld) {
  GemmDesc g{};
  g.A = Qm;
  g.lda = ld;
  g.ta = T_D2;
  g.B = Pm;
  g.ldb = ld;
  g.tb = T_D2;
  g.bmode = 1;
  g.C = out;
  g.ldc = ld;
  g.tc = T_D2;
  g.M = n;
  g.N = n;
  g.K = n;
  g.nsplit = 1;
  g.kchunk = n;
  g.prec = G_F64;
  return launch_cgemm(g, c->stream);
}

// out(:, 0:ncol) = P Q(:, 0:ncol), P n x n, Q n x ncol (column-major, ld).
hipError_t square_product_cols(const qeh_ctx *c, const double2 *Qm, const double2 *Pm,
                               double2 *out, int n, int ncol, int ld) {
  GemmDesc g{};
  g.A = Qm;
  g.lda = ld;
  g.ta = T_D2;
  g.B = Pm;
  g.ldb = ld;
  g.tb = T_D2;
  g.bmode = 1;
  g.C = out;
  g.ldc = ld;
  g.tc = T_D2;
  g.M = ncol;
  g.N = n;
  g.K = n;
  g.nsplit = 1;
  g.kchunk = n;
  g.prec = G_F64;
  return launch_cgemm(g, c->stream);
}

// rows b < nb: out_b = sum_j Y(j, b) X_j  (Y col-major ld, j < n)
hipError_t rotate(const qeh_ctx *c, const double2 *Y, int ld, int n, int nb, const double2 *X,
                  double2 *out) {
  GemmDesc g{};
  g.A = Y;
  g.lda = ld;
  g.ta = T_D2;
  g.B = X;
  g.ldb = c->npw;
  g.tb = T_D2;
  g.bmode = 1;
  g.C = out;
  g.ldc = c->npw;
  g.tc = T_D2;
  g.M = nb;
  g.N = c->npw;
  g.K = n;
  g.nsplit = 1;
  g.kchunk = n;
  g.prec = G_F64;
  return launch_cgemm(g, c->stream);
}


void EvPool::start(hipStream_t s) {
  while (ev.size() < used + 2) {
    hipEvent_t x;
    if (hipEventCreate(&x) != hipSuccess) return;
    ev.push_back(x);
  }
  (void)hipEventRecord(ev[used], s);
}

void EvPool::stop(hipStream_t s) {
  if (ev.size() < used + 2) return;
  (void)hipEventRecord(ev[used + 1], s);
  used += 2;
}

void EvPool::harvest() {
  for (size_t i = 0; i + 1 < used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) acc += ms * 1e-3;
  }
  used = 0;
}

void EvPool::destroy() {
  for (auto x : ev) (void)hipEventDestroy(x);
  ev.clear();
  used = 0;
}

qeh_status dav_check_opts(const qeh_ctx *c, int nb, const qeh_dav_opts *o, int *nvecx,
                          double *rtol, int *maxiter, bool *own) {
  if (!c) {
    set_error("ctx is null");
    return QEH_ERR_INVALID;
  }
  if (nb < 1 || nb > c->npw) {
    set_error("nb must be in [1, npw]");
    return QEH_ERR_INVALID;
  }
  *nvecx = (o && o->nvecx > 0) ? o->nvecx : 2 * nb;
  *rtol = (o && o->rtol > 0) ? o->rtol : 1e-8;
  *maxiter = (o && o->maxiter > 0) ? o->maxiter : 200;
  if (*nvecx < 2 * nb || *nvecx > c->npw) {
    set_error("nvecx must be in [2 nb, npw]");
    return QEH_ERR_INVALID;
  }
  const int sub = o ? o->subspace : QEH_SUBSPACE_AUTO;
  if (sub != QEH_SUBSPACE_AUTO && sub != QEH_SUBSPACE_OWN && sub != QEH_SUBSPACE_ROCSOLVER) {
    set_error("subspace must be QEH_SUBSPACE_AUTO, _OWN or _ROCSOLVER");
    return QEH_ERR_INVALID;
  }
  if (sub == QEH_SUBSPACE_OWN && *nvecx > kEigMaxN) {
    set_error("the own subspace solver takes nvecx <= " + std::to_string(kEigMaxN));
    return QEH_ERR_INVALID;
  }
  *own = sub == QEH_SUBSPACE_OWN || (sub == QEH_SUBSPACE_AUTO && *nvecx <= kEigAutoMaxN);
  if (o && o->refine) {
    const qeh_ctx *r = o->refine;
    if (c->prec != QEH_MIXED || r->prec != QEH_FP64) {
      set_error("refine: a QEH_FP64 context for a QEH_MIXED solve");
      return QEH_ERR_INVALID;
    }
    if (r->npw != c->npw || r->gamma != c->gamma || r->n1 != c->n1 || r->n2 != c->n2 ||
        r->n3 != c->n3 || r->nkb != c->nkb || r->nat != c->nat || r->has_q != c->has_q) {
      set_error("refine: context of a different cell (npw, box, projectors or Gamma flag)");
      return QEH_ERR_INVALID;
    }
  }
  return QEH_OK;
}

qeh_status dav_layout(const qeh_ctx *c, int nb, int nvecx, bool own, DavLayout *L) {
  size_t cur = 0;
  const size_t row = 16 * (size_t)c->npw;
  L->V = bump2(&cur, row * nvecx);
  L->W = bump2(&cur, row * nvecx);
  L->P = bump2(&cur, row * nb);
  L->Q = bump2(&cur, row * nb);
  const size_t mat = 16 * (size_t)nvecx * nvecx;
  L->Hr = bump2(&cur, mat);
  L->Sr = bump2(&cur, mat);
  L->Hw = bump2(&cur, mat);
  L->Sw = bump2(&cur, mat);
  L->X = bump2(&cur, mat);
  L->Lc = bump2(&cur, mat);
  L->LcH = bump2(&cur, mat);
  L->Y = bump2(&cur, mat);
  L->part = bump2(&cur, 16 * (size_t)kMaxSplit * nb * nvecx);
  L->eps = bump2(&cur, 8 * (size_t)nvecx);
  L->E = bump2(&cur, 8 * (size_t)nvecx);
  L->norms = bump2(&cur, 8 * (size_t)nb);
  L->idx = bump2(&cur, 4 * (size_t)nb);
  L->info = bump2(&cur, 16);
  L->flag = bump2(&cur, 4);
  // generalized problem: S V and S P beside V and P
  L->U = bump2(&cur, c->has_q ? row * nvecx : 0);
  L->SP = bump2(&cur, c->has_q ? row * nb : 0);
  L->own = own;
  if (own) {
    L->solver_bytes = 0;
    L->solver = bump2(&cur, 0);
    L->tri = bump2(&cur, 8 * 4 * (size_t)nvecx);
    L->Zt = bump2(&cur, 8 * (size_t)nvecx * nb);
    L->escr = bump2(&cur, 8 * eig_scratch_doubles(nvecx));
  } else {
    qeh_status st = solver_bytes(nvecx, c->gamma != 0, &L->solver_bytes);
    if (st != QEH_OK) return st;
    L->solver = bump2(&cur, std::max<size_t>(L->solver_bytes, 256));
    L->tri = L->Zt = L->escr = bump2(&cur, 0);
  }
  L->total = cur;
  return QEH_OK;
}

qeh_status DavRun::init(qeh_ctx *c, int nb, double2 *psi, int ldpsi, double *eig,
                        const qeh_dav_opts *o, void *work, size_t work_bytes) {
  t0_ = std::chrono::steady_clock::now();
  double rtol;
  qeh_status st = dav_check_opts(c, nb, o, &nvecx_, &rtol, &maxiter_, &own_);
  if (st != QEH_OK) return st;
  if (!psi || !eig || !work) {
    set_error("psi_inout, eig and work must be non-null");
    return QEH_ERR_INVALID;
  }
  if (ldpsi < c->npw) {
    set_error("ldpsi < npw");
    return QEH_ERR_INVALID;
  }
  if (reinterpret_cast<uintptr_t>(work) % kAlign) {
    set_error("work not 256-byte aligned");
    return QEH_ERR_INVALID;
  }
  st = dav_layout(c, nb, nvecx_, own_, &L_);
  if (st != QEH_OK) return st;
  if (work_bytes < L_.total) {
    set_error("work area has " + std::to_string(work_bytes) + " bytes, plan needs " +
              std::to_string(L_.total));
    return QEH_ERR_NOMEM;
  }
  c_ = c;
  nb_ = nb;
  psi_ = psi;
  ldpsi_ = ldpsi;
  eig_ = eig;
  npw_ = c->npw;
  mixed_ = c->prec == QEH_MIXED;
  c64_ = o ? o->refine : nullptr;
  if (c64_ && c64_->stream != c->stream) {
    set_error("refine: the FP64 context must use the same HIP stream");
    return QEH_ERR_INVALID;
  }
  phase64_ = false;
  it64_ = 0;
  thr_ = mixed_ ? std::max(rtol, 1e-5) : rtol;
  char *w = reinterpret_cast<char *>(work);
  V_ = reinterpret_cast<double2 *>(w + L_.V);
  W_ = reinterpret_cast<double2 *>(w + L_.W);
  P_ = reinterpret_cast<double2 *>(w + L_.P);
  Q_ = reinterpret_cast<double2 *>(w + L_.Q);
  Hr_ = reinterpret_cast<double2 *>(w + L_.Hr);
  Sr_ = reinterpret_cast<double2 *>(w + L_.Sr);
  Hw_ = reinterpret_cast<double2 *>(w + L_.Hw);
  Sw_ = reinterpret_cast<double2 *>(w + L_.Sw);
  part_ = reinterpret_cast<double2 *>(w + L_.part);
  X_ = reinterpret_cast<double2 *>(w + L_.X);
  Lc_ = reinterpret_cast<double2 *>(w + L_.Lc);
  LcH_ = reinterpret_cast<double2 *>(w + L_.LcH);
  Y_ = reinterpret_cast<double2 *>(w + L_.Y);
  eps_d_ = reinterpret_cast<double *>(w + L_.eps);
  E_d_ = reinterpret_cast<double *>(w + L_.E);
  norms_d_ = reinterpret_cast<double *>(w + L_.norms);
  idx_d_ = reinterpret_cast<int *>(w + L_.idx);
  info_d_ = reinterpret_cast<int *>(w + L_.info);
  flag_d_ = reinterpret_cast<int *>(w + L_.flag);
  gen_ = c->has_q != 0;
  U_ = gen_ ? reinterpret_cast<double2 *>(w + L_.U) : nullptr;
  SP_ = gen_ ? reinterpret_cast<double2 *>(w + L_.SP) : nullptr;
  tri_ = reinterpret_cast<double *>(w + L_.tri);
  Zt_ = reinterpret_cast<double *>(w + L_.Zt);
  escr_ = reinterpret_cast<double *>(w + L_.escr);
  // pinned host readback: eps, norms (nb doubles each), idx (nb ints), 2 ints
  void *h = nullptr;
  const size_t hb = 16 * (size_t)nb + 4 * (size_t)nb + 32;
  hipError_t e = hipHostMalloc(&h, hb, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(e, "pinned host buffer");
  h_eps_ = reinterpret_cast<double *>(h);
  h_nrm_ = h_eps_ + nb;
  h_idx_ = reinterpret_cast<int *>(h_nrm_ + nb);
  h_int_ = h_idx_ + nb;
  eps_prev_.assign(nb, INFINITY);
  best_res_.assign(nb, INFINITY);
  stall_.assign(nb, 0);
  phase_ = kStart;
  notconv_ = nb;
  resid_max_ = INFINITY;
  if (own_) return QEH_OK;   // no library handle: the own solver needs none
  if (rocblas_create_handle(&rh_) != rocblas_status_success) {
    rh_ = nullptr;
    release();
    set_error("rocblas_create_handle failed");
    return QEH_ERR_DEVICE;
  }
  // library reductions with atomics sum in an order that depends on timing:
  // forbid them, so that a solve gives the same bits whatever else runs
  if (rocblas_set_stream(rh_, c->stream) != rocblas_status_success ||
      rocblas_set_atomics_mode(rh_, rocblas_atomics_not_allowed) != rocblas_status_success) {
    release();
    set_error("rocblas_set_stream / rocblas_set_atomics_mode failed");
    return QEH_ERR_DEVICE;
  }
  if (rocblas_set_workspace(rh_, w + L_.solver, std::max<size_t>(L_.solver_bytes, 256)) !=
      rocblas_status_success) {
    release();
    set_error("rocblas_set_workspace failed");
    return QEH_ERR_DEVICE;
  }
  phase_ = kStart;
  notconv_ = nb;
  resid_max_ = INFINITY;
  return QEH_OK;
}

void DavRun::release() {
  ev_h_.destroy();
  ev_s_.destroy();
  if (rh_) rocblas_destroy_handle(rh_);
  rh_ = nullptr;
  if (h_eps_) (void)hipHostFree(h_eps_);
  h_eps_ = nullptr;
}

qeh_status DavRun::hpsi(const double2 *x, double2 *y, int n) {
  band_applies_ += n;
  if (rci_) {   // the caller applies H before the next advance()
    req_x_ = x;
    req_y_ = y;
    req_n_ = n;
    pending_ = true;
    return QEH_OK;
  }
  ev_h_.start(c_->stream);
  qeh_status r = apply_h_impl(phase64_ ? c64_ : c_, 2, n, reinterpret_cast<const double *>(x),
                              npw_, reinterpret_cast<double *>(y), npw_);
  ev_h_.stop(c_->stream);
  return r;
}

bool DavRun::take_request(const double2 **x, double2 **y, int *n) {
  if (!pending_) return false;
  pending_ = false;
  *x = req_x_;
  *y = req_y_;
  *n = req_n_;
  return true;
}

// Hr y = eps Sr y on the library's kernels: Sr = L L^H, A = L^-1 Hr L^-H by
// two triangular solves (L^-1 Hr, then L^-1 of its adjoint), A = Q T Q^H,
// the nb lowest eigenpairs of T, Z = Q Z_T, Y = L^-H Z.  Works in the
// arena's n x n matrices: Sw (factor, then A before symmetrising), Lc / LcH
// (L, L^H), X (L^-1 Hr, then Z), Hw (A, then its reflectors), Y.
void DavRun::rr_own() {
  hipStream_t s = c_->stream;
  const int n = nbase_, nb = nb_, ld = nvecx_;
  ok(launch_hermitise_copy(Hr_, ld, Hw_, ld, n, s));
  ok(launch_hermitise_copy(Sr_, ld, Sw_, ld, n, s));
  ok(launch_chol(Sw_, ld, n, info_d_ + 1, escr_, wide_, s));
  ok(launch_tril_adjoint(Sw_, Lc_, LcH_, ld, n, s));
  ok(launch_trsm(0, Lc_, ld, n, Hw_, ld, n, X_, ld, s));    // X = L^-1 Hr
  ok(launch_trsm(1, Lc_, ld, n, X_, ld, n, Sw_, ld, s));    // Sw = L^-1 X^H = A
  ok(launch_hermitise_copy(Sw_, ld, Hw_, ld, n, s));        // Hw = (A + A^H) / 2
  ok(launch_tridiag(Hw_, ld, n, tri_, escr_, info_d_ + 1, wide_, s));
  ok(launch_trieig(tri_, n, nb, eps_d_, Zt_, n, escr_, info_d_ + 3, info_d_ + 1, wide_, s));
  ok(launch_backtr(Hw_, ld, n, tri_, Zt_, n, nb, X_, ld, info_d_ + 1, info_d_ + 3, s));
  ok(launch_trsm(2, LcH_, ld, n, X_, ld, nb, Y_, ld, s));   // Y = L^-H Z
}

// Basis = the current Ritz vectors (orthonormal), W = H V through the active
// context, reduced matrices rebuilt from them.
void DavRun::restart_from_ritz() {
  hipStream_t s = c_->stream;
  ++restarts_;
  ok(launch_copy_rows(P_, npw_, V_, npw_, npw_, nb_, s));
  nbase_ = nb_;
  if (phase64_) {
    qeh_status st = hpsi(V_, W_, nb_);
    if (st == QEH_OK && gen_) st = spsi(V_, U_, nb_);
    if (st != QEH_OK && result_ == QEH_OK) result_ = st;
  } else {
    ok(launch_copy_rows(Q_, npw_, W_, npw_, npw_, nb_, s));
    if (gen_) ok(launch_copy_rows(SP_, npw_, U_, npw_, npw_, nb_, s));
  }
  ok(reduce_cols(c_, V_, nb_, W_, nb_, Hr_, nvecx_, part_));
  ok(reduce_cols(c_, V_, nb_, gen_ ? U_ : V_, nb_, Sr_, nvecx_, part_));
}

qeh_status DavRun::spsi(const double2 *x, double2 *y, int n) {
  // timed with H (t_hpsi), except under reverse communication, where that
  // figure is left to the caller
  if (!rci_) ev_h_.start(c_->stream);
  qeh_status r = apply_s_impl(phase64_ ? c64_ : c_, n, reinterpret_cast<const double *>(x), npw_,
                              reinterpret_cast<double *>(y), npw_);
  if (!rci_) ev_h_.stop(c_->stream);
  return r;
}

bool DavRun::fail_device(const char *what) {
  result_ = hip_fail(err_, what);
  phase_ = kDone;
  return true;
}

bool DavRun::advance() {
  hipStream_t s = c_->stream;
  const int nb = nb_, npw = npw_, nvecx = nvecx_;
  while (true) {
    if (err_ != hipSuccess) return fail_device("davidson");
    switch (phase_) {
      case kStart: {
        // finiteness of psi0, V = psi0
        ok(launch_fill_int(flag_d_, 1, 0, s));
        ok(launch_fill_int(info_d_, 4, 0, s));
        for (int b = 0; b < nb; ++b)
          ok(launch_check_finite(reinterpret_cast<const double *>(psi_ + (size_t)b * ldpsi_),
                                 2 * (long)npw, flag_d_, s));
        ok(launch_copy_rows(psi_, ldpsi_, V_, npw, npw, nb, s));
        if (c_->gamma) ok(launch_zero_g0_imag(V_, npw, nb, s));   // psi(G = 0) real
        ok(hipMemcpyAsync(h_int_, flag_d_, 4, hipMemcpyDeviceToHost, s));
        phase_ = kCheckInput;
        return false;
      }
      case kCheckInput: {
        if (h_int_[0]) {
          set_error("psi0 has a non-finite value");
          result_ = QEH_ERR_NUMERIC;
          phase_ = kDone;
          return true;
        }
        qeh_status st = hpsi(V_, W_, nb);
        if (st != QEH_OK) {
          result_ = st;
          phase_ = kDone;
          return true;
        }
        phase_ = kCheckInputPost;
        if (rci_) return false;
        break;
      }
      case kCheckInputPost: {
        qeh_status st = gen_ ? spsi(V_, U_, nb) : QEH_OK;
        if (st != QEH_OK) {
          result_ = st;
          phase_ = kDone;
          return true;
        }
        ok(reduce_cols(c_, V_, nb, W_, nb, Hr_, nvecx, part_));
        ok(reduce_cols(c_, V_, nb, gen_ ? U_ : V_, nb, Sr_, nvecx, part_));
        nbase_ = nb;
        phase_ = kRR;
        break;
      }
      case kRR: {
        // Hr y = eps Sr y: Sr = L L^H (Cholesky; its status is checked on the
        // host before anything consumes L), A = L^-1 Hr L^-H (two MFMA
        // products with the explicit inverse), A z = eps z (Hermitian
        // eigensolver), y = L^-H z (one more product).
        ++it_;
        if (phase64_) ++it64_;
        if (own_) {
          // the whole reduced solve is enqueued at once: the kernels after
          // the Cholesky skip their work when it failed, and the host reads
          // all status words after one drain
          ev_s_.start(s);
          rr_own();
          ev_s_.stop(s);
          h_int_[1] = h_int_[2] = h_int_[3] = 0;
          ok(hipMemcpyAsync(h_int_ + 1, info_d_ + 1, 12, hipMemcpyDeviceToHost, s));
          phase_ = kRRCheck;
          return false;
        }
        ev_s_.start(s);
        const int n = nbase_;
        ok(launch_hermitise_copy(Hr_, nvecx, Hw_, nvecx, n, s));
        ok(launch_hermitise_copy(Sr_, nvecx, Sw_, nvecx, n, s));
        rocblas_status rs;
        if (c_->gamma) {
          // Gamma: the reduced matrices are real symmetric; the real routines
          // work on a real copy in X's space (rocSOLVER's complex eigensolver
          // returned non-finite vectors for complex input with all imaginary
          // parts zero at n >= 128)
          double *xr = reinterpret_cast<double *>(X_);
          ok(launch_real_part(Sw_, nvecx, xr, nvecx, n, s));
          rs = rocsolver_dpotrf(rh_, rocblas_fill_lower, n, xr, nvecx, info_d_ + 1);
          ok(launch_real_to_complex(xr, nvecx, Sw_, nvecx, n, s));
        } else {
          rs = rocsolver_zpotrf(rh_, rocblas_fill_lower, n,
                                reinterpret_cast<rocblas_double_complex *>(Sw_), nvecx,
                                info_d_ + 1);
        }
        ev_s_.stop(s);
        if (rs != rocblas_status_success) {
          set_error("rocsolver_zpotrf failed to launch");
          result_ = QEH_ERR_DEVICE;
          phase_ = kDone;
          return true;
        }
        h_int_[2] = h_int_[3] = 0;
        ok(hipMemcpyAsync(h_int_ + 1, info_d_ + 1, 4, hipMemcpyDeviceToHost, s));
        phase_ = kRRSolve;
        return false;
      }
      case kRRSolve: {
        if (h_int_[1] != 0) {   // not positive definite: handled in kRRCheck
          phase_ = kRRCheck;
          break;
        }
        const int n = nbase_;
        ev_s_.start(s);
        double *xr = reinterpret_cast<double *>(X_);   // Gamma: real scratch
        rocblas_status rs;
        if (c_->gamma) {
          ok(launch_real_part(Sw_, nvecx, xr, nvecx, n, s));
          rs = rocsolver_dtrtri(rh_, rocblas_fill_lower, rocblas_diagonal_non_unit, n, xr, nvecx,
                                info_d_ + 2);
          ok(launch_real_to_complex(xr, nvecx, Sw_, nvecx, n, s));
        } else {
          rs = rocsolver_ztrtri(rh_, rocblas_fill_lower, rocblas_diagonal_non_unit, n,
                                reinterpret_cast<rocblas_double_complex *>(Sw_), nvecx,
                                info_d_ + 2);
        }
        ok(launch_tril_adjoint(Sw_, Lc_, LcH_, nvecx, n, s));
        ok(square_product(c_, Hw_, Lc_, X_, n, nvecx));     // X = L^-1 Hr
        ok(square_product(c_, LcH_, X_, Hw_, n, nvecx));    // A = X L^-H
        if (rs == rocblas_status_success && c_->gamma) {
          ok(launch_real_part(Hw_, nvecx, xr, nvecx, n, s));
          rs = rocsolver_dsyevd(rh_, rocblas_evect_original, rocblas_fill_upper, n, xr, nvecx,
                                eps_d_, E_d_, info_d_ + 3);
          ok(launch_real_to_complex(xr, nvecx, Hw_, nvecx, n, s));
        } else if (rs == rocblas_status_success) {
          rs = rocsolver_zheevd(rh_, rocblas_evect_original, rocblas_fill_upper, n,
                                reinterpret_cast<rocblas_double_complex *>(Hw_), nvecx, eps_d_,
                                E_d_, info_d_ + 3);
        }
        ok(square_product_cols(c_, Hw_, LcH_, Y_, n, nb, nvecx));   // Y = L^-H Z
        ev_s_.stop(s);
        if (rs != rocblas_status_success) {
          set_error("rocSOLVER call failed to launch");
          result_ = QEH_ERR_DEVICE;
          phase_ = kDone;
          return true;
        }
        ok(hipMemcpyAsync(h_int_ + 2, info_d_ + 2, 8, hipMemcpyDeviceToHost, s));
        phase_ = kRRCheck;
        return false;
      }
      case kRRCheck: {
        if (h_int_[1] != 0 || h_int_[2] != 0 || h_int_[3] != 0) {
          // reduced overlap not positive definite (or solver failure)
          if (chol_prev_ || !have_ritz_) {
            set_error("reduced overlap matrix not positive definite");
            result_ = QEH_ERR_CHOLESKY;
            if (!have_ritz_) {
              phase_ = kDone;
              return true;
            }
            ok(launch_copy_rows(P_, npw, psi_, ldpsi_, npw, nb, s));
            phase_ = kFinish;
            return false;
          }
          // restart from the last Ritz vectors (orthonormal)
          chol_prev_ = true;
          restart_from_ritz();
          phase_ = kRR;
          break;
        }
        chol_prev_ = false;
        ev_s_.start(s);
        ok(rotate(c_, Y_, nvecx, nbase_, nb, V_, P_));
        ok(rotate(c_, Y_, nvecx, nbase_, nb, W_, Q_));
        if (gen_) ok(rotate(c_, Y_, nvecx, nbase_, nb, U_, SP_));
        // residuals H psi - eps S psi (S psi = psi for S = 1)
        ok(launch_resid_norms(gen_ ? SP_ : P_, Q_, npw, npw, nb, eps_d_, norms_d_, c_->gamma, s));
        ev_s_.stop(s);
        have_ritz_ = true;
        ok(hipMemcpyAsync(h_eps_, eps_d_, 8 * (size_t)nb, hipMemcpyDeviceToHost, s));
        ok(hipMemcpyAsync(h_nrm_, norms_d_, 8 * (size_t)nb, hipMemcpyDeviceToHost, s));
        phase_ = kConverge;
        return false;
      }
      case kConverge: {
        ev_h_.harvest();
        ev_s_.harvest();
        int nc = 0;
        resid_max_ = 0.0;
        bool finite = true;
        for (int b = 0; b < nb; ++b) {
          const double r = std::sqrt(std::max(h_nrm_[b], 0.0));
          if (!std::isfinite(r) || !std::isfinite(h_eps_[b])) finite = false;
          resid_max_ = std::max(resid_max_, r);
          bool conv = r <= thr_;
          if (r < 0.9 * best_res_[b]) {
            best_res_[b] = r;
            stall_[b] = 0;
          } else {
            ++stall_[b];
          }
          // mixed form, single-precision phase: the floor stops the residual
          // (noise at the floor can keep resetting the stall count, so a Ritz
          // value that has settled to 1e-8 Ry counts as stalled too).  With a
          // refinement context a stalled band is handed over to the FP64
          // phase, whatever its residual; without one it is accepted at the
          // floor only while that floor is <= 10x the threshold (3 iterations)
          // or <= 100x (5 iterations, or a settled Ritz value): the floor
          // grows with the cutoff and the number of projectors
          if (mixed_ && !phase64_) {
            const bool settled = std::fabs(h_eps_[b] - eps_prev_[b]) <= 1e-8;
            if (c64_ && (stall_[b] >= 3 || settled)) conv = true;
            if (!c64_ && stall_[b] >= 3 && r <= 10.0 * thr_) conv = true;
            if (!c64_ && (stall_[b] >= 5 || settled) && r <= 100.0 * thr_) conv = true;
          }
          if (!conv) h_idx_[nc++] = b;
        }
        for (int b = 0; b < nb; ++b) eps_prev_[b] = h_eps_[b];
        notconv_ = nc;
        if (!finite) {
          set_error("non-finite residual or eigenvalue");
          result_ = QEH_ERR_NUMERIC;
        } else if (nc > 0 && it_ >= maxiter_) {
          set_error("Davidson reached maxiter");
          result_ = QEH_ERR_NOT_CONVERGED;
        }
        if (nc == 0 && result_ == QEH_OK && c64_ && !phase64_) {
          // single precision has done what it can: continue on the same basis
          // with H (and S) applied in FP64 until the FP64 residuals meet thr.
          // W = H V is recomputed for every basis vector (the subspace is
          // kept, only the operator's rounding changes); Sr = V^H V stands
          // unless S != 1, whose S V is recomputed as well
          phase64_ = true;
          for (int b = 0; b < nb; ++b) {
            best_res_[b] = INFINITY;
            stall_[b] = 0;
          }
          qeh_status st = hpsi(V_, W_, nbase_);
          if (st == QEH_OK && gen_) st = spsi(V_, U_, nbase_);
          if (st != QEH_OK) {
            result_ = st;
            phase_ = kDone;
            return true;
          }
          ok(reduce_cols(c_, V_, nbase_, W_, nbase_, Hr_, nvecx, part_));
          if (gen_) ok(reduce_cols(c_, V_, nbase_, U_, nbase_, Sr_, nvecx, part_));
          phase_ = kRR;
          break;
        }
        if (nc == 0 || result_ != QEH_OK) {
          ok(launch_copy_rows(P_, npw, psi_, ldpsi_, npw, nb, s));
          phase_ = kFinish;
          return false;
        }
        ok(hipMemcpyAsync(idx_d_, h_idx_, 4 * (size_t)nc, hipMemcpyHostToDevice, s));
        if (nbase_ + nc > nvecx) {
          ++restarts_;
          ok(launch_copy_rows(P_, npw, V_, npw, npw, nb, s));
          ok(launch_copy_rows(Q_, npw, W_, npw, npw, nb, s));
          if (gen_) ok(launch_copy_rows(SP_, npw, U_, npw, npw, nb, s));
          ok(launch_set_diag(Hr_, nvecx, nb, eps_d_, s));
          ok(launch_set_diag(Sr_, nvecx, nb, nullptr, s));
          nbase_ = nb;
        }
        ok(launch_precond(gen_ ? SP_ : P_, Q_, npw, npw, idx_d_, nc, eps_d_, c_->d.hdiag,
                          V_ + (size_t)nbase_ * npw, npw, c_->gamma, s));
        qeh_status st = hpsi(V_ + (size_t)nbase_ * npw, W_ + (size_t)nbase_ * npw, nc);
        if (st != QEH_OK) {
          result_ = st;
          phase_ = kDone;
          return true;
        }
        nc_ = nc;
        phase_ = kConvergePost;
        if (rci_) return false;
        break;
      }
      case kConvergePost: {
        const int nc = nc_;
        qeh_status st =
            gen_ ? spsi(V_ + (size_t)nbase_ * npw, U_ + (size_t)nbase_ * npw, nc) : QEH_OK;
        if (st != QEH_OK) {
          result_ = st;
          phase_ = kDone;
          return true;
        }
        ev_s_.start(s);
        ok(reduce_cols(c_, V_, nbase_ + nc, W_ + (size_t)nbase_ * npw, nc,
                       Hr_ + (size_t)nbase_ * nvecx, nvecx, part_));
        ok(reduce_cols(c_, V_, nbase_ + nc, (gen_ ? U_ : V_) + (size_t)nbase_ * npw, nc,
                       Sr_ + (size_t)nbase_ * nvecx, nvecx, part_));
        ok(launch_herm_fill(Hr_, nvecx, nbase_, nbase_ + nc, s));
        ok(launch_herm_fill(Sr_, nvecx, nbase_, nbase_ + nc, s));
        ev_s_.stop(s);
        nbase_ += nc;
        phase_ = kRR;
        break;
      }
      case kFinish: {
        ev_h_.harvest();
        ev_s_.harvest();
        for (int b = 0; b < nb; ++b) eig_[b] = h_eps_[b];
        t_total_ = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
        phase_ = kDone;
        return true;
      }
      case kDone:
        return true;
    }
  }
}

void DavRun::fill_info(qeh_dav_info *info) const {
  if (!info) return;
  info->iters = it_;
  info->notconv = notconv_;
  info->restarts = restarts_;
  info->band_applies = band_applies_;
  info->resid_max = resid_max_;
  info->t_hpsi = ev_h_.acc;
  info->t_subspace = ev_s_.acc;
  info->refine_iters = it64_;
  info->t_total = t_total_ > 0.0 ? t_total_
                                 : std::chrono::duration<double>(
                                       std::chrono::steady_clock::now() - t0_).count();
}

}  // namespace qeh

using namespace qeh;

extern "C" {

qeh_status qeh_davidson_plan(const qeh_ctx *c, int nb, const qeh_dav_opts *o,
                             size_t *work_bytes) {
  if (!work_bytes) {
    set_error("work_bytes is null");
    return QEH_ERR_INVALID;
  }
  int nvecx, maxiter;
  double rtol;
  bool own = false;
  qeh_status st = dav_check_opts(c, nb, o, &nvecx, &rtol, &maxiter, &own);
  if (st != QEH_OK) return st;
  DavLayout L;
  st = dav_layout(c, nb, nvecx, own, &L);
  if (st != QEH_OK) return st;
  *work_bytes = L.total;
  return QEH_OK;
}

qeh_status qeh_davidson(qeh_ctx *c, int nb, double *psi_inout, int ldpsi, double *eig,
                        const qeh_dav_opts *o, void *work, size_t work_bytes,
                        qeh_dav_info *info) {
  DavRun run;
  qeh_status st = run.init(c, nb, reinterpret_cast<double2 *>(psi_inout), ldpsi, eig, o, work,
                           work_bytes);
  if (st != QEH_OK) return st;
  while (!run.advance()) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      run.release();
      return hip_fail(e, "davidson sync");
    }
  }
  run.fill_info(info);
  const qeh_status r = run.result();
  run.release();
  return r;
}

}  // extern "C"

struct qeh_dav_rci {
  qeh::DavRun run;
  qeh_ctx *ctx = nullptr;
  bool ended = false;
  qeh_status final_status = QEH_OK;
};

extern "C" {

qeh_status qeh_dav_rci_create(qeh_ctx *c, int nb, double *psi_inout, int ldpsi, double *eig,
                              const qeh_dav_opts *o, void *work, size_t work_bytes,
                              qeh_dav_rci **out) {
  if (!out) {
    set_error("out is null");
    return QEH_ERR_INVALID;
  }
  *out = nullptr;
  if (o && o->refine) {
    set_error("reverse communication: the caller applies H, opts->refine must be NULL");
    return QEH_ERR_INVALID;
  }
  qeh_dav_rci *r = new (std::nothrow) qeh_dav_rci;
  if (!r) {
    set_error("no host memory for the reverse-communication handle");
    return QEH_ERR_NOMEM;
  }
  qeh_status st = r->run.init(c, nb, reinterpret_cast<double2 *>(psi_inout), ldpsi, eig, o,
                              work, work_bytes);
  if (st != QEH_OK) {
    delete r;
    return st;
  }
  r->run.set_rci();
  r->ctx = c;
  *out = r;
  return QEH_OK;
}

qeh_status qeh_dav_rci_step(qeh_dav_rci *r, qeh_rci_request *req) {
  if (!r || !req) {
    set_error("rci and req must be non-null");
    return QEH_ERR_INVALID;
  }
  req->x = nullptr;
  req->y = nullptr;
  req->n = 0;
  req->ld = 0;
  if (r->ended) return r->final_status;
  while (!r->run.advance()) {
    const double2 *x;
    double2 *y;
    int n;
    if (r->run.take_request(&x, &y, &n)) {
      req->x = reinterpret_cast<const double *>(x);
      req->y = reinterpret_cast<double *>(y);
      req->n = n;
      req->ld = r->ctx->npw;
      return QEH_RCI_APPLY_H;
    }
    hipError_t e = hipStreamSynchronize(r->ctx->stream);
    if (e != hipSuccess) {
      r->ended = true;
      r->final_status = hip_fail(e, "davidson sync");
      return r->final_status;
    }
  }
  r->ended = true;
  r->final_status = r->run.result();
  return r->final_status;
}

qeh_status qeh_dav_rci_destroy(qeh_dav_rci *r, qeh_dav_info *info) {
  if (!r) {
    set_error("rci is null");
    return QEH_ERR_INVALID;
  }
  // work still enqueued (an abandoned solve) reads the handle's pinned buffers
  hipError_t e = hipStreamSynchronize(r->ctx->stream);
  r->run.fill_info(info);
  r->run.release();
  delete r;
  return e == hipSuccess ? QEH_OK : hip_fail(e, "davidson rci destroy");
}

namespace {
struct EighLayout {
  size_t Sw, Lc, LcH, X, Hw, tri, Zt, escr, info, total;
};
EighLayout eigh_layout(int n, int nb) {
  EighLayout L{};
  size_t cur = 0;
  const size_t mat = 16 * (size_t)n * n;
  L.Sw = bump2(&cur, mat);
  L.Lc = bump2(&cur, mat);
  L.LcH = bump2(&cur, mat);
  L.X = bump2(&cur, mat);
  L.Hw = bump2(&cur, mat);
  L.tri = bump2(&cur, 8 * 4 * (size_t)n);
  L.Zt = bump2(&cur, 8 * (size_t)n * nb);
  L.escr = bump2(&cur, 8 * eig_scratch_doubles(n));
  L.info = bump2(&cur, 16);
  L.total = cur;
  return L;
}
}  // namespace

qeh_status qeh_subspace_plan(int n, int nb, size_t *work_bytes) {
  if (!work_bytes) {
    set_error("work_bytes is null");
    return QEH_ERR_INVALID;
  }
  if (n < 1 || n > kEigMaxN || nb < 1 || nb > n) {
    set_error("need 1 <= nb <= n <= " + std::to_string(kEigMaxN));
    return QEH_ERR_INVALID;
  }
  *work_bytes = eigh_layout(n, nb).total;
  return QEH_OK;
}

qeh_status qeh_subspace_eigh(int n, int nb, const double *H, const double *S, int ld, double *eig,
                             double *Y, int ldy, void *work, size_t work_bytes,
                             void *hip_stream) {
  size_t need = 0;
  qeh_status st = qeh_subspace_plan(n, nb, &need);
  if (st != QEH_OK) return st;
  if (!H || !S || !eig || !Y || !work) {
    set_error("H, S, eig, Y and work must be non-null");
    return QEH_ERR_INVALID;
  }
  if (ld < n || ldy < n) {
    set_error("ld and ldy must be >= n");
    return QEH_ERR_INVALID;
  }
  if (reinterpret_cast<uintptr_t>(work) % kAlign || work_bytes < need) {
    set_error("work must be 256-byte aligned with qeh_subspace_plan bytes");
    return QEH_ERR_NOMEM;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const EighLayout L = eigh_layout(n, nb);
  char *w = static_cast<char *>(work);
  auto M = [&](size_t off) { return reinterpret_cast<double2 *>(w + off); };
  double *tri = reinterpret_cast<double *>(w + L.tri), *zt = reinterpret_cast<double *>(w + L.Zt),
         *escr = reinterpret_cast<double *>(w + L.escr);
  int *info = reinterpret_cast<int *>(w + L.info);
  const double2 *h = reinterpret_cast<const double2 *>(H), *sm = reinterpret_cast<const double2 *>(S);
  hipError_t e = launch_fill_int(info, 4, 0, s);
  auto run = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  run(launch_hermitise_copy(h, ld, M(L.Hw), n, n, s));
  run(launch_hermitise_copy(sm, ld, M(L.Sw), n, n, s));
  run(launch_chol(M(L.Sw), n, n, info, escr, true, s));
  run(launch_tril_adjoint(M(L.Sw), M(L.Lc), M(L.LcH), n, n, s));
  run(launch_trsm(0, M(L.Lc), n, n, M(L.Hw), n, n, M(L.X), n, s));
  run(launch_trsm(1, M(L.Lc), n, n, M(L.X), n, n, M(L.Sw), n, s));
  run(launch_hermitise_copy(M(L.Sw), n, M(L.Hw), n, n, s));
  run(launch_tridiag(M(L.Hw), n, n, tri, escr, info, true, s));
  run(launch_trieig(tri, n, nb, eig, zt, n, escr, info + 2, info, true, s));
  run(launch_backtr(M(L.Hw), n, n, tri, zt, n, nb, M(L.X), n, info, info + 2, s));
  run(launch_trsm(2, M(L.LcH), n, n, M(L.X), n, nb, reinterpret_cast<double2 *>(Y), ldy, s));
  int hinfo[4] = {0, 0, 0, 0};
  run(hipMemcpyAsync(hinfo, info, 16, hipMemcpyDeviceToHost, s));
  run(hipStreamSynchronize(s));
  if (e != hipSuccess) return hip_fail(e, "qeh_subspace_eigh");
  if (hinfo[0] != 0) {
    set_error("S is not positive definite (leading minor " + std::to_string(hinfo[0]) + ")");
    return QEH_ERR_CHOLESKY;
  }
  if (hinfo[2] != 0) {
    set_error("tridiagonal eigensolver failed (status " + std::to_string(hinfo[2]) + ")");
    return QEH_ERR_NUMERIC;
  }
  return QEH_OK;
}

}  // extern "C"
