// Block Davidson eigensolver on one GPU.
//
// The paper names the Davidson method among the GPU-accelerated iterative
// solvers, runs the small dense generalized eigenproblem on a GPU dense
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
// the library's MFMA complex GEMMs in FP64; the dense Hermitian generalized
// eigensolve of the reduced pair uses rocSOLVER (the GPU counterpart of the
// dense solver library the paper uses for this step), with its workspace
// taken from the caller's work area so the library allocates nothing.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "qeh_internal.h"

namespace qeh {
qeh_status apply_h_impl(qeh_ctx *c, int part, int nb, const double *psi, int ldpsi,
                        double *hpsi, int ldh);
}

using namespace qeh;

namespace {

struct DavLayout {
  size_t V, W, P, Q, Hr, Sr, Hw, Sw, eps, E, norms, idx, info, flag, solver;
  size_t solver_bytes;
  size_t total;
};

size_t bump2(size_t *cur, size_t bytes) {
  const size_t o = *cur;
  *cur += (bytes + kAlign - 1) / kAlign * kAlign;
  return o;
}

qeh_status solver_bytes(int n, size_t *out) {
  rocblas_handle h;
  if (rocblas_create_handle(&h) != rocblas_status_success) {
    set_error("rocblas_create_handle failed");
    return QEH_ERR_DEVICE;
  }
  rocblas_start_device_memory_size_query(h);
  rocsolver_zhegvd(h, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_upper, n, nullptr,
                   n, nullptr, n, nullptr, nullptr, nullptr);
  size_t sz = 0;
  rocblas_stop_device_memory_size_query(h, &sz);
  rocblas_destroy_handle(h);
  *out = sz;
  return QEH_OK;
}

qeh_status dav_layout(const qeh_ctx *c, int nb, int nvecx, DavLayout *L) {
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
  L->eps = bump2(&cur, 8 * (size_t)nvecx);
  L->E = bump2(&cur, 8 * (size_t)nvecx);
  L->norms = bump2(&cur, 8 * (size_t)nb);
  L->idx = bump2(&cur, 4 * (size_t)nb);
  L->info = bump2(&cur, 4);
  L->flag = bump2(&cur, 4);
  qeh_status st = solver_bytes(nvecx, &L->solver_bytes);
  if (st != QEH_OK) return st;
  L->solver = bump2(&cur, std::max<size_t>(L->solver_bytes, 256));
  L->total = cur;
  return QEH_OK;
}

qeh_status check_opts(const qeh_ctx *c, int nb, const qeh_dav_opts *o, int *nvecx, double *rtol,
                      int *maxiter) {
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
  return QEH_OK;
}

// C[j][i] style reduction: out(i, j0+j) = sum_G conj(X_i[G]) Y_j[G],
// i < nrow, j < ncol; out col-major with ld.
hipError_t reduce_cols(const qeh_ctx *c, const double2 *X, int nrow, const double2 *Y, int ncol,
                       double2 *out, int ld) {
  GemmDesc g{};
  g.A = Y;
  g.lda = c->npw;
  g.ta = T_D2;
  g.B = X;
  g.ldb = c->npw;
  g.tb = T_D2;
  g.bmode = 0;
  g.conjB = 1;
  g.C = out;
  g.ldc = ld;
  g.tc = T_D2;
  g.M = ncol;
  g.N = nrow;
  g.K = c->npw;
  g.nsplit = 1;
  g.kchunk = c->npw;
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

// Device-time accumulator: event pairs are recorded around enqueued work and
// read back only after the host has synchronised the stream.
struct EvPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  double acc = 0.0;
  void start(hipStream_t s) {
    while (ev.size() < used + 2) {
      hipEvent_t x;
      if (hipEventCreate(&x) != hipSuccess) return;
      ev.push_back(x);
    }
    (void)hipEventRecord(ev[used], s);
  }
  void stop(hipStream_t s) {
    if (ev.size() < used + 2) return;
    (void)hipEventRecord(ev[used + 1], s);
    used += 2;
  }
  void harvest() {   // call after a stream synchronisation
    for (size_t i = 0; i + 1 < used; i += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) acc += ms * 1e-3;
    }
    used = 0;
  }
  void destroy() {
    for (auto x : ev) (void)hipEventDestroy(x);
    ev.clear();
  }
};

}  // namespace

extern "C" {

qeh_status qeh_davidson_plan(const qeh_ctx *c, int nb, const qeh_dav_opts *o,
                             size_t *work_bytes) {
  if (!work_bytes) {
    set_error("work_bytes is null");
    return QEH_ERR_INVALID;
  }
  int nvecx, maxiter;
  double rtol;
  qeh_status st = check_opts(c, nb, o, &nvecx, &rtol, &maxiter);
  if (st != QEH_OK) return st;
  DavLayout L;
  st = dav_layout(c, nb, nvecx, &L);
  if (st != QEH_OK) return st;
  *work_bytes = L.total;
  return QEH_OK;
}

qeh_status qeh_davidson(qeh_ctx *c, int nb, double *psi_inout, int ldpsi, double *eig,
                        const qeh_dav_opts *o, void *work, size_t work_bytes,
                        qeh_dav_info *info) {
  const auto t0 = std::chrono::steady_clock::now();
  int nvecx, maxiter;
  double rtol;
  qeh_status st = check_opts(c, nb, o, &nvecx, &rtol, &maxiter);
  if (st != QEH_OK) return st;
  if (!psi_inout || !eig || !work) {
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
  DavLayout L;
  st = dav_layout(c, nb, nvecx, &L);
  if (st != QEH_OK) return st;
  if (work_bytes < L.total) {
    set_error("work area has " + std::to_string(work_bytes) + " bytes, plan needs " +
              std::to_string(L.total));
    return QEH_ERR_NOMEM;
  }
  const bool mixed = c->prec == QEH_MIXED;
  const double thr = mixed ? std::max(rtol, 1e-5) : rtol;
  const int npw = c->npw;
  hipStream_t s = c->stream;
  char *w = reinterpret_cast<char *>(work);
  double2 *V = reinterpret_cast<double2 *>(w + L.V);
  double2 *W = reinterpret_cast<double2 *>(w + L.W);
  double2 *P = reinterpret_cast<double2 *>(w + L.P);
  double2 *Q = reinterpret_cast<double2 *>(w + L.Q);
  double2 *Hr = reinterpret_cast<double2 *>(w + L.Hr);
  double2 *Sr = reinterpret_cast<double2 *>(w + L.Sr);
  double2 *Hw = reinterpret_cast<double2 *>(w + L.Hw);
  double2 *Sw = reinterpret_cast<double2 *>(w + L.Sw);
  double *eps_d = reinterpret_cast<double *>(w + L.eps);
  double *E_d = reinterpret_cast<double *>(w + L.E);
  double *norms_d = reinterpret_cast<double *>(w + L.norms);
  int *idx_d = reinterpret_cast<int *>(w + L.idx);
  int *info_d = reinterpret_cast<int *>(w + L.info);
  int *flag_d = reinterpret_cast<int *>(w + L.flag);
  double2 *psi = reinterpret_cast<double2 *>(psi_inout);

  rocblas_handle rh = nullptr;
  if (rocblas_create_handle(&rh) != rocblas_status_success) {
    set_error("rocblas_create_handle failed");
    return QEH_ERR_DEVICE;
  }
  rocblas_set_stream(rh, s);
  if (rocblas_set_workspace(rh, w + L.solver, std::max<size_t>(L.solver_bytes, 256)) !=
      rocblas_status_success) {
    rocblas_destroy_handle(rh);
    set_error("rocblas_set_workspace failed");
    return QEH_ERR_DEVICE;
  }
  EvPool ev_h, ev_s;
  auto cleanup = [&]() {
    ev_h.destroy();
    ev_s.destroy();
    rocblas_destroy_handle(rh);
  };

  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  long band_applies = 0;
  auto hpsi = [&](const double2 *x, double2 *y, int n) -> qeh_status {
    ev_h.start(s);
    qeh_status r = apply_h_impl(c, 2, n, reinterpret_cast<const double *>(x), npw,
                                reinterpret_cast<double *>(y), npw);
    ev_h.stop(s);
    band_applies += n;
    return r;
  };

  // ---- start: finiteness of psi0, V = psi0, W = H V
  ok(hipMemsetAsync(flag_d, 0, 4, s));
  for (int b = 0; b < nb; ++b)
    ok(launch_check_finite(psi_inout + 2 * (size_t)b * ldpsi, 2 * (long)npw, flag_d, s));
  ok(launch_copy_rows(psi, ldpsi, V, npw, npw, nb, s));
  int hflag = 0;
  ok(hipMemcpyAsync(&hflag, flag_d, 4, hipMemcpyDeviceToHost, s));
  ok(hipStreamSynchronize(s));
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "davidson start");
  }
  if (hflag) {
    cleanup();
    set_error("psi0 has a non-finite value");
    return QEH_ERR_NUMERIC;
  }
  st = hpsi(V, W, nb);
  if (st != QEH_OK) {
    cleanup();
    return st;
  }
  ok(reduce_cols(c, V, nb, W, nb, Hr, nvecx));
  ok(reduce_cols(c, V, nb, V, nb, Sr, nvecx));
  int nbase = nb;

  std::vector<double> eps(nb), eps_prev(nb, INFINITY), nrm(nb);
  std::vector<int> idx(nb);
  int it = 0, restarts = 0, notconv = nb;
  bool chol_prev = false, have_ritz = false;
  double resid_max = INFINITY;
  qeh_status result = QEH_OK;
  while (true) {
    ++it;
    // ---- Rayleigh-Ritz on the reduced pair
    ev_s.start(s);
    ok(launch_hermitise_copy(Hr, nvecx, Hw, nvecx, nbase, s));
    ok(launch_hermitise_copy(Sr, nvecx, Sw, nvecx, nbase, s));
    rocblas_status rs = rocsolver_zhegvd(
        rh, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_upper, nbase,
        reinterpret_cast<rocblas_double_complex *>(Hw), nvecx,
        reinterpret_cast<rocblas_double_complex *>(Sw), nvecx, eps_d, E_d, info_d);
    if (rs != rocblas_status_success) {
      cleanup();
      set_error("rocsolver_zhegvd failed to launch");
      return QEH_ERR_DEVICE;
    }
    int hinfo = 0;
    ok(hipMemcpyAsync(&hinfo, info_d, 4, hipMemcpyDeviceToHost, s));
    ok(hipStreamSynchronize(s));
    if (e != hipSuccess) break;
    if (hinfo != 0) {
      ev_s.stop(s);
      // overlap matrix not positive definite (or no convergence of the solver)
      if (chol_prev || !have_ritz) {
        result = QEH_ERR_CHOLESKY;
        set_error("reduced overlap matrix not positive definite");
        break;
      }
      chol_prev = true;
      ++restarts;
      ok(launch_copy_rows(P, npw, V, npw, npw, nb, s));
      ok(launch_copy_rows(Q, npw, W, npw, npw, nb, s));
      nbase = nb;
      ok(reduce_cols(c, V, nb, W, nb, Hr, nvecx));
      ok(reduce_cols(c, V, nb, V, nb, Sr, nvecx));
      continue;
    }
    chol_prev = false;
    // ---- Ritz vectors, residual norms
    ok(rotate(c, Hw, nvecx, nbase, nb, V, P));
    ok(rotate(c, Hw, nvecx, nbase, nb, W, Q));
    ok(launch_resid_norms(P, Q, npw, npw, nb, eps_d, norms_d, s));
    ev_s.stop(s);
    have_ritz = true;
    ok(hipMemcpyAsync(eps.data(), eps_d, 8 * (size_t)nb, hipMemcpyDeviceToHost, s));
    ok(hipMemcpyAsync(nrm.data(), norms_d, 8 * (size_t)nb, hipMemcpyDeviceToHost, s));
    ok(hipStreamSynchronize(s));
    if (e != hipSuccess) break;
    ev_h.harvest();
    ev_s.harvest();
    int nc = 0;
    resid_max = 0.0;
    for (int b = 0; b < nb; ++b) {
      const double r = std::sqrt(std::max(nrm[b], 0.0));
      if (!std::isfinite(r)) {
        result = QEH_ERR_NUMERIC;
        set_error("non-finite residual");
      }
      resid_max = std::max(resid_max, r);
      bool conv = r <= thr;
      if (mixed && std::fabs(eps[b] - eps_prev[b]) <= 1e-8) conv = true;
      if (!conv) idx[nc++] = b;
    }
    eps_prev = eps;
    notconv = nc;
    if (result != QEH_OK) break;
    if (nc == 0) break;
    if (it >= maxiter) {
      result = QEH_ERR_NOT_CONVERGED;
      set_error("Davidson reached maxiter");
      break;
    }
    ok(hipMemcpyAsync(idx_d, idx.data(), 4 * (size_t)nc, hipMemcpyHostToDevice, s));
    if (nbase + nc > nvecx) {
      ++restarts;
      ok(launch_copy_rows(P, npw, V, npw, npw, nb, s));
      ok(launch_copy_rows(Q, npw, W, npw, npw, nb, s));
      ok(launch_set_diag(Hr, nvecx, nb, eps_d, s));
      ok(launch_set_diag(Sr, nvecx, nb, nullptr, s));
      nbase = nb;
    }
    ok(launch_precond(P, Q, npw, npw, idx_d, nc, eps_d, c->d.hdiag, V + (size_t)nbase * npw, npw,
                      s));
    st = hpsi(V + (size_t)nbase * npw, W + (size_t)nbase * npw, nc);
    if (st != QEH_OK) {
      result = st;
      break;
    }
    ev_s.start(s);
    ok(reduce_cols(c, V, nbase + nc, W + (size_t)nbase * npw, nc, Hr + (size_t)nbase * nvecx,
                   nvecx));
    ok(reduce_cols(c, V, nbase + nc, V + (size_t)nbase * npw, nc, Sr + (size_t)nbase * nvecx,
                   nvecx));
    ok(launch_herm_fill(Hr, nvecx, nbase, nbase + nc, s));
    ok(launch_herm_fill(Sr, nvecx, nbase, nbase + nc, s));
    ev_s.stop(s);
    nbase += nc;
    if (e != hipSuccess) break;
  }
  if (e == hipSuccess && have_ritz) {
    ok(launch_copy_rows(P, npw, psi, ldpsi, npw, nb, s));
    ok(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b) eig[b] = eps[b];
  }
  ev_h.harvest();
  ev_s.harvest();
  if (info) {
    info->iters = it;
    info->notconv = notconv;
    info->restarts = restarts;
    info->band_applies = band_applies;
    info->resid_max = resid_max;
    info->t_hpsi = ev_h.acc;
    info->t_subspace = ev_s.acc;
    info->t_total =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "davidson");
  return result;
}

}  // extern "C"
