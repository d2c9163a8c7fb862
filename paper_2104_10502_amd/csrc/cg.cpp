// Band-by-band preconditioned conjugate-gradient eigensolver: the paper's
// other iterative solver of the Kohn-Sham problem beside Davidson (section
// "Evolution of the GPU-enabled version").  The paper gives no algorithm; this
// is the textbook form, step for step that of the FP64 oracle:
//   1. X = psi0, HX = H X, Rayleigh-Ritz on the block (orthonormal, ordered);
//   2. for band m = 0, 1, ...: x = X_m orthogonalised against the bands below
//      and normalised, hx = H x, lam = <x|hx>; then repeat
//        r = hx - lam x (stop when ||r|| <= thr or at maxiter),
//        g = P(lam) r (the Davidson preconditioner), g kept orthogonal to the
//        bands below and to x,
//        d = g + beta d (Polak-Ribiere, restarted when negative), d kept
//        orthogonal to x, dn = d / ||d||, hd = H dn,
//        the lower eigenpair of the 2 x 2 problem over (x, dn): x, hx, lam
//        rotated (the Rayleigh quotient never rises);
//   3. a final Rayleigh-Ritz of the block.
// H is applied one band at a time through the context's H|psi> path; the
// vector work runs on the CG kernels, the reductions in fixed orders, and the
// host waits once per iteration (for ||r||).  The block Rayleigh-Ritz steps
// use the library's own subspace solver, so nb <= 512.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <string>
#include <utility>
#include <vector>

#include "davidson.h"
#include "qeh_internal.h"

namespace qeh {
qeh_status apply_h_impl(qeh_ctx *c, int part, int nb, const double *psi, int ldpsi,
                        double *hpsi, int ldh);

namespace {

size_t bump_cg(size_t *cur, size_t bytes) {
  const size_t o = *cur;
  *cur += (bytes + kAlign - 1) / kAlign * kAlign;
  return o;
}

struct CgLayout {
  size_t X, HX, Xr, HXr, r, g, gp, d, dn, hd, coef, part, Hr, Sr, Y, eig, norms, sc, dotp, flag,
      eigw, eigw_bytes, total;
};

qeh_status cg_check(const qeh_ctx *c, int nb) {
  if (!c) {
    set_error("ctx is null");
    return QEH_ERR_INVALID;
  }
  if (nb < 1 || nb > kEigMaxN) {
    set_error("CG: need 1 <= nb <= " + std::to_string(kEigMaxN));
    return QEH_ERR_INVALID;
  }
  if (nb > c->npw) {
    set_error("CG: nb > npw");
    return QEH_ERR_INVALID;
  }
  if (c->has_q) {
    set_error("CG solves the standard problem: the context has an overlap operator (q blocks)");
    return QEH_ERR_INVALID;
  }
  return QEH_OK;
}

qeh_status cg_layout(const qeh_ctx *c, int nb, CgLayout *L) {
  size_t cur = 0;
  const size_t vec = 16 * (size_t)c->npw;
  const size_t blk = vec * nb;
  L->X = bump_cg(&cur, blk);
  L->HX = bump_cg(&cur, blk);
  L->Xr = bump_cg(&cur, blk);
  L->HXr = bump_cg(&cur, blk);
  L->r = bump_cg(&cur, vec);
  L->g = bump_cg(&cur, vec);
  L->gp = bump_cg(&cur, vec);
  L->d = bump_cg(&cur, vec);
  L->dn = bump_cg(&cur, vec);
  L->hd = bump_cg(&cur, vec);
  L->coef = bump_cg(&cur, 16 * (size_t)nb);
  L->part = bump_cg(&cur, 16 * (size_t)kReduceMaxSplit * nb * nb);
  L->Hr = bump_cg(&cur, 16 * (size_t)nb * nb);
  L->Sr = bump_cg(&cur, 16 * (size_t)nb * nb);
  L->Y = bump_cg(&cur, 16 * (size_t)nb * nb);
  L->eig = bump_cg(&cur, 8 * (size_t)nb);
  L->norms = bump_cg(&cur, 8 * (size_t)nb);
  L->sc = bump_cg(&cur, 8 * (size_t)kCgSlots);
  L->dotp = bump_cg(&cur, 16 * (size_t)kCgDotBlocks * kCgMaxDots);
  L->flag = bump_cg(&cur, 16);
  size_t eb = 0;
  qeh_status st = qeh_subspace_plan(nb, nb, &eb);
  if (st != QEH_OK) return st;
  L->eigw = bump_cg(&cur, eb);
  L->eigw_bytes = eb;
  L->total = cur;
  return QEH_OK;
}

// One run of the solver over caller-provided work memory.
class CgRun {
 public:
  CgRun(qeh_ctx *c, int nb, char *w, const CgLayout &L) : c_(c), nb_(nb), L_(L), w_(w) {
    s_ = c->stream;
    npw_ = c->npw;
  }
  ~CgRun() {
    // an early error return can leave work enqueued that reads the pinned
    // buffer or records the events
    (void)hipStreamSynchronize(s_);
    ev_h_.destroy();
    ev_s_.destroy();
    if (h_) (void)hipHostFree(h_);
  }

  qeh_status run(double2 *psi, int ldpsi, double *eig, double thr, int maxiter,
                 qeh_dav_info *info);

 private:
  template <typename T> T *at(size_t off) { return reinterpret_cast<T *>(w_ + off); }
  void ok(hipError_t e) {
    if (err_ == hipSuccess) err_ = e;
  }
  qeh_status hpsi(const double2 *x, double2 *y, int n) {
    applies_ += n;
    ev_h_.start(s_);
    qeh_status st = apply_h_impl(c_, 2, n, reinterpret_cast<const double *>(x), npw_,
                                 reinterpret_cast<double *>(y), npw_);
    ev_h_.stop(s_);
    return st;
  }
  void dots(std::initializer_list<std::pair<std::pair<const double2 *, const double2 *>, int>> l) {
    CgDots p{};
    int n = 0;
    for (const auto &e : l) {
      p.a[n] = e.first.first;
      p.b[n] = e.first.second;
      p.dst[n] = e.second;
      ++n;
    }
    ok(launch_cg_dots(p, n, npw_, c_->gamma, at<double>(L_.dotp), at<double>(L_.sc), s_));
  }
  // Rayleigh-Ritz of the block (X, HX) into (Xr, HXr) and eigenvalues on the
  // device; returns the subspace solver's status
  qeh_status block_rr();
  qeh_status read_scalar(int slot, double *v) {
    ok(hipMemcpyAsync(h_, at<double>(L_.sc) + slot, 8, hipMemcpyDeviceToHost, s_));
    ok(hipStreamSynchronize(s_));
    if (err_ != hipSuccess) return hip_fail(err_, "CG");
    *v = h_[0];
    return QEH_OK;
  }

  qeh_ctx *c_;
  int nb_, npw_ = 0;
  const CgLayout &L_;
  char *w_;
  hipStream_t s_;
  hipError_t err_ = hipSuccess;
  double *h_ = nullptr;
  long applies_ = 0;
  EvPool ev_h_, ev_s_;   // device time of H and of the block Rayleigh-Ritz steps
};

qeh_status CgRun::block_rr() {
  double2 *X = at<double2>(L_.X), *HX = at<double2>(L_.HX);
  ev_s_.start(s_);
  ok(reduce_cols(c_, X, nb_, HX, nb_, at<double2>(L_.Hr), nb_, at<double2>(L_.part)));
  ok(reduce_cols(c_, X, nb_, X, nb_, at<double2>(L_.Sr), nb_, at<double2>(L_.part)));
  if (err_ != hipSuccess) return hip_fail(err_, "CG Rayleigh-Ritz products");
  qeh_status st = qeh_subspace_eigh(nb_, nb_, at<double>(L_.Hr), at<double>(L_.Sr), nb_,
                                    at<double>(L_.eig), at<double>(L_.Y), nb_, w_ + L_.eigw,
                                    L_.eigw_bytes, s_);
  if (st != QEH_OK) return st;
  ok(rotate(c_, at<double2>(L_.Y), nb_, nb_, nb_, X, at<double2>(L_.Xr)));
  ok(rotate(c_, at<double2>(L_.Y), nb_, nb_, nb_, HX, at<double2>(L_.HXr)));
  ev_s_.stop(s_);
  return err_ == hipSuccess ? QEH_OK : hip_fail(err_, "CG rotation");
}

qeh_status CgRun::run(double2 *psi, int ldpsi, double *eig, double thr, int maxiter,
                      qeh_dav_info *info) {
  const auto t0 = std::chrono::steady_clock::now();
  void *hp = nullptr;
  const hipError_t he = hipHostMalloc(&hp, 64, hipHostMallocDefault);
  if (he != hipSuccess) return hip_fail(he, "pinned buffer");
  h_ = static_cast<double *>(hp);
  const int nb = nb_, npw = npw_;
  double2 *X = at<double2>(L_.X), *HX = at<double2>(L_.HX);
  double2 *r = at<double2>(L_.r), *g = at<double2>(L_.g), *gp = at<double2>(L_.gp);
  double2 *d = at<double2>(L_.d), *dn = at<double2>(L_.dn), *hd = at<double2>(L_.hd);
  double2 *coef = at<double2>(L_.coef);
  double *sc = at<double>(L_.sc);
  int *flag = at<int>(L_.flag);

  // input: finite, psi(G = 0) real on Gamma contexts
  ok(launch_fill_int(flag, 1, 0, s_));
  for (int b = 0; b < nb; ++b)
    ok(launch_check_finite(reinterpret_cast<const double *>(psi + (size_t)b * ldpsi),
                           2 * (long)npw, flag, s_));
  int hflag = 0;
  ok(hipMemcpyAsync(h_, flag, 4, hipMemcpyDeviceToHost, s_));
  ok(hipStreamSynchronize(s_));
  if (err_ != hipSuccess) return hip_fail(err_, "CG input check");
  std::memcpy(&hflag, h_, 4);
  if (hflag) {
    set_error("psi0 has a non-finite value");
    return QEH_ERR_NUMERIC;
  }
  ok(launch_copy_rows(psi, ldpsi, X, npw, npw, nb, s_));
  if (c_->gamma) ok(launch_zero_g0_imag(X, npw, nb, s_));
  qeh_status st = hpsi(X, HX, nb);
  if (st != QEH_OK) return st;
  st = block_rr();
  if (st != QEH_OK) return st;
  ok(launch_copy_rows(at<double2>(L_.Xr), npw, X, npw, npw, nb, s_));
  ok(launch_copy_rows(at<double2>(L_.HXr), npw, HX, npw, npw, nb, s_));

  long iters = 0;
  int notconv = 0;
  for (int m = 0; m < nb; ++m) {
    double2 *x = X + (size_t)m * npw, *hx = HX + (size_t)m * npw;
    if (m > 0) {
      ok(reduce_cols(c_, X, m, x, 1, coef, nb, at<double2>(L_.part)));
      ok(launch_cg_project(x, X, npw, coef, m, npw, s_));
    }
    dots({{{x, x}, kCgXX}});
    ok(launch_cg_scalar(sc, 0, s_));
    ok(launch_cg_scale(x, sc, npw, s_));
    st = hpsi(x, hx, 1);
    if (st != QEH_OK) return st;
    dots({{{x, hx}, kCgLam}});
    int it = 0;
    double rr = 0.0;
    while (true) {
      ok(launch_cg_resid(x, hx, c_->d.hdiag, sc, r, g, npw, c_->gamma, s_));
      if (it > 0)
        dots({{{r, r}, kCgRR}, {{gp, r}, kCgGpr}});
      else
        dots({{{r, r}, kCgRR}});
      st = read_scalar(kCgRR, &rr);
      if (st != QEH_OK) return st;
      const double rn = std::sqrt(std::max(rr, 0.0));
      if (!std::isfinite(rn)) {
        set_error("CG: non-finite residual");
        return QEH_ERR_NUMERIC;
      }
      if (rn <= thr || it >= maxiter) {
        if (rn > thr) ++notconv;
        break;
      }
      ++it;
      ok(reduce_cols(c_, X, m + 1, g, 1, coef, nb, at<double2>(L_.part)));
      ok(launch_cg_project(g, X, npw, coef, m + 1, npw, s_));
      dots({{{g, r}, kCgGam}});
      ok(launch_cg_scalar(sc, 1, s_));
      ok(launch_cg_dir(g, d, gp, sc, npw, s_));
      dots({{{x, d}, kCgXD}, {{d, d}, kCgDD}});
      ok(launch_cg_scalar(sc, 2, s_));
      ok(launch_cg_dnorm(d, x, dn, sc, npw, s_));
      st = hpsi(dn, hd, 1);
      if (st != QEH_OK) return st;
      dots({{{x, hd}, kCgB}, {{dn, hd}, kCgC}});
      ok(launch_cg_scalar(sc, 3, s_));
      ok(launch_cg_update(x, hx, dn, hd, sc, npw, s_));
    }
    iters += it;
  }

  // final Rayleigh-Ritz: ordered eigenpairs of the block
  st = block_rr();
  if (st != QEH_OK) return st;
  double *eig_d = at<double>(L_.eig), *norms = at<double>(L_.norms);
  ok(launch_resid_norms(at<double2>(L_.Xr), at<double2>(L_.HXr), npw, npw, nb, eig_d, norms,
                        c_->gamma, s_));
  ok(launch_copy_rows(at<double2>(L_.Xr), npw, psi, ldpsi, npw, nb, s_));
  std::vector<double> hn(nb);
  ok(hipMemcpyAsync(eig, eig_d, 8 * (size_t)nb, hipMemcpyDeviceToHost, s_));
  ok(hipMemcpyAsync(hn.data(), norms, 8 * (size_t)nb, hipMemcpyDeviceToHost, s_));
  ok(hipStreamSynchronize(s_));
  if (err_ != hipSuccess) return hip_fail(err_, "CG results");
  ev_h_.harvest();
  ev_s_.harvest();
  double rmax = 0.0;
  for (int b = 0; b < nb; ++b) rmax = std::max(rmax, std::sqrt(std::max(hn[b], 0.0)));
  if (info) {
    info->iters = (int)iters;
    info->notconv = notconv;
    info->restarts = 0;
    info->band_applies = applies_;
    info->resid_max = rmax;
    info->t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->t_hpsi = ev_h_.acc;
    info->t_subspace = ev_s_.acc;
    info->refine_iters = 0;
  }
  if (notconv > 0) {
    set_error("CG: " + std::to_string(notconv) + " band(s) reached maxiter");
    return QEH_ERR_NOT_CONVERGED;
  }
  return QEH_OK;
}

}  // namespace
}  // namespace qeh

using namespace qeh;

extern "C" {

qeh_status qeh_cg_plan(const qeh_ctx *c, int nb, size_t *work_bytes) {
  if (!work_bytes) {
    set_error("work_bytes is null");
    return QEH_ERR_INVALID;
  }
  qeh_status st = cg_check(c, nb);
  if (st != QEH_OK) return st;
  CgLayout L;
  st = cg_layout(c, nb, &L);
  if (st != QEH_OK) return st;
  *work_bytes = L.total;
  return QEH_OK;
}

qeh_status qeh_cg(qeh_ctx *c, int nb, double *psi_inout, int ldpsi, double *eig,
                  const qeh_cg_opts *o, void *work, size_t work_bytes, qeh_dav_info *info) {
  qeh_status st = cg_check(c, nb);
  if (st != QEH_OK) return st;
  if (!psi_inout || !eig || !work) {
    set_error("psi_inout, eig and work must be non-null");
    return QEH_ERR_INVALID;
  }
  if (ldpsi < c->npw) {
    set_error("ldpsi < npw");
    return QEH_ERR_INVALID;
  }
  double rtol = o ? o->rtol : 0.0;
  int maxiter = o ? o->maxiter : 0;
  if (!(rtol >= 0.0) || maxiter < 0) {
    set_error("CG: rtol must be >= 0 and maxiter >= 0");
    return QEH_ERR_INVALID;
  }
  if (rtol == 0.0) rtol = 1e-8;
  if (maxiter == 0) maxiter = 100;
  const double thr = c->prec == QEH_MIXED ? std::max(rtol, 1e-5) : rtol;
  CgLayout L;
  st = cg_layout(c, nb, &L);
  if (st != QEH_OK) return st;
  if (reinterpret_cast<uintptr_t>(work) % kAlign) {
    set_error("work not 256-byte aligned");
    return QEH_ERR_INVALID;
  }
  if (work_bytes < L.total) {
    set_error("work area has " + std::to_string(work_bytes) + " bytes, plan needs " +
              std::to_string(L.total));
    return QEH_ERR_NOMEM;
  }
  CgRun run(c, nb, static_cast<char *>(work), L);
  return run.run(reinterpret_cast<double2 *>(psi_inout), ldpsi, eig, thr, maxiter, info);
}

}  // extern "C"
