// Resumable block-Davidson run (internal).  advance() enqueues device work on
// the context stream up to the next point where the host needs device
// results, and returns false; after the stream has drained the caller calls
// advance() again.  It returns true once the run is finished.  The blocking
// qeh_davidson(), the request server and the reverse-communication handle all
// drive this one state machine.  In reverse-communication mode every H
// application becomes a request (take_request) that the caller serves before
// the next advance(); the work enqueued before and after it is the same as
// when the run applies H itself.
#pragma once

#include <rocblas/rocblas.h>

#include <chrono>
#include <vector>

#include "qeh_internal.h"

namespace qeh {

struct DavLayout {
  size_t V, W, P, Q, Hr, Sr, Hw, Sw, X, Lc, LcH, Y, part, eps, E, norms, idx, info, flag,
      solver, tri, Zt, escr, U, SP;
  size_t solver_bytes;
  bool own;   // the library's own subspace solver (else rocSOLVER)
  size_t total;
};

// Device-time accumulator: event pairs recorded around enqueued work, read
// back only after the host has seen the stream drain.
struct EvPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  double acc = 0.0;
  void start(hipStream_t s);
  void stop(hipStream_t s);
  void harvest();
  void destroy();
};

qeh_status dav_check_opts(const qeh_ctx *c, int nb, const qeh_dav_opts *o, int *nvecx,
                          double *rtol, int *maxiter, bool *own);
qeh_status dav_layout(const qeh_ctx *c, int nb, int nvecx, bool own, DavLayout *L);

class DavRun {
 public:
  // Validates and binds; nothing is enqueued yet.  eig is a host array of nb.
  qeh_status init(qeh_ctx *c, int nb, double2 *psi, int ldpsi, double *eig,
                  const qeh_dav_opts *o, void *work, size_t work_bytes);
  bool advance();
  // reverse communication: H is applied by the caller (set before the first
  // advance); after advance() returns false, take_request reports whether it
  // stopped for an H application rather than for a stream drain
  void set_rci() { rci_ = true; }
  // own subspace solver on one workgroup per step (least device time: for
  // runs that share the device, as the request server's jobs do)
  void set_narrow_solver() { wide_ = false; }
  bool take_request(const double2 **x, double2 **y, int *n);
  qeh_status result() const { return result_; }
  void fill_info(qeh_dav_info *info) const;
  void release();
  ~DavRun() { release(); }

 private:
  enum Phase {
    kStart,
    kCheckInput,
    kCheckInputPost,   // after H V of the starting block
    kRR,
    kRRSolve,
    kRRCheck,
    kConverge,
    kConvergePost,     // after H of the new correction vectors
    kFinish,
    kDone
  };
  void rr_own();   // enqueue the whole Rayleigh-Ritz solve on the own kernels
  void restart_from_ritz();   // V = P, W = H P, reduced matrices rebuilt
  qeh_status hpsi(const double2 *x, double2 *y, int n);
  qeh_status spsi(const double2 *x, double2 *y, int n);   // S x (generalized problem)
  void ok(hipError_t e) {
    if (err_ == hipSuccess) err_ = e;
  }
  bool fail_device(const char *what);

  qeh_ctx *c_ = nullptr;
  int nb_ = 0, ldpsi_ = 0, nvecx_ = 0, maxiter_ = 0, npw_ = 0;
  double thr_ = 0.0;
  bool mixed_ = false;
  double2 *psi_ = nullptr;
  double *eig_ = nullptr;
  DavLayout L_{};
  double2 *V_ = nullptr, *W_ = nullptr, *P_ = nullptr, *Q_ = nullptr;
  double2 *Hr_ = nullptr, *Sr_ = nullptr, *Hw_ = nullptr, *Sw_ = nullptr, *part_ = nullptr;
  double2 *X_ = nullptr, *Lc_ = nullptr, *LcH_ = nullptr, *Y_ = nullptr;
  double *tri_ = nullptr, *Zt_ = nullptr, *escr_ = nullptr;   // own subspace solver
  bool own_ = false;
  bool wide_ = true;   // own solver's steps over many workgroups
  double2 *U_ = nullptr, *SP_ = nullptr;   // S V and S P (overlap S != 1)
  bool gen_ = false;                       // generalized problem H psi = eps S psi
  qeh_ctx *c64_ = nullptr;   // mixed form: FP64 context of the refinement phase
  bool phase64_ = false;     // H applied through c64_
  int it64_ = 0;             // iterations of the refinement phase
  double *eps_d_ = nullptr, *E_d_ = nullptr, *norms_d_ = nullptr;
  int *idx_d_ = nullptr, *info_d_ = nullptr, *flag_d_ = nullptr;
  // pinned host mirrors of the per-iteration readback
  double *h_eps_ = nullptr, *h_nrm_ = nullptr;
  int *h_idx_ = nullptr, *h_int_ = nullptr;   // [0] flag, [1..3] potrf/trtri/heevd info
  std::vector<double> eps_prev_, best_res_;
  std::vector<int> stall_;
  rocblas_handle rh_ = nullptr;
  EvPool ev_h_, ev_s_;
  Phase phase_ = kStart;
  int it_ = 0, restarts_ = 0, notconv_ = 0, nbase_ = 0, nc_ = 0;
  bool rci_ = false, pending_ = false;   // reverse communication
  const double2 *req_x_ = nullptr;
  double2 *req_y_ = nullptr;
  int req_n_ = 0;
  bool chol_prev_ = false, have_ritz_ = false;
  double resid_max_ = 0.0;
  long band_applies_ = 0;
  qeh_status result_ = QEH_OK;
  hipError_t err_ = hipSuccess;
  std::chrono::steady_clock::time_point t0_;
  double t_total_ = 0.0;
};

}  // namespace qeh
