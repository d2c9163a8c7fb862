// Projectors built on the device (the pseudopotential terms of the
// quantum-engine modules): validation of the radial-table description, the
// staging of its small inputs into a device workspace, and the C entry points
// qeh_beta_plan / qeh_beta_generate.  qeh_ctx_create calls the same staging
// when a cell comes without a host beta.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "qeh_internal.h"

namespace qeh {
namespace {

qeh_status bad(const std::string &m) {
  set_error(m);
  return QEH_ERR_INVALID;
}

size_t up256(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

void recip_rows(const double *a, double *b) {
  const double *a1 = a, *a2 = a + 3, *a3 = a + 6;
  auto cross = [](const double *u, const double *v, double *w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                     a[2] * (a[3] * a[7] - a[4] * a[6]);
  cross(a2, a3, b);
  cross(a3, a1, b + 3);
  cross(a1, a2, b + 6);
  for (int i = 0; i < 9; ++i) b[i] *= 2.0 * M_PI / det;
}

long total_channels(const qeh_projgen *p) {
  long n = 0;
  for (int s = 0; s < p->nsp; ++s) n += p->nchan[s];
  return n;
}

// q = k + G for every G, SoA [3][npw]
std::vector<double> qvectors(const qeh_cell *c) {
  double b[9];
  recip_rows(c->lattice, b);
  const size_t npw = c->npw;
  std::vector<double> q(3 * npw);
  for (size_t g = 0; g < npw; ++g) {
    const int *m = c->miller + 3 * g;
    for (int i = 0; i < 3; ++i)
      q[i * npw + g] = c->kpt[i] + m[0] * b[i] + m[1] * b[3 + i] + m[2] * b[6 + i];
  }
  return q;
}

}  // namespace

ProjgenLayout projgen_layout(const qeh_cell *c) {
  ProjgenLayout L{};
  const qeh_projgen *p = c->projgen;
  const long nch = total_channels(p);
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t o = cur;
    cur += up256(bytes);
    return o;
  };
  L.off_q = take(24 * (size_t)c->npw);
  L.off_atom = take(16 * (size_t)std::max(c->nat, 1));
  L.off_tau = take(24 * (size_t)std::max(c->nat, 1));
  L.off_chan0 = take(4 * (size_t)(p->nsp + 1));
  L.off_lchan = take(4 * (size_t)std::max(nch, 1L));
  L.off_tab = take(8 * (size_t)std::max(nch, 1L) * p->nq);
  L.total = cur;
  return L;
}

qeh_status projgen_validate(const qeh_cell *c) {
  const qeh_projgen *p = c->projgen;
  if (!p) return bad("projgen is null");
  if (c->nat < 1 || c->nat > 65535) return bad("projgen needs 1 <= nat <= 65535");
  if (!c->nproj) return bad("nproj is null");
  if (!p->tau || !p->ityp || !p->nchan || !p->tab) return bad("projgen array is null");
  if (p->nsp < 1) return bad("projgen nsp < 1");
  if (p->nq < 4) return bad("projgen nq < 4");
  if (!(p->dq > 0.0) || !std::isfinite(p->dq)) return bad("projgen dq must be finite and > 0");
  long nch = 0;
  for (int s = 0; s < p->nsp; ++s) {
    if (p->nchan[s] < 0 || p->nchan[s] > 64) return bad("projgen nchan must be in [0, 64]");
    nch += p->nchan[s];
  }
  if (nch > 0 && !p->lchan) return bad("projgen lchan is null");
  std::vector<int> per_sp(p->nsp, 0);
  {
    long cc = 0;
    for (int s = 0; s < p->nsp; ++s)
      for (int k = 0; k < p->nchan[s]; ++k, ++cc) {
        const int l = p->lchan[cc];
        if (l < 0 || l > 2) return bad("projgen l must be 0, 1 or 2");
        per_sp[s] += 2 * l + 1;
      }
  }
  for (int a = 0; a < c->nat; ++a) {
    const int s = p->ityp[a];
    if (s < 0 || s >= p->nsp) return bad("projgen ityp out of range at atom " + std::to_string(a));
    if (c->nproj[a] != per_sp[s])
      return bad("nproj[" + std::to_string(a) + "] does not match its species' channels");
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(p->tau[3 * a + i])) {
        set_error("projgen tau has a non-finite value");
        return QEH_ERR_NUMERIC;
      }
  }
  for (long i = 0; i < nch * (long)p->nq; ++i)
    if (!std::isfinite(p->tab[i])) {
      set_error("projgen tab has a non-finite value");
      return QEH_ERR_NUMERIC;
    }
  // every |k+G| inside the table's interpolation range
  const std::vector<double> q = qvectors(c);
  const size_t npw = c->npw;
  double qmax = 0.0;
  for (size_t g = 0; g < npw; ++g) {
    const double x = q[g], y = q[npw + g], z = q[2 * npw + g];
    qmax = std::max(qmax, std::sqrt(x * x + y * y + z * z));
  }
  if (qmax > (p->nq - 3) * p->dq)
    return bad("projgen table ends at " + std::to_string((p->nq - 3) * p->dq) +
               " bohr^-1 but the sphere reaches |k+G| = " + std::to_string(qmax));
  return QEH_OK;
}

qeh_status projgen_run(const qeh_cell *c, bool f64, void *out, long ldb, char *work,
                       hipStream_t s, const double2 *dmat_dev, double *hdiag_dev) {
  const qeh_projgen *p = c->projgen;
  const ProjgenLayout L = projgen_layout(c);
  const long nch = total_channels(p);
  const std::vector<double> q = qvectors(c);
  std::vector<int> chan0(p->nsp + 1, 0);
  for (int sp = 0; sp < p->nsp; ++sp) chan0[sp + 1] = chan0[sp] + p->nchan[sp];
  std::vector<int4> atoms(c->nat);
  {
    int row = 0, doff = 0;
    for (int a = 0; a < c->nat; ++a) {
      const int n = c->nproj[a];
      atoms[a] = make_int4(p->ityp[a], row, n, doff);
      row += n;
      doff += n * n;
    }
  }
  const double *A = c->lattice;
  const double omega =
      std::fabs(A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                A[2] * (A[3] * A[7] - A[4] * A[6]));
  const double pref = 4.0 * M_PI / std::sqrt(omega);
  hipError_t e = hipSuccess;
  auto up = [&](size_t off, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes)
      e = hipMemcpyAsync(work + off, src, bytes, hipMemcpyHostToDevice, s);
  };
  up(L.off_q, q.data(), 8 * q.size());
  up(L.off_atom, atoms.data(), sizeof(int4) * atoms.size());
  up(L.off_tau, p->tau, 24 * (size_t)c->nat);
  up(L.off_chan0, chan0.data(), 4 * chan0.size());
  if (nch > 0) {
    up(L.off_lchan, p->lchan, 4 * (size_t)nch);
    up(L.off_tab, p->tab, 8 * (size_t)nch * p->nq);
  }
  const int4 *atoms_d = reinterpret_cast<const int4 *>(work + L.off_atom);
  if (e == hipSuccess)
    e = launch_beta_gen(f64, reinterpret_cast<const double *>(work + L.off_q), c->npw, c->nat,
                        atoms_d, reinterpret_cast<const double *>(work + L.off_tau),
                        reinterpret_cast<const int *>(work + L.off_chan0),
                        reinterpret_cast<const int *>(work + L.off_lchan),
                        reinterpret_cast<const double *>(work + L.off_tab), p->nq, p->dq, pref,
                        out, ldb, s);
  if (e == hipSuccess && hdiag_dev)
    e = launch_nl_diag(f64, out, ldb, c->npw, c->nat, atoms_d, dmat_dev, hdiag_dev, s);
  // the staging vectors are host locals: wait before they go
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "projector generation");
  return QEH_OK;
}

}  // namespace qeh

using namespace qeh;

namespace {

qeh_status check_sphere(const qeh_cell *c) {
  if (!c) return bad("cell is null");
  if (c->npw < 1 || !c->miller) return bad("npw must be >= 1 with a Miller list");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(c->lattice[i])) return bad("lattice not finite");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(c->kpt[i])) return bad("kpt not finite");
  return projgen_validate(c);
}

}  // namespace

extern "C" {

qeh_status qeh_beta_plan(const qeh_cell *cell, size_t *work_bytes) {
  if (!work_bytes) return bad("work_bytes is null");
  const qeh_status st = check_sphere(cell);
  if (st != QEH_OK) return st;
  *work_bytes = projgen_layout(cell).total;
  return QEH_OK;
}

qeh_status qeh_beta_generate(const qeh_cell *cell, int precision, void *beta, long ldb,
                             void *work, size_t work_bytes, void *hip_stream) {
  const qeh_status st = check_sphere(cell);
  if (st != QEH_OK) return st;
  if (precision != QEH_FP64 && precision != QEH_MIXED)
    return bad("precision must be QEH_FP64 or QEH_MIXED");
  if (!beta) return bad("beta is null");
  if (ldb < cell->npw) return bad("ldb < npw");
  if (!work || reinterpret_cast<uintptr_t>(work) % kAlign)
    return bad("work must be a 256-byte aligned device pointer");
  const size_t need = projgen_layout(cell).total;
  if (work_bytes < need)
    return bad("work has " + std::to_string(work_bytes) + " bytes, plan needs " +
               std::to_string(need));
  return projgen_run(cell, precision == QEH_FP64, beta, ldb, static_cast<char *>(work),
                     reinterpret_cast<hipStream_t>(hip_stream), nullptr, nullptr);
}

qeh_status qeh_beta_generate_static(const qeh_cell *cell, int precision, void *beta, long ldb,
                                    void *hip_stream) {
  const qeh_status st = check_sphere(cell);
  if (st != QEH_OK) return st;
  if (precision != QEH_FP64 && precision != QEH_MIXED)
    return bad("precision must be QEH_FP64 or QEH_MIXED");
  if (!beta) return bad("beta is null");
  if (ldb < cell->npw) return bad("ldb < npw");
  const size_t need = projgen_layout(cell).total;
  if (need > (size_t)QEH_BETA_STATIC_BYTES) {
    set_error("qeh_beta_generate_static: the generator inputs need " + std::to_string(need) +
              " bytes of staging, the static array holds " +
              std::to_string((size_t)QEH_BETA_STATIC_BYTES) + " (use qeh_beta_generate)");
    return QEH_ERR_NOMEM;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char *work = nullptr;
  const hipError_t e = beta_static_scratch(s, &work);
  if (e != hipSuccess) return hip_fail(e, "static staging array address");
  // every staged field is written before the generator reads it: nothing in
  // the array needs clearing between calls
  return projgen_run(cell, precision == QEH_FP64, beta, ldb, work, s, nullptr, nullptr);
}

}  // extern "C"
