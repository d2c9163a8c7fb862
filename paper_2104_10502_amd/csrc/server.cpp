// Request server: continuous batching of block-Davidson solves on one GPU.
//
// The paper expects throughput from many independent calculations and notes
// that several small runs sharing one GPU pay off (sections "Outlook and
// conclusions" and "Evolution of the GPU-enabled version").  Design:
//
// * qeh_submit (any thread) deep-copies the request, plans its footprint
//   (context arena + Davidson work + psi per k-point) and queues it.
// * One server thread admits queued requests first-come first-served as soon
//   as the free arena (first-fit over an offset free list) and nk free slots
//   allow; a request that fits may pass a head request that has waited less
//   than kBackfillWindow seconds.
// * Every admitted k-point (job) owns a slot = a HIP stream and a worker
//   thread that drives its DavRun state machine (advance() enqueues work up
//   to the next host decision, then the worker waits for its own stream).
//   Jobs therefore never wait on each other's host-side synchronisation (the
//   dense eigensolver synchronises its calling thread), and the device
//   interleaves the kernels of every running request.
// * Finished jobs release their arena range and slot immediately.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "davidson.h"

namespace qeh {
namespace {

constexpr double kBackfillWindow = 0.25;
constexpr int kMaxSlots = 64;

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Host copy of one k-point's cell.
struct HostCell {
  qeh_cell cell{};
  std::vector<int> miller, nproj;
  std::vector<double> vloc, beta, dmat, qmat, psi0;
  // radial-table description when beta is built on the device
  bool has_pg = false;
  qeh_projgen pg{};
  std::vector<double> tau, tab;
  std::vector<int> ityp, nchan, lchan;
  void bind() {
    cell.miller = miller.data();
    cell.vloc = vloc.data();
    cell.nproj = nproj.empty() ? nullptr : nproj.data();
    cell.beta = beta.empty() ? nullptr : beta.data();
    cell.dmat = dmat.empty() ? nullptr : dmat.data();
    cell.qmat = qmat.empty() ? nullptr : qmat.data();
    if (has_pg) {
      pg.tau = tau.data();
      pg.ityp = ityp.data();
      pg.nchan = nchan.data();
      pg.lchan = lchan.empty() ? nullptr : lchan.data();
      pg.tab = tab.data();
      cell.projgen = &pg;
    } else {
      cell.projgen = nullptr;
    }
  }
};

struct Request;

struct Job {
  Request *req = nullptr;
  int k = 0;
  HostCell hc;
  size_t ctx_bytes = 0, ctx64_bytes = 0, dav_bytes = 0, psi_bytes = 0, total = 0;
  size_t off = 0;
  int slot = -1;
  qeh_ctx *ctx = nullptr;
  qeh_ctx *ctx64 = nullptr;   // mixed-form requests: FP64 context of the refinement phase
  qeh_dav_opts opts{};
  std::unique_ptr<DavRun> run;
  bool started = false, finished = false, reaped = false;
  std::thread th;
  std::vector<double> eig;
  qeh_dav_info info{};
  qeh_status st = QEH_OK;
};

struct Request {
  uint64_t id = 0;
  int nk = 0, nb = 0;
  qeh_dav_opts opts{};
  std::vector<std::unique_ptr<Job>> jobs;
  size_t footprint = 0;
  double t[4] = {0, 0, 0, 0};   // arrive, admit, start, finish
  int remaining = 0;
  bool admitted = false, done = false, cancelled = false;
  qeh_status st = QEH_OK;
  std::string msg;   // error text of the first failing job
};

}  // namespace
}  // namespace qeh

struct qeh_server {
  char *arena = nullptr;
  size_t arena_bytes = 0;
  int max_slots = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<int> slot_free;
  std::chrono::steady_clock::time_point t0;
  // free list of the arena: offset -> length
  std::map<size_t, size_t> free_ranges;
  size_t in_use = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<qeh::Request *> queue;                       // submitted, not admitted
  std::map<uint64_t, std::unique_ptr<qeh::Request>> all;  // every live request
  std::vector<qeh::Job *> running;                        // admitted, not reaped
  uint64_t next_id = 1;
  bool stop = false;
  long finished = 0;
  int peak_running = 0;
  double busy_s = 0.0;
  std::thread th;
};

namespace qeh {
namespace {

bool alloc_range(qeh_server *s, size_t n, size_t *off) {
  for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it) {
    if (it->second >= n) {
      *off = it->first;
      const size_t rest = it->second - n;
      const size_t o2 = it->first + n;
      s->free_ranges.erase(it);
      if (rest) s->free_ranges[o2] = rest;
      s->in_use += n;
      return true;
    }
  }
  return false;
}

void free_range(qeh_server *s, size_t off, size_t n) {
  s->in_use -= n;
  auto it = s->free_ranges.emplace(off, n).first;
  // merge with the next range
  auto nx = std::next(it);
  if (nx != s->free_ranges.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    s->free_ranges.erase(nx);
  }
  // merge with the previous range
  if (it != s->free_ranges.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      s->free_ranges.erase(it);
    }
  }
}

// Try to place every job of r; all or nothing.
bool try_admit(qeh_server *s, Request *r) {
  int free_slots = 0;
  for (int f : s->slot_free) free_slots += f;
  if (free_slots < r->nk) return false;
  std::vector<size_t> offs;
  for (auto &j : r->jobs) {
    size_t off;
    if (!alloc_range(s, j->total, &off)) {
      for (size_t i = 0; i < offs.size(); ++i) free_range(s, offs[i], r->jobs[i]->total);
      return false;
    }
    offs.push_back(off);
  }
  for (size_t i = 0; i < r->jobs.size(); ++i) {
    Job *j = r->jobs[i].get();
    j->off = offs[i];
    for (int sl = 0; sl < s->max_slots; ++sl)
      if (s->slot_free[sl]) {
        s->slot_free[sl] = 0;
        j->slot = sl;
        break;
      }
  }
  r->admitted = true;
  r->t[1] = now_s(s->t0);
  return true;
}

// Set up a job on its stream: context, psi0 upload, Davidson init.
// Returns false (status in j->st) on failure.
bool start_job(qeh_server *s, Job *j) {
  hipStream_t st = s->streams[j->slot];
  char *base = s->arena + j->off;
  j->started = true;
  j->hc.bind();
  qeh_status rc = qeh_ctx_create(&j->hc.cell, base, j->ctx_bytes, st, &j->ctx);
  if (rc != QEH_OK) {
    j->st = rc;
    return false;
  }
  j->opts = j->req->opts;
  j->opts.refine = nullptr;
  if (j->ctx64_bytes) {
    qeh_cell c64 = j->hc.cell;
    c64.precision = QEH_FP64;
    rc = qeh_ctx_create(&c64, base + j->ctx_bytes, j->ctx64_bytes, st, &j->ctx64);
    if (rc != QEH_OK) {
      j->st = rc;
      return false;
    }
    j->opts.refine = j->ctx64;
  }
  char *after = base + j->ctx_bytes + j->ctx64_bytes;
  double2 *psi = reinterpret_cast<double2 *>(after);
  // exactly the host copy's bytes (psi_bytes is that size rounded up to the
  // arena alignment; reading that far would run past the end of the vector)
  hipError_t e = hipMemcpyAsync(psi, j->hc.psi0.data(), sizeof(double) * j->hc.psi0.size(),
                                hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    j->st = hip_fail(e, "psi0 upload");
    return false;
  }
  j->eig.assign(j->req->nb, 0.0);
  j->run.reset(new DavRun());
  // served jobs share the device: the subspace solver's least-device-time form
  j->run->set_narrow_solver();
  rc = j->run->init(j->ctx, j->req->nb, psi, j->hc.cell.npw, j->eig.data(), &j->opts,
                    after + j->psi_bytes, j->dav_bytes);
  if (rc != QEH_OK) {
    j->st = rc;
    return false;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (j->req->t[2] == 0.0) j->req->t[2] = now_s(s->t0);
  return true;
}

void finish_job(qeh_server *s, Job *j) {
  // make sure nothing of this job is still in flight before its range is reused
  if (j->slot >= 0) (void)hipStreamSynchronize(s->streams[j->slot]);
  if (j->run) j->run->release();
  j->run.reset();
  if (j->ctx) qeh_ctx_destroy(j->ctx);
  j->ctx = nullptr;
  if (j->ctx64) qeh_ctx_destroy(j->ctx64);
  j->ctx64 = nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  free_range(s, j->off, j->total);
  s->slot_free[j->slot] = 1;
  Request *r = j->req;
  if (j->st != QEH_OK && r->st == QEH_OK) {
    r->st = j->st;
    r->msg = qeh_last_error();   // thread-local text of this (server) thread
  }
  if (--r->remaining == 0) r->t[3] = now_s(s->t0);   // results ready
  j->finished = true;
  s->cv_work.notify_all();
}

// Coordinator, lock held, after joining j's worker: a request becomes visible
// to qeh_poll only once every worker thread of it has been joined.
void reap_job(qeh_server *s, Job *j) {
  j->reaped = true;
  Request *r = j->req;
  if (r->remaining != 0) return;
  for (auto &jj : r->jobs)
    if (!jj->reaped) return;
  r->done = true;
  s->finished++;
  for (auto &jj : r->jobs) jj->hc = HostCell();   // host copies no longer needed
  s->cv_done.notify_all();
}

// Worker thread of one job: set up, drive the Davidson state machine to the
// end (waiting on this job's stream between steps), release.
void job_main(qeh_server *s, Job *j) {
  if (start_job(s, j)) {
    hipStream_t st = s->streams[j->slot];
    while (!j->run->advance()) {
      hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        j->st = hip_fail(e, "device work of a served job");
        break;
      }
    }
    if (j->st == QEH_OK) {
      j->run->fill_info(&j->info);
      j->st = j->run->result();
    }
  }
  finish_job(s, j);
}

void server_loop(qeh_server *s) {
  auto last = std::chrono::steady_clock::now();
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    // reap finished workers
    for (auto it = s->running.begin(); it != s->running.end();) {
      Job *j = *it;
      if (j->finished) {
        lk.unlock();
        if (j->th.joinable()) j->th.join();
        lk.lock();
        reap_job(s, j);
        it = s->running.erase(it);
      } else {
        ++it;
      }
    }
    const auto tn = std::chrono::steady_clock::now();
    if (!s->running.empty()) s->busy_s += std::chrono::duration<double>(tn - last).count();
    last = tn;
    if (s->stop && s->running.empty()) break;
    // admit: first come first served, backfill while the head is young
    std::vector<Job *> fresh;
    if (!s->stop) {
      const double t = now_s(s->t0);
      bool head_blocked = false;
      for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request *r = *it;
        if (r->cancelled) {
          it = s->queue.erase(it);
          continue;
        }
        if (head_blocked && t - s->queue.front()->t[0] >= kBackfillWindow) break;
        if (try_admit(s, r)) {
          for (auto &j : r->jobs) fresh.push_back(j.get());
          it = s->queue.erase(it);
        } else {
          if (it == s->queue.begin()) head_blocked = true;
          ++it;
        }
      }
    }
    for (Job *j : fresh) {
      s->running.push_back(j);
      j->th = std::thread(job_main, s, j);
    }
    s->peak_running = std::max<int>(s->peak_running, (int)s->running.size());
    // sleep until a submission or a job end; wake periodically for backfill
    s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
  }
}

qeh_status plan_job(const qeh_cell *cell, int nb, const qeh_dav_opts *o, Job *j) {
  qeh_status st = qeh_ctx_plan(cell, &j->ctx_bytes);
  if (st != QEH_OK) return st;
  j->ctx64_bytes = 0;
  if (cell->precision == QEH_MIXED) {
    // mixed-form solves finish with H in FP64 (refinement phase)
    qeh_cell c64 = *cell;
    c64.precision = QEH_FP64;
    st = qeh_ctx_plan(&c64, &j->ctx64_bytes);
    if (st != QEH_OK) return st;
    j->ctx64_bytes = align_up(j->ctx64_bytes);
  }
  // the Davidson plan needs only npw, the Gamma flag and whether S != 1
  qeh_ctx probe;
  probe.npw = cell->npw;
  probe.gamma = cell->gamma ? 1 : 0;
  probe.has_q = cell->qmat ? 1 : 0;   // S != 1: the plan holds S V and S P too
  int nvecx, maxiter;
  double rtol;
  bool own = false;
  st = dav_check_opts(&probe, nb, o, &nvecx, &rtol, &maxiter, &own);
  if (st != QEH_OK) return st;
  DavLayout L;
  st = dav_layout(&probe, nb, nvecx, own, &L);
  if (st != QEH_OK) return st;
  j->ctx_bytes = align_up(j->ctx_bytes);
  j->psi_bytes = align_up(16 * (size_t)nb * cell->npw);
  j->dav_bytes = align_up(L.total);
  j->total = j->ctx_bytes + j->ctx64_bytes + j->psi_bytes + j->dav_bytes;
  return QEH_OK;
}

void copy_cell(const qeh_cell *c, const double *psi0, int nb, HostCell *h) {
  h->cell = *c;
  const size_t npw = c->npw;
  h->miller.assign(c->miller, c->miller + 3 * npw);
  const size_t nfft = (size_t)c->fft[0] * c->fft[1] * c->fft[2];
  h->vloc.assign(c->vloc, c->vloc + nfft);
  long nkb = 0, nd = 0;
  if (c->nat > 0) {
    h->nproj.assign(c->nproj, c->nproj + c->nat);
    for (int a = 0; a < c->nat; ++a) {
      nkb += c->nproj[a];
      nd += (long)c->nproj[a] * c->nproj[a];
    }
  }
  if (nkb && c->beta) {
    h->beta.assign(c->beta, c->beta + 2 * nkb * npw);
  } else if (nkb && c->projgen) {
    const qeh_projgen *p = c->projgen;
    h->has_pg = true;
    h->pg = *p;
    h->tau.assign(p->tau, p->tau + 3 * (size_t)c->nat);
    h->ityp.assign(p->ityp, p->ityp + c->nat);
    h->nchan.assign(p->nchan, p->nchan + p->nsp);
    long nch = 0;
    for (int s2 = 0; s2 < p->nsp; ++s2) nch += p->nchan[s2];
    if (nch) h->lchan.assign(p->lchan, p->lchan + nch);
    h->tab.assign(p->tab, p->tab + (size_t)nch * p->nq);
  }
  if (nd) h->dmat.assign(c->dmat, c->dmat + 2 * nd);
  if (nd && c->qmat) h->qmat.assign(c->qmat, c->qmat + 2 * nd);
  h->psi0.assign(psi0, psi0 + 2 * (size_t)nb * npw);
  h->bind();
}

}  // namespace
}  // namespace qeh

using namespace qeh;

extern "C" {

qeh_status qeh_server_create(void *arena, size_t arena_bytes, int max_slots, qeh_server **out) {
  if (!out) return (set_error("out is null"), QEH_ERR_INVALID);
  *out = nullptr;
  if (!arena || reinterpret_cast<uintptr_t>(arena) % kAlign)
    return (set_error("arena must be a 256-byte aligned device pointer"), QEH_ERR_INVALID);
  if (max_slots < 1 || max_slots > kMaxSlots)
    return (set_error("max_slots must be in [1, 64]"), QEH_ERR_INVALID);
  std::unique_ptr<qeh_server> s(new qeh_server());
  s->arena = reinterpret_cast<char *>(arena);
  s->arena_bytes = arena_bytes / kAlign * kAlign;
  s->max_slots = max_slots;
  s->free_ranges[0] = s->arena_bytes;
  s->slot_free.assign(max_slots, 1);
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t st;
    hipEvent_t ev;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      for (auto x : s->events) (void)hipEventDestroy(x);
      return hip_fail(e, "server streams");
    }
    s->streams.push_back(st);
    s->events.push_back(ev);
  }
  s->t0 = std::chrono::steady_clock::now();
  qeh_server *raw = s.get();
  s->th = std::thread(server_loop, raw);
  *out = s.release();
  return QEH_OK;
}

qeh_status qeh_submit(qeh_server *s, const qeh_cell *cells, int nk, int nb, const double *psi0,
                      const qeh_dav_opts *opts, uint64_t *ticket) {
  if (!s || !cells || !psi0 || !ticket) return (set_error("null argument"), QEH_ERR_INVALID);
  if (nk < 1 || nb < 1) return (set_error("nk and nb must be >= 1"), QEH_ERR_INVALID);
  std::unique_ptr<Request> r(new Request());
  r->nk = nk;
  r->nb = nb;
  if (opts) r->opts = *opts;
  r->opts.refine = nullptr;   // the server attaches its own FP64 context per job
  r->t[0] = now_s(s->t0);
  size_t off = 0;
  for (int k = 0; k < nk; ++k) {
    std::unique_ptr<Job> j(new Job());
    j->req = r.get();
    j->k = k;
    qeh_status st = plan_job(&cells[k], nb, opts, j.get());
    if (st != QEH_OK) return st;
    copy_cell(&cells[k], psi0 + 2 * off, nb, &j->hc);
    off += (size_t)nb * cells[k].npw;
    r->footprint += j->total;
    r->jobs.push_back(std::move(j));
  }
  r->remaining = nk;
  if (r->footprint > s->arena_bytes || nk > s->max_slots) {
    set_error("request needs " + std::to_string(r->footprint) + " bytes / " +
              std::to_string(nk) + " slots; the server has " + std::to_string(s->arena_bytes) +
              " / " + std::to_string(s->max_slots));
    return QEH_ERR_REJECTED;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  *ticket = r->id;
  s->queue.push_back(r.get());
  s->all[r->id] = std::move(r);
  s->cv_work.notify_all();
  return QEH_OK;
}

qeh_status qeh_poll(qeh_server *s, uint64_t ticket, double *eig, qeh_dav_info *info,
                    double *t_stamps) {
  if (!s) return (set_error("server is null"), QEH_ERR_INVALID);
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return (set_error("unknown ticket"), QEH_ERR_INVALID);
  Request *r = it->second.get();
  if (r->cancelled) {
    s->all.erase(it);
    set_error("request was cancelled");
    return QEH_ERR_REJECTED;
  }
  if (!r->done) return QEH_ERR_BUSY;
  for (int k = 0; k < r->nk; ++k) {
    Job *j = r->jobs[k].get();
    if (eig) std::copy(j->eig.begin(), j->eig.end(), eig + (size_t)k * r->nb);
    if (info) info[k] = j->info;
  }
  if (t_stamps) std::copy(r->t, r->t + 4, t_stamps);
  const qeh_status st = r->st;
  if (st != QEH_OK) set_error(r->msg);
  s->all.erase(it);
  return st;
}

qeh_status qeh_cancel(qeh_server *s, uint64_t ticket) {
  if (!s) return (set_error("server is null"), QEH_ERR_INVALID);
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return (set_error("unknown ticket"), QEH_ERR_INVALID);
  Request *r = it->second.get();
  if (r->admitted || r->done) return QEH_ERR_BUSY;
  r->cancelled = true;
  s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), r), s->queue.end());
  return QEH_OK;
}

qeh_status qeh_server_stats(qeh_server *s, double *out, int n) {
  if (!s || !out) return (set_error("null argument"), QEH_ERR_INVALID);
  std::lock_guard<std::mutex> lk(s->mu);
  int running = 0;
  for (int f : s->slot_free) running += f ? 0 : 1;
  const double v[8] = {(double)s->queue.size(), (double)running, (double)s->finished,
                       (double)s->in_use, (double)s->arena_bytes, (double)s->peak_running,
                       s->busy_s, now_s(s->t0)};
  for (int i = 0; i < n && i < 8; ++i) out[i] = v[i];
  return QEH_OK;
}

qeh_status qeh_server_destroy(qeh_server *s) {
  if (!s) return QEH_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  for (auto x : s->streams) (void)hipStreamDestroy(x);
  for (auto x : s->events) (void)hipEventDestroy(x);
  delete s;
  return QEH_OK;
}

}  // extern "C"
