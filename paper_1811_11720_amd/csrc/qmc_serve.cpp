// qmc_serve.cpp -- continuous batching of integration requests on one context.
//
// qmc_submit queues a ticket (a group of requests) and returns at once.  A
// scheduler thread per context runs rounds: before each round it admits
// queued tickets in arrival order while their estimated device memory fits
// the context's budget; one round evaluates the current lattice of every
// admitted, unfinished request with the persistent batch kernels
// (run_batch), then applies each request's own error goal and growth rule
// (Sec. 3.3.1; at the largest lattice a request stops instead of adding
// shifts, so its memory stays within what admission reserved).  A request
// that finishes returns its reserved memory to the budget at once, so
// tickets that arrive while others are on the GPU join the next round.  A request's
// results do not depend on what it was batched with (its tiling depends only
// on its own n and m).  Descriptors stay resident on the device between
// rounds; a request's state between rounds is (n, z, shifts, round count).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <list>

#include "qmc_host.h"

namespace {

using clk = std::chrono::steady_clock;

struct Req {
  qmc_request q;
  qmc_integrand* f;
  std::vector<double> shifts;
  std::vector<uint64_t> z;
  uint64_t n = 0;
  bool done = false;
  qmc_result r{};
  qmch::BatchJob job;
  size_t bytes = 0;
  // progress on the current lattice when it is evaluated over several rounds
  uint32_t tiles_total = 0, tiles_done = 0;  // tiles_total 0: the lattice has not started
  double tile_cost = 0.0;                     // cost units of one tile
  double* d_part = nullptr;                   // its tile partials, kept between rounds
  size_t part_bytes = 0;
  uint64_t lat_signs = 0;                     // points with Im F(z) > 0 so far on this lattice
};

struct Ticket {
  uint64_t id;
  std::vector<Req> reqs;
  clk::time_point t_submit, t_admit;
  bool admitted = false, finished = false, cancelled = false;
  int status = QMC_OK;
  size_t bytes = 0;  // reservation of all requests (admission test)
  size_t held = 0;   // part of the reservation still counted in in_use
};

}  // namespace

struct qmc_serve_state {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread thr;
  bool stop = false;
  uint64_t next_id = 1;
  std::list<std::shared_ptr<Ticket>> queue;   // submitted, not admitted
  std::list<std::shared_ptr<Ticket>> active;  // admitted, running
  std::map<uint64_t, std::shared_ptr<Ticket>> all;
  size_t in_use = 0;
  uint64_t rounds = 0;
  std::vector<double*> to_free;  // partial buffers of finished requests, freed before the next round
};

namespace qmch {

// Device bytes admitted requests may hold: QMC_SERVE_MEM, and no more than a
// caller-owned workspace (which cannot grow), less the per-round arena
// headers (launch counters, prefix tables, alignment).
size_t serve_budget(const qmc_context* c) {
  const size_t cap = c->own_ws ? c->serve_mem_limit : std::min(c->serve_mem_limit, c->ws_bytes);
  const size_t reserve = 64 * 1024;
  return cap > reserve ? cap - reserve : 0;
}

// Device bytes one request can need in a round at lattice size n, whatever
// schedule run_batch picks (tuned, cached or default tiles, specialised or
// table-driven kernel): batch_ktiles_bound bounds its tile count.
static size_t request_bytes(const qmc_integrand* f, uint64_t n, uint32_t m, const qmc_context* c) {
  const bool cplx = (f->flags & QMC_DEFORM) != 0;
  const uint64_t kt = batch_ktiles_bound(c, n);
  const size_t rows = cplx ? 2 * (size_t)m : m;
  return batch_job_bytes(rows, kt, m, f->dim, (f->flags & QMC_EVAL_FP32) != 0);
}

static void release(qmc_serve_state* s, Ticket& t, size_t bytes) {
  bytes = std::min(bytes, t.held);
  t.held -= bytes;
  s->in_use -= bytes;
}

static void drop_partials(qmc_serve_state* s, Req& r) {
  if (r.d_part) s->to_free.push_back(r.d_part);
  r.d_part = nullptr;
  r.part_bytes = 0;
}

static void finish_ticket(qmc_serve_state* s, Ticket& t, int status) {
  t.finished = true;
  t.status = status;
  for (auto& r : t.reqs) {
    r.f->refs -= 1;
    drop_partials(s, r);
  }
  release(s, t, t.held);  // nothing is held by a ticket that was never admitted
  s->cv_done.notify_all();
}

// Cost units of one evaluation of f (the batch planner's ordering weight).
static double eval_cost(const qmc_integrand* f) {
  double cst = (double)(f->n_u + f->n_f) * f->dim + 10.0 * f->dim;
  if (f->flags & QMC_DEFORM) cst = cst * 6.0 + 2.0 * f->dim * f->dim * f->dim;
  return cst;
}

// The part of a request's current lattice that runs this round: all of it
// when it fits its share of the round's cost budget (or the context has a
// caller-owned workspace), else the next tiles that fit (at least one), with
// the tile partials in a buffer kept until the lattice is done.
static int plan_slice(qmc_context* c, qmc_serve_state* s, Req& r, double share) {
  BatchJob& j = r.job;
  j.tile_first = 0;
  j.tile_count = 0;
  j.ext_partial = nullptr;
  j.finish = true;
  if (r.tiles_total == 0) {
    BatchShape sh;
    int rc = batch_job_shape(c, j, sh);
    if (rc) return rc;
    r.tiles_total = sh.ktiles * sh.groups;
    r.tiles_done = 0;
    r.lat_signs = 0;
    r.tile_cost = (double)sh.tile_points * std::min<uint32_t>(sh.group_size, r.q.m) * eval_cost(r.f);
    const double whole = (double)r.n * r.q.m * eval_cost(r.f);
    if (whole <= share || !c->own_ws || r.tiles_total == 1) {
      r.tiles_total = 0;  // one round: no state kept
      return QMC_OK;
    }
    const size_t need = (size_t)sh.rows * sh.ktiles * sizeof(double);
    if (need > r.part_bytes) {
      if (r.d_part) HIPCHK(hipFree(r.d_part));
      r.d_part = nullptr;
      r.part_bytes = 0;
      hipError_t e = hipMalloc((void**)&r.d_part, need);
      if (e != hipSuccess) return fail(QMC_ENOMEM, "hipMalloc(%zu) for tile partials: %s", need, hipGetErrorString(e));
      r.part_bytes = need;
    }
  }
  const uint32_t left = r.tiles_total - r.tiles_done;
  const double fit = std::floor(share / std::max(r.tile_cost, 1.0));
  const uint32_t take = (uint32_t)std::max(1.0, std::min((double)left, fit));
  j.tile_first = r.tiles_done;
  j.tile_count = take;
  j.ext_partial = r.d_part;
  j.finish = take == left;
  return QMC_OK;
}

static void scheduler(qmc_context* c, qmc_serve_state* s) {
  (void)hipSetDevice(c->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // admission: arrival order, while the memory budget allows
    while (!s->queue.empty()) {
      auto& t = s->queue.front();
      if (t->cancelled) {
        finish_ticket(s, *t, QMC_ECANCELED);
        s->queue.pop_front();
        continue;
      }
      if (s->in_use + t->bytes > serve_budget(c) && !s->active.empty()) break;
      t->admitted = true;
      t->t_admit = clk::now();
      s->in_use += t->bytes;
      t->held = t->bytes;
      s->active.push_back(t);
      s->queue.pop_front();
    }
    // drop cancelled tickets at the round boundary
    for (auto it = s->active.begin(); it != s->active.end();) {
      if ((*it)->cancelled) {
        finish_ticket(s, **it, QMC_ECANCELED);
        it = s->active.erase(it);
      } else {
        ++it;
      }
    }
    if (s->active.empty()) {
      if (s->stop) return;
      s->cv_work.wait(lk);
      continue;
    }
    // one round over every unfinished request of the admitted tickets: each
    // gets about an equal share of the round's cost budget (its whole current
    // lattice when that fits, else the next slice of its tiles), so rounds,
    // and with them the wait of a ticket that arrives meanwhile, stay bounded
    std::vector<BatchJob*> jobs;
    std::vector<std::pair<Ticket*, Req*>> refs;
    for (auto& t : s->active)
      for (auto& r : t->reqs)
        if (!r.done) {
          r.job.f = r.f;
          r.job.n = r.n;
          r.job.z = r.z.data();
          r.job.m = r.q.m;
          r.job.shifts = r.shifts.data();
          r.job.t = r.q.t;
          jobs.push_back(&r.job);
          refs.push_back({t.get(), &r});
        }
    std::vector<double*> frees;
    frees.swap(s->to_free);
    lk.unlock();
    double ks = 0.0;
    int rc = QMC_OK;
    {
      // API calls waiting for the context go first: they wait at most one round
      for (int spin = 0; c->lock_waiters.load(std::memory_order_acquire) > 0; ++spin) {
        if (spin < 64)
          std::this_thread::yield();
        else
          std::this_thread::sleep_for(std::chrono::microseconds(50));
      }
      std::lock_guard<std::recursive_mutex> g(c->mu);
      for (double* q : frees) (void)hipFree(q);
      const double share = c->serve_round_cost / (double)std::max<size_t>(1, refs.size());
      for (auto& pr : refs)
        if (rc == QMC_OK) rc = plan_slice(c, s, *pr.second, share);
      if (rc == QMC_OK) rc = c->broken ? QMC_EDEVICE : run_batch(c, jobs, &ks);
      if (rc == QMC_EDEVICE) c->broken = true;
    }
    lk.lock();
    s->rounds += 1;
    if (rc != QMC_OK) {
      for (auto& t : s->active) finish_ticket(s, *t, rc);
      s->active.clear();
      continue;
    }
    for (auto& pr : refs) {
      Req& r = *pr.second;
      Ticket& tk = *pr.first;
      const bool cplx = (r.f->flags & QMC_DEFORM) != 0;
      const uint32_t m = r.q.m;
      r.r.device_seconds += ks;
      r.lat_signs += r.job.sign_points;
      if (r.tiles_total) {  // a lattice evaluated over several rounds
        r.tiles_done += r.job.tile_count;
        if (!r.job.finish) continue;
        r.tiles_total = 0;
      }
      r.r.iterations += 1;
      r.r.evaluations += r.n * (uint64_t)m;
      r.r.n = r.n;
      std::vector<double> qs(m);
      for (uint32_t k = 0; k < m; ++k) qs[k] = r.job.sums_at[k] / (double)r.n;
      estimate(qs.data(), m, r.r.re, r.r.err_re);
      r.r.im = r.r.err_im = 0.0;
      if (cplx) {
        for (uint32_t k = 0; k < m; ++k) qs[k] = r.job.sums_at[m + k] / (double)r.n;
        estimate(qs.data(), m, r.r.im, r.r.err_im);
      }
      if (!r.job.fp32_dev.empty()) {
        const std::vector<double> zero(m, 0.0);
        fp32_error(r.job.fp32_dev.data(), cplx ? r.job.fp32_dev.data() + m : zero.data(), r.job.fp32_ref.data(),
                   cplx ? r.job.fp32_ref.data() + m : zero.data(), m, r.job.fp32_dev_points, r.r);
      }
      r.r.flags &= ~(uint32_t)(QMC_NONFINITE | QMC_DEFORM_SIGN);
      if (r.lat_signs) r.r.flags |= QMC_DEFORM_SIGN;
      r.lat_signs = 0;
      if (r.f->has_vr && r.f->vr_fallback) r.r.flags |= QMC_VR_FALLBACK;
      const bool finite = std::isfinite(r.r.re) && std::isfinite(r.r.im);
      if (!finite) r.r.flags |= QMC_NONFINITE;
      const bool grow = r.q.rel_tol > 0 || r.q.abs_tol > 0;
      if (!grow) {
        r.done = true;
        drop_partials(s, r);
        release(s, tk, r.bytes);
        continue;
      }
      if (finite && goal_met(r.r, r.q.rel_tol, r.q.abs_tol, r.q.errormode, cplx)) {
        r.r.flags |= QMC_CONVERGED;
        r.done = true;
        drop_partials(s, r);
        release(s, tk, r.bytes);
        continue;
      }
      // no added shifts here (max_m = m): a request's device memory stays
      // within its admission estimate
      GrowthStep g = growth_step(c, r.q, r.r, r.n, m, r.f->dim, cplx, c->serve_max_n, m);
      if (g.kind != GrowthStep::LATTICE) {
        r.r.flags |= QMC_MAXEVAL_HIT;
        r.done = true;
        drop_partials(s, r);
        release(s, tk, r.bytes);
        continue;
      }
      r.n = g.n;
      r.z.swap(g.z);
    }
    for (auto it = s->active.begin(); it != s->active.end();) {
      Ticket& t = **it;
      bool all_done = true;
      for (auto& r : t.reqs) all_done = all_done && r.done;
      if (all_done) {
        const double wall = std::chrono::duration<double>(clk::now() - t.t_submit).count();
        const double queue = std::chrono::duration<double>(t.t_admit - t.t_submit).count();
        for (auto& r : t.reqs) {
          r.r.wall_seconds = wall;
          r.r.queue_seconds = queue;
          r.r.path = 2;
        }
        finish_ticket(s, t, QMC_OK);
        it = s->active.erase(it);
      } else {
        ++it;
      }
    }
  }
}

void serve_shutdown(qmc_context* c) {
  qmc_serve_state* s = c->serve.load();
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->thr.joinable()) s->thr.join();
  (void)hipSetDevice(c->device);
  for (double* q : s->to_free) (void)hipFree(q);
  for (auto& kv : s->all)
    for (auto& r : kv.second->reqs)
      if (r.d_part) (void)hipFree(r.d_part);
  delete s;
  c->serve = nullptr;
}

int serve_inflight(qmc_context* c) {
  qmc_serve_state* s = c->serve.load();
  if (!s) return 0;
  std::lock_guard<std::mutex> g(s->mu);
  return (int)(s->queue.size() + s->active.size());
}

}  // namespace qmch

using namespace qmch;

extern "C" {

int qmc_submit(qmc_context* c, const qmc_request* reqs, uint32_t count, uint64_t* ticket) {
  if (!c || !reqs || !ticket || count == 0) return fail(QMC_EINVAL, "bad arguments");
  const clk::time_point t_entry = clk::now();
  auto t = std::make_shared<Ticket>();
  t->reqs.resize(count);
  {
    // Validation needs only the lattice table's lock: a submission never
    // waits for a round that is running on the device.
    if (c->closing) return fail(QMC_EINVAL, "context has been destroyed");
    if (c->broken) return fail(QMC_EDEVICE, "context is unusable after a device error");
    for (uint32_t i = 0; i < count; ++i) {
      const qmc_request& q = reqs[i];
      Req& r = t->reqs[i];
      if (!q.f) return fail(QMC_EINVAL, "request %u has no integrand", i);
      r.q = q;
      r.f = const_cast<qmc_integrand*>(q.f);
      if (r.f->ctx != c) return fail(QMC_EINVAL, "request %u: integrand belongs to another context", i);
      if (r.f->genz) return fail(QMC_EUNSUPPORTED, "request %u: Genz integrands run through qmc_integrate", i);
      if (q.m < 1 || q.m > QMC_MAX_SHIFTS) return fail(QMC_EINVAL, "request %u: m=%u", i, q.m);
      const uint32_t dim = r.f->dim;
      if (q.z) {
        int rc = check_lattice(q.n, dim, q.z);
        if (rc) return rc;
        r.n = q.n;
        r.z.assign(q.z, q.z + dim);
      } else {
        uint64_t nn = 0;
        if (next_registered(c, q.n, dim, &nn, true, &r.z) != QMC_OK)
          return fail(QMC_ENOTFOUND, "request %u: no registered lattice with %u components", i, dim);
        r.n = nn;
      }
      r.q.z = nullptr;  // the caller's array may be freed after return
      r.shifts.resize((size_t)q.m * dim);
      make_shifts(q.seed, q.m, dim, r.shifts.data());
      r.r.m = q.m;
      // memory at the largest lattice the request may reach
      const bool grow = q.rel_tol > 0 || q.abs_tol > 0;
      uint64_t nmax = r.n;
      if (grow) {
        const uint64_t top = largest_registered(c);
        nmax = std::max<uint64_t>(r.n, std::min<uint64_t>(c->serve_max_n, top ? top : r.n));
      }
      r.bytes = request_bytes(r.f, nmax, q.m, c);
      t->bytes += r.bytes;
    }
    if (t->bytes > serve_budget(c))
      return fail(QMC_ENOMEM, "ticket needs %zu bytes, the serving budget is %zu", t->bytes, serve_budget(c));
    std::lock_guard<std::mutex> g(c->serve_init);
    if (!c->serve) {
      qmc_serve_state* s = new qmc_serve_state();
      s->thr = std::thread(scheduler, c, s);
      c->serve = s;
    }
  }
  qmc_serve_state* s = c->serve;
  {
    std::lock_guard<std::mutex> g(s->mu);
    t->id = s->next_id++;
    t->t_submit = t_entry;
    for (auto& r : t->reqs) r.f->refs += 1;
    s->queue.push_back(t);
    s->all[t->id] = t;
    *ticket = t->id;
  }
  s->cv_work.notify_all();
  return QMC_OK;
}

static int collect(qmc_serve_state* s, uint64_t ticket, qmc_result* out) {
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return fail(QMC_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Ticket& t = *it->second;
  if (!t.finished) return QMC_PENDING;
  int st = t.status;
  if (out && st == QMC_OK)
    for (size_t i = 0; i < t.reqs.size(); ++i) out[i] = t.reqs[i].r;
  s->all.erase(it);
  if (st != QMC_OK) return fail(st, "ticket %llu %s", (unsigned long long)ticket,
                                st == QMC_ECANCELED ? "was cancelled" : "failed on the device");
  return QMC_OK;
}

int qmc_poll(qmc_context* c, uint64_t ticket, qmc_result* out) {
  if (!c) return fail(QMC_EINVAL, "context is NULL");
  qmc_serve_state* s = c->serve.load();
  if (!s) return fail(QMC_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  std::lock_guard<std::mutex> g(s->mu);
  return collect(s, ticket, out);
}

int qmc_wait(qmc_context* c, uint64_t ticket, double timeout_s, qmc_result* out) {
  if (!c) return fail(QMC_EINVAL, "context is NULL");
  qmc_serve_state* s = c->serve.load();
  if (!s) return fail(QMC_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  std::unique_lock<std::mutex> lk(s->mu);
  auto deadline = clk::now() + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(
                                   timeout_s < 0 ? 1e9 : timeout_s));
  for (;;) {
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(QMC_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->finished) return collect(s, ticket, out);
    if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
      it = s->all.find(ticket);
      if (it != s->all.end() && it->second->finished) return collect(s, ticket, out);
      return QMC_PENDING;
    }
  }
}

int qmc_cancel(qmc_context* c, uint64_t ticket) {
  qmc_serve_state* s = c ? c->serve.load() : nullptr;
  if (!s) return fail(QMC_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(QMC_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->finished) return QMC_OK;
    it->second->cancelled = true;
  }
  s->cv_work.notify_all();
  return QMC_OK;
}

int qmc_serve_stats(qmc_context* c, uint64_t* rounds, uint64_t* queued, uint64_t* active, uint64_t* bytes_in_use) {
  if (!c) return fail(QMC_EINVAL, "context is NULL");
  uint64_t r = 0, q = 0, a = 0, b = 0;
  if (qmc_serve_state* s = c->serve.load()) {
    std::lock_guard<std::mutex> g(s->mu);
    r = s->rounds;
    q = s->queue.size();
    a = s->active.size();
    b = s->in_use;
  }
  if (rounds) *rounds = r;
  if (queued) *queued = q;
  if (active) *active = a;
  if (bytes_in_use) *bytes_in_use = b;
  return QMC_OK;
}

}  // extern "C"
