// Serving: continuous batching of PCG solves (Sec. 4.2) over device-resident
// preconditioners. Host-side policy only; the device work runs in the engines
// of device.hip (one batch of PCG columns per preconditioner, own stream).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <future>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "handles.hpp"

namespace {

using spnet::ColumnStatus;
using spnet::Engine;
using spnet::HostFactors;
using spnet::Precond;

struct Request;

// the engine of one preconditioner and the request column each batch column holds
struct EngineSlot {
  std::shared_ptr<Precond> pre;
  Engine *eng = nullptr;
  bool uploaded_here = false;  // the server factored and uploaded pre
  int64_t bytes = 0;           // engine + (uploaded factors)
  std::vector<Request *> col_req;
  std::vector<int> col_j;
  int64_t last_tick = 0;
  bool ticking = false;
  int active_columns() const {
    int a = 0;
    for (auto *r : col_req) a += r != nullptr;
    return a;
  }
  ~EngineSlot() {
    if (eng) spnet::engine_destroy(eng);
  }
};

struct Request {
  uint64_t ticket = 0;
  std::shared_ptr<Precond> pre;
  int k = 1;
  std::vector<double> f, u;
  double rtol = 1e-8;
  int64_t max_iter = 1000;
  std::vector<sn_solve_info> info;
  enum { QUEUED, RUNNING, DONE, FAILED } state = QUEUED;
  sn_status err = SN_OK;
  std::string msg;
  int remaining = 0;
  std::chrono::steady_clock::time_point t_submit, t_admit;
};

}  // namespace

struct sn_server_s {
  sn_server_opts o{};
  uint64_t next_ticket = 1;
  int64_t tick_no = 0;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::deque<Request *> queue;
  std::vector<std::unique_ptr<EngineSlot>> engines;
  // host factorisations in flight or done, per preconditioner
  std::unordered_map<Precond *, std::shared_future<std::shared_ptr<HostFactors>>> factoring;
  // every call holds mu; the driver thread (sn_server_run) steps the server
  // while there is work and sleeps on cv_work otherwise; cv_done wakes waiters
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread driver;
  bool driving = false, stop = false;
  sn_status drive_err = SN_OK;
  std::string drive_msg;

  int64_t used() const {
    int64_t b = 0;
    for (auto &e : engines) b += e->bytes;
    return b;
  }
  EngineSlot *slot_of(Precond *p) {
    for (auto &e : engines)
      if (e->pre.get() == p) return e.get();
    return nullptr;
  }
  bool has_work() const {
    if (!queue.empty()) return true;
    for (auto &e : engines)
      if (e->ticking || e->active_columns() > 0) return true;
    return false;
  }
  void stop_driver() {
    {
      std::lock_guard<std::mutex> lk(mu);
      if (!driving) return;
      stop = true;
    }
    cv_work.notify_all();
    driver.join();
    std::lock_guard<std::mutex> lk(mu);
    driving = false;
    stop = false;
  }
  ~sn_server_s() {
    stop_driver();
    for (auto &e : engines)
      if (e->eng) spnet::engine_wait(e->eng);
    for (auto &f : factoring) f.second.wait();
    engines.clear();
  }
};

namespace {

int64_t factor_estimate(const Precond &pre, const HostFactors &hf, int precision) {
  // both star layouts (band streams, supernodal blobs with about 20 bytes of
  // index per position and update), per-position arrays, matrix, coarse operator
  // (dense and packed)
  const int64_t ts = precision == SN_PREC_FP64 ? 8 : 4;
  int64_t vals = 0, pos = 0, upd = 0;
  for (const auto &F : hf.stars) {
    vals += (int64_t)(F.colvals.size() + F.rowvals.size() + F.sn.S.size());
    pos += F.n;
    upd += F.sn.nu;
  }
  const int64_t n = pre.sys->n, nnz = (int64_t)pre.sys->col.size();
  return (vals * ts + pos * (40 + 2 * ts) + upd * 8 + n * pre.nvert_per_elem * 16 + nnz * 12 +
          pre.m0 * pre.m0 * 12) * 13 / 10;  // the coarse inverse dense and packed
}

// start the host factorisation of pre on a worker thread (once)
void start_factor(sn_server_s &S, const std::shared_ptr<Precond> &pre) {
  if (pre->dev || S.factoring.count(pre.get())) return;
  std::shared_ptr<Precond> keep = pre;
  S.factoring[pre.get()] = std::async(std::launch::async, [keep]() {
                             return std::make_shared<HostFactors>(spnet::factor_host(*keep));
                           }).share();
}

void fail_request(Request *r, sn_status code, const std::string &msg) {
  r->state = Request::FAILED;
  r->err = code;
  r->msg = msg;
}

// evict idle engines, least recently ticked first, until `need` more bytes fit
bool make_room(sn_server_s &S, int64_t need) {
  while (S.used() + need > S.o.hbm_budget) {
    EngineSlot *victim = nullptr;
    for (auto &e : S.engines)
      if (e->active_columns() == 0 && !e->ticking && (!victim || e->last_tick < victim->last_tick)) victim = e.get();
    if (!victim) return false;
    std::shared_ptr<Precond> pre = victim->pre;
    const bool drop_factors = victim->uploaded_here;
    for (size_t i = 0; i < S.engines.size(); ++i)
      if (S.engines[i].get() == victim) {
        S.engines.erase(S.engines.begin() + (ptrdiff_t)i);
        break;
      }
    if (drop_factors && pre->dev) {
      spnet::device_release(pre->dev.release());
      pre->precision = -1;
    }
  }
  return true;
}

// engine for the request's preconditioner: existing, or created within the budget
EngineSlot *engine_for(sn_server_s &S, Request *r) {
  if (EngineSlot *e = S.slot_of(r->pre.get())) return e;
  Precond &pre = *r->pre;
  std::shared_ptr<HostFactors> hf;
  int64_t need = 0;
  if (!pre.dev) {
    auto it = S.factoring.find(&pre);
    if (it == S.factoring.end()) {
      start_factor(S, r->pre);
      return nullptr;
    }
    if (it->second.wait_for(std::chrono::seconds(0)) != std::future_status::ready) return nullptr;
    try {
      hf = it->second.get();
    } catch (const spnet::Error &e) {
      S.factoring.erase(it);
      fail_request(r, e.code, e.what());
      return nullptr;
    }
    need += factor_estimate(pre, *hf, S.o.precision);
  }
  const int64_t eng_bytes = spnet::engine_footprint(pre, S.o.max_columns);
  need += eng_bytes;
  if (need > S.o.hbm_budget) {
    fail_request(r, SN_EBUSY, "request exceeds the server's device-memory budget");
    return nullptr;
  }
  if (!make_room(S, need)) return nullptr;
  auto slot = std::make_unique<EngineSlot>();
  slot->pre = r->pre;
  // a failure to upload the factors or to create the engine fails this
  // request only; the others keep running
  try {
    if (!pre.dev) {
      S.factoring.erase(&pre);
      spnet::device_setup(pre, *hf, S.o.precision);
      slot->uploaded_here = true;
    }
    slot->eng = spnet::engine_create(pre, S.o.max_columns);
  } catch (const spnet::Error &e) {
    if (slot->uploaded_here && pre.dev) {
      spnet::device_release(pre.dev.release());
      pre.precision = -1;
    }
    fail_request(r, e.code, e.what());
    return nullptr;
  }
  slot->bytes = spnet::engine_footprint(pre, S.o.max_columns) + (slot->uploaded_here ? spnet::device_bytes(pre) : 0);
  slot->col_req.assign((size_t)S.o.max_columns, nullptr);
  slot->col_j.assign((size_t)S.o.max_columns, -1);
  S.engines.push_back(std::move(slot));
  return S.engines.back().get();
}

void retire_finished(sn_server_s &S, EngineSlot &e) {
  const int kc = S.o.max_columns;
  std::vector<ColumnStatus> st((size_t)kc);
  spnet::engine_status(e.eng, st.data());
  for (int c = 0; c < kc; ++c) {
    Request *r = e.col_req[c];
    if (!r) continue;
    const ColumnStatus &x = st[c];
    if (!(x.active && x.done && !x.verify)) continue;
    const int j = e.col_j[c];
    spnet::engine_retire(e.eng, c, r->u.data() + j, r->k);
    const double fn = std::sqrt(x.f2);
    sn_solve_info &in = r->info[j];
    in.iters = x.iters;
    in.res_rec = fn > 0 ? std::sqrt(x.rr) / fn : std::sqrt(x.rr);
    in.res_true = fn > 0 ? std::sqrt(x.t2) / fn : std::sqrt(x.t2);
    in.converged = spnet::column_converged(x.rr, x.t2, x.tol2);
    in.replacements = x.replacements;
    in.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - r->t_submit).count();
    e.col_req[c] = nullptr;
    e.col_j[c] = -1;
    if (--r->remaining == 0) r->state = Request::DONE;
  }
}

// One scheduling step (see sn_server_step). block: wait for the first tick
// to complete (or a host factorisation, when nothing iterates); else only
// look. Returns whether anything changed.
bool step_once(sn_server_s &S, bool block) {
  ++S.tick_no;
  bool any_ticking = false, progressed = false;
  for (auto &e : S.engines) any_ticking |= e->ticking;
  // 1. engines whose tick has completed: retire their converged columns.
  //    Engines advance independently: a small network does not wait for the
  //    ticks of a large one.
  do {
    for (auto &e : S.engines)
      if (e->ticking && spnet::engine_query(e->eng)) {
        e->ticking = false;
        retire_finished(S, *e);
        progressed = true;
      }
    if (block && any_ticking && !progressed) std::this_thread::yield();
  } while (block && any_ticking && !progressed);
  // nothing iterates but requests wait for their host factorisation: wait
  // for the first of those to finish, so that a blocking step makes progress
  if (block && !any_ticking) {
    bool running = false;
    for (auto &e : S.engines) running |= e->active_columns() > 0;
    if (!running)
      for (Request *r : S.queue) {
        auto it = S.factoring.find(r->pre.get());
        if (it != S.factoring.end()) {
          it->second.wait();
          break;
        }
      }
  }
  // 2. admit queued requests that fit (in arrival order; a request that
  //    cannot start yet does not hold back later ones)
  for (auto it = S.queue.begin(); it != S.queue.end();) {
    Request *r = *it;
    EngineSlot *e = engine_for(S, r);
    if (r->state == Request::FAILED) {
      it = S.queue.erase(it);
      progressed = true;
      continue;
    }
    if (!e || e->ticking) {
      ++it;
      continue;
    }
    std::vector<int32_t> cols;
    for (int c = 0; c < S.o.max_columns && (int)cols.size() < r->k; ++c)
      if (!e->col_req[c]) cols.push_back(c);
    if ((int)cols.size() < r->k) {
      ++it;
      continue;
    }
    std::vector<double> rt((size_t)r->k, r->rtol);
    std::vector<int64_t> mi((size_t)r->k, r->max_iter);
    spnet::engine_admit(e->eng, r->k, cols.data(), r->f.data(), rt.data(), mi.data());
    for (int j = 0; j < r->k; ++j) {
      e->col_req[cols[j]] = r;
      e->col_j[cols[j]] = j;
    }
    r->remaining = r->k;
    r->state = Request::RUNNING;
    r->t_admit = std::chrono::steady_clock::now();
    r->f.clear();
    r->f.shrink_to_fit();
    it = S.queue.erase(it);
    progressed = true;
  }
  // 3. queue the next iterations of every idle engine with running columns
  for (auto &e : S.engines)
    if (!e->ticking && e->active_columns() > 0) {
      spnet::engine_tick(e->eng, S.o.iters_per_tick, S.o.use_graph != 0);
      e->ticking = true;
      e->last_tick = S.tick_no;
      progressed = true;
    }
  return progressed;
}

void counts(sn_server_s &S, int32_t *n_active, int32_t *n_queued) {
  int32_t act = 0;
  for (auto &kv : S.reqs) act += kv.second->state == Request::RUNNING;
  if (n_active) *n_active = act;
  if (n_queued) *n_queued = (int32_t)S.queue.size();
}

// The driver thread: steps the server while it has work (without blocking,
// so that calls from other threads get the lock between steps), sleeps on
// cv_work otherwise. A device error stops it
// and fails every request not yet done.
void drive(sn_server_s *S, int device) {
  std::unique_lock<std::mutex> lk(S->mu);
  try {
    spnet::device_bind(device);
  } catch (const spnet::Error &e) {
    S->drive_err = e.code;
    S->drive_msg = e.what();
    S->stop = true;
  }
  while (!S->stop) {
    if (!S->has_work()) {
      S->cv_work.wait(lk);
      continue;
    }
    bool progressed = false;
    try {
      progressed = step_once(*S, false);
    } catch (const spnet::Error &e) {
      S->drive_err = e.code;
      S->drive_msg = e.what();
    } catch (const std::exception &e) {
      S->drive_err = SN_EDEVICE;
      S->drive_msg = e.what();
    }
    if (S->drive_err != SN_OK) {
      for (auto &kv : S->reqs)
        if (kv.second->state == Request::QUEUED || kv.second->state == Request::RUNNING)
          fail_request(kv.second.get(), S->drive_err, "server thread stopped: " + S->drive_msg);
      S->queue.clear();
      S->cv_done.notify_all();
      break;
    }
    if (progressed) S->cv_done.notify_all();
    // let other callers take the lock between steps; while ticks are in
    // flight the thread spins (a sleep would add the timer's slack, tens of
    // microseconds, to every tick)
    lk.unlock();
    std::this_thread::yield();
    lk.lock();
  }
}

}  // namespace

extern "C" {

void sn_server_opts_default(sn_server_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->hbm_budget = (int64_t)64 << 30;
  o->max_columns = 8;
  o->iters_per_tick = 4;
  o->precision = SN_PREC_FP32_STARS;
  o->use_graph = 1;
}

sn_status sn_server_create(const sn_server_opts *opts, sn_server *out) {
  return spnet::guarded([&] {
    if (!out) spnet::fail(SN_EINVAL, "out is NULL");
    sn_server_opts o;
    if (opts) o = *opts;
    else sn_server_opts_default(&o);
    if (o.max_columns != 1 && o.max_columns != 2 && o.max_columns != 4 && o.max_columns != 8 && o.max_columns != 16)
      spnet::fail(SN_EINVAL, "max_columns must be 1, 2, 4, 8 or 16");
    if (o.iters_per_tick < 1) spnet::fail(SN_EINVAL, "iters_per_tick must be positive");
    if (o.hbm_budget <= 0) spnet::fail(SN_EINVAL, "hbm_budget must be positive");
    if (o.precision != SN_PREC_FP64 && o.precision != SN_PREC_FP32_STARS &&
        o.precision != SN_PREC_FP32_STARS_COARSE)
      spnet::fail(SN_EINVAL, "unknown precision");
    auto *s = new sn_server_s;
    s->o = o;
    *out = s;
  });
}

sn_status sn_server_submit(sn_server srv, sn_precond pre, int k, const double *f, double rtol, int64_t max_iter,
                           uint64_t *ticket) {
  return spnet::guarded([&] {
    if (!srv || !pre || !f || !ticket) spnet::fail(SN_EINVAL, "null argument");
    if (k < 1 || k > srv->o.max_columns) spnet::fail(SN_EINVAL, "k must be in 1..max_columns");
    if (!(rtol >= 0.0) || !std::isfinite(rtol)) spnet::fail(SN_EINVAL, "bad rtol");
    const int64_t n = pre->p->sys->n;
    for (int64_t i = 0; i < n * k; ++i)
      if (!std::isfinite(f[i])) spnet::fail(SN_EINVAL, "non-finite right-hand side");
    if (pre->p->dev &&
        spnet::engine_footprint(*pre->p, srv->o.max_columns) > srv->o.hbm_budget)
      spnet::fail(SN_EBUSY, "request exceeds the server's device-memory budget");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->drive_err != SN_OK) spnet::fail(srv->drive_err, "server thread stopped: " + srv->drive_msg);
    auto r = std::make_unique<Request>();
    r->ticket = srv->next_ticket++;
    r->pre = pre->p;
    r->k = k;
    r->f.assign(f, f + n * k);
    r->u.assign((size_t)(n * k), 0.0);
    r->rtol = rtol;
    r->max_iter = max_iter > 0 ? max_iter : 1000;
    r->info.assign((size_t)k, sn_solve_info{});
    r->t_submit = std::chrono::steady_clock::now();
    start_factor(*srv, r->pre);
    srv->queue.push_back(r.get());
    *ticket = r->ticket;
    srv->reqs[r->ticket] = std::move(r);
    srv->cv_work.notify_all();
  });
}

sn_status sn_server_step(sn_server srv, int32_t *n_active, int32_t *n_queued) {
  return spnet::guarded([&] {
    if (!srv) spnet::fail(SN_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->driving) spnet::fail(SN_EBUSY, "the server's own thread steps it (sn_server_run)");
    step_once(*srv, true);
    srv->cv_done.notify_all();
    counts(*srv, n_active, n_queued);
  });
}

sn_status sn_server_poll(sn_server srv, uint64_t ticket, double *u, sn_solve_info *info) {
  sn_status rc = SN_OK;
  const sn_status g = spnet::guarded([&] {
    if (!srv) spnet::fail(SN_EINVAL, "null server");
    std::unique_ptr<Request> done;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      auto it = srv->reqs.find(ticket);
      if (it == srv->reqs.end()) spnet::fail(SN_EINVAL, "unknown ticket");
      Request &r = *it->second;
      if (r.state == Request::FAILED) {
        const sn_status code = r.err;
        const std::string msg = r.msg;
        srv->reqs.erase(it);
        spnet::fail(code, msg);
      }
      if (r.state != Request::DONE) {
        rc = SN_EBUSY;
        return;
      }
      if (!u && !info) return;  // status query: the result stays
      // the result leaves the server; it is copied out without the lock
      done = std::move(it->second);
      srv->reqs.erase(it);
    }
    if (u) std::memcpy(u, done->u.data(), done->u.size() * sizeof(double));
    if (info) std::memcpy(info, done->info.data(), done->info.size() * sizeof(sn_solve_info));
  });
  return g != SN_OK ? g : rc;
}

sn_status sn_server_usage(sn_server srv, int64_t *device_bytes, int32_t *n_engines) {
  return spnet::guarded([&] {
    if (!srv) spnet::fail(SN_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (device_bytes) *device_bytes = srv->used();
    if (n_engines) *n_engines = (int32_t)srv->engines.size();
  });
}

sn_status sn_server_run(sn_server srv, int enable) {
  return spnet::guarded([&] {
    if (!srv) spnet::fail(SN_EINVAL, "null server");
    if (!enable) {
      srv->stop_driver();
      return;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->driving) return;
    if (srv->drive_err != SN_OK) spnet::fail(srv->drive_err, "server thread stopped: " + srv->drive_msg);
    const int device = spnet::device_current();
    srv->stop = false;
    srv->driver = std::thread(drive, srv, device);
    srv->driving = true;
  });
}

sn_status sn_server_wait(sn_server srv, uint64_t ticket, double timeout_s) {
  sn_status rc = SN_OK;
  const sn_status g = spnet::guarded([&] {
    if (!srv) spnet::fail(SN_EINVAL, "null server");
    if (!(timeout_s >= 0.0)) spnet::fail(SN_EINVAL, "timeout must be non-negative");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto finished = [&]() {
      if (ticket != 0) {
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end()) spnet::fail(SN_EINVAL, "unknown ticket");
        return it->second->state == Request::DONE || it->second->state == Request::FAILED;
      }
      for (auto &kv : srv->reqs)
        if (kv.second->state == Request::DONE || kv.second->state == Request::FAILED) return true;
      return false;
    };
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                           std::chrono::duration<double>(std::min(timeout_s, 1e6)));
    while (!finished()) {
      if (srv->driving) {
        if (srv->cv_done.wait_until(lk, until) == std::cv_status::timeout && !finished()) {
          rc = SN_EBUSY;
          return;
        }
      } else {
        if (!srv->has_work() || std::chrono::steady_clock::now() >= until) {
          rc = SN_EBUSY;
          return;
        }
        step_once(*srv, true);
      }
    }
  });
  return g != SN_OK ? g : rc;
}

void sn_server_destroy(sn_server srv) { delete srv; }

}  // extern "C"
