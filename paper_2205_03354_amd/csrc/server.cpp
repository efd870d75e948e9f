// Request server: continuous batching of biharmonic / Cahn-Hilliard solves.
//
// One worker thread issues every device call. It keeps up to max_slots
// requests resident, each as a SolveTask on its own stream, and cycles over
// them: a request whose last chunk has completed (its event has fired) is
// advanced and its next chunk enqueued; a finished request is copied back
// and retired, which frees its slot and budget; queued requests are admitted
// in arrival order as soon as a slot and enough budget are free. Requests
// never share device buffers or reductions, so each one computes exactly
// what it would compute alone.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "task.hpp"

struct sc_server;

namespace sc {

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  TaskSpec spec;
  std::vector<double> f, g, u0;   // host copies (contiguous)
  int g_halo = 0;
  double* u_out = nullptr;
  size_t bytes = 0;               // device footprint charged to the budget
  double t_submit = 0, t_admit = 0;
  bool cancelled = false;
  double fake_seconds = 0;        // fake-device mode: modelled run time
};

enum SlotPhase { S_FREE, S_RUNNING, S_DRAINING };

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  SlotPhase phase = S_FREE;
  std::unique_ptr<Request> req;
  std::unique_ptr<SolveTask> task;
  void* staging = nullptr;        // f | g | u0/u_out, contiguous FP64
  size_t staging_bytes = 0;
  double fake_done_at = 0;
};

int64_t points(const TaskSpec& sp) { return sp.n[0] * sp.n[1] * sp.n[2]; }

int64_t ring_points(const TaskSpec& sp, int halo) {
  int64_t p = 1;
  for (int a = 0; a < sp.dim; ++a) p *= sp.n[a] + 2 * halo;
  return p;
}

}  // namespace

}  // namespace sc

struct sc_server {
  sc_server_opts opts{};
  bool inner_tol_set = false;  // the caller chose inner_tol (else each precision's default)
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_done;   // results available
  std::condition_variable cv_work;   // work for the worker
  std::deque<std::unique_ptr<sc::Request>> pending;
  std::vector<sc::Slot> slots;
  std::vector<sc_result> finished;
  std::map<uint64_t, sc::Request*> live;  // queued or resident, by id
  size_t used = 0;
  uint64_t next_id = 1;
  bool stop = false;
  int device = 0;
  std::thread worker;
  sc::Clock::time_point t0 = sc::Clock::now();

  double now() const { return std::chrono::duration<double>(sc::Clock::now() - t0).count(); }
  void run();
  void retire(sc::Slot& sl, sc_status st, const sc_solve_stats* stats);
  void admit_locked(std::vector<int>* newly);
  bool start_slot(sc::Slot& sl);
};

namespace sc {

namespace {

void emit_result(sc_server* S, const Request& r, sc_status st, const sc_solve_stats* stats) {
  sc_result res{};
  res.id = r.id;
  res.status = st;
  if (stats) {
    res.iterations = stats->iterations;
    res.outer = stats->outer;
    res.rel_residual = stats->rel_residual;
  }
  res.t_submit = r.t_submit;
  res.t_admit = r.t_admit;
  res.t_done = S->now();
  res.device_bytes = r.bytes;
  S->finished.push_back(res);
  S->live.erase(r.id);
}

}  // namespace

}  // namespace sc

void sc_server::retire(sc::Slot& sl, sc_status st, const sc_solve_stats* stats) {
  sl.task.reset();  // waits for the slot's stream, returns the workspace
  if (sl.staging) {
    if (sl.st) (void)hipStreamSynchronize(sl.st);
    sc::pool_free(sl.staging);
    sl.staging = nullptr;
  }
  std::lock_guard<std::mutex> g(mu);
  used -= sl.req->bytes;
  sc::emit_result(this, *sl.req, st, stats);
  sl.req.reset();
  sl.phase = sc::S_FREE;
  cv_done.notify_all();
}

// Admit queued requests in arrival order while a slot and budget are free.
void sc_server::admit_locked(std::vector<int>* newly) {
  for (size_t i = 0; i < slots.size() && !pending.empty(); ++i) {
    if (slots[i].phase != sc::S_FREE || slots[i].req) continue;
    while (!pending.empty()) {
      auto& head = pending.front();
      if (head->cancelled) {
        sc::emit_result(this, *head, SC_ECANCELLED, nullptr);
        pending.pop_front();
        cv_done.notify_all();
        continue;
      }
      if (head->bytes > budget) {
        sc::emit_result(this, *head, SC_ENOMEM, nullptr);
        pending.pop_front();
        cv_done.notify_all();
        continue;
      }
      break;
    }
    if (pending.empty()) break;
    if (used + pending.front()->bytes > budget) break;  // wait for memory
    used += pending.front()->bytes;
    pending.front()->t_admit = now();
    slots[i].req = std::move(pending.front());
    pending.pop_front();
    newly->push_back((int)i);
  }
}

// Stage the inputs and start the solve on the slot's stream.
bool sc_server::start_slot(sc::Slot& sl) {
  sc::Request& r = *sl.req;
  if (opts.fake_device) {
    sl.phase = sc::S_RUNNING;
    sl.fake_done_at = now() + r.fake_seconds;
    return true;
  }
  const int64_t np = sc::points(r.spec);
  const int64_t ng = r.g.empty() ? 0 : sc::ring_points(r.spec, r.g_halo);
  sl.staging_bytes = (size_t)(2 * np + ng) * sizeof(double) + 512;
  sl.staging = sc::pool_alloc(sl.staging_bytes);
  sc_status s = SC_ENOMEM;
  if (sl.staging) {
    double* f = static_cast<double*>(sl.staging);
    double* u = f + np;
    double* g = u + np;
    const int64_t p0 = r.spec.n[0], z0 = r.spec.n[0] * r.spec.n[1];
    bool ok = hipMemsetAsync(u, 0, np * sizeof(double), sl.st) == hipSuccess;
    if (ok && !r.f.empty()) ok = hipMemcpyAsync(f, r.f.data(), np * sizeof(double), hipMemcpyHostToDevice, sl.st) == hipSuccess;
    if (ok && !r.u0.empty())
      ok = hipMemcpyAsync(u, r.u0.data(), np * sizeof(double), hipMemcpyHostToDevice, sl.st) == hipSuccess;
    if (ok && ng) ok = hipMemcpyAsync(g, r.g.data(), ng * sizeof(double), hipMemcpyHostToDevice, sl.st) == hipSuccess;
    if (ok) {
      sl.task = std::make_unique<sc::SolveTask>();
      s = sl.task->init(r.spec, sl.st);
      if (s == SC_OK) {
        const sc::GridView uv{u, p0, z0};
        const sc::GridView fv{f, p0, z0};
        const int64_t gp = r.spec.n[0] + 2 * r.g_halo;
        const int64_t gz = gp * (r.spec.n[1] + 2 * r.g_halo);
        const int64_t goff = (r.spec.dim == 3 ? r.g_halo * gz : 0) + r.g_halo * gp + r.g_halo;
        const sc::GridView gv{g + goff, gp, gz};
        s = sl.task->start(uv, fv, ng ? &gv : nullptr);
      }
    } else {
      s = SC_EDEVICE;
      (void)hipGetLastError();
    }
  }
  if (s != SC_OK) {
    retire(sl, s, nullptr);
    return false;
  }
  (void)hipEventRecord(sl.ev, sl.st);
  sl.phase = sc::S_RUNNING;
  return true;
}

void sc_server::run() {
  if (!opts.fake_device) (void)hipSetDevice(device);
  for (;;) {
    std::vector<int> newly;
    {
      std::unique_lock<std::mutex> lk(mu);
      bool any_active = false;
      for (auto& sl : slots) any_active = any_active || sl.req != nullptr;
      if (stop && !any_active) {
        while (!pending.empty()) {
          sc::emit_result(this, *pending.front(), SC_ECANCELLED, nullptr);
          pending.pop_front();
        }
        cv_done.notify_all();
        break;
      }
      if (stop) {
        for (auto& q : pending) q->cancelled = true;
      }
      admit_locked(&newly);
      if (!any_active && newly.empty()) {
        cv_work.wait_for(lk, std::chrono::milliseconds(5));
        continue;
      }
    }
    for (int i : newly) start_slot(slots[i]);
    bool progress = !newly.empty();
    for (auto& sl : slots) {
      if (!sl.req) continue;
      bool cancelled;
      {
        std::lock_guard<std::mutex> g(mu);
        cancelled = sl.req->cancelled;
      }
      if (opts.fake_device) {
        if (cancelled) {
          retire(sl, SC_ECANCELLED, nullptr);
          progress = true;
        } else if (now() >= sl.fake_done_at) {
          sc_solve_stats st{};
          st.iterations = opts.solve.check_every;
          st.outer = 1;
          retire(sl, SC_OK, &st);
          progress = true;
        }
        continue;
      }
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipErrorNotReady) continue;
      progress = true;
      if (q != hipSuccess) {
        sc::set_error("device error in request %llu: %s", (unsigned long long)sl.req->id, hipGetErrorString(q));
        retire(sl, SC_EDEVICE, nullptr);
        continue;
      }
      if (sl.phase == sc::S_DRAINING) {
        retire(sl, sl.task->status(), &sl.task->stats());
        continue;
      }
      if (cancelled) {
        retire(sl, SC_ECANCELLED, nullptr);
        continue;
      }
      bool done = false;
      const sc_status s = sl.task->advance(&done);
      if (s != SC_OK) {
        retire(sl, s, nullptr);
        continue;
      }
      if (done) {
        const sc_status st = sl.task->status();
        if ((st == SC_OK || st == SC_ENOTCONV || st == SC_EBREAKDOWN) && sl.req->u_out) {
          const int64_t np = sc::points(sl.req->spec);
          double* u = static_cast<double*>(sl.staging) + np;
          const int64_t p0 = sl.req->spec.n[0], z0 = sl.req->spec.n[0] * sl.req->spec.n[1];
          if (sl.task->enqueue_copy_out(u, p0, z0) != SC_OK ||
              hipMemcpyAsync(sl.req->u_out, u, np * sizeof(double), hipMemcpyDeviceToHost, sl.st) != hipSuccess) {
            retire(sl, SC_EDEVICE, nullptr);
            continue;
          }
        }
        sl.phase = sc::S_DRAINING;
      }
      (void)hipEventRecord(sl.ev, sl.st);
    }
    if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

namespace sc {

namespace {

sc_status make_spec(const sc_server* S, const sc_request* r, Request* q) {
  if (!r || !r->op) {
    set_error("NULL request or operator");
    return SC_EINVAL;
  }
  if ((r->dim != 2 && r->dim != 3) || r->n[0] < 1 || r->n[1] < 1 || r->n[2] < 1 || (r->dim == 2 && r->n[2] != 1)) {
    set_error("bad request shape");
    return SC_EINVAL;
  }
  if (r->op->dim != r->dim) {
    set_error("operator dimension does not match the request");
    return SC_EINVAL;
  }
  TaskSpec& sp = q->spec;
  sp.o = S->opts.solve;
  if (r->precision != -1) {
    sc_status ps = check_precision(r->precision);
    if (ps != SC_OK) return ps;
    sc_solve_opts o = S->opts.solve;
    o.precision = r->precision;
    if (!S->inner_tol_set) o.inner_tol = 0.0;  // the default of the request's precision
    fill_opts(&o, &sp.o);
  }
  sp.dim = r->dim;
  sp.h = r->kind == SC_REQ_CH_STEP ? r->ch.h : r->h;
  for (int a = 0; a < 3; ++a) sp.n[a] = r->n[a];
  const int64_t np = r->n[0] * r->n[1] * r->n[2];
  sc_status s;
  if (r->kind == SC_REQ_BVP) {
    sp.kind = TASK_BVP;
    if (!r->f) {
      set_error("BVP request without forcing");
      return SC_EINVAL;
    }
    if ((s = make_kstencil(r->op, r->h, &sp.ksA)) != SC_OK) return s;
    q->f.assign(r->f, r->f + np);
    if (r->u0) q->u0.assign(r->u0, r->u0 + np);
    if (r->g) {
      q->g_halo = sp.ksA.R;
      int64_t ng = 1;
      for (int a = 0; a < r->dim; ++a) ng *= r->n[a] + 2 * q->g_halo;
      q->g.assign(r->g, r->g + ng);
    }
  } else if (r->kind == SC_REQ_CH_STEP) {
    sp.kind = TASK_CH;
    if (!r->u0) {
      set_error("Cahn-Hilliard request without u0");
      return SC_EINVAL;
    }
    if ((s = check_ch(r->op, &r->ch, r->dim)) != SC_OK) return s;
    if ((s = ch_operator(r->op, &r->ch, &sp.ksA, &sp.ksL)) != SC_OK) return s;
    sp.dt = r->ch.dt;
    sp.S = r->ch.S;
    q->u0.assign(r->u0, r->u0 + np);
  } else {
    set_error("unknown request kind %d", r->kind);
    return SC_EINVAL;
  }
  q->u_out = r->u_out;
  const int64_t ng = q->g.size();
  q->bytes = task_footprint(sp) + (((size_t)(2 * np + ng) * sizeof(double) + 512 + 4095) & ~(size_t)4095);
  q->fake_seconds = 2e-8 * (double)np;  // a modelled 20 ns per unknown
  return SC_OK;
}

}  // namespace

sc_status server_create(const sc_server_opts* opts, sc_server** out) {
  if (!opts || !out) {
    set_error("NULL argument");
    return SC_EINVAL;
  }
  *out = nullptr;
  if (opts->max_slots < 1 || opts->max_slots > 256) {
    set_error("max_slots must be in 1..256");
    return SC_EINVAL;
  }
  auto S = std::make_unique<sc_server>();
  S->opts = *opts;
  fill_opts(&opts->solve, &S->opts.solve);
  S->inner_tol_set = opts->solve.inner_tol > 0;
  if (check_opts(S->opts.solve) != SC_OK) return SC_EINVAL;
  S->slots.resize(opts->max_slots);
  if (!opts->fake_device) {
    SC_HIP_CHECK(hipGetDevice(&S->device));
    for (auto& sl : S->slots) {
      SC_HIP_CHECK(hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking));
      SC_HIP_CHECK(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    }
    size_t free_b = 0, total_b = 0;
    SC_HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
    S->budget = opts->hbm_budget ? (size_t)opts->hbm_budget : (size_t)(0.8 * (double)free_b);
  } else {
    S->budget = opts->hbm_budget ? (size_t)opts->hbm_budget : ((size_t)1 << 34);
  }
  S->worker = std::thread([p = S.get()] { p->run(); });
  *out = S.release();
  return SC_OK;
}

sc_status server_submit(sc_server* S, const sc_request* r, uint64_t* id) {
  if (!S || !id) {
    set_error("NULL argument");
    return SC_EINVAL;
  }
  auto q = std::make_unique<Request>();
  sc_status s = make_spec(S, r, q.get());
  if (s != SC_OK) return s;
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) {
    set_error("server is shutting down");
    return SC_EINVAL;
  }
  q->id = S->next_id++;
  q->t_submit = S->now();
  *id = q->id;
  S->live[q->id] = q.get();
  S->pending.push_back(std::move(q));
  S->cv_work.notify_one();
  return SC_OK;
}

sc_status server_poll(sc_server* S, sc_result* out, int32_t max, int32_t* n, int32_t wait_ms) {
  if (!S || !n || (max > 0 && !out)) {
    set_error("NULL argument");
    return SC_EINVAL;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->finished.empty() && wait_ms > 0)
    S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !S->finished.empty(); });
  const int32_t k = std::min<int32_t>(max, (int32_t)S->finished.size());
  for (int32_t i = 0; i < k; ++i) out[i] = S->finished[i];
  S->finished.erase(S->finished.begin(), S->finished.begin() + k);
  *n = k;
  return SC_OK;
}

sc_status server_cancel(sc_server* S, uint64_t id) {
  if (!S) {
    set_error("NULL server");
    return SC_EINVAL;
  }
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->live.find(id);
  if (it == S->live.end()) {
    set_error("request %llu is not queued or running", (unsigned long long)id);
    return SC_EINVAL;
  }
  it->second->cancelled = true;
  S->cv_work.notify_one();
  return SC_OK;
}

sc_status server_load(sc_server* S, int32_t* queued, int32_t* active, int32_t* fin, uint64_t* bytes) {
  if (!S) {
    set_error("NULL server");
    return SC_EINVAL;
  }
  std::lock_guard<std::mutex> g(S->mu);
  int32_t a = 0;
  for (auto& sl : S->slots) a += sl.req ? 1 : 0;
  if (queued) *queued = (int32_t)S->pending.size();
  if (active) *active = a;
  if (fin) *fin = (int32_t)S->finished.size();
  if (bytes) *bytes = S->used;
  return SC_OK;
}

void server_destroy(sc_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  for (auto& sl : S->slots) {
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
  }
  delete S;
}

}  // namespace sc
