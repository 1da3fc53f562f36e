// Serving loop of libmlc (the mlc_server_* calls of include/mlc.h).
//
// Built only on the public C ABI: a request queue filled by the caller, one
// host thread that builds plans on first use, admits queued requests in
// arrival order when a stream slot and arena memory are free, launches the
// head request together with the queued requests of its patch-work class
// through mlc_solve_batched, and retires launches by polling their end
// events.  Launches on different streams overlap on the device, so requests
// that arrive while others run start as soon as a slot and memory free up
// (continuous batching), without waiting for the running ones.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/mlc.h"

// libmlc.hip internals used here
void mlc_set_error(mlc_context* ctx, const std::string& msg);
int mlc_context_device(const mlc_context* ctx);
bool mlc_budget_take(mlc_context* ctx, size_t bytes);
void mlc_budget_give(mlc_context* ctx, size_t bytes);
bool mlc_check_enabled();
mlc_status mlc_check_charge(mlc_context* ctx, const double* f, const mlc_plan_info& I, void* stream);

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// A plan serves exactly one problem description.
using PlanKey = std::tuple<int, double, int, double, double, int, int, int, int, int, int, int, double, double,
                           double, int, int, int, int, int>;
PlanKey plan_key(const mlc_problem& p) {
  // levels and the coarser radii as given: 0 and 2 both mean two levels, and
  // a 0 radius equals the finer level's, so equal problems may still get two
  // plans (never one plan for two different problems)
  return PlanKey{p.n_cells, p.h, p.patch, p.alpha, p.beta, p.P, p.Q, p.interp_b, p.conv_precision, p.fft_size,
                 p.dgf_half_width, p.levels, p.level_alpha[0], p.level_alpha[1], p.level_alpha[2], p.rhs_order,
                 p.skip_empty, p.box_cells[0], p.box_cells[1], p.box_cells[2]};
}

// Requests whose patch-level work is identical may share a launch.
bool same_class(const mlc_plan_info& a, const mlc_plan_info& b) {
  return a.n == b.n && a.d_alpha == b.d_alpha && a.d_beta == b.d_beta && a.P == b.P && a.Q == b.Q &&
         a.b == b.b && a.conv_precision == b.conv_precision && a.M == b.M && a.Z == b.Z;
}

constexpr size_t kAlign = 256;
size_t round_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit sub-allocator over the device arena (offsets only).
class Arena {
 public:
  void reset(size_t n) {
    free_.clear();
    if (n) free_[0] = n;
  }
  bool alloc(size_t n, size_t* off) {
    n = round_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, next = it->first + n;
      free_.erase(it);
      if (rest) free_[next] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = round_up(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;   // offset -> length
};

enum State { QUEUED = 0, RUNNING = 1, FINISHED = 2 };

struct Request {
  uint64_t ticket = 0;
  mlc_problem prob{};
  mlc_plan_info info{};
  const double* f = nullptr;
  double* phi = nullptr;
  Clock::time_point t_submit, t_launch, t_done;
  double device_ms = 0.0;
  int batch = 0;
  mlc_status status = MLC_OK;
  State state = QUEUED;
};

struct Launch {
  std::vector<Request*> reqs;
  int stream = 0;
  size_t off = 0, bytes = 0;
  hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace

struct mlc_server {
  mlc_context* ctx = nullptr;
  mlc_server_config cfg{};
  int device = 0;
  // shared between the caller and the server thread
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> tickets;
  uint64_t next_ticket = 1;
  int64_t unfinished = 0;
  bool stop = false;
  // plans: built by the server thread or by mlc_server_prepare
  std::mutex plans_mu;
  std::map<PlanKey, mlc_plan*> plans;
  // owned by the server thread after start
  char* arena_base = nullptr;
  size_t arena_bytes = 0;
  Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<char> stream_busy;
  std::vector<Launch> running;
  std::vector<hipEvent_t> events;
  std::thread worker;
};

namespace {

mlc_plan* plan_for(mlc_server* S, const mlc_problem& p, mlc_status* st) {
  std::lock_guard<std::mutex> lk(S->plans_mu);
  const PlanKey key = plan_key(p);
  auto it = S->plans.find(key);
  if (it != S->plans.end()) return it->second;
  mlc_plan* P = nullptr;
  *st = mlc_plan_create(S->ctx, &p, &P);
  if (*st != MLC_OK) return nullptr;
  S->plans[key] = P;
  return P;
}

hipEvent_t take_event(mlc_server* S) {
  if (!S->events.empty()) {
    hipEvent_t e = S->events.back();
    S->events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

void finish_locked(mlc_server* S, Request* r, mlc_status st, Clock::time_point now) {
  r->status = st;
  r->t_done = now;
  r->state = FINISHED;
  --S->unfinished;
}

void remove_from_queue_locked(mlc_server* S, Request* r) {
  for (auto it = S->queue.begin(); it != S->queue.end(); ++it)
    if (*it == r) { S->queue.erase(it); return; }
}

// Retire every launch whose end event has completed.
void retire(mlc_server* S) {
  for (size_t i = 0; i < S->running.size();) {
    Launch& L = S->running[i];
    hipError_t q = hipEventQuery(L.b);
    if (q == hipErrorNotReady) { ++i; continue; }
    float ms = 0.0f;
    mlc_status st = MLC_OK;
    if (q == hipSuccess) {
      hipEventElapsedTime(&ms, L.a, L.b);
    } else {
      st = MLC_ERR_DEVICE;
      mlc_set_error(S->ctx, std::string("server launch: ") + hipGetErrorString(q));
    }
    const auto now = Clock::now();
    S->arena.release(L.off, L.bytes);
    S->stream_busy[L.stream] = 0;
    S->events.push_back(L.a);
    S->events.push_back(L.b);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (Request* r : L.reqs) {
        r->device_ms = ms;
        finish_locked(S, r, st, now);
      }
    }
    S->cv_done.notify_all();
    S->running.erase(S->running.begin() + long(i));
  }
}

// Try to start one launch; true if one was started (or requests failed).
bool admit(mlc_server* S) {
  int stream = -1;
  for (int k = 0; k < int(S->streams.size()); ++k)
    if (!S->stream_busy[k]) { stream = k; break; }
  if (stream < 0) return false;
  std::vector<Request*> group;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->queue.empty()) return false;
    Request* head = S->queue.front();
    group.push_back(head);
    for (auto it = S->queue.begin() + 1; it != S->queue.end() && int(group.size()) < S->cfg.max_batch; ++it)
      if (same_class(head->info, (*it)->info)) group.push_back(*it);
  }
  // plans (a first use builds one: slow, and outside the queue lock); with
  // MLC_CHECK each request's charge is checked alone, so that a bad one
  // fails by itself and not the launch it would have joined
  std::vector<mlc_plan*> plans;
  std::vector<Request*> ok;
  bool failed = false;
  const bool check = mlc_check_enabled();
  for (Request* r : group) {
    mlc_status st = MLC_OK;
    mlc_plan* P = plan_for(S, r->prob, &st);
    size_t own = 0;
    if (P && mlc_plan_workspace_bytes(P, &own) == MLC_OK && round_up(own) > S->arena_bytes) {
      mlc_set_error(S->ctx, "request workspace exceeds the server's workspace budget");
      st = MLC_ERR_OUT_OF_MEMORY;
      P = nullptr;
    }
    if (P && check) st = mlc_check_charge(S->ctx, r->f, r->info, S->streams[stream]);
    if (!P || st != MLC_OK) {
      std::lock_guard<std::mutex> lk(S->mu);
      remove_from_queue_locked(S, r);
      finish_locked(S, r, st, Clock::now());
      failed = true;
      continue;
    }
    {
      // the plan's sizes (its torus may be autotuned) decide the class of
      // later groupings
      std::lock_guard<std::mutex> lk(S->mu);
      mlc_plan_get_info(P, &r->info);
    }
    plans.push_back(P);
    ok.push_back(r);
  }
  if (failed) S->cv_done.notify_all();
  // the largest prefix of the group whose workspace fits in the arena now
  size_t off = 0, need = 0;
  while (!ok.empty()) {
    if (mlc_batch_workspace_bytes(int32_t(ok.size()), plans.data(), &need) == MLC_OK && S->arena.alloc(need, &off))
      break;
    ok.pop_back();
    plans.pop_back();
  }
  if (ok.empty()) return failed;
  const auto now = Clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (Request* r : ok) {
      remove_from_queue_locked(S, r);
      r->state = RUNNING;
      r->t_launch = now;
      r->batch = int(ok.size());
    }
  }
  Launch L;
  L.reqs = ok;
  L.stream = stream;
  L.off = off;
  L.bytes = need;
  L.a = take_event(S);
  L.b = take_event(S);
  std::vector<const double*> fs;
  std::vector<double*> phis;
  for (Request* r : ok) {
    fs.push_back(r->f);
    phis.push_back(r->phi);
  }
  hipStream_t s = S->streams[stream];
  hipEventRecord(L.a, s);
  mlc_status st = mlc_solve_batched(int32_t(ok.size()), plans.data(), fs.data(), phis.data(),
                                    S->arena_base + off, need, s);
  hipEventRecord(L.b, s);
  if (st != MLC_OK) {
    // wait for whatever part of the solve was enqueued before the arena is reused
    hipStreamSynchronize(s);
    S->arena.release(off, need);
    S->events.push_back(L.a);
    S->events.push_back(L.b);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (Request* r : ok) finish_locked(S, r, st, Clock::now());
    }
    S->cv_done.notify_all();
    return true;
  }
  S->stream_busy[stream] = 1;
  S->running.push_back(L);
  return true;
}

void worker_main(mlc_server* S) {
  hipSetDevice(S->device);
  for (;;) {
    retire(S);
    if (admit(S)) continue;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->running.empty()) {
      // idle: sleep until a request arrives or the server stops
      if (S->queue.empty() && S->stop) break;
      S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
      if (S->queue.empty() && S->stop) break;
    } else {
      // launches in flight: look at their events again shortly
      S->cv_work.wait_for(lk, std::chrono::microseconds(50));
    }
  }
}

}  // namespace

extern "C" mlc_status mlc_server_create(mlc_context* ctx, const mlc_server_config* cfg, mlc_server** out) {
  if (!ctx || !out) return MLC_ERR_INVALID_ARG;
  mlc_server_config c{};
  if (cfg) c = *cfg;
  if (c.streams < 0 || c.streams > 8 || c.max_batch < 0 || c.max_queue < 0) {
    mlc_set_error(ctx, "server config out of range");
    return MLC_ERR_INVALID_ARG;
  }
  if (c.workspace_budget_bytes == 0) c.workspace_budget_bytes = size_t(16) << 30;
  if (c.streams == 0) c.streams = 2;
  if (c.max_batch == 0) c.max_batch = 16;
  if (c.max_queue == 0) c.max_queue = 4096;
  const int device = mlc_context_device(ctx);
  if (hipSetDevice(device) != hipSuccess) return MLC_ERR_DEVICE;
  auto* S = new (std::nothrow) mlc_server;
  if (!S) return MLC_ERR_OUT_OF_MEMORY;
  S->ctx = ctx;
  S->cfg = c;
  S->device = device;
  S->arena_bytes = round_up(c.workspace_budget_bytes);
  if (!mlc_budget_take(ctx, S->arena_bytes)) {
    delete S;
    mlc_set_error(ctx, "server arena exceeds the context's budget");
    return MLC_ERR_OUT_OF_MEMORY;
  }
  if (hipMalloc(reinterpret_cast<void**>(&S->arena_base), S->arena_bytes) != hipSuccess) {
    mlc_budget_give(ctx, S->arena_bytes);
    delete S;
    mlc_set_error(ctx, "server arena allocation failed");
    return MLC_ERR_OUT_OF_MEMORY;
  }
  S->arena.reset(S->arena_bytes);
  for (int k = 0; k < c.streams; ++k) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t t : S->streams) hipStreamDestroy(t);
      hipFree(S->arena_base);
      mlc_budget_give(ctx, S->arena_bytes);
      delete S;
      mlc_set_error(ctx, "server stream creation failed");
      return MLC_ERR_DEVICE;
    }
    S->streams.push_back(s);
  }
  S->stream_busy.assign(c.streams, 0);
  S->worker = std::thread(worker_main, S);
  *out = S;
  return MLC_OK;
}

extern "C" mlc_status mlc_server_prepare(mlc_server* srv, const mlc_problem* prob) {
  if (!srv || !prob) return MLC_ERR_INVALID_ARG;
  if (prob->max_live > 0) {
    mlc_set_error(srv->ctx, "the server batches its requests: max_live plans solve alone (mlc_solve)");
    return MLC_ERR_UNSUPPORTED;
  }
  mlc_status st = MLC_OK;
  return plan_for(srv, *prob, &st) ? MLC_OK : st;
}

extern "C" mlc_status mlc_server_submit(mlc_server* srv, const mlc_problem* prob, const double* f, double* phi,
                                        uint64_t* ticket) {
  if (!srv || !prob || !f || !phi || !ticket) return MLC_ERR_INVALID_ARG;
  if (prob->max_live > 0) {
    mlc_set_error(srv->ctx, "the server batches its requests: max_live plans solve alone (mlc_solve)");
    return MLC_ERR_UNSUPPORTED;
  }
  mlc_plan_info info{};
  mlc_status st = mlc_problem_info(prob, &info);
  if (st != MLC_OK) return st;
  size_t ws = 0;
  st = mlc_problem_workspace_bytes(prob, &ws);
  if (st != MLC_OK) return st;
  if (round_up(ws) > srv->arena_bytes) {
    mlc_set_error(srv->ctx, "request workspace exceeds the server's workspace budget");
    return MLC_ERR_OUT_OF_MEMORY;
  }
  auto* r = new (std::nothrow) Request;
  if (!r) return MLC_ERR_OUT_OF_MEMORY;
  r->prob = *prob;
  r->info = info;
  r->f = f;
  r->phi = phi;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->unfinished >= srv->cfg.max_queue) {
      delete r;
      return MLC_ERR_BUSY;
    }
    r->ticket = srv->next_ticket++;
    srv->queue.push_back(r);
    srv->tickets[r->ticket] = r;
    ++srv->unfinished;
    *ticket = r->ticket;
  }
  srv->cv_work.notify_one();
  return MLC_OK;
}

extern "C" mlc_status mlc_server_poll(mlc_server* srv, uint64_t ticket, int32_t* done, mlc_timing* t) {
  if (!srv || !done) return MLC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return MLC_ERR_INVALID_ARG;
  Request* r = it->second;
  if (r->state != FINISHED) {
    *done = 0;
    return MLC_ERR_NOT_READY;
  }
  *done = 1;
  if (t) {
    t->status = r->status;
    t->batch_size = r->batch;
    t->queue_ms = r->batch ? ms_between(r->t_submit, r->t_launch) : ms_between(r->t_submit, r->t_done);
    t->device_ms = r->device_ms;
    t->total_ms = ms_between(r->t_submit, r->t_done);
  }
  const mlc_status st = r->status;
  srv->tickets.erase(it);
  delete r;
  return st;
}

extern "C" mlc_status mlc_server_drain(mlc_server* srv) {
  if (!srv) return MLC_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] { return srv->unfinished == 0; });
  return MLC_OK;
}

extern "C" mlc_status mlc_server_destroy(mlc_server* srv) {
  if (!srv) return MLC_ERR_INVALID_ARG;
  mlc_server_drain(srv);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  for (auto& kv : srv->plans) mlc_plan_destroy(kv.second);
  for (hipEvent_t e : srv->events) hipEventDestroy(e);
  for (hipStream_t s : srv->streams) hipStreamDestroy(s);
  hipFree(srv->arena_base);
  mlc_budget_give(srv->ctx, srv->arena_bytes);
  for (auto& kv : srv->tickets) delete kv.second;
  delete srv;
  return MLC_OK;
}
