// Serving: a persistent request loop that keeps the grids and operators of the
// admitted requests on the device and overlaps their work.
//
// Requests queue on submission.  Worker threads (each owning a share of the
// slots, each slot with its own stream and pinned history buffer) admit them
// in arrival order, skipping ahead to later requests that fit when the head
// does not, as long as one of the worker's slots is free and the request's
// workspace fits in the free part of the HBM budget.  The budget is reserved
// on the device once, when the server starts, and workspaces are carved from
// it, so admission and retirement allocate and free nothing on the device.
// An admitted request's grid is created, its operators built and its cycles
// enqueued in batches (replayed HIP graphs) without blocking the worker; the
// worker polls each of its active requests' batch event, sets up the next
// batch or retires the request (solution copied out, memory returned to the
// budget) and admits waiting requests as slots and memory free up.  Each
// request's arithmetic is exactly the single-grid path, so a result does not
// depend on what else is in the mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qmg_internal.hpp"

using namespace qmg;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

thread_local std::string g_server_err;

constexpr int kServerWorkers = 8;  // host threads driving the slots

struct Req {
  uint64_t id = 0;
  qmg_grid_desc desc{};
  qmg_solver_opts opts{};
  std::vector<double> eps, f;
  double tol = 1e-8;
  int max_cycles = 0;
  size_t bytes = 0;
  double t_submit = 0, t_arrive = 0, t_admit = 0, t_done = 0;
  int state = 0;  // 0 queued, 1 active, 2 done
  bool deferred = false;  // arrived and found no slot or memory at least once
  int status = QMG_OK;
  std::string err;
  qmg_grid_t* g = nullptr;
  int slot = -1;
  size_t off = 0;  // workspace offset in the server's arena
  SolveState st;
  std::vector<double> u;
  qmg_solve_report rep{};
};

}  // namespace

struct qmg_server {
  size_t budget = 0, in_use = 0, peak = 0;
  double t0 = 0;                            // server clock origin (arrival times count from it)
  hipStream_t user = nullptr;               // the caller's stream (nullable)
  int max_slots = 0;
  int device = 0;
  int nworkers = 1;
  std::vector<hipStream_t> streams;
  std::vector<double*> hist;                // pinned residual history per slot
  std::vector<std::vector<int>> slot_free;  // per worker; slot s belongs to worker s % nworkers
  char* arena = nullptr;                    // the budget, reserved on the device
  std::map<size_t, size_t> holes;           // free arena ranges: offset -> size
  std::mutex mu;
  std::condition_variable cv_done, cv_work;
  std::deque<Req*> queue;
  std::vector<Req*> active;
  std::unordered_map<uint64_t, Req*> all;
  uint64_t next_id = 1;
  int64_t submitted = 0, completed = 0, failed = 0, deferred = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::string err;
};

namespace {

constexpr size_t kArenaAlign = 256;

size_t arena_size(size_t bytes) { return (bytes + kArenaAlign - 1) & ~(kArenaAlign - 1); }

// First fit in the arena (caller holds the lock); false when no hole is large
// enough (fragmentation: the request waits like one over the budget).
bool arena_take(qmg_server* s, size_t bytes, size_t* off) {
  const size_t need = arena_size(bytes);
  for (auto it = s->holes.begin(); it != s->holes.end(); ++it) {
    if (it->second < need) continue;
    *off = it->first;
    const size_t rest = it->second - need;
    const size_t at = it->first + need;
    s->holes.erase(it);
    if (rest > 0) s->holes[at] = rest;
    return true;
  }
  return false;
}

// Returns a range to the arena, merging it with its free neighbours.
void arena_give(qmg_server* s, size_t off, size_t bytes) {
  size_t size = arena_size(bytes);
  auto next = s->holes.lower_bound(off);
  if (next != s->holes.end() && off + size == next->first) {
    size += next->second;
    next = s->holes.erase(next);
  }
  if (next != s->holes.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += size;
      return;
    }
  }
  s->holes[off] = size;
}

void fail(Req* r, int code, const std::string& msg) {
  if (r->status == QMG_OK) {
    r->status = code;
    r->err = msg;
  }
}

void release_grid(Req* r) {
  if (r->g) {
    qmg_destroy_grid(r->g);
    r->g = nullptr;
  }
}

// Creates, fills and builds the grid of an admitted request and enqueues its
// first batch; any error retires the request with that status.
void start(qmg_server* s, Req* r) {
  const int rc = [&]() -> int {
    int c = create_grid(&r->desc, &r->opts, s->arena + r->off, r->bytes, s->streams[r->slot], s->hist[r->slot],
                        &r->g);
    if (c != QMG_OK) return c;
    c = qmg_set_coefficients(r->g, r->eps.data(), 1, r->f.data(), QMG_HOST);
    if (c != QMG_OK) return c;
    c = qmg_build_operators(r->g, nullptr);
    if (c != QMG_OK) return c;
    try {
      solve_begin(r->g, r->st, r->tol, r->max_cycles);
      if (!r->st.done) solve_enqueue(r->g, r->st);
    } catch (const ApiError& e) {
      fail(r, e.code, e.what());
      return e.code;
    } catch (const std::exception& e) {
      fail(r, QMG_EHIP, e.what());
      return QMG_EHIP;
    }
    return QMG_OK;
  }();
  if (rc != QMG_OK) fail(r, rc, r->g ? qmg_last_error(r->g) : qmg_last_error(nullptr));
  r->eps.clear();
  r->eps.shrink_to_fit();
  r->f.clear();
  r->f.shrink_to_fit();
}

// Copies the solution out, frees the device memory and marks the request done.
void finish(qmg_server* s, Req* r) {
  if (r->g && r->status == QMG_OK) {
    int64_t nu = 0;
    qmg_sizes(r->g, &nu, nullptr, nullptr);
    r->u.resize((size_t)nu);
    const int c = qmg_get_solution(r->g, r->u.data(), QMG_HOST);
    if (c != QMG_OK) fail(r, c, qmg_last_error(r->g));
    solve_fill_report(r->g, r->st, &r->rep);
    if (!(r->st.rr <= r->tol)) fail(r, QMG_ENOTCONV, "tolerance not reached");
  }
  release_grid(r);
  std::lock_guard<std::mutex> lk(s->mu);
  r->t_done = now_s();
  r->state = 2;
  s->in_use -= r->bytes;
  arena_give(s, r->off, r->bytes);
  s->slot_free[r->slot % s->nworkers].push_back(r->slot);
  s->active.erase(std::remove(s->active.begin(), s->active.end(), r), s->active.end());
  ++s->completed;
  if (r->status != QMG_OK) ++s->failed;
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

// Worker w drives the slots s with s % nworkers == w.
void loop(qmg_server* s, int w) {
  (void)hipSetDevice(s->device);
  std::vector<int>& mine = s->slot_free[w];
  for (;;) {
    std::vector<Req*> admitted, running;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop && s->queue.empty() && s->active.empty()) break;
      const double tnow = now_s();
      for (auto it = s->queue.begin(); it != s->queue.end() && !mine.empty();) {
        Req* r = *it;
        size_t off = 0;
        if (r->t_arrive <= tnow && s->in_use + r->bytes <= s->budget && arena_take(s, r->bytes, &off)) {
          r->off = off;
          r->slot = mine.back();
          mine.pop_back();
          s->in_use += r->bytes;
          s->peak = std::max(s->peak, s->in_use);
          r->state = 1;
          r->t_admit = now_s();
          s->active.push_back(r);
          admitted.push_back(r);
          it = s->queue.erase(it);
        } else {
          if (r->t_arrive <= tnow && !r->deferred) {  // arrived, but no memory for it
            r->deferred = true;
            ++s->deferred;
          }
          ++it;
        }
      }
      size_t free_slots = 0;
      for (const std::vector<int>& f : s->slot_free) free_slots += f.size();
      if (free_slots == 0)  // arrived, but every slot is busy
        for (Req* r : s->queue)
          if (!r->deferred && r->t_arrive <= tnow) {
            r->deferred = true;
            ++s->deferred;
          }
      for (Req* r : s->active)
        if (r->slot % s->nworkers == w) running.push_back(r);
    }
    bool progress = !admitted.empty();
    for (Req* r : admitted) {
      start(s, r);
      if (r->status != QMG_OK || r->st.done) finish(s, r);
    }
    for (Req* r : running) {
      if (std::find(admitted.begin(), admitted.end(), r) != admitted.end()) continue;
      try {
        if (!solve_ready(r->g)) continue;
        progress = true;
        solve_collect(r->g, r->st);
        if (r->st.done) finish(s, r);
        else solve_enqueue(r->g, r->st);
      } catch (const ApiError& e) {
        fail(r, e.code, e.what());
        finish(s, r);
      } catch (const std::exception& e) {
        fail(r, QMG_EHIP, e.what());
        finish(s, r);
      }
    }
    if (!progress) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait_for(lk, std::chrono::microseconds(50));
    }
  }
}

template <class F>
int sguard(qmg_server* s, F&& f) {
  try {
    f();
    return QMG_OK;
  } catch (const ApiError& e) {
    g_server_err = e.what();
    if (s) s->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_server_err = e.what();
    if (s) s->err = e.what();
    return QMG_EHIP;
  }
}

}  // namespace

extern "C" {

int qmg_server_create(size_t hbm_budget, int max_slots, void* stream, qmg_server_t** out) {
  return sguard(nullptr, [&] {
    if (!out) throw ApiError(QMG_EINVAL, "null output handle");
    if (max_slots < 1 || max_slots > 256) throw ApiError(QMG_EINVAL, "max_slots must lie in 1..256");
    if (hbm_budget == 0) throw ApiError(QMG_EINVAL, "zero HBM budget");
    qmg_server* s = new qmg_server();
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    s->user = (hipStream_t)stream;
    s->nworkers = std::min(max_slots, kServerWorkers);
    auto release = [s] {
      for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
      for (double* h : s->hist) (void)hipHostFree(h);
      if (s->arena) (void)hipFree(s->arena);
    };
    try {
      QMG_HIP(hipGetDevice(&s->device));
      void* p = nullptr;
      if (hipMalloc(&p, hbm_budget) != hipSuccess) {
        (void)hipGetLastError();
        throw ApiError(QMG_ENOMEM, "cannot reserve the HBM budget of " + std::to_string(hbm_budget) + " bytes");
      }
      s->arena = (char*)p;
      s->holes[0] = hbm_budget & ~(kArenaAlign - 1);
      s->slot_free.resize(s->nworkers);
      for (int i = 0; i < max_slots; ++i) {
        hipStream_t st = nullptr;
        QMG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        s->streams.push_back(st);
        double* h = nullptr;
        QMG_HIP(hipHostMalloc((void**)&h, kHistCap * sizeof(double), hipHostMallocDefault));
        s->hist.push_back(h);
      }
      if (s->user) {  // served work starts after what the caller enqueued before
        hipEvent_t ev = nullptr;
        QMG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        QMG_HIP(hipEventRecord(ev, s->user));
        for (hipStream_t st : s->streams) QMG_HIP(hipStreamWaitEvent(st, ev, 0));
        QMG_HIP(hipEventDestroy(ev));
      }
      for (int i = max_slots - 1; i >= 0; --i) s->slot_free[i % s->nworkers].push_back(i);
      s->t0 = now_s();
      for (int w = 0; w < s->nworkers; ++w) s->workers.emplace_back(loop, s, w);
    } catch (...) {
      release();
      delete s;
      throw;
    }
    *out = s;
  });
}

int qmg_server_submit(qmg_server_t* s, const qmg_grid_desc* desc, const qmg_solver_opts* opts,
                      const double* eps, const double* f, double rel_tol, int max_cycles,
                      double t_arrival, uint64_t* ticket) {
  return sguard(s, [&] {
    if (!s || !desc || !opts || !eps || !f || !ticket) throw ApiError(QMG_EINVAL, "null argument");
    if (!(rel_tol >= 0.0) || max_cycles < 0) throw ApiError(QMG_EINVAL, "bad tolerance or cycle limit");
    if (std::isnan(t_arrival)) throw ApiError(QMG_EINVAL, "arrival time is NaN");
    if (desc->base_level != 0 && desc->base_level != desc->max_level)
      throw ApiError(QMG_EINVAL, "the server takes regular grids");
    size_t bytes = 0;
    const int rc = qmg_workspace_bytes(desc, opts, &bytes);
    if (rc != QMG_OK) throw ApiError(rc, qmg_last_error(nullptr));
    if (bytes > s->budget) throw ApiError(QMG_EINVAL, "request workspace exceeds the whole HBM budget");
    Req* r = new Req();
    r->desc = *desc;
    r->desc.refine = nullptr;
    r->desc.regions = nullptr;
    r->desc.n_regions = 0;
    r->opts = *opts;
    int64_t nc = 1, cells = 1, unk = 1;
    for (int i = 0; i < desc->max_level; ++i) nc *= 3;
    for (int i = 0; i < desc->dim; ++i) {
      cells *= nc;
      unk *= nc - 1;
    }
    r->eps.assign(eps, eps + cells);
    r->f.assign(f, f + unk);
    r->tol = rel_tol;
    r->max_cycles = max_cycles;
    r->bytes = bytes;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete r;
      throw ApiError(QMG_ESTATE, "server is shutting down");
    }
    r->id = s->next_id++;
    r->t_submit = now_s();
    r->t_arrive = t_arrival >= 0.0 ? s->t0 + t_arrival : r->t_submit;
    s->queue.push_back(r);
    s->all[r->id] = r;
    ++s->submitted;
    *ticket = r->id;
    s->cv_work.notify_all();
  });
}

int qmg_server_poll(qmg_server_t* s, uint64_t ticket, int* done, double* u_out,
                    qmg_solve_report* report, double* latency_s) {
  int status = QMG_OK;
  const int rc = sguard(s, [&] {
    if (!s || !done) throw ApiError(QMG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) throw ApiError(QMG_EINVAL, "unknown or already collected ticket");
    Req* r = it->second;
    *done = r->state == 2;
    if (!*done) return;
    if (u_out && !r->u.empty()) std::memcpy(u_out, r->u.data(), r->u.size() * sizeof(double));
    if (report) *report = r->rep;
    if (latency_s) *latency_s = r->t_done - r->t_arrive;
    status = r->status;
    if (status != QMG_OK) {
      g_server_err = r->err;
      s->err = r->err;
    }
    s->all.erase(it);
    delete r;
  });
  return rc != QMG_OK ? rc : status;
}

int qmg_server_drain(qmg_server_t* s) {
  return sguard(s, [&] {
    if (!s) throw ApiError(QMG_EINVAL, "null server");
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_done.wait(lk, [&] { return s->queue.empty() && s->active.empty(); });
    }
    if (s->user) {  // later work on the caller's stream follows the served work
      for (hipStream_t st : s->streams) {
        hipEvent_t ev = nullptr;
        QMG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        QMG_HIP(hipEventRecord(ev, st));
        QMG_HIP(hipStreamWaitEvent(s->user, ev, 0));
        QMG_HIP(hipEventDestroy(ev));
      }
    }
  });
}

int qmg_server_stats(qmg_server_t* s, qmg_server_stats_t* st) {
  return sguard(s, [&] {
    if (!s || !st) throw ApiError(QMG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->active = (int64_t)s->active.size();
    st->queued = (int64_t)s->queue.size();
    st->deferred = s->deferred;
    st->hbm_budget = s->budget;
    st->hbm_in_use = s->in_use;
    st->hbm_peak = s->peak;
    st->max_slots = s->max_slots;
  });
}

const char* qmg_server_last_error(const qmg_server_t* s) {
  if (s) return s->err.c_str();
  return g_server_err.c_str();
}

int qmg_server_destroy(qmg_server_t* s) {
  if (!s) return QMG_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // requests not yet admitted are dropped
    for (Req* r : s->queue) {
      s->all.erase(r->id);
      delete r;
    }
    s->queue.clear();
    s->cv_work.notify_all();
  }
  for (std::thread& t : s->workers)
    if (t.joinable()) t.join();
  for (auto& kv : s->all) {
    release_grid(kv.second);
    delete kv.second;
  }
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  for (double* h : s->hist) (void)hipHostFree(h);
  if (s->arena) (void)hipFree(s->arena);
  delete s;
  return QMG_OK;
}

}  // extern "C"
