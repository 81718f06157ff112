// Solve server with continuous batching (pserve_* in include/pcheb.h).
//
// Requests that share an operator and parameters form a group: one resident
// handle (operator data, bounds, workspace for `cap` right-hand sides), one
// stream, and a slot table.  A set-up thread builds groups (allocation and the
// bound estimate) while a worker thread loops over
//   * cancellations and completions (non-blocking event queries),
//   * admission of queued requests into free slots; a request without a group
//     reserves the group's memory (evicting idle groups, least recently used,
//     when the budget requires) and queues its set-up,
//   * one launch of a pair of PCG iterations per group with work in flight,
//     replayed from the handle's HIP graph over all of the group's slots.
// A slot's scalars and stop flag live on the device; a slot joins between
// launches (its start kernels are ordered on the group stream) and leaves
// when its readback shows it finished: then its true residual is computed and
// its solution copied to the caller.  Idle slots are marked finished, so the
// launches skip them.  Every right-hand side sees the same kernels and the
// same reduction order whatever else runs, so its result is the same alone or
// batched.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "handle.hpp"
#include "rng.hpp"
#include "solver.hpp"

namespace pcheb {

using Clock = std::chrono::steady_clock;

enum class RState { Queued, Active, Draining, Done };

struct Request {
  uint64_t id = 0;
  pserve_request req{};
  RState state = RState::Queued;
  Clock::time_point t_submit;
  pcg_stats stats{};
  pcheb_status result = PCHEB_PENDING;
  int group = -1;
  int slot = -1;
  bool cancel = false;
  std::string error;
};

struct GroupKey {
  pcheb_operator op;
  int32_t k, prec, fuse;
  double lmin, lmax, s;
  uint64_t op_key;
  bool operator==(const GroupKey& o) const {
    const pcheb_operator &a = op, &b = o.op;
    const bool same_op = a.kind == b.kind && a.n == b.n && a.rowptr == b.rowptr && a.colind == b.colind &&
                         a.values == b.values && a.nnz == b.nnz && a.nx == b.nx && a.ny == b.ny && a.nz == b.nz &&
                         a.cell_coeff == b.cell_coeff && a.sell_C == b.sell_C && a.sell_sigma == b.sell_sigma;
    return same_op && k == o.k && prec == o.prec && fuse == o.fuse && lmin == o.lmin && lmax == o.lmax && s == o.s &&
           op_key == o.op_key;
  }
};

static GroupKey key_of(const pserve_request& r) {
  GroupKey g{};
  g.op = r.op;
  g.k = r.k;
  g.prec = r.prec;
  g.fuse = r.fuse_steps;
  g.lmin = r.lambda_max > 0 ? r.lambda_min : 0.0;
  g.lmax = r.lambda_max > 0 ? r.lambda_max : 0.0;
  g.s = r.theta_scale;
  g.op_key = r.op_key;
  return g;
}

struct Group {
  GroupKey key;
  Handle* h = nullptr;
  hipStream_t stream = nullptr;
  double* X = nullptr;  // cap vectors, stride ldw (solutions)
  double* B = nullptr;  // cap vectors, stride ldw (right-hand sides)
  DeviceBuffer xb, bb;  // the blocks of X and B
  int cap = 0;
  std::vector<uint64_t> slot_req;       // request id, 0 = free
  std::vector<int64_t> slot_since;      // launch sequence number when the slot joined
  std::vector<int> slot_draining;       // 1 while its completion is in flight
  std::vector<hipEvent_t> slot_ev;      // completion copy done
  DevState* poll = nullptr;             // pinned: states after the last launch
  DevState* fin = nullptr;              // pinned: final state per slot
  hipEvent_t ev = nullptr;
  bool in_flight = false;
  int64_t launch_seq = 0;               // sequence number of the launch in flight
  size_t bytes = 0;
  Clock::time_point last_used;

  int busy() const {
    int c = 0;
    for (int i = 0; i < cap; ++i) c += slot_req[i] != 0;
    return c;
  }
};

// Set-up of a group (operator data, bound estimate, workspace), done by the
// set-up thread while the worker keeps the running groups going.
struct SetupJob {
  GroupKey key;
  pserve_request req;
  size_t bytes = 0;  // reserved against the budget when the job was queued
  std::unique_ptr<Group> group;
  pcheb_status status = PCHEB_OK;
  std::string msg;
  bool done = false;
};

struct Server {
  size_t budget = 0;
  int max_nrhs = 1;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_done, cv_work, cv_setup;
  std::deque<std::shared_ptr<SetupJob>> setup_q;  // waiting for the set-up thread
  std::vector<std::shared_ptr<SetupJob>> setups;  // queued, running or finished, not yet collected
  std::thread setup_thread;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs;
  std::deque<uint64_t> queue;
  std::vector<std::unique_ptr<Group>> groups;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  pserve_stats st{};
  size_t used = 0;
};

static const int kPairsPerLaunch = 1;  // two PCG iterations between readbacks

static pcheb_params params_of(const pserve_request& r, double lmin, double lmax) {
  pcheb_params p{};
  p.k = r.k;
  p.lambda_min = lmin;
  p.lambda_max = lmax;
  p.theta_scale = r.theta_scale;
  p.prec = r.prec;
  p.fuse_steps = r.fuse_steps;
  return p;
}

static size_t request_bytes(const pserve_request& r, int cap) {
  const pcheb_params p = params_of(r, 0.5, 1.5);
  const size_t ldw = size_t((r.op.n + 63) / 64 * 64);
  return footprint_bytes(&r.op, &p, cap) + 2 * size_t(cap) * ldw * sizeof(double);
}

static void hist_add(pserve_stats& st, int active) {
  int b = 0;
  for (int lim = 1; b < 7 && active > lim; lim *= 2) ++b;
  st.batch_hist[b] += 1;
}

static void destroy_group(Group& g) {
  if (g.stream) (void)hipStreamSynchronize(g.stream);
  if (g.ev) (void)hipEventDestroy(g.ev);
  for (hipEvent_t e : g.slot_ev)
    if (e) (void)hipEventDestroy(e);
  if (g.poll) (void)hipHostFree(g.poll);
  if (g.fin) (void)hipHostFree(g.fin);
  std::vector<DeviceBuffer> blocks{g.xb, g.bb};
  device_free_all(blocks);
  g.xb = g.bb = DeviceBuffer{};
  g.X = g.B = nullptr;
  destroy_handle(g.h);
  g.h = nullptr;
  if (g.stream) (void)hipStreamDestroy(g.stream);
  g.stream = nullptr;
}

// Resident data for a request's operator and parameters (bounds estimated here if asked).
static std::unique_ptr<Group> create_group(Server& sv, const pserve_request& r) {
  auto g = std::make_unique<Group>();
  g->key = key_of(r);
  g->cap = sv.max_nrhs;
  try {
    PCHEB_HIP_CHECK(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
    double lmin = r.lambda_min, lmax = r.lambda_max;
    if (!(lmax > 0)) {
      std::vector<DeviceBuffer> start{device_alloc(size_t(r.op.n) * sizeof(double))};
      double* v0 = static_cast<double*>(start[0].ptr);
      launch_fill_uniform(v0, r.op.n, 7, 0.5, 1.5, g->stream);  // Lanczos start: U[0.5, 1.5), seed 7
      const pcheb_status e = pcheb_estimate_bounds(&r.op, v0, 30, &lmin, &lmax, g->stream);
      device_free_all(start);
      if (e != PCHEB_OK) fail(e, std::string("bound estimate: ") + last_error_cstr());
      lmax *= 1.01;
    }
    const pcheb_params p = params_of(r, lmin, lmax);
    g->h = create_handle(&r.op, &p, g->stream);
    ensure_workspace(*g->h, g->cap, g->stream);
    const size_t lw = size_t(g->h->ldw) * size_t(g->cap);
    g->xb = device_alloc(lw * sizeof(double));
    g->X = static_cast<double*>(g->xb.ptr);
    g->bb = device_alloc(lw * sizeof(double));
    g->B = static_cast<double*>(g->bb.ptr);
    PCHEB_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&g->poll), size_t(g->cap) * sizeof(DevState),
                                  hipHostMallocDefault));
    PCHEB_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&g->fin), size_t(g->cap) * sizeof(DevState),
                                  hipHostMallocDefault));
    PCHEB_HIP_CHECK(hipEventCreateWithFlags(&g->ev, hipEventDisableTiming));
    g->slot_req.assign(size_t(g->cap), 0);
    g->slot_since.assign(size_t(g->cap), 0);
    g->slot_draining.assign(size_t(g->cap), 0);
    g->slot_ev.assign(size_t(g->cap), nullptr);
    for (auto& e : g->slot_ev) PCHEB_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const Slots all{0, g->cap};
    solver_init_states(*g->h, all, 1e-8, 1, 1, g->stream);
    solver_retire(*g->h, all, g->stream);
    PCHEB_HIP_CHECK(hipStreamSynchronize(g->stream));
    solver_prepare_graph(*g->h, all, g->X, g->h->ldw, 1);
    g->bytes = request_bytes(r, g->cap);
    g->last_used = Clock::now();
  } catch (...) {
    destroy_group(*g);
    throw;
  }
  return g;
}

static void finish_request(Server& sv, Request& rq, pcheb_status result) {
  rq.result = result;
  rq.state = RState::Done;
  rq.stats.seconds = std::chrono::duration<double>(Clock::now() - rq.t_submit).count();
  if (!rq.cancel && (result == PCHEB_OK || result == PCHEB_NOT_CONVERGED || result == PCHEB_BREAKDOWN))
    sv.st.completed += 1;
  sv.cv_done.notify_all();
}

// One pass of the worker loop; returns true if anything happened.
static bool worker_step(Server& sv) {
  bool progress = false;
  std::unique_lock<std::mutex> lk(sv.mu);

  // cancellations
  for (auto& kv : sv.reqs) {
    Request& rq = *kv.second;
    if (!rq.cancel || rq.state == RState::Done || rq.state == RState::Draining) continue;
    if (rq.state == RState::Queued) {
      sv.queue.erase(std::remove(sv.queue.begin(), sv.queue.end(), rq.id), sv.queue.end());
    } else {
      Group& g = *sv.groups[size_t(rq.group)];
      solver_retire(*g.h, Slots{rq.slot, 1}, g.stream);
      g.slot_req[size_t(rq.slot)] = 0;
    }
    sv.st.cancelled += 1;
    rq.stats.status = PCHEB_NOT_CONVERGED;
    finish_request(sv, rq, PCHEB_NOT_CONVERGED);
    progress = true;
  }

  // groups whose set-up finished: add them, or fail the requests waiting for them
  for (auto it = sv.setups.begin(); it != sv.setups.end();) {
    SetupJob& job = **it;
    if (!job.done) {
      ++it;
      continue;
    }
    progress = true;
    if (job.group) {
      size_t at = sv.groups.size();
      for (size_t gi = 0; gi < sv.groups.size(); ++gi)
        if (!sv.groups[gi]) at = gi;
      if (at == sv.groups.size()) sv.groups.emplace_back();
      sv.groups[at] = std::move(job.group);
      sv.st.groups_created += 1;
    } else {
      sv.used -= job.bytes;
      const std::vector<uint64_t> waiting(sv.queue.begin(), sv.queue.end());
      for (const uint64_t id : waiting) {
        Request& rq = *sv.reqs.at(id);
        if (rq.cancel || !(key_of(rq.req) == job.key)) continue;
        rq.stats.status = job.status;
        rq.error = job.msg;
        sv.st.rejected += 1;
        sv.queue.erase(std::find(sv.queue.begin(), sv.queue.end(), id));
        finish_request(sv, rq, job.status);
      }
    }
    it = sv.setups.erase(it);
  }

  for (size_t gi = 0; gi < sv.groups.size(); ++gi) {
    Group* gp = sv.groups[gi].get();
    if (!gp) continue;
    Group& g = *gp;
    // completions whose copies have landed
    for (int j = 0; j < g.cap; ++j) {
      if (!g.slot_draining[size_t(j)]) continue;
      if (hipEventQuery(g.slot_ev[size_t(j)]) != hipSuccess) continue;
      auto it = sv.reqs.find(g.slot_req[size_t(j)]);
      if (it != sv.reqs.end()) {
        Request& rq = *it->second;
        fill_stats(*g.h, g.fin[j], PCG_FLEXIBLE, &rq.stats);
        finish_request(sv, rq, pcheb_status(rq.stats.status));
      }
      g.slot_draining[size_t(j)] = 0;
      g.slot_req[size_t(j)] = 0;
      progress = true;
    }
    // readback of the last launch: start draining the slots that finished
    if (g.in_flight && hipEventQuery(g.ev) == hipSuccess) {
      g.in_flight = false;
      progress = true;
      for (int j = 0; j < g.cap; ++j) {
        const uint64_t id = g.slot_req[size_t(j)];
        if (!id || g.slot_draining[size_t(j)] || g.slot_since[size_t(j)] >= g.launch_seq) continue;
        if (g.poll[j].done == kRunning) continue;
        Request& rq = *sv.reqs.at(id);
        const Slots one{j, 1};
        const int64_t ldw = g.h->ldw;
        solver_finish(*g.h, one, g.B, ldw, g.X, ldw, g.stream);
        PCHEB_HIP_CHECK(hipMemcpyAsync(rq.req.x, g.X + int64_t(j) * ldw, size_t(g.h->n) * sizeof(double),
                                       hipMemcpyDeviceToDevice, g.stream));
        PCHEB_HIP_CHECK(hipMemcpyAsync(&g.fin[j], g.h->st + j, sizeof(DevState), hipMemcpyDeviceToHost, g.stream));
        PCHEB_HIP_CHECK(hipEventRecord(g.slot_ev[size_t(j)], g.stream));
        g.slot_draining[size_t(j)] = 1;
        rq.state = RState::Draining;
      }
    }
  }

  // admission in arrival order; a request that cannot get memory stops group creation
  bool may_create = true;
  const std::vector<uint64_t> pending(sv.queue.begin(), sv.queue.end());
  auto dequeue = [&](uint64_t id) { sv.queue.erase(std::find(sv.queue.begin(), sv.queue.end(), id)); };
  for (const uint64_t id : pending) {
    const std::shared_ptr<Request> rp = sv.reqs.at(id);
    Request& rq = *rp;
    if (rq.cancel || rq.state != RState::Queued) continue;  // cancellations are handled on the next pass
    const GroupKey key = key_of(rq.req);
    int gidx = -1;
    for (size_t gi = 0; gi < sv.groups.size(); ++gi)
      if (sv.groups[gi] && sv.groups[gi]->key == key) gidx = int(gi);
    if (gidx < 0) {
      bool pending = false;
      for (const auto& job : sv.setups) pending = pending || job->key == key;
      if (pending || !may_create) continue;  // its group is being set up, or memory is short
      const size_t need = request_bytes(rq.req, sv.max_nrhs);
      while (sv.used + need > sv.budget) {  // evict the least recently used idle group
        int victim = -1;
        for (size_t gi = 0; gi < sv.groups.size(); ++gi) {
          Group* c = sv.groups[gi].get();
          if (!c || c->busy() || c->in_flight) continue;
          if (victim < 0 || c->last_used < sv.groups[size_t(victim)]->last_used) victim = int(gi);
        }
        if (victim < 0) break;
        sv.used -= sv.groups[size_t(victim)]->bytes;
        destroy_group(*sv.groups[size_t(victim)]);
        sv.groups[size_t(victim)].reset();
        sv.st.groups_evicted += 1;
      }
      if (sv.used + need > sv.budget) {
        may_create = false;
        continue;
      }
      auto job = std::make_shared<SetupJob>();
      job->key = key;
      job->req = rq.req;
      job->bytes = need;
      sv.used += need;  // reserved now, so later admissions see it
      sv.st.bytes_high_water = std::max<int64_t>(sv.st.bytes_high_water, int64_t(sv.used));
      sv.setups.push_back(job);
      sv.setup_q.push_back(job);
      sv.cv_setup.notify_one();
      progress = true;
      continue;  // admitted once the group exists
    }
    Group& g = *sv.groups[size_t(gidx)];
    int slot = -1;
    for (int j = 0; j < g.cap && slot < 0; ++j)
      if (g.slot_req[size_t(j)] == 0) slot = j;
    if (slot < 0) continue;
    const Slots one{slot, 1};
    const int64_t ldw = g.h->ldw;
    PCHEB_HIP_CHECK(hipMemcpyAsync(g.B + int64_t(slot) * ldw, rq.req.b, size_t(g.h->n) * sizeof(double),
                                   hipMemcpyDeviceToDevice, g.stream));
    solver_init_states(*g.h, one, rq.req.tol, rq.req.maxit, 1, g.stream);
    solver_start(*g.h, one, g.B, ldw, g.X, ldw, false, 1, g.stream);
    g.slot_req[size_t(slot)] = rq.id;
    // the readback of a launch already in flight predates this slot's start
    g.slot_since[size_t(slot)] = g.launch_seq;
    g.last_used = Clock::now();
    rq.state = RState::Active;
    rq.group = gidx;
    rq.slot = slot;
    sv.st.admitted += 1;
    dequeue(id);
    progress = true;
  }

  // launches
  for (auto& gptr : sv.groups) {
    if (!gptr) continue;
    Group& g = *gptr;
    if (g.in_flight) continue;
    int running = 0;
    for (int j = 0; j < g.cap; ++j) running += g.slot_req[size_t(j)] != 0 && !g.slot_draining[size_t(j)];
    if (!running) continue;
    solver_iteration_pairs(*g.h, Slots{0, g.cap}, g.X, g.h->ldw, kPairsPerLaunch, 1, g.stream);
    PCHEB_HIP_CHECK(hipMemcpyAsync(g.poll, g.h->st, size_t(g.cap) * sizeof(DevState), hipMemcpyDeviceToHost,
                                   g.stream));
    PCHEB_HIP_CHECK(hipEventRecord(g.ev, g.stream));
    g.in_flight = true;
    g.launch_seq += 1;
    g.last_used = Clock::now();
    sv.st.launches += 1;
    hist_add(sv.st, running);
    progress = true;
  }

  if (!progress) sv.cv_work.wait_for(lk, std::chrono::microseconds(50));
  return progress;
}

static void worker_main(Server* sv) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      if (sv->stop) break;
    }
    try {
      worker_step(*sv);
    } catch (...) {
      // a device failure ends every request that has not finished; the server stays usable
      // only for new groups (the failed groups are dropped)
      pcheb_status st = PCHEB_HIP;
      std::string msg = "unexpected internal error";
      try {
        throw;
      } catch (const Error& e) {
        st = e.status;
        msg = e.msg;
      } catch (...) {
      }
      std::lock_guard<std::mutex> lk(sv->mu);
      for (auto& kv : sv->reqs) {
        Request& rq = *kv.second;
        if (rq.state != RState::Done) {
          rq.stats.status = st;
          rq.error = msg;
          finish_request(*sv, rq, st);
        }
      }
      sv->queue.clear();
      for (auto& g : sv->groups)
        if (g) {
          destroy_group(*g);
          g.reset();
        }
      sv->used = 0;  // what remains reserved: set-ups not collected yet
      for (const auto& job : sv->setups) sv->used += job->bytes;
    }
  }
}

static void setup_main(Server* sv) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    std::shared_ptr<SetupJob> job;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_setup.wait(lk, [&] { return sv->stop || !sv->setup_q.empty(); });
      if (sv->stop) break;
      job = sv->setup_q.front();
      sv->setup_q.pop_front();
    }
    std::unique_ptr<Group> g;
    pcheb_status status = PCHEB_OK;
    std::string msg;
    try {
      g = create_group(*sv, job->req);
    } catch (const Error& e) {
      status = e.status;
      msg = e.msg;
    } catch (const std::bad_alloc&) {
      status = PCHEB_OOM;
      msg = "host allocation failed";
    } catch (...) {
      status = PCHEB_HIP;
      msg = "unexpected internal error";
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    job->group = std::move(g);
    job->status = status;
    job->msg = msg;
    job->done = true;
    sv->cv_work.notify_one();
  }
}

}  // namespace pcheb

using namespace pcheb;

template <class F>
static pcheb_status guarded_srv(F&& f) {
  try {
    set_last_error("");
    return f();
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return PCHEB_OOM;
  } catch (...) {
    set_last_error("unexpected internal error");
    return PCHEB_HIP;
  }
}

static Server* as_server(pserve_handle s) {
  if (!s) fail(PCHEB_INVALID, "null server");
  return reinterpret_cast<Server*>(s);
}

extern "C" {

pcheb_status pserve_create(size_t hbm_budget, int32_t max_nrhs, pserve_handle* out) {
  return guarded_srv([&]() -> pcheb_status {
    if (!out) fail(PCHEB_INVALID, "out is null");
    if (max_nrhs < 1 || max_nrhs > 64) fail(PCHEB_INVALID, "max_nrhs must be in [1, 64]");
    if (hbm_budget == 0) fail(PCHEB_INVALID, "budget must be positive");
    auto* sv = new Server();
    sv->budget = hbm_budget;
    sv->max_nrhs = max_nrhs;
    sv->st.budget = int64_t(hbm_budget);
    PCHEB_HIP_CHECK(hipGetDevice(&sv->device));
    sv->worker = std::thread(worker_main, sv);
    sv->setup_thread = std::thread(setup_main, sv);
    *out = reinterpret_cast<pserve_handle>(sv);
    return PCHEB_OK;
  });
}

pcheb_status pserve_submit(pserve_handle s, const pserve_request* req, uint64_t* id) {
  return guarded_srv([&]() -> pcheb_status {
    Server* sv = as_server(s);
    if (!req || !id || !req->b || !req->x) fail(PCHEB_INVALID, "null request, id, b or x");
    if (!(req->tol > 0) || req->maxit < 1) fail(PCHEB_INVALID, "tol must be positive and maxit >= 1");
    if ((reinterpret_cast<uintptr_t>(req->b) | reinterpret_cast<uintptr_t>(req->x)) % 16 != 0)
      fail(PCHEB_INVALID, "vectors must be 16-byte aligned");
    const size_t need = request_bytes(*req, sv->max_nrhs);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->st.submitted += 1;
    if (need > sv->budget) {
      sv->st.rejected += 1;
      fail(PCHEB_BUDGET, "request needs " + std::to_string(need) + " bytes, budget is " + std::to_string(sv->budget));
    }
    auto rq = std::make_shared<Request>();
    rq->id = sv->next_id++;
    rq->req = *req;
    rq->t_submit = Clock::now();
    sv->reqs[rq->id] = rq;
    sv->queue.push_back(rq->id);
    *id = rq->id;
    sv->cv_work.notify_one();
    return PCHEB_OK;
  });
}

pcheb_status pserve_poll(pserve_handle s, uint64_t id, int32_t* done, pcg_stats* stats) {
  return guarded_srv([&]() -> pcheb_status {
    Server* sv = as_server(s);
    if (!done) fail(PCHEB_INVALID, "done is null");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) fail(PCHEB_NOT_FOUND, "unknown request id");
    *done = it->second->state == RState::Done ? 1 : 0;
    if (*done) {
      const Request& rq = *it->second;
      if (stats) *stats = rq.stats;
      if (rq.result != PCHEB_OK)
        set_last_error(rq.cancel ? "request cancelled" : !rq.error.empty() ? rq.error : "request did not converge");
      sv->reqs.erase(it);  // reported: the id is released
    }
    return PCHEB_OK;
  });
}

pcheb_status pserve_wait(pserve_handle s, uint64_t id, pcg_stats* stats) {
  return guarded_srv([&]() -> pcheb_status {
    Server* sv = as_server(s);
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) fail(PCHEB_NOT_FOUND, "unknown request id");
    std::shared_ptr<Request> rq = it->second;
    sv->cv_done.wait(lk, [&] { return rq->state == RState::Done; });
    if (stats) *stats = rq->stats;
    sv->reqs.erase(rq->id);  // reported: the id is released
    if (rq->result != PCHEB_OK)
      set_last_error(rq->cancel ? "request cancelled" : !rq->error.empty() ? rq->error : "request did not converge");
    return rq->result;
  });
}

pcheb_status pserve_cancel(pserve_handle s, uint64_t id) {
  return guarded_srv([&]() -> pcheb_status {
    Server* sv = as_server(s);
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) fail(PCHEB_NOT_FOUND, "unknown request id");
    it->second->cancel = true;
    sv->cv_work.notify_one();
    return PCHEB_OK;
  });
}

pcheb_status pserve_get_stats(pserve_handle s, pserve_stats* out) {
  return guarded_srv([&]() -> pcheb_status {
    Server* sv = as_server(s);
    if (!out) fail(PCHEB_INVALID, "out is null");
    std::lock_guard<std::mutex> lk(sv->mu);
    pserve_stats st = sv->st;
    st.queued = int64_t(sv->queue.size());
    st.active = 0;
    st.groups = 0;
    for (auto& g : sv->groups)
      if (g) {
        st.groups += 1;
        st.active += g->busy();
      }
    st.bytes_in_use = int64_t(sv->used);
    st.bytes_high_water = std::max<int64_t>(sv->st.bytes_high_water, int64_t(sv->used));
    sv->st.bytes_high_water = st.bytes_high_water;
    *out = st;
    return PCHEB_OK;
  });
}

pcheb_status pserve_destroy(pserve_handle s) {
  return guarded_srv([&]() -> pcheb_status {
    if (!s) return PCHEB_OK;
    Server* sv = reinterpret_cast<Server*>(s);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stop = true;
      sv->cv_work.notify_all();
      sv->cv_setup.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    if (sv->setup_thread.joinable()) sv->setup_thread.join();
    for (auto& g : sv->groups)
      if (g) destroy_group(*g);
    for (auto& job : sv->setups)
      if (job->group) destroy_group(*job->group);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      for (auto& kv : sv->reqs)
        if (kv.second->state != RState::Done) {
          kv.second->stats.status = PCHEB_NOT_CONVERGED;
          finish_request(*sv, *kv.second, PCHEB_NOT_CONVERGED);
        }
    }
    delete sv;
    return PCHEB_OK;
  });
}

}  // extern "C"
