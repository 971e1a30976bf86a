// Request loop with continuous batching over the library's own C ABI: a
// worker thread admits queued cases by device footprint, steps every resident
// case through one ib_lbm_batch, and retires cases as they reach their step
// counts.  No arithmetic of the method happens here; every step runs in the
// batch's HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ib_lbm.h"
#include "../../include/ib_lbm_server.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  ib_lbm_request req;
  ib_lbm_result res;
  ib_lbm_sim *sim = nullptr;
  int64_t remaining = 0;
  bool done = false;
};

}  // namespace

struct ib_lbm_server {
  ib_lbm_server_config cfg;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  ib_lbm_batch *batch = nullptr;
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;
  std::unordered_map<int64_t, std::unique_ptr<Request>> all;
  int64_t next_id = 1;
  bool stop = false;
  bool broken = false;
  std::string err;
  ib_lbm_server_stats st{};
  std::thread worker;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

void set_err_locked(ib_lbm_server *S, const std::string &msg) { S->err = msg; }

// Completes a request: result fields already set by the caller.
void complete(ib_lbm_server *S, Request *r, int32_t status, bool was_resident) {
  r->res.t_finish = S->now();
  r->res.status = status;
  std::lock_guard<std::mutex> lk(S->mu);
  r->done = true;
  if (was_resident) {
    S->st.resident -= 1;
    S->st.resident_bytes -= r->res.footprint;
  }
  S->st.completed += 1;
  if (status != IB_LBM_OK) S->st.failed += 1;
  S->st.node_updates += (int64_t)r->req.lattice.nx * r->req.lattice.ny * r->res.steps_done;
  S->cv_done.notify_all();
}

// Creates the request's sim, adds its bodies and attaches it to the batch
// with its step count as target.  Returns a failure status, or OK.
int32_t start_request(ib_lbm_server *S, Request *r) {
  ib_lbm_config cfg = r->req.lattice;
  cfg.stream = (void *)S->stream;
  cfg.alloc = nullptr;
  ib_lbm_status st = ib_lbm_create(&cfg, &r->sim);
  if (st) return st;
  if (S->cfg.launch.block_x > 0 && (st = ib_lbm_set_launch(r->sim, &S->cfg.launch))) return st;
  if ((st = ib_lbm_set_spread(r->sim, S->cfg.spread))) return st;
  for (int b = 0; b < r->req.n_bodies; b++) {
    int32_t id = 0;
    if ((st = ib_lbm_add_body(r->sim, &r->req.bodies[b], &id))) return st;
  }
  if ((st = ib_lbm_batch_attach(S->batch, r->sim))) return st;
  if ((st = ib_lbm_batch_set_target(S->batch, r->sim, r->req.steps))) return st;
  return IB_LBM_OK;
}

// Reads the final state of a resident request to the host and releases it.
int32_t finish_request(ib_lbm_server *S, Request *r) {
  int32_t status = IB_LBM_OK;
  int64_t done = 0;
  ib_lbm_status st = ib_lbm_steps_done(r->sim, &done);
  if (st) status = st;
  r->res.steps_done = done;
  for (int b = 0; b < r->req.n_bodies; b++) {
    st = ib_lbm_forces(r->sim, b, &r->res.body[b]);
    if (st && status == IB_LBM_OK) status = st;
  }
  if (r->req.rho && r->req.ux && r->req.uy) {
    st = ib_lbm_fields(r->sim, r->req.rho, r->req.ux, r->req.uy);
    if (st && status == IB_LBM_OK) status = st;
  }
  (void)ib_lbm_batch_detach(S->batch, r->sim);
  (void)ib_lbm_destroy(r->sim);
  r->sim = nullptr;
  return status;
}

void release_failed_start(ib_lbm_server *S, Request *r) {
  if (!r->sim) return;
  (void)ib_lbm_batch_detach(S->batch, r->sim);  // no-op when it was never attached
  (void)ib_lbm_destroy(r->sim);
  r->sim = nullptr;
}

void worker_main(ib_lbm_server *S) {
  (void)hipSetDevice(S->device);
  std::vector<Request *> res;  // resident, in admission order
  for (;;) {
    std::vector<Request *> admit, reject;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty() || !res.empty(); });
      if (S->stop && S->pending.empty() && res.empty()) break;
      // Admission in arrival order: the head of the queue waits until the
      // budget and the resident cap allow it (no overtaking, so a large case
      // is not starved by smaller ones behind it).
      while (!S->pending.empty()) {
        Request *r = S->pending.front();
        if (S->broken || r->res.footprint > S->cfg.hbm_budget) {
          S->pending.pop_front();
          reject.push_back(r);
          continue;
        }
        if ((int64_t)(res.size() + admit.size()) >= S->cfg.max_resident ||
            S->st.resident_bytes + r->res.footprint > S->cfg.hbm_budget)
          break;
        S->pending.pop_front();
        S->st.resident_bytes += r->res.footprint;
        S->st.resident += 1;
        S->st.admitted += 1;
        admit.push_back(r);
      }
      S->st.queued = (int64_t)S->pending.size();
      S->st.peak_resident = std::max<int64_t>(S->st.peak_resident, S->st.resident);
      S->st.peak_resident_bytes = std::max(S->st.peak_resident_bytes, S->st.resident_bytes);
    }
    for (Request *r : reject) complete(S, r, S->broken ? IB_LBM_E_STATE : IB_LBM_E_NOMEM, false);
    for (Request *r : admit) {
      r->res.t_admit = S->now();
      const int32_t st = start_request(S, r);
      if (st) {
        release_failed_start(S, r);
        complete(S, r, st, true);
      } else {
        r->remaining = r->req.steps;
        res.push_back(r);
      }
    }
    if (res.empty()) continue;
    // One scheduling round: every resident case advances together; the
    // round ends when the first of them reaches its step count.
    int64_t q = S->cfg.quantum;
    for (Request *r : res) q = std::min(q, r->remaining);
    const double tb = S->now();
    ib_lbm_status st = IB_LBM_OK;
    if (q > 0) {
      st = ib_lbm_batch_step(S->batch, q);
      if (!st) st = ib_lbm_batch_sync(S->batch);
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->st.busy_seconds += S->now() - tb;
      S->st.rounds += 1;
      if (st) {
        S->broken = true;
        set_err_locked(S, std::string("batch step failed: ") + ib_lbm_batch_last_error(S->batch));
      }
    }
    std::vector<Request *> keep;
    for (Request *r : res) {
      r->remaining -= q;
      if (st || r->remaining <= 0) {
        const int32_t fs = finish_request(S, r);
        complete(S, r, st ? (int32_t)IB_LBM_E_DEVICE : fs, true);
      } else {
        keep.push_back(r);
      }
    }
    res.swap(keep);
  }
}

}  // namespace

extern "C" {

ib_lbm_status ib_lbm_server_create(const ib_lbm_server_config *cfg, ib_lbm_server **out) {
  if (!cfg || !out) return IB_LBM_E_INVALID;
  *out = nullptr;
  if (cfg->abi_version != IB_LBM_ABI_VERSION ||
      (cfg->precision != IB_LBM_FP64 && cfg->precision != IB_LBM_FP32_SHIFTED) ||
      cfg->max_resident < 0 || cfg->quantum < 0 || cfg->graph_steps < 0 ||
      (cfg->spread != IB_LBM_SPREAD_GATHER && cfg->spread != IB_LBM_SPREAD_ATOMIC))
    return IB_LBM_E_INVALID;
  auto S = std::make_unique<ib_lbm_server>();
  S->cfg = *cfg;
  if (S->cfg.hbm_budget == 0) S->cfg.hbm_budget = 16ull << 30;
  if (S->cfg.max_resident == 0) S->cfg.max_resident = 64;
  if (S->cfg.quantum == 0) S->cfg.quantum = 256;
  if (hipGetDevice(&S->device) != hipSuccess) return IB_LBM_E_DEVICE;
  if (cfg->stream) {
    S->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) return IB_LBM_E_DEVICE;
    S->own_stream = true;
  }
  ib_lbm_status st = ib_lbm_batch_create((void *)S->stream, cfg->precision, &S->batch);
  if (st) {
    if (S->own_stream) (void)hipStreamDestroy(S->stream);
    return st;
  }
  if (S->cfg.launch.block_x > 0 && (st = ib_lbm_batch_set_launch(S->batch, &S->cfg.launch))) {
    (void)ib_lbm_batch_destroy(S->batch);
    if (S->own_stream) (void)hipStreamDestroy(S->stream);
    return st;
  }
  (void)ib_lbm_batch_set_spread(S->batch, S->cfg.spread);
  if (S->cfg.graph_steps > 0) (void)ib_lbm_batch_set_graph(S->batch, S->cfg.graph_steps);
  S->t0 = Clock::now();
  ib_lbm_server *raw = S.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_server_submit(ib_lbm_server *srv, const ib_lbm_request *req, int64_t *id) {
  if (!srv || !req || !id) return IB_LBM_E_INVALID;
  if (req->n_bodies < 0 || req->n_bodies > IB_LBM_SERVER_MAX_BODIES || req->steps < 0 ||
      req->lattice.precision != srv->cfg.precision)
    return IB_LBM_E_INVALID;
  auto r = std::make_unique<Request>();
  r->req = *req;
  memset(&r->res, 0, sizeof r->res);
  r->res.n_bodies = req->n_bodies;
  int32_t nm[IB_LBM_SERVER_MAX_BODIES];
  for (int b = 0; b < req->n_bodies; b++) {
    const ib_lbm_body_desc &d = req->bodies[b];
    nm[b] = d.n_markers > 0 ? d.n_markers : (int32_t)std::lround(M_PI * d.diameter);
  }
  r->res.footprint = ib_lbm_footprint(&req->lattice, req->n_bodies, nm);
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return IB_LBM_E_STATE;
  r->res.id = srv->next_id++;
  r->res.t_submit = srv->now();
  *id = r->res.id;
  srv->pending.push_back(r.get());
  srv->all.emplace(r->res.id, std::move(r));
  srv->st.submitted += 1;
  srv->st.queued = (int64_t)srv->pending.size();
  srv->cv_work.notify_one();
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_server_wait(ib_lbm_server *srv, int64_t id, double timeout_s, ib_lbm_result *out) {
  if (!srv || !out) return IB_LBM_E_INVALID;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->all.find(id);
  if (it == srv->all.end()) return IB_LBM_E_INVALID;
  Request *r = it->second.get();
  auto ready = [&] { return r->done; };
  if (timeout_s < 0) {
    srv->cv_done.wait(lk, ready);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return (ib_lbm_status)IB_LBM_PENDING;
  }
  *out = r->res;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_server_stats_get(ib_lbm_server *srv, ib_lbm_server_stats *out) {
  if (!srv || !out) return IB_LBM_E_INVALID;
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->st;
  out->now = srv->now();
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_server_drain(ib_lbm_server *srv) {
  if (!srv) return IB_LBM_E_INVALID;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] { return srv->st.completed == srv->st.submitted; });
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_server_destroy(ib_lbm_server *srv) {
  if (!srv) return IB_LBM_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  if (srv->worker.joinable()) srv->worker.join();
  (void)ib_lbm_batch_destroy(srv->batch);
  if (srv->own_stream) (void)hipStreamDestroy(srv->stream);
  delete srv;
  return IB_LBM_OK;
}

const char *ib_lbm_server_last_error(const ib_lbm_server *srv) {
  return srv ? srv->err.c_str() : "null server";
}

}  // extern "C"
