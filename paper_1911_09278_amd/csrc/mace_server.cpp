// Reconstruction service: scans arrive at any time, are admitted into scan
// slots while the HBM budget allows, and advance by continuous batching --
// every Mann iteration (Algorithm 1) of a system's admitted scans runs as one
// round of launches over all of them, a scan leaves as soon as its own
// residual test passes, and a waiting scan takes its slot at the next
// iteration.  Each system (geometry) has its own worker thread and HIP
// stream, so the iterations of scans of different sizes overlap on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "mace_runtime.h"

using namespace mace;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int kGroupSlots = 32;  // scans of one group in flight at once

struct Request {
  int64_t ticket = 0;
  int sys = 0;
  std::vector<float> y, lam;
  mace_prior prior{};
  double rho = 0, sigma = 0, tol = 0;
  int sweeps = 1, max_iters = 0;
  Clock::time_point t_submit, t_done;
  std::vector<float> x;
  mace_info info{};
  int status = MACE_OK;
  bool done = false;
  std::atomic<bool> cancel{false};  // set by mace_server_cancel while in flight
};

// Scans of one system that share the solver parameters (prior, rho, sigma,
// sweeps): they run in the same launches.
struct Group {
  mace_prior prior{};
  double rho = 0, sigma = 0;
  int sweeps = 1;
  Batch batch;
  std::vector<Request*> req;  // per slot; nullptr = free
  std::vector<int> iters;
  std::vector<int> tail_iters;  // iterations run with the FP32 values after the switch
  std::vector<int64_t> bytes;  // device bytes held by each slot (0 = none)
  int ticks = 0;
  DevBuf<float> yin, lin;   // staging of admitted scans' y and Lambda
  double* hlast = nullptr;  // pinned read-back of the slots' residuals
  hipEvent_t ev = nullptr;
  ~Group() {
    std::lock_guard<std::mutex> lk(capture_mutex());
    if (hlast) (void)hipHostFree(hlast);
    if (ev) (void)hipEventDestroy(ev);
  }
  int active() const {
    int k = 0;
    for (auto* r : req) k += r != nullptr;
    return k;
  }
  // field by field: the struct's padding bytes are whatever the caller's
  // copy held
  bool same(const Request& r) const {
    const mace_prior& a = prior;
    const mace_prior& b = r.prior;
    return rho == r.rho && sigma == r.sigma && sweeps == r.sweeps && a.kind == b.kind &&
           a.sigma_x == b.sigma_x && a.p == b.p && a.q == b.q && a.T == b.T &&
           a.b_edge == b.b_edge && a.b_diag == b.b_diag;
  }
};

}  // namespace

struct mace_server {
  std::vector<mace_system*> sys;
  int64_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  std::vector<std::vector<std::unique_ptr<Group>>> groups;  // per system
  std::vector<std::thread> workers;
  bool stop = false;
  int err = MACE_OK;
  std::string err_text;
  int64_t next_ticket = 1;
  int64_t used = 0, peak = 0;
  int64_t submitted = 0, completed = 0;
  int in_flight = 0, max_in_flight = 0;

  void worker(int k);
  int tick(int k, std::vector<std::pair<Group*, int>>& admitted);
  bool fits(int64_t need) const { return budget <= 0 || used + need <= budget; }
};

namespace {

int64_t state_bytes(const mace_system* s) { return slot_bytes(s, 1); }

// Picks (group, slot) for r in system k's groups (creating a group when no
// existing one shares its parameters).  Host only; called under the lock.
std::pair<Group*, int> place(mace_server* sv, int k, const Request& r) {
  auto& gs = sv->groups[k];
  Group* g = nullptr;
  for (auto& c : gs)
    if (c->same(r)) g = c.get();
  if (!g) {
    gs.push_back(std::make_unique<Group>());
    g = gs.back().get();
    g->prior = r.prior;
    g->rho = r.rho;
    g->sigma = r.sigma;
    g->sweeps = r.sweeps;
  }
  for (int i = 0; i < (int)g->req.size(); ++i)
    if (!g->req[i]) return {g, i};
  if ((int)g->req.size() < kGroupSlots) {
    g->req.push_back(nullptr);
    g->iters.push_back(0);
    g->tail_iters.push_back(0);
    g->bytes.push_back(0);
    return {g, (int)g->req.size() - 1};
  }
  return {nullptr, -1};
}

}  // namespace

// One round of system k's worker: start the newly admitted scans, run one
// Mann iteration of every group with scans in flight, read the residuals,
// finish the scans whose test passed.  Runs without the lock.
int mace_server::tick(int k, std::vector<std::pair<Group*, int>>& admitted) {
  mace_system* s = sys[k];
  hipStream_t st = s->stream;
  const bool fp16 = s->precision == 1;
  const bool tail = fp16 && s->fp32_tail > 0;
  for (auto& [g, i] : admitted) {
    Request* r = g->req[i];
    if (!g->hlast) {
      std::lock_guard<std::mutex> lk(capture_mutex());
      HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&g->hlast), sizeof(double) * kMaxScanSlots,
                           hipHostMallocDefault));
      HIP_OK(hipEventCreateWithFlags(&g->ev, hipEventDisableTiming));
    }
    int rc = ensure_slot(s, g->batch, i, 1);
    if (rc) return rc;
    const size_t m = (size_t)s->n_views * s->n_ch;
    if (g->yin.count != m) {
      HIP_OK(g->yin.alloc(m));
      HIP_OK(g->lin.alloc(m));
    }
    // the request keeps its host copies until it is waited for; the staging
    // buffers are reused in stream order
    HIP_OK(hipMemcpyAsync(g->yin.p, r->y.data(), sizeof(float) * m, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(g->lin.p, r->lam.data(), sizeof(float) * m, hipMemcpyHostToDevice, st));
    SvArgs a;
    fill_args(s, a, &g->prior, g->rho, g->sigma, fp16);
    rc = start_slot(s, g->batch, i, g->yin.p, g->lin.p, nullptr, a, st);
    if (rc) return rc;
    g->iters[i] = 0;
    g->tail_iters[i] = 0;
  }
  std::vector<Group*> ran;
  for (auto& gp : groups[k]) {
    Group* g = gp.get();
    const int act = g->active();
    if (act == 0) continue;
    int n_occ = 0;
    for (int i = 0; i < (int)g->req.size(); ++i)
      if (g->req[i]) n_occ = i + 1;
    const int P = batch_rows_per_agent(s, act, true);
    Schedule* sch = get_schedule(s, n_occ, -1, P);
    if (!sch) return fail(MACE_E_HIP, "schedule upload failed");
    SvArgs a;
    fill_args(s, a, &g->prior, g->rho, g->sigma, fp16);
    a.strict = P == 1 ? 1 : 0;
    if (s->refresh_every > 0 && g->ticks > 0 && g->ticks % s->refresh_every == 0) {
      int rc = refresh_slots(s, g->batch, n_occ, sch, a, st);
      if (rc) return rc;
    }
    // eager launches: a worker thread captures no graph (see capture_mutex)
    int rc = run_iteration(s, g->batch, sch, n_occ, a, g->sweeps, P, st, false);
    if (rc) return rc;
    ++g->ticks;
    HIP_OK(hipMemcpyAsync(g->hlast, g->batch.lastres.p, sizeof(double) * n_occ,
                          hipMemcpyDeviceToHost, st));
    HIP_OK(hipEventRecord(g->ev, st));
    ran.push_back(g);
  }
  std::vector<std::pair<Group*, int>> fin;
  for (Group* g : ran) {
    HIP_OK(hipEventSynchronize(g->ev));
    for (int i = 0; i < (int)g->req.size(); ++i) {
      Request* r = g->req[i];
      if (!r) continue;
      const int it = ++g->iters[i];
      const bool in16 = g->batch.htable[i].prec == 1;
      if (tail && !in16) ++g->tail_iters[i];
      const double res = g->hlast[i];
      int status = -100;
      if (r->cancel.load())
        status = MACE_E_CANCELLED;
      else if (!std::isfinite(res))
        status = MACE_E_NONFINITE;
      else if (r->tol > 0 && res < r->tol)
        status = MACE_OK;
      else if (it >= r->max_iters)
        status = r->tol > 0 ? MACE_W_MAXITER : MACE_OK;
      // an FP16 scan with an FP32 tail: it switches to the FP32 values when
      // it first meets tol, or fp32_tail iterations before max_iters
      if (tail && in16 && it < r->max_iters &&
          (status == MACE_OK || (status == -100 && it >= r->max_iters - s->fp32_tail))) {
        SvArgs a;
        fill_args(s, a, &g->prior, g->rho, g->sigma, false);
        int rc = switch_slot_fp32(s, g->batch, i, a, st);
        if (rc) return rc;
        continue;
      }
      if (status == -100) continue;
      if (status != MACE_E_CANCELLED) {
        r->x.resize(s->n);
        HIP_OK(hipMemcpyAsync(r->x.data(), g->batch.scan[i]->wbar.p, sizeof(float) * s->n,
                              hipMemcpyDeviceToHost, st));
      }
      int rc = write_slot(s, g->batch, i, 0, st);
      if (rc) return rc;
      r->status = status;
      r->info.iters = it;
      r->info.residual = res;
      r->info.equits = (double)g->sweeps * it;
      r->info.fp32_tail_iters = g->tail_iters[i];
      r->info.status = status;
      fin.emplace_back(g, i);
    }
  }
  if (!fin.empty()) HIP_OK(hipStreamSynchronize(st));
  std::lock_guard<std::mutex> lk(mu);
  for (auto& [g, i] : fin) {
    Request* r = g->req[i];
    r->t_done = Clock::now();
    r->done = true;
    g->req[i] = nullptr;
    --in_flight;
    ++completed;
  }
  if (!fin.empty()) {
    cv_done.notify_all();
    cv_work.notify_all();
  }
  return MACE_OK;
}

void mace_server::worker(int k) {
  mace_system* s = sys[k];
  if (hipSetDevice(s->device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(mu);
    err = MACE_E_HIP;
    err_text = "hipSetDevice failed in a server worker";
    cv_done.notify_all();
    return;
  }
  const int64_t need = state_bytes(s);
  std::unique_lock<std::mutex> lk(mu);
  while (err == MACE_OK) {
    // admission, oldest first: a scan that does not fit the budget blocks
    // every later one, so large scans are not starved by small ones
    std::vector<std::pair<Group*, int>> admitted;
    bool blocked = false;  // the oldest waiting scan does not fit the budget
    for (auto itq = pending.begin(); itq != pending.end();) {
      Request* r = *itq;
      const int64_t rneed = state_bytes(sys[r->sys]);
      if (r->sys != k) {
        // another worker's scan: it holds back this worker's later scans
        // while it waits for memory (unless it can never fit: then its own
        // worker fails it)
        if (!fits(rneed) && !(budget > 0 && rneed > budget)) {
          blocked = true;
          break;
        }
        ++itq;
        continue;
      }
      auto [g, i] = place(this, k, *r);
      if (!g) {  // the group is full: wait for a slot
        ++itq;
        continue;
      }
      const int64_t extra = g->bytes[i] ? 0 : need;
      if (!fits(extra)) {
        if (budget > 0 && need > budget) {  // can never fit
          r->status = MACE_E_NOMEM;
          r->info.status = MACE_E_NOMEM;
          r->t_done = Clock::now();
          r->done = true;
          itq = pending.erase(itq);
          cv_done.notify_all();
          cv_work.notify_all();
          continue;
        }
        blocked = true;
        break;
      }
      used += extra;
      peak = std::max(peak, used);
      g->bytes[i] = need;
      g->req[i] = r;
      admitted.emplace_back(g, i);
      ++in_flight;
      max_in_flight = std::max(max_in_flight, in_flight);
      itq = pending.erase(itq);
    }
    if (blocked) {
      // give back the memory of this system's idle slots
      for (auto& g : groups[k])
        for (int i = 0; i < (int)g->req.size(); ++i)
          if (!g->req[i] && g->bytes[i]) {
            release_slot(g->batch, i);
            used -= g->bytes[i];
            g->bytes[i] = 0;
            cv_work.notify_all();
          }
    }
    bool busy = !admitted.empty();
    for (auto& g : groups[k]) busy = busy || g->active() > 0;
    if (!busy) {
      if (stop) break;
      cv_work.wait(lk);
      continue;
    }
    lk.unlock();
    const int rc = tick(k, admitted);
    lk.lock();
    if (rc != MACE_OK) {
      err = rc;
      err_text = last_error_text();
    }
  }
  if (err != MACE_OK) {
    // fail everything this worker holds or will never run
    for (auto& g : groups[k])
      for (auto*& r : g->req)
        if (r) {
          r->status = err;
          r->info.status = err;
          r->done = true;
          r = nullptr;
        }
    for (auto* r : pending) {
      r->status = err;
      r->info.status = err;
      r->done = true;
    }
    pending.clear();
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

extern "C" int mace_server_create(mace_system* const* systems, int32_t n_systems,
                                  int64_t hbm_budget_bytes, mace_server** out) {
  if (!out) return fail(MACE_E_ARG, "out is NULL");
  *out = nullptr;
  if (!systems || n_systems < 1) return fail(MACE_E_ARG, "need at least one system");
  if (hbm_budget_bytes < 0) return fail(MACE_E_ARG, "hbm_budget_bytes must be >= 0");
  auto sv = std::make_unique<mace_server>();
  for (int k = 0; k < n_systems; ++k) {
    if (!systems[k]) return fail(MACE_E_ARG, "system %d is NULL", k);
    for (int j = 0; j < k; ++j)
      if (systems[j] == systems[k]) return fail(MACE_E_ARG, "system %d is listed twice", k);
    sv->sys.push_back(systems[k]);
  }
  sv->budget = hbm_budget_bytes;
  sv->groups.resize(n_systems);
  for (int k = 0; k < n_systems; ++k) sv->workers.emplace_back(&mace_server::worker, sv.get(), k);
  *out = sv.release();
  return MACE_OK;
}

extern "C" int mace_server_submit(mace_server* sv, int32_t system_idx, const float* y,
                                  const float* lam, const mace_prior* pr, double rho,
                                  double sigma, int32_t sweeps, double tol, int32_t max_iters,
                                  int64_t* ticket) {
  if (!sv || !y || !lam || !ticket) return fail(MACE_E_ARG, "NULL argument");
  if (system_idx < 0 || system_idx >= (int)sv->sys.size())
    return fail(MACE_E_ARG, "system index %d out of range", system_idx);
  int rc = check_prior(pr);
  if (rc) return rc;
  if (!(rho > 0 && rho < 1)) return fail(MACE_E_ARG, "rho must be in (0, 1)");
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(MACE_E_ARG, "sigma must be > 0");
  if (sweeps < 1) return fail(MACE_E_ARG, "sweeps must be >= 1");
  if (max_iters < 1) return fail(MACE_E_ARG, "max_iters must be >= 1");
  if (!(tol >= 0) || !std::isfinite(tol)) return fail(MACE_E_ARG, "tol must be >= 0");
  const mace_system* s = sv->sys[system_idx];
  const size_t m = (size_t)s->n_views * s->n_ch;
  auto r = std::make_unique<Request>();
  r->sys = system_idx;
  r->y.assign(y, y + m);
  r->lam.assign(lam, lam + m);
  r->prior = *pr;
  r->rho = rho;
  r->sigma = sigma;
  r->sweeps = sweeps;
  r->tol = tol;
  r->max_iters = max_iters;
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->err != MACE_OK) return fail(sv->err, "server failed: %s", sv->err_text.c_str());
  if (sv->stop) return fail(MACE_E_ARG, "server is shutting down");
  r->ticket = sv->next_ticket++;
  *ticket = r->ticket;
  sv->pending.push_back(r.get());
  sv->reqs[r->ticket] = std::move(r);
  ++sv->submitted;
  sv->cv_work.notify_all();
  return MACE_OK;
}

extern "C" int mace_server_wait(mace_server* sv, int64_t ticket, float* x_out, mace_info* info,
                                double* latency_s) {
  if (!sv) return fail(MACE_E_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(MACE_E_ARG, "unknown ticket %lld", (long long)ticket);
  Request* r = it->second.get();
  sv->cv_done.wait(lk, [&] { return r->done; });
  const int status = r->status;
  if (x_out && r->x.size() == (size_t)sv->sys[r->sys]->n)
    std::memcpy(x_out, r->x.data(), sizeof(float) * r->x.size());
  if (info) *info = r->info;
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  const std::string text = sv->err_text;
  sv->reqs.erase(it);
  if (status < 0) {
    if (status == MACE_E_NOMEM) return fail(status, "the scan's state exceeds the HBM budget");
    if (status == MACE_E_CANCELLED) return fail(status, "the scan was cancelled");
    return fail(status, "scan failed: %s", text.c_str());
  }
  return status;
}

extern "C" int mace_server_cancel(mace_server* sv, int64_t ticket) {
  if (!sv) return fail(MACE_E_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(MACE_E_ARG, "unknown ticket %lld", (long long)ticket);
  Request* r = it->second.get();
  if (r->done) return MACE_OK;  // finished already: its result stands
  auto pit = std::find(sv->pending.begin(), sv->pending.end(), r);
  if (pit != sv->pending.end()) {
    // not admitted yet: it leaves the queue now
    sv->pending.erase(pit);
    r->status = MACE_E_CANCELLED;
    r->info.status = MACE_E_CANCELLED;
    r->t_done = Clock::now();
    r->done = true;
    ++sv->completed;
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
    return MACE_OK;
  }
  // in flight: its worker releases the slot after the current iteration
  r->cancel.store(true);
  return MACE_OK;
}

extern "C" int mace_server_stats(mace_server* sv, mace_server_counters* out) {
  if (!sv || !out) return fail(MACE_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  out->submitted = sv->submitted;
  out->completed = sv->completed;
  out->queued = (int64_t)sv->pending.size();
  out->in_flight = sv->in_flight;
  out->max_in_flight = sv->max_in_flight;
  out->bytes_in_use = sv->used;
  out->peak_bytes = sv->peak;
  return sv->err;
}

extern "C" void mace_server_destroy(mace_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    // scans not yet admitted are dropped
    for (auto* r : sv->pending) {
      r->status = MACE_E_ARG;
      r->info.status = MACE_E_ARG;
      r->done = true;
    }
    sv->pending.clear();
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
  }
  for (auto& t : sv->workers) t.join();
  for (size_t k = 0; k < sv->groups.size(); ++k) {
    (void)hipSetDevice(sv->sys[k]->device);
    sv->groups[k].clear();
  }
  delete sv;
}
