// Host runtime of the MACE library, part 2: scan slots, the Mann-iteration
// driver (Algorithm 1) for one scan or a batch of scans of one geometry, the
// single-agent partial prox, and state read-back.
//
// All launches of a solve run on the system's private stream.  One Mann
// iteration (4 colour-phase sweep launches per ICD pass, then the consensus /
// residual epilogue) is captured once in a hipGraph and replayed; the slot
// table lives in device memory, so a slot that has converged is switched off
// without re-capturing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <tuple>

#include "mace_runtime.h"

using namespace mace;

namespace mace {

int64_t slot_bytes(const mace_system* s, int resid_cap) {
  const int64_t nimg = (int64_t)s->N * s->n, nrow = (int64_t)s->N * s->estride;
  return 4 * (3 * nrow + 3 * nimg + 2 * s->n) +
         8 * ((int64_t)s->N * s->n_sv * 4 + (int64_t)epilogue_scratch_doubles() + std::max(1, resid_cap)) + 8;
}

int ensure_slot(mace_system* s, Batch& b, int idx, int resid_cap) {
  if (idx >= kMaxScanSlots) return fail(MACE_E_ARG, "slot %d out of range", idx);
  while ((int)b.scan.size() <= idx) b.scan.push_back(std::make_unique<ScanSlot>());
  ScanSlot& q = *b.scan[idx];
  const size_t nimg = (size_t)s->N * s->n;
  const size_t nrow = (size_t)s->N * s->estride;
  const size_t npart = (size_t)s->N * s->n_sv * 4 + epilogue_scratch_doubles();
  // Any buffer missing or of the wrong size (a previous call may have failed
  // half way): the whole slot is allocated again.  On a failure the slot is
  // left empty, so no table entry can point at a missing buffer.
  const bool whole = q.e.count == nrow && q.lam.count == nrow && q.yb.count == nrow &&
                     q.X.count == nimg && q.w.count == nimg && q.th2.count == nimg &&
                     q.wbar.count == (size_t)s->n && q.aux.count == (size_t)s->n &&
                     q.part.count == npart && q.counter.count == 2;
  auto fill = [&]() -> int {
    if (!whole) {
      HIP_OK(q.e.alloc(nrow));
      HIP_OK(q.lam.alloc(nrow));
      HIP_OK(q.yb.alloc(nrow));
      HIP_OK(q.X.alloc(nimg));
      HIP_OK(q.w.alloc(nimg));
      HIP_OK(q.th2.alloc(nimg));
      HIP_OK(q.wbar.alloc(s->n));
      HIP_OK(q.aux.alloc(s->n));
      HIP_OK(q.part.alloc(npart));
      HIP_OK(q.counter.alloc(2));
      HIP_OK(hipMemset(q.counter.p, 0, 2 * sizeof(int)));  // the epilogue ticket starts at 0
    }
    const int cap = std::max(1, resid_cap);
    if (q.resid_cap < cap || !q.resid.p) {
      q.resid_cap = 0;
      HIP_OK(q.resid.alloc((size_t)cap));
      q.resid_cap = cap;
    }
    return MACE_OK;
  };
  const int rc = fill();
  if (rc) {
    release_slot(b, idx);
    return rc;
  }
  // allocated once at the maximum size: captured graphs hold these addresses
  if (b.lastres.count < (size_t)kMaxScanSlots) HIP_OK(b.lastres.alloc(kMaxScanSlots));
  if (b.sums.count < (size_t)kMaxScanSlots * 4) HIP_OK(b.sums.alloc((size_t)kMaxScanSlots * 4));
  if (b.table.count < (size_t)kMaxScanSlots) {
    HIP_OK(b.table.alloc(kMaxScanSlots));
    b.htable.assign(kMaxScanSlots, SlotDesc{});
    HIP_OK(hipMemset(b.table.p, 0, b.table.bytes()));  // every slot inactive
  }
  return MACE_OK;
}

void release_slot(Batch& b, int idx) {
  if (idx < (int)b.scan.size()) b.scan[idx] = std::make_unique<ScanSlot>();
}

int write_slot(mace_system* s, Batch& b, int i, int active, hipStream_t st, int prec) {
  SlotDesc d{};
  if (active) {
    ScanSlot& q = *b.scan[i];
    d.e = q.e.p;
    d.lam = q.lam.p;
    d.X = q.X.p;
    d.w = q.w.p;
    d.wbar = q.wbar.p;
    d.aux = q.aux.p;
    d.th2 = q.th2.p;
    d.part = q.part.p;
    d.resid = q.resid.p;
    d.last = b.lastres.p + i;
    d.counter = q.counter.p;
    d.resid_cap = q.resid_cap;
    d.active = 1;
    d.prec = prec >= 0 ? prec : (s->precision == 1 ? 1 : 0);
  }
  b.htable[i] = d;
  HIP_OK(launch_write_slot(b.table.p, i, d, st));
  return MACE_OK;
}

}  // namespace mace

namespace {

// Launches over all four colour phases in one mode, with the slot table seen
// from `slot_base`.
int launch_phases(mace_system* s, const Schedule* sch, SvArgs a, int mode, hipStream_t st,
                  const SlotDesc* slot_base) {
  const size_t lds = sv_lds_bytes(s->bmax, s->S, s->kpad, s->format, s->wmax, s->nzp, a.vol_nz > 0);
  a.R = sch->R;
  a.slots = slot_base;
  for (int c = 0; c < 4; ++c) {
    a.tasks = sch->tasks[c].p;
    a.T = sch->T[c];
    HIP_OK(launch_sv(a, mode, s->slots, sch->grid, lds, st));
  }
  return MACE_OK;
}

// The launches of one Mann iteration: `sweeps` ICD passes (the last one with
// the reflection + Mann update) and the epilogue.  prec_mask says which
// record precisions the active slots read (bit 0: FP32, bit 1: FP16); each
// colour phase runs one launch per precision present, each launch only the
// slots of its precision (the scans are independent, so their order within
// a phase does not matter).
int enqueue_iteration(mace_system* s, Batch& b, const Schedule* sch, int n_slots, SvArgs a,
                      int sweeps, int prec_mask, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const size_t lds = sv_lds_bytes(s->bmax, s->S, s->kpad, s->format, s->wmax, s->nzp, a.vol_nz > 0);
  a.R = sch->R;
  a.slots = b.table.p;
  if (ev0) HIP_OK(hipEventRecord(ev0, st));
  for (int sw = 0; sw < sweeps; ++sw) {
    a.mann = (sw == sweeps - 1) ? 1 : 0;
    for (int c = 0; c < 4; ++c) {
      a.tasks = sch->tasks[c].p;
      a.T = sch->T[c];
      for (int pr = 0; pr < 2; ++pr) {
        if (!(prec_mask & (1 << pr))) continue;
        a.fp16 = pr;
        HIP_OK(launch_sv(a, kSweep, s->slots, sch->grid, lds, st));
      }
    }
  }
  if (ev1) HIP_OK(hipEventRecord(ev1, st));
  HIP_OK(launch_epilogue(b.table.p, n_slots, s->N, s->n, s->N * s->n_sv, st));
  if (a.hpass > 0) HIP_OK(launch_smooth(b.table.p, n_slots, s->nx, s->ny, a.hpass, st));
  return MACE_OK;
}

uint64_t args_key(const SvArgs& a) {
  uint64_t h = 1469598103934665603ULL;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ULL;
  };
  mix(&a.kind, sizeof a.kind);
  mix(&a.invN, sizeof(float) * 4);  // invN, is2, rho, relax
  mix(&a.bedge, sizeof(float) * 6);
  mix(&a.strict, sizeof a.strict);
  mix(&a.hpass, sizeof a.hpass);
  return h;
}

}  // namespace

namespace mace {

// Theta2 = sum_r A_rs^2 Lambda_r and, from y and w_init, the initial state of
// slot i: w = w_init (or 0), X = G(w) -- or X = X_init when a solve is
// resumed from a checkpoint of (w, X) --, e = y - A X (y, lam: device,
// global row order).  The slot's table entry is written and switched on.
int start_slot(mace_system* s, Batch& b, int i, const float* y, const float* lam,
               const float* w_init, const SvArgs& base, hipStream_t st, const float* X_init) {
  ScanSlot& q = *b.scan[i];
  const int64_t nrow = (int64_t)s->N * s->estride;
  HIP_OK(launch_gather_rows(q.yb.p, y, s->row_src.p, nrow, st));
  HIP_OK(launch_copy(q.e.p, q.yb.p, nrow, st));
  HIP_OK(launch_gather_rows(q.lam.p, lam, s->row_src.p, nrow, st));
  const int64_t nimg = (int64_t)s->N * s->n;
  if (w_init)
    HIP_OK(launch_copy(q.w.p, w_init, nimg, st));
  else
    HIP_OK(launch_fill(q.w.p, 0.f, nimg, st));
  HIP_OK(launch_broadcast_mean(q.w.p, q.wbar.p, q.X.p, s->N, s->n, st));
  if (X_init) HIP_OK(launch_copy(q.X.p, X_init, nimg, st));
  HIP_OK(hipMemsetAsync(q.counter.p, 0, 2 * sizeof(int), st));
  HIP_OK(hipMemsetAsync(b.lastres.p + i, 0, sizeof(double), st));
  int rc = write_slot(s, b, i, 1, st);
  if (rc) return rc;
  // theta2 (and e = y - A X when X != 0) through a one-slot schedule that
  // sees the table from this slot on
  const int P = default_rows_per_agent(s);
  Schedule* one = get_schedule(s, 1, -1, P);
  if (!one) return fail(MACE_E_HIP, "schedule upload failed");
  SvArgs a = base;
  a.strict = P == 1 ? 1 : 0;
  a.fp16 = b.htable[i].prec;
  rc = launch_phases(s, one, a, kTheta2, st, b.table.p + i);
  if (rc) return rc;
  if (w_init || X_init) {
    rc = launch_phases(s, one, a, kRefresh, st, b.table.p + i);
    if (rc) return rc;
  }
  return MACE_OK;
}

// e = y - A X for every active slot (FP32 drift), each slot with the matrix
// values of its own precision.
int refresh_slots(mace_system* s, Batch& b, int n_slots, const Schedule* sch, const SvArgs& base,
                  hipStream_t st) {
  int mask = 0;
  for (int i = 0; i < n_slots; ++i) {
    if (!b.htable[i].active) continue;
    ScanSlot& q = *b.scan[i];
    HIP_OK(launch_copy(q.e.p, q.yb.p, (int64_t)s->N * s->estride, st));
    mask |= 1 << b.htable[i].prec;
  }
  for (int pr = 0; pr < 2; ++pr) {
    if (!(mask & (1 << pr))) continue;
    SvArgs a = base;
    a.fp16 = pr;
    int rc = launch_phases(s, sch, a, kRefresh, st, b.table.p);
    if (rc) return rc;
  }
  return MACE_OK;
}

// The precision switch of an FP16 scan (slot i): from here on its sweeps read
// the FP32 matrix values; theta2 and e = y - A X_i are rebuilt with them, so
// the FP32 iterations start from the exact error sinogram of the current
// state.  Only slot i is touched (one-slot schedule seeing the table from
// slot i on).
int switch_slot_fp32(mace_system* s, Batch& b, int i, const SvArgs& base, hipStream_t st) {
  int rc = write_slot(s, b, i, 1, st, 0);
  if (rc) return rc;
  ScanSlot& q = *b.scan[i];
  HIP_OK(launch_copy(q.e.p, q.yb.p, (int64_t)s->N * s->estride, st));
  const int P = default_rows_per_agent(s);
  Schedule* one = get_schedule(s, 1, -1, P);
  if (!one) return fail(MACE_E_HIP, "schedule upload failed");
  SvArgs a = base;
  a.fp16 = 0;
  a.strict = P == 1 ? 1 : 0;
  rc = launch_phases(s, one, a, kTheta2, st, b.table.p + i);
  if (rc) return rc;
  return launch_phases(s, one, a, kRefresh, st, b.table.p + i);
}

int slot_prec_mask(const Batch& b, int n_slots) {
  int mask = 0;
  for (int i = 0; i < n_slots; ++i)
    if (b.htable[i].active) mask |= 1 << b.htable[i].prec;
  return mask;
}

// One Mann iteration through a captured graph.  The first iteration with a
// given configuration runs eagerly (it also performs the one-time kernel
// attribute set-up, which stays out of the capture); the second captures.
int run_iteration(mace_system* s, Batch& b, const Schedule* sch, int n_slots, const SvArgs& a,
                  int sweeps, int P, hipStream_t st, bool use_graph) {
  const int mask = slot_prec_mask(b, n_slots);
  if (!use_graph)
    return enqueue_iteration(s, b, sch, n_slots, a, sweeps, mask, st, nullptr, nullptr);
  const auto key = std::make_tuple(n_slots, P, sweeps, mask, args_key(a));
  auto it = b.graphs.find(key);
  if (it == b.graphs.end()) {
    b.graphs[key] = nullptr;
    return enqueue_iteration(s, b, sch, n_slots, a, sweeps, mask, st, nullptr, nullptr);
  }
  if (!it->second) {
    auto ng = std::make_unique<IterGraph>();
    hipGraph_t graph = nullptr;
    int rc;
    hipError_t e;
    {
      std::lock_guard<std::mutex> lk(capture_mutex());
      HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      rc = enqueue_iteration(s, b, sch, n_slots, a, sweeps, mask, st, nullptr, nullptr);
      e = hipStreamEndCapture(st, &graph);
    }
    ng->graph = graph;  // destroyed with ng on every return below
    if (rc) return rc;
    HIP_OK(e);
    {
      std::lock_guard<std::mutex> lk(capture_mutex());
      HIP_OK(hipGraphInstantiate(&ng->exec, graph, nullptr, nullptr, 0));
    }
    it->second = std::move(ng);
  }
  HIP_OK(hipGraphLaunch(it->second->exec, st));
  return MACE_OK;
}

// Rows per (scan, agent) for n scans in flight.  A batch that owns the GPU
// divides the automatic value by n: about the same number of rows in total,
// each row sweeping many super-voxels with all scans in step (the matrix
// records are shared in L2).  Scans that share the GPU with other streams
// (the server) keep the single-scan value: more, shorter workgroups, which
// lets the other streams' launches in between.
int batch_rows_per_agent(const mace_system* s, int n, bool share_gpu) {
  const int P = default_rows_per_agent(s);
  if (share_gpu || s->rows_per_agent > 0 || n <= 1) return P;
  return std::max(1, P / n);
}

}  // namespace mace

namespace {

struct BatchIO {
  const float* y;
  const float* lam;
  const float* w_init;
  float* x_out;
  mace_info* info;
  const float* X_init = nullptr;  // resume: the agents' states of a checkpoint
};

// Partial-update MACE (Algorithm 1) for `n` scans of this geometry at once.
// Each scan stops on its own residual; finished scans are switched off in the
// slot table while the others continue.
int solve_batch_impl(mace_system* s, int n, const BatchIO* io, const mace_prior* pr, double rho,
                     double sigma, int sweeps, int max_iters, double tol, hipStream_t user,
                     int hpass = 0) {
  // MACE-PnP (Algorithm 3, eq. (FG_PnP)): the agents' proximal maps of the
  // data terms alone (beta = 0) at sqrt(N) sigma; the consensus is
  // H(mean w), `hpass` passes of the binomial smoother after each epilogue
  const mace_prior none{0, 1.0, 2.0, 2.0, 1.0, 0.0, 0.0};
  if (hpass > 0) pr = &none;
  int rc = check_prior(pr);
  if (rc) return rc;
  if (n < 1 || n > kMaxScanSlots) return fail(MACE_E_ARG, "batch size must be in [1, %d]", kMaxScanSlots);
  if (!(rho > 0 && rho < 1)) return fail(MACE_E_ARG, "rho must be in (0, 1)");
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(MACE_E_ARG, "sigma must be > 0");
  if (sweeps < 1) return fail(MACE_E_ARG, "sweeps must be >= 1");
  if (max_iters < 0) return fail(MACE_E_ARG, "max_iters must be >= 0");
  for (int i = 0; i < n; ++i)
    if (!io[i].y || !io[i].lam || !io[i].x_out) return fail(MACE_E_ARG, "NULL scan argument");
  Batch& b = s->batch;
  hipStream_t st = s->stream;
  if (user) HIP_OK(hipStreamSynchronize(user));  // the caller's inputs are ready
  const int P = batch_rows_per_agent(s, n, false);
  Schedule* sch = get_schedule(s, n, -1, P);
  if (!sch) return fail(MACE_E_HIP, "schedule upload failed");
  for (int i = 0; i < n; ++i) {
    rc = ensure_slot(s, b, i, max_iters);
    if (rc) return rc;
  }
  const bool fp16 = s->precision == 1;
  SvArgs a;
  fill_args(s, a, pr, rho, hpass > 0 ? sigma * std::sqrt((double)s->N) : sigma, fp16);
  a.strict = P == 1 ? 1 : 0;
  if (hpass > 0) {
    a.c0 = 0.0f;  // no prior term in the agents
    a.hpass = hpass;
  }
  for (int i = 0; i < n; ++i) {
    rc = start_slot(s, b, i, io[i].y, io[i].lam, io[i].w_init, a, st, io[i].X_init);
    if (rc) return rc;
  }
  for (int i = n; i < (int)b.htable.size(); ++i)
    if (b.htable[i].active) {
      rc = write_slot(s, b, i, 0, st);
      if (rc) return rc;
    }
  const bool timing = s->timing;
  if (timing && (int)s->ev.size() < 2 * max_iters + 2) {
    std::lock_guard<std::mutex> lk(capture_mutex());
    for (auto e : s->ev) (void)hipEventDestroy(e);
    s->ev.assign(2 * max_iters + 2, nullptr);
    for (auto& e : s->ev) HIP_OK(hipEventCreate(&e));
  }
  if (timing) HIP_OK(hipEventRecord(s->ev[2 * max_iters], st));
  std::vector<int> iters(n, 0), status(n, MACE_OK), tail_iters(n, 0);
  std::vector<double> last(n, 0.0);
  // FP16 scans with an FP32 tail switch to the FP32 values when they first
  // meet tol, or fp32_tail iterations before max_iters; they stop when they
  // meet tol again in FP32 (or at max_iters).
  const bool tail = fp16 && s->fp32_tail > 0;
  const int tail_at = std::max(0, max_iters - s->fp32_tail);
  int live = n, it = 0;
  for (; it < max_iters && live > 0; ++it) {
    if (tail && it >= tail_at)
      for (int i = 0; i < n; ++i)
        if (b.htable[i].active && b.htable[i].prec == 1) {
          rc = switch_slot_fp32(s, b, i, a, st);
          if (rc) return rc;
        }
    if (s->refresh_every > 0 && it > 0 && it % s->refresh_every == 0) {
      rc = refresh_slots(s, b, n, sch, a, st);
      if (rc) return rc;
    }
    if (timing)
      rc = enqueue_iteration(s, b, sch, n, a, sweeps, slot_prec_mask(b, n), st, s->ev[2 * it],
                             s->ev[2 * it + 1]);
    else
      rc = run_iteration(s, b, sch, n, a, sweeps, P, st);
    if (rc) return rc;
    for (int i = 0; i < n; ++i)
      if (b.htable[i].active) {
        iters[i] = it + 1;
        if (tail && b.htable[i].prec == 0) ++tail_iters[i];
      }
    if (tol > 0) {
      HIP_OK(hipMemcpyAsync(last.data(), b.lastres.p, sizeof(double) * n, hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      for (int i = 0; i < n; ++i) {
        if (!b.htable[i].active) continue;
        const bool bad = !std::isfinite(last[i]);
        if (!bad && last[i] < tol && tail && b.htable[i].prec == 1) {
          // met tol with the FP16 values: continue with the FP32 ones
          if (it + 1 < max_iters) {
            rc = switch_slot_fp32(s, b, i, a, st);
            if (rc) return rc;
          }
          continue;
        }
        if (bad || last[i] < tol) {
          if (bad) status[i] = MACE_E_NONFINITE;
          rc = write_slot(s, b, i, 0, st);
          if (rc) return rc;
          --live;
        }
      }
    }
  }
  if (timing) HIP_OK(hipEventRecord(s->ev[2 * max_iters + 1], st));
  HIP_OK(hipMemcpyAsync(last.data(), b.lastres.p, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  double sweep_ms = 0.0, iter_ms = 0.0;
  if (timing) {
    for (int k = 0; k < it; ++k) {
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, s->ev[2 * k], s->ev[2 * k + 1]));
      sweep_ms += ms;
    }
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, s->ev[2 * max_iters], s->ev[2 * max_iters + 1]));
    iter_ms = ms;
  }
  int worst = MACE_OK;
  for (int i = 0; i < n; ++i) {
    ScanSlot& q = *b.scan[i];
    if (max_iters == 0) HIP_OK(launch_broadcast_mean(q.w.p, q.wbar.p, q.X.p, s->N, s->n, st));
    // x = mean_i w_i: wbar holds it after the scan's last epilogue
    HIP_OK(hipMemcpyAsync(io[i].x_out, q.wbar.p, sizeof(float) * s->n, hipMemcpyDeviceToDevice, st));
    if (status[i] == MACE_OK && !std::isfinite(last[i])) status[i] = MACE_E_NONFINITE;
    // no iteration run (max_iters = 0): tol is not met
    if (status[i] == MACE_OK && tol > 0 && (iters[i] == 0 || !(last[i] < tol)))
      status[i] = MACE_W_MAXITER;
    if (io[i].info) {
      io[i].info->iters = iters[i];
      io[i].info->residual = last[i];
      io[i].info->equits = (double)sweeps * iters[i];
      io[i].info->status = status[i];
      io[i].info->sweep_ms = sweep_ms;
      io[i].info->sweep_launches = timing ? it * sweeps * 4 : 0;
      io[i].info->iter_ms = iter_ms;
      io[i].info->fp32_tail_iters = tail_iters[i];
    }
    if (status[i] == MACE_E_NONFINITE) worst = MACE_E_NONFINITE;
    else if (status[i] == MACE_W_MAXITER && worst == MACE_OK) worst = MACE_W_MAXITER;
  }
  HIP_OK(hipStreamSynchronize(st));
  if (worst == MACE_E_NONFINITE) return fail(MACE_E_NONFINITE, "non-finite residual");
  return worst;
}

// A volume (nz slices measured by this system's 2-D matrix, coupled by the
// axial cliques of the 3-D prior): slice z runs in slot z.  Each colour
// phase is two launches, the even slices and then the odd ones, so a slice's
// axial neighbours hold still while it sweeps and both see the other
// parity's latest values (a red-black order over the slices).  The Mann
// iteration, the consensus and the residual are those of the stacked volume
// (Algorithm 1 over all nz * n voxels): the slices stop together, when
// r_k = ||X^{k+1} - G w^k|| / ||w^k|| over the whole volume is below tol.
// y, lam: device, nz blocks of the global row order; x_out: device, nz * n.
int solve_volume_impl(mace_system* s, int nz, const float* y, const float* lam,
                      const mace_prior* pr, double b_axial, double rho, double sigma, int sweeps,
                      int max_iters, double tol, float* x_out, mace_info* info) {
  int rc = check_prior(pr);
  if (rc) return rc;
  if (s->precision != 0)
    return fail(MACE_E_ARG, "volumes run with FP32 matrix values (load the system with precision 0)");
  if (nz < 1 || nz > kMaxScanSlots) return fail(MACE_E_ARG, "nz must be in [1, %d]", kMaxScanSlots);
  if (!(b_axial >= 0) || !std::isfinite(b_axial)) return fail(MACE_E_ARG, "b_axial must be >= 0");
  if (!(rho > 0 && rho < 1)) return fail(MACE_E_ARG, "rho must be in (0, 1)");
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(MACE_E_ARG, "sigma must be > 0");
  if (sweeps < 1) return fail(MACE_E_ARG, "sweeps must be >= 1");
  if (max_iters < 0) return fail(MACE_E_ARG, "max_iters must be >= 0");
  Batch& b = s->batch;
  hipStream_t st = s->stream;
  // slices in groups of Z (1: each slice its own group); rows per agent
  // for the groups of one parity together
  const int Z = std::max(1, std::min(s->slice_group, nz));
  const int ngroups = (nz + Z - 1) / Z;
  const int P = batch_rows_per_agent(s, (ngroups + 1) / 2, false);
  const Schedule* sch[2] = {get_schedule(s, nz, -1, P, 0, Z),
                            ngroups > 1 ? get_schedule(s, nz, -1, P, 1, Z) : nullptr};
  if (!sch[0] || (ngroups > 1 && !sch[1])) return fail(MACE_E_HIP, "schedule upload failed");
  for (int z = 0; z < nz; ++z) {
    rc = ensure_slot(s, b, z, max_iters);
    if (rc) return rc;
  }
  SvArgs a;
  fill_args(s, a, pr, rho, sigma, false);
  // a row sweeps a super-voxel through its group's slices in turn: each
  // task's stores complete before the next reads its axial neighbours
  a.strict = (P == 1 || Z > 1) ? 1 : 0;
  a.vol_nz = nz;
  a.baxial = (float)b_axial;
  const size_t m = (size_t)s->n_views * s->n_ch;
  for (int z = 0; z < nz; ++z) {
    rc = start_slot(s, b, z, y + z * m, lam + z * m, nullptr, a, st, nullptr);
    if (rc) return rc;
  }
  for (int i = nz; i < (int)b.htable.size(); ++i)
    if (b.htable[i].active) {
      rc = write_slot(s, b, i, 0, st);
      if (rc) return rc;
    }
  const size_t lds = sv_lds_bytes(s->bmax, s->S, s->kpad, s->format, s->wmax, s->nzp, a.vol_nz > 0);
  a.slots = b.table.p;
  std::vector<double> sums((size_t)nz * 4);
  double r = 0.0;
  int it = 0, status = MACE_OK;
  auto residual = [&]() -> int {
    HIP_OK(hipMemcpyAsync(sums.data(), b.sums.p, sizeof(double) * 4 * nz, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    double num = 0.0, den = 0.0, xx = 0.0;
    for (int z = 0; z < nz; ++z) {  // slice order: a fixed summation order
      num += sums[z * 4 + 0];
      den += sums[z * 4 + 1];
      xx += sums[z * 4 + 2];
    }
    const double d = den > 0.0 ? den : xx;
    r = !(std::isfinite(num) && std::isfinite(den) && std::isfinite(xx)) ? std::nan("")
        : d > 0.0 ? std::sqrt(num) / std::sqrt(d) : 0.0;
    return MACE_OK;
  };
  for (; it < max_iters; ++it) {
    for (int sw = 0; sw < sweeps; ++sw) {
      a.mann = (sw == sweeps - 1) ? 1 : 0;
      for (int c = 0; c < 4; ++c)
        for (int par = 0; par < 2; ++par) {
          if (!sch[par]) continue;
          a.R = sch[par]->R;
          a.tasks = sch[par]->tasks[c].p;
          a.T = sch[par]->T[c];
          HIP_OK(launch_sv(a, kSweep, s->slots, sch[par]->grid, lds, st));
        }
    }
    HIP_OK(launch_epilogue(b.table.p, nz, s->N, s->n, s->N * s->n_sv, st, b.sums.p));
    if (tol > 0) {
      rc = residual();
      if (rc) return rc;
      if (!std::isfinite(r)) {
        status = MACE_E_NONFINITE;
        ++it;
        break;
      }
      if (r < tol) {
        ++it;
        break;
      }
    }
  }
  if (it > 0 && tol <= 0) {
    rc = residual();
    if (rc) return rc;
    if (!std::isfinite(r)) status = MACE_E_NONFINITE;
  }
  for (int z = 0; z < nz; ++z) {
    ScanSlot& q = *b.scan[z];
    if (it == 0) HIP_OK(launch_broadcast_mean(q.w.p, q.wbar.p, q.X.p, s->N, s->n, st));
    HIP_OK(hipMemcpyAsync(x_out + (size_t)z * s->n, q.wbar.p, sizeof(float) * s->n,
                          hipMemcpyDeviceToDevice, st));
  }
  HIP_OK(hipStreamSynchronize(st));
  if (status == MACE_OK && tol > 0 && (it == 0 || !(r < tol))) status = MACE_W_MAXITER;
  if (info) {
    *info = mace_info{};
    info->iters = it;
    info->residual = r;
    info->equits = (double)sweeps * it;
    info->status = status;
  }
  if (status == MACE_E_NONFINITE) return fail(MACE_E_NONFINITE, "non-finite residual");
  return status;
}

}  // namespace

extern "C" int mace_solve_volume(mace_system* s, int32_t nz, const float* y, const float* lam,
                                 const mace_prior* pr, double b_axial, double rho, double sigma,
                                 int32_t sweeps, int32_t max_iters, double tol, float* x_out,
                                 mace_info* info) {
  if (!s || !y || !lam || !x_out) return fail(MACE_E_ARG, "NULL argument");
  if (nz < 1 || nz > kMaxScanSlots) return fail(MACE_E_ARG, "nz must be in [1, %d]", kMaxScanSlots);
  const size_t m = (size_t)s->n_views * s->n_ch;
  DevBuf<float> dy, dl, dx;
  HIP_OK(dy.upload(y, m * nz));
  HIP_OK(dl.upload(lam, m * nz));
  HIP_OK(dx.alloc((size_t)s->n * nz));
  int rc = solve_volume_impl(s, nz, dy.p, dl.p, pr, b_axial, rho, sigma, sweeps, max_iters, tol,
                             dx.p, info);
  if (rc < 0 && rc != MACE_E_NONFINITE) return rc;
  const std::string saved = last_error_text();
  HIP_OK(hipMemcpy(x_out, dx.p, sizeof(float) * s->n * nz, hipMemcpyDeviceToHost));
  if (rc == MACE_E_NONFINITE) return fail(MACE_E_NONFINITE, "%s", saved.c_str());
  return rc;
}

extern "C" int mace_solve_dev(mace_system* s, const float* y, const float* lam,
                              const mace_prior* pr, double rho, double sigma, int32_t sweeps,
                              int32_t max_iters, double tol, const float* w_init, float* x_out,
                              mace_info* info, void* stream) {
  if (!s || !y || !lam || !x_out) return fail(MACE_E_ARG, "NULL argument");
  BatchIO io{y, lam, w_init, x_out, info};
  return solve_batch_impl(s, 1, &io, pr, rho, sigma, sweeps, max_iters, tol, (hipStream_t)stream);
}

extern "C" int mace_solve_batch_dev(mace_system* s, int32_t n_scans, const float* const* y,
                                    const float* const* lam, const mace_prior* pr, double rho,
                                    double sigma, int32_t sweeps, int32_t max_iters, double tol,
                                    float* const* x_out, mace_info* info, void* stream) {
  if (!s || !y || !lam || !x_out) return fail(MACE_E_ARG, "NULL argument");
  if (n_scans < 1 || n_scans > kMaxScanSlots) return fail(MACE_E_ARG, "n_scans must be in [1, %d]", kMaxScanSlots);
  std::vector<BatchIO> io(n_scans);
  for (int i = 0; i < n_scans; ++i) io[i] = BatchIO{y[i], lam[i], nullptr, x_out[i], info ? info + i : nullptr};
  return solve_batch_impl(s, n_scans, io.data(), pr, rho, sigma, sweeps, max_iters, tol,
                          (hipStream_t)stream);
}

extern "C" int mace_solve_batch(mace_system* s, int32_t n_scans, const float* const* y,
                                const float* const* lam, const mace_prior* pr, double rho,
                                double sigma, int32_t sweeps, int32_t max_iters, double tol,
                                float* const* x_out, mace_info* info) {
  if (!s || !y || !lam || !x_out) return fail(MACE_E_ARG, "NULL argument");
  if (n_scans < 1 || n_scans > kMaxScanSlots) return fail(MACE_E_ARG, "n_scans must be in [1, %d]", kMaxScanSlots);
  const size_t m = (size_t)s->n_views * s->n_ch;
  std::vector<std::unique_ptr<DevBuf<float>>> bufs;
  std::vector<BatchIO> io(n_scans);
  for (int i = 0; i < n_scans; ++i) {
    if (!y[i] || !lam[i] || !x_out[i]) return fail(MACE_E_ARG, "NULL scan argument");
    auto dy = std::make_unique<DevBuf<float>>(), dl = std::make_unique<DevBuf<float>>(),
         dx = std::make_unique<DevBuf<float>>();
    HIP_OK(dy->upload(y[i], m));
    HIP_OK(dl->upload(lam[i], m));
    HIP_OK(dx->alloc(s->n));
    io[i] = BatchIO{dy->p, dl->p, nullptr, dx->p, info ? info + i : nullptr};
    bufs.push_back(std::move(dy));
    bufs.push_back(std::move(dl));
    bufs.push_back(std::move(dx));
  }
  int rc = solve_batch_impl(s, n_scans, io.data(), pr, rho, sigma, sweeps, max_iters, tol, nullptr);
  if (rc < 0 && rc != MACE_E_NONFINITE) return rc;
  const std::string saved = last_error_text();
  for (int i = 0; i < n_scans; ++i)
    HIP_OK(hipMemcpy(x_out[i], io[i].x_out, sizeof(float) * s->n, hipMemcpyDeviceToHost));
  if (rc == MACE_E_NONFINITE) return fail(MACE_E_NONFINITE, "%s", saved.c_str());
  return rc;
}

extern "C" int mace_solve(mace_system* s, const float* y, const float* lam, const mace_prior* pr,
                          double rho, double sigma, int32_t sweeps, int32_t max_iters, double tol,
                          const float* w_init, float* x_out, mace_info* info) {
  if (!s || !y || !lam || !x_out) return fail(MACE_E_ARG, "NULL argument");
  const size_t m = (size_t)s->n_views * s->n_ch, nimg = (size_t)s->N * s->n;
  DevBuf<float> dy, dl, dw, dx;
  HIP_OK(dy.upload(y, m));
  HIP_OK(dl.upload(lam, m));
  if (w_init) HIP_OK(dw.upload(w_init, nimg));
  HIP_OK(dx.alloc(s->n));
  BatchIO io{dy.p, dl.p, w_init ? dw.p : nullptr, dx.p, info};
  int rc = solve_batch_impl(s, 1, &io, pr, rho, sigma, sweeps, max_iters, tol, nullptr);
  if (rc < 0 && rc != MACE_E_NONFINITE) return rc;
  const std::string saved = last_error_text();
  HIP_OK(hipMemcpy(x_out, dx.p, sizeof(float) * s->n, hipMemcpyDeviceToHost));
  if (rc == MACE_E_NONFINITE) return fail(MACE_E_NONFINITE, "%s", saved.c_str());
  return rc;
}

extern "C" int mace_solve_resume(mace_system* s, const float* y, const float* lam,
                                 const mace_prior* pr, double rho, double sigma, int32_t sweeps,
                                 int32_t max_iters, double tol, const float* w0, const float* X0,
                                 float* x_out, mace_info* info) {
  if (!s || !y || !lam || !w0 || !X0 || !x_out) return fail(MACE_E_ARG, "NULL argument");
  const size_t m = (size_t)s->n_views * s->n_ch, nimg = (size_t)s->N * s->n;
  DevBuf<float> dy, dl, dw, dX, dx;
  HIP_OK(dy.upload(y, m));
  HIP_OK(dl.upload(lam, m));
  HIP_OK(dw.upload(w0, nimg));
  HIP_OK(dX.upload(X0, nimg));
  HIP_OK(dx.alloc(s->n));
  BatchIO io{dy.p, dl.p, dw.p, dx.p, info, dX.p};
  int rc = solve_batch_impl(s, 1, &io, pr, rho, sigma, sweeps, max_iters, tol, nullptr);
  if (rc < 0 && rc != MACE_E_NONFINITE) return rc;
  const std::string saved = last_error_text();
  HIP_OK(hipMemcpy(x_out, dx.p, sizeof(float) * s->n, hipMemcpyDeviceToHost));
  if (rc == MACE_E_NONFINITE) return fail(MACE_E_NONFINITE, "%s", saved.c_str());
  return rc;
}

extern "C" int mace_solve_pnp(mace_system* s, const float* y, const float* lam, double rho,
                              double sigma, int32_t sweeps, int32_t max_iters, double tol,
                              int32_t h_passes, float* x_out, mace_info* info) {
  if (!s || !y || !lam || !x_out) return fail(MACE_E_ARG, "NULL argument");
  if (h_passes < 1 || h_passes > 64) return fail(MACE_E_ARG, "h_passes must be in [1, 64]");
  const size_t m = (size_t)s->n_views * s->n_ch;
  DevBuf<float> dy, dl, dx;
  HIP_OK(dy.upload(y, m));
  HIP_OK(dl.upload(lam, m));
  HIP_OK(dx.alloc(s->n));
  BatchIO io{dy.p, dl.p, nullptr, dx.p, info};
  int rc = solve_batch_impl(s, 1, &io, nullptr, rho, sigma, sweeps, max_iters, tol, nullptr, h_passes);
  if (rc < 0 && rc != MACE_E_NONFINITE) return rc;
  const std::string saved = last_error_text();
  HIP_OK(hipMemcpy(x_out, dx.p, sizeof(float) * s->n, hipMemcpyDeviceToHost));
  if (rc == MACE_E_NONFINITE) return fail(MACE_E_NONFINITE, "%s", saved.c_str());
  return rc;
}

extern "C" int mace_prox(mace_system* s, int32_t agent, const float* y, const float* lam,
                         const mace_prior* pr, double sigma, const float* v,
                         const float* x_init, int32_t sweeps, float* x_out) {
  if (!s || !y || !lam || !v || !x_init || !x_out) return fail(MACE_E_ARG, "NULL argument");
  if (agent < 0 || agent >= s->N) return fail(MACE_E_ARG, "agent %d out of range", agent);
  int rc = check_prior(pr);
  if (rc) return rc;
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(MACE_E_ARG, "sigma must be > 0");
  if (sweeps < 1) return fail(MACE_E_ARG, "sweeps must be >= 1");
  const int P = default_rows_per_agent(s);
  Schedule* sch = get_schedule(s, 1, agent, P);
  if (!sch) return fail(MACE_E_HIP, "schedule upload failed");
  Batch& b = s->batch;
  rc = ensure_slot(s, b, 0, 1);
  if (rc) return rc;
  hipStream_t st = s->stream;
  rc = write_slot(s, b, 0, 1, st);
  if (rc) return rc;
  ScanSlot& q = *b.scan[0];
  const size_t m = (size_t)s->n_views * s->n_ch;
  const int64_t nrow = (int64_t)s->N * s->estride;
  DevBuf<float> dy, dl, dv;
  HIP_OK(dy.upload(y, m));
  HIP_OK(dl.upload(lam, m));
  HIP_OK(dv.upload(v, s->n));
  HIP_OK(launch_gather_rows(q.yb.p, dy.p, s->row_src.p, nrow, st));
  HIP_OK(launch_copy(q.e.p, q.yb.p, nrow, st));
  HIP_OK(launch_gather_rows(q.lam.p, dl.p, s->row_src.p, nrow, st));
  // the agent's image = x_init, its w = wbar = v, so that 2 wbar - w = v
  HIP_OK(hipMemcpyAsync(q.X.p + (size_t)agent * s->n, x_init, sizeof(float) * s->n,
                        hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(q.wbar.p, dv.p, sizeof(float) * s->n, hipMemcpyDeviceToDevice, st));
  HIP_OK(hipMemcpyAsync(q.w.p + (size_t)agent * s->n, dv.p, sizeof(float) * s->n,
                        hipMemcpyDeviceToDevice, st));
  const bool fp16 = s->precision == 1;
  SvArgs a;
  fill_args(s, a, pr, 0.5, sigma, fp16);
  a.strict = P == 1 ? 1 : 0;
  rc = launch_phases(s, sch, a, kTheta2, st, b.table.p);
  if (rc) return rc;
  rc = launch_phases(s, sch, a, kRefresh, st, b.table.p);
  if (rc) return rc;
  a.mann = 0;
  for (int sw = 0; sw < sweeps; ++sw) {
    rc = launch_phases(s, sch, a, kSweep, st, b.table.p);
    if (rc) return rc;
  }
  HIP_OK(hipMemcpyAsync(x_out, q.X.p + (size_t)agent * s->n, sizeof(float) * s->n,
                        hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  return MACE_OK;
}

extern "C" int64_t mace_scan_bytes(const mace_system* s) { return s ? slot_bytes(s, 1) : 0; }

extern "C" int mace_get_state(const mace_system* s, float* w, float* X) {
  if (!s) return fail(MACE_E_ARG, "NULL system");
  if (s->batch.scan.empty() || !s->batch.scan[0]->w.p)
    return fail(MACE_E_ARG, "no solve has run on this system");
  const size_t bytes = (size_t)s->N * s->n * sizeof(float);
  if (w) HIP_OK(hipMemcpy(w, s->batch.scan[0]->w.p, bytes, hipMemcpyDeviceToHost));
  if (X) HIP_OK(hipMemcpy(X, s->batch.scan[0]->X.p, bytes, hipMemcpyDeviceToHost));
  return MACE_OK;
}

extern "C" int mace_get_slot_state(const mace_system* s, int32_t slot, float* w, float* X) {
  if (!s) return fail(MACE_E_ARG, "NULL system");
  if (slot < 0 || slot >= (int)s->batch.scan.size() || !s->batch.scan[slot]->w.p)
    return fail(MACE_E_ARG, "slot %d holds no state", slot);
  const size_t bytes = (size_t)s->N * s->n * sizeof(float);
  if (w) HIP_OK(hipMemcpy(w, s->batch.scan[slot]->w.p, bytes, hipMemcpyDeviceToHost));
  if (X) HIP_OK(hipMemcpy(X, s->batch.scan[slot]->X.p, bytes, hipMemcpyDeviceToHost));
  return MACE_OK;
}

extern "C" int mace_get_error_sinogram(const mace_system* s, float* e) {
  if (!s || !e) return fail(MACE_E_ARG, "NULL argument");
  if (s->batch.scan.empty() || !s->batch.scan[0]->e.p)
    return fail(MACE_E_ARG, "no solve has run on this system");
  const ScanSlot& q = *s->batch.scan[0];
  std::vector<float> blk(q.e.count);
  HIP_OK(hipMemcpy(blk.data(), q.e.p, q.e.bytes(), hipMemcpyDeviceToHost));
  for (int a = 0; a < s->N; ++a)
    for (size_t kl = 0; kl < s->views[a].size(); ++kl)
      memcpy(e + (size_t)s->views[a][kl] * s->n_ch, blk.data() + (size_t)a * s->estride + kl * s->n_ch,
             sizeof(float) * s->n_ch);
  return MACE_OK;
}
