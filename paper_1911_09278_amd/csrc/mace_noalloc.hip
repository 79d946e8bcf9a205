// mace_solve_dev_noalloc: mace_solve_dev for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid allocation).  The scan state that mace_solve_dev keeps in
// buffers it allocates (error sinogram, weights, agent images, Mann state,
// theta2, residual partials, the slot table) lives here in one file-scope
// device array of fixed size; the call allocates nothing, captures no graph
// and creates no event or stream.  It runs the same kernels as mace_solve_dev
// on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "mace_runtime.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;  // 16 MiB per GPU
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  In host code the name is
// only a handle for hipGetSymbolAddress: kernels get the device address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up once per device,
// with that device current).
int scratch_ptr(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return mace::fail(MACE_E_HIP, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    HIP_OK(hipGetDevice(&cur));
    if (cur != device) HIP_OK(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    HIP_OK(e);
    if (!p) return mace::fail(MACE_E_HIP, "scratch array has no device address");
    g_ptr[device] = p;
  }
  *out = static_cast<unsigned char*>(g_ptr[device]);
  return MACE_OK;
}

__global__ void zero_words_kernel(uint32_t* __restrict__ dst, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = 0u;
}

hipError_t zero_words(void* dst, int64_t count, hipStream_t st) {
  int64_t g = (count + 255) / 256;
  g = std::max<int64_t>(1, std::min<int64_t>(g, 4096));
  hipLaunchKernelGGL(zero_words_kernel, dim3((int)g), dim3(256), 0, st,
                     static_cast<uint32_t*>(dst), count);
  return hipGetLastError();
}

// Carves the scan state out of the scratch array, 256-byte aligned pieces
// (with base 0 it only measures).
struct Carve {
  uintptr_t base;
  size_t used = 0;
  template <class T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + used);
    used += (count * sizeof(T) + 255) & ~size_t(255);
    return p;
  }
};

struct Layout {
  mace::SlotDesc* table;
  double* lastres;
  float *e, *lam, *yb, *X, *w, *wbar, *aux, *th2;
  double *part, *resid;
  int* counter;
  size_t bytes;
};

Layout carve(const mace_system* s, uintptr_t base) {
  const size_t nimg = (size_t)s->N * s->n, nrow = (size_t)s->N * s->estride;
  Carve c{base};
  Layout L;
  L.table = c.take<mace::SlotDesc>(1);
  L.lastres = c.take<double>(1);
  L.counter = c.take<int>(2);
  L.resid = c.take<double>(1);
  L.part = c.take<double>((size_t)s->N * s->n_sv * 4 + mace::epilogue_scratch_doubles());
  L.e = c.take<float>(nrow);
  L.lam = c.take<float>(nrow);
  L.yb = c.take<float>(nrow);
  L.X = c.take<float>(nimg);
  L.w = c.take<float>(nimg);
  L.th2 = c.take<float>(nimg);
  L.wbar = c.take<float>(s->n);
  L.aux = c.take<float>(s->n);
  L.bytes = c.used;
  return L;
}

int phases(const mace_system* s, const mace::Schedule* sch, mace::SvArgs a, int mode,
           hipStream_t st) {
  const size_t lds = mace::sv_lds_bytes(s->bmax, s->S, s->kpad, s->format, s->wmax, s->nzp, a.vol_nz > 0);
  a.R = sch->R;
  for (int c = 0; c < 4; ++c) {
    a.tasks = sch->tasks[c].p;
    a.T = sch->T[c];
    HIP_OK(mace::launch_sv(a, mode, s->slots, sch->grid, lds, st));
  }
  return MACE_OK;
}

}  // namespace

namespace mace {
// Called by mace_load_system on the system's device: looks up the scratch
// array's address there once, so that the entry point below finds it.
int noalloc_prepare(int device) {
  unsigned char* p = nullptr;
  return scratch_ptr(device, &p);
}
size_t noalloc_capacity() { return kScratchBytes; }
size_t noalloc_bytes(const mace_system* s) { return carve(s, 0).bytes; }
}  // namespace mace

using namespace mace;

extern "C" int mace_solve_dev_noalloc(mace_system* s, const float* y, const float* lam,
                                      const mace_prior* pr, double rho, double sigma,
                                      int32_t sweeps, int32_t max_iters, double tol,
                                      const float* w_init, float* x_out, mace_info* info,
                                      void* stream) {
  if (!s || !y || !lam || !x_out) return fail(MACE_E_ARG, "NULL argument");
  int rc = check_prior(pr);
  if (rc) return rc;
  if (!(rho > 0 && rho < 1)) return fail(MACE_E_ARG, "rho must be in (0, 1)");
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(MACE_E_ARG, "sigma must be > 0");
  if (sweeps < 1) return fail(MACE_E_ARG, "sweeps must be >= 1");
  if (max_iters < 0) return fail(MACE_E_ARG, "max_iters must be >= 0");
  unsigned char* base = nullptr;
  rc = scratch_ptr(s->device, &base);
  if (rc) return rc;
  const Layout L = carve(s, reinterpret_cast<uintptr_t>(base));
  if (L.bytes > kScratchBytes)
    return fail(MACE_E_NOMEM,
                "the scan state needs %zu bytes; the allocation-free workspace holds %zu",
                L.bytes, kScratchBytes);
  // the one-slot schedule of the automatic rows per agent, built at load
  const int P = default_rows_per_agent(s);
  auto it = s->schedules.find(std::make_tuple(1, -1, P, -1, 1));
  if (it == s->schedules.end() || !it->second)
    return fail(MACE_E_HIP, "the system's one-scan schedule is missing");
  const Schedule* sch = it->second.get();
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool fp16 = s->precision == 1;
  const int64_t nrow = (int64_t)s->N * s->estride, nimg = (int64_t)s->N * s->n;

  SvArgs a;
  fill_args(s, a, pr, rho, sigma, fp16);
  a.strict = P == 1 ? 1 : 0;
  a.slots = L.table;

  // scan state: agent-block y and Lambda, e = y, w = w_init or 0, X = G(w);
  // the counters and the residual start at zero (the previous call's
  // contents are still there)
  SlotDesc d{};
  d.e = L.e;
  d.lam = L.lam;
  d.X = L.X;
  d.w = L.w;
  d.wbar = L.wbar;
  d.aux = L.aux;
  d.th2 = L.th2;
  d.part = L.part;
  d.resid = L.resid;
  d.last = L.lastres;
  d.counter = L.counter;
  d.resid_cap = 1;
  d.active = 1;
  d.prec = fp16 ? 1 : 0;
  HIP_OK(zero_words(L.counter, 2, st));
  HIP_OK(zero_words(L.lastres, 2, st));
  HIP_OK(launch_gather_rows(L.yb, y, s->row_src.p, nrow, st));
  HIP_OK(launch_copy(L.e, L.yb, nrow, st));
  HIP_OK(launch_gather_rows(L.lam, lam, s->row_src.p, nrow, st));
  if (w_init)
    HIP_OK(launch_copy(L.w, w_init, nimg, st));
  else
    HIP_OK(launch_fill(L.w, 0.f, nimg, st));
  HIP_OK(launch_broadcast_mean(L.w, L.wbar, L.X, s->N, s->n, st));
  HIP_OK(launch_write_slot(L.table, 0, d, st));
  rc = phases(s, sch, a, kTheta2, st);
  if (rc) return rc;
  if (w_init) {
    rc = phases(s, sch, a, kRefresh, st);
    if (rc) return rc;
  }

  // FP16 values with an FP32 tail: the switch (theta2 and e rebuilt with the
  // FP32 values) when tol is first met, or fp32_tail iterations before
  // max_iters
  const bool tail = fp16 && s->fp32_tail > 0;
  const int tail_at = std::max(0, max_iters - s->fp32_tail);
  bool in16 = fp16;
  int tail_iters = 0;
  auto to_fp32 = [&]() -> int {
    in16 = false;
    a.fp16 = 0;
    d.prec = 0;
    HIP_OK(launch_write_slot(L.table, 0, d, st));
    HIP_OK(launch_copy(L.e, L.yb, nrow, st));
    int r2 = phases(s, sch, a, kTheta2, st);
    if (r2) return r2;
    return phases(s, sch, a, kRefresh, st);
  };

  // Algorithm 1, eager launches on the caller's stream
  double last = 0.0;
  int k = 0;
  int status = MACE_OK;
  for (; k < max_iters; ++k) {
    if (tail && in16 && k >= tail_at) {
      rc = to_fp32();
      if (rc) return rc;
    }
    if (!in16 && tail) ++tail_iters;
    for (int sw = 0; sw < sweeps; ++sw) {
      a.mann = (sw == sweeps - 1) ? 1 : 0;
      rc = phases(s, sch, a, kSweep, st);
      if (rc) return rc;
    }
    HIP_OK(launch_epilogue(L.table, 1, s->N, s->n, s->N * s->n_sv, st));
    if (tol > 0) {
      HIP_OK(hipMemcpyAsync(&last, L.lastres, sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      if (!std::isfinite(last)) {
        status = MACE_E_NONFINITE;
        ++k;
        break;
      }
      if (last < tol) {
        if (tail && in16) {
          if (k + 1 < max_iters) {
            rc = to_fp32();
            if (rc) return rc;
          }
          continue;
        }
        ++k;
        break;
      }
    }
  }
  if (max_iters == 0) HIP_OK(launch_broadcast_mean(L.w, L.wbar, L.X, s->N, s->n, st));
  HIP_OK(launch_copy(x_out, L.wbar, s->n, st));
  HIP_OK(hipMemcpyAsync(&last, L.lastres, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (status == MACE_OK && !std::isfinite(last)) status = MACE_E_NONFINITE;
  // no iteration run (max_iters = 0): tol is not met
  if (status == MACE_OK && tol > 0 && (k == 0 || !(last < tol))) status = MACE_W_MAXITER;
  if (info) {
    *info = mace_info{};
    info->iters = k;
    info->residual = last;
    info->equits = (double)sweeps * k;
    info->status = status;
    info->fp32_tail_iters = tail_iters;
  }
  if (status == MACE_E_NONFINITE) return fail(MACE_E_NONFINITE, "non-finite residual");
  return status;
}

extern "C" int64_t mace_noalloc_capacity(void) { return (int64_t)kScratchBytes; }
