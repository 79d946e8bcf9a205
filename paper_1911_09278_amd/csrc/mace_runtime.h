// Host-side runtime types shared by the library's translation units.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mace.h"
#include "mace_internal.h"

namespace mace {

// Allocation-failure hook for tests: when the countdown is k >= 0, the k-th
// next device allocation (0 = the next one) fails with hipErrorOutOfMemory.
std::atomic<int>& alloc_fail_countdown();
inline bool alloc_should_fail() {
  std::atomic<int>& c = alloc_fail_countdown();
  int v = c.load();
  while (v >= 0) {
    if (c.compare_exchange_weak(v, v - 1)) return v == 0;
  }
  return false;
}

// Records the calling thread's error message and returns code.
int fail(int code, const char* fmt, ...);
const std::string& last_error_text();

// Held while a stream captures an iteration graph and around the library's
// device and pinned-host allocations and frees: in this runtime such a call
// on one thread can invalidate a capture running on another.
std::mutex& capture_mutex();

#define HIP_OK(expr)                                                                       \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess)                                                                  \
      return ::mace::fail(_e == hipErrorOutOfMemory ? MACE_E_NOMEM : MACE_E_HIP,           \
                          "%s: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
  } while (0)

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t count = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { reset(); }
  void reset() {
    if (p) {
      std::lock_guard<std::mutex> lk(capture_mutex());
      (void)hipFree(p);
    }
    p = nullptr;
    count = 0;
  }
  // On failure the buffer stays empty (p == nullptr, count == 0), so a later
  // size check sees it as missing and allocates again.
  hipError_t alloc(size_t n) {
    reset();
    if (n == 0) return hipSuccess;
    std::lock_guard<std::mutex> lk(capture_mutex());
    if (alloc_should_fail()) return hipErrorOutOfMemory;
    T* q = nullptr;
    const hipError_t e = hipMalloc(reinterpret_cast<void**>(&q), n * sizeof(T));
    if (e != hipSuccess) return e;
    p = q;
    count = n;
    return hipSuccess;
  }
  hipError_t upload(const T* h, size_t n) {
    hipError_t e = alloc(n);
    if (e != hipSuccess || n == 0) return e;
    return hipMemcpy(p, h, n * sizeof(T), hipMemcpyHostToDevice);
  }
  size_t bytes() const { return count * sizeof(T); }
};

// Task tables of one schedule: one [R][T] table per colour phase.
struct Schedule {
  DevBuf<int> tasks[4];
  int R = 0, T[4] = {0, 0, 0, 0}, grid = 0;
};

// Device state of one scan.
struct ScanSlot {
  DevBuf<float> e, lam, yb, X, w, wbar, aux, th2;
  DevBuf<double> part, resid;
  DevBuf<int> counter;
  int resid_cap = 0;
  int64_t bytes() const {
    return (int64_t)(e.bytes() + lam.bytes() + yb.bytes() + X.bytes() + w.bytes() + wbar.bytes() +
                     aux.bytes() + th2.bytes() + part.bytes() + resid.bytes() + counter.bytes());
  }
};

// Iteration graph: the launches of one Mann iteration, captured once.
struct IterGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~IterGraph() {
    std::lock_guard<std::mutex> lk(capture_mutex());
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// A set of scan slots that advance together: slot table, residual read-back,
// captured iteration graphs.  A system holds one for its own solves; a
// server holds one per group of scans that share the solver parameters.
struct Batch {
  std::vector<std::unique_ptr<ScanSlot>> scan;
  DevBuf<SlotDesc> table;  // device slot table, kMaxScanSlots entries
  std::vector<SlotDesc> htable;
  DevBuf<double> lastres;  // latest residual of each slot
  DevBuf<double> sums;     // volumes: each slot's residual sums, [kMaxScanSlots][4]
  std::map<std::tuple<int, int, int, int, uint64_t>, std::unique_ptr<IterGraph>> graphs;
};

}  // namespace mace

struct mace_system {
  int nx = 0, ny = 0, n = 0, n_views = 0, n_ch = 0, N = 0;
  int Kmax = 0, slots = 0, kpad = 0;  // record values are stored at stride Kmax
  int S = 0, gx = 0, gy = 0, n_sv = 0;
  int bmax = 0;
  int rpb = 0;  // rows per workgroup of the sweep kernel (16, 8 or 4)
  int wmax = 0;
  int precision = 0;
  int rows_per_agent = 0;
  int fp32_tail = 0;
  int refresh_every = 0;
  int format = 0;  // 0: compact records (sv_kernel), 1: general records (sv_kernel_gen)
  int nzp = 0;     // general records: entries per (agent, pixel)
  int64_t estride = 0;
  std::vector<int> view_agent;          // [n_views]
  std::vector<std::vector<int>> views;  // agent -> its views, ascending
  std::vector<int> sv_pix0;             // [n_sv + 1]
  std::vector<int> colour_svs[4];       // SVs of each colour in schedule order
  // device copies of the matrix
  mace::DevBuf<float2> aval;
  mace::DevBuf<__half2> hval;
  mace::DevBuf<float> hscale;
  mace::DevBuf<uint32_t> adel;
  mace::DevBuf<float> gval;     // general records
  mace::DevBuf<uint16_t> grow;
  mace::DevBuf<mace::BandEnt> band;
  mace::DevBuf<int> band_rows;
  mace::DevBuf<int> d_sv_pix0;
  mace::DevBuf<int> row_src;  // agent-block row -> global row (or -1)
  // key: (slots, only agent, rows per agent, parity, slice group)
  std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<mace::Schedule>> schedules;
  // slot 0 serves mace_solve / mace_prox; mace_solve_batch uses 0..B-1
  mace::Batch batch;
  hipStream_t stream = nullptr;
  int device = 0;  // HIP device the system lives on
  int64_t matrix_bytes = 0;
  bool timing = false;
  double relax = 0.0;  // 0: automatic (1 for the sequential schedule, 0.5 otherwise)
  int slice_group = 1;  // volumes: consecutive slices per super-voxel group
  std::vector<hipEvent_t> ev;
  ~mace_system();
};

namespace mace {
int default_rows_per_agent(const mace_system* s);
// Task tables for n_slots slots (parity 0 / 1: only the even / odd slots).
Schedule* get_schedule(mace_system* s, int n_slots, int only_agent, int P, int parity = -1,
                       int group = 1);
int check_prior(const mace_prior* pr);
void fill_args(const mace_system* s, SvArgs& a, const mace_prior* pr, double rho, double sigma,
               bool fp16);

// Scan-slot machinery (mace_solve.cpp), shared by the batch solve and the server.
int64_t slot_bytes(const mace_system* s, int resid_cap);
int ensure_slot(mace_system* s, Batch& b, int idx, int resid_cap);
void release_slot(Batch& b, int idx);
// Writes the device table entry of slot i (stream-ordered, by a kernel).
// prec: the matrix values the slot reads (-1: the system's precision).
int write_slot(mace_system* s, Batch& b, int i, int active, hipStream_t st, int prec = -1);
int start_slot(mace_system* s, Batch& b, int i, const float* y, const float* lam,
               const float* w_init, const SvArgs& base, hipStream_t st,
               const float* X_init = nullptr);
int refresh_slots(mace_system* s, Batch& b, int n_slots, const Schedule* sch, const SvArgs& base,
                  hipStream_t st);
// Switches slot i to the FP32 matrix values (theta2 and e rebuilt with them).
int switch_slot_fp32(mace_system* s, Batch& b, int i, const SvArgs& base, hipStream_t st);
// Bit p set when an active slot among the first n_slots reads precision p.
int slot_prec_mask(const Batch& b, int n_slots);
// One Mann iteration; through a captured graph when use_graph (the batch
// solve), eager launches otherwise (the server's worker threads).
int run_iteration(mace_system* s, Batch& b, const Schedule* sch, int n_slots, const SvArgs& a,
                  int sweeps, int P, hipStream_t st, bool use_graph = true);
// Rows per (scan, agent) when n scans run together (share_gpu: other
// streams run launches beside them).
int batch_rows_per_agent(const mace_system* s, int n, bool share_gpu);
// Allocation-free entry point (mace_noalloc.hip): looks up this device's
// static workspace once; its capacity and the bytes a scan of s needs there.
int noalloc_prepare(int device);
size_t noalloc_capacity();
size_t noalloc_bytes(const mace_system* s);
}  // namespace mace
