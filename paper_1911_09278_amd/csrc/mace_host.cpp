// Host runtime of the MACE library: argument checks, repacking of the system
// matrix into the device layout, super-voxel schedules, per-scan workspace
// and the Mann-iteration driver.  The C ABI is declared in include/mace.h.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mace.h"
#include "mace_internal.h"

using namespace mace;

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(_e == hipErrorOutOfMemory ? MACE_E_NOMEM : MACE_E_HIP, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(_e), __FILE__, __LINE__);                   \
  } while (0)

extern "C" const char* mace_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------- device buffers
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t count = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
    count = 0;
  }
  hipError_t alloc(size_t n) {
    reset();
    count = n;
    if (n == 0) return hipSuccess;
    return hipMalloc(reinterpret_cast<void**>(&p), n * sizeof(T));
  }
  hipError_t upload(const T* h, size_t n) {
    hipError_t e = alloc(n);
    if (e != hipSuccess || n == 0) return e;
    return hipMemcpy(p, h, n * sizeof(T), hipMemcpyHostToDevice);
  }
  size_t bytes() const { return count * sizeof(T); }
};

// ---------------------------------------------------------------- system
struct Schedule {
  DevBuf<int> tasks[4];  // one table per colour phase: [R][T]
  int R = 0, T[4] = {0, 0, 0, 0}, grid = 0;
};

struct mace_system {
  int nx = 0, ny = 0, n = 0, n_views = 0, n_ch = 0, N = 0;
  int Kmax = 0, slots = 0, kpad = 0;
  int S = 4, gx = 0, gy = 0, n_sv = 0;
  int bmax = 0;
  int wmax = 0;
  int precision = 0;
  int rows_per_agent = 0;
  int fp32_tail = 0;
  int refresh_every = 0;
  int64_t estride = 0;
  std::vector<int> view_agent;             // [n_views]
  std::vector<std::vector<int>> views;     // agent -> its views, ascending
  std::vector<int> sv_pix0;                // [n_sv + 1]
  std::vector<int> colour_svs[4];          // SVs of each colour in schedule order
  // device copies of the matrix
  DevBuf<float2> aval;
  DevBuf<__half2> hval;
  DevBuf<float> hscale;
  DevBuf<uint16_t> aoff;
  DevBuf<BandEnt> band;
  DevBuf<int> band_rows;
  DevBuf<int> d_sv_pix0;
  DevBuf<int> row_src;                     // agent-block row -> global row (or -1)
  std::map<int64_t, std::unique_ptr<Schedule>> schedules;
  // scan workspace
  DevBuf<float> e, lam, yb, X, w, wbar, th2;
  DevBuf<double> part, resid;
  DevBuf<int> counter;
  int resid_cap = 0, part_cap = 0;
  int64_t matrix_bytes = 0;
  bool timing = false;
  double relax = 0.0;  // 0: automatic (1 for the sequential schedule, 0.5 otherwise)
  std::vector<hipEvent_t> ev;  // timing events, created on demand
  ~mace_system() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// ---------------------------------------------------------------- repacking
static int build_partition(mace_system* s, const int32_t* view_to_agent) {
  s->view_agent.resize(s->n_views);
  for (int k = 0; k < s->n_views; ++k) {
    int a = view_to_agent ? view_to_agent[k] : k % s->N;
    if (a < 0 || a >= s->N)
      return fail(MACE_E_PARTITION, "view %d assigned to agent %d (N = %d)", k, a, s->N);
    s->view_agent[k] = a;
  }
  s->views.assign(s->N, {});
  for (int k = 0; k < s->n_views; ++k) s->views[s->view_agent[k]].push_back(k);
  s->Kmax = 0;
  for (int a = 0; a < s->N; ++a) {
    if (s->views[a].empty()) return fail(MACE_E_PARTITION, "agent %d owns no view", a);
    s->Kmax = std::max<int>(s->Kmax, (int)s->views[a].size());
  }
  if (s->Kmax > kRowLanes * kMaxSlots)
    return fail(MACE_E_PARTITION, "an agent owns %d views; at most %d are supported", s->Kmax,
                kRowLanes * kMaxSlots);
  s->slots = (s->Kmax + kRowLanes - 1) / kRowLanes;
  s->kpad = s->slots * kRowLanes;
  s->estride = (int64_t)s->Kmax * s->n_ch;
  return MACE_OK;
}

static int check_matrix(const mace_system* s, const int64_t* cp, const int32_t* row,
                        const float* val) {
  const int64_t m = (int64_t)s->n_views * s->n_ch;
  if (cp[0] != 0) return fail(MACE_E_MATRIX, "col_ptr[0] = %lld, expected 0", (long long)cp[0]);
  for (int64_t c = 0; c < s->n; ++c)
    if (cp[c + 1] < cp[c]) return fail(MACE_E_MATRIX, "col_ptr decreases at column %lld", (long long)c);
  const int64_t nnz = cp[s->n];
  const int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::atomic<int> bad{0};
  std::atomic<int64_t> bad_col{-1};
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t] {
      for (int64_t c = t; c < s->n && !bad; c += nth) {
        int32_t prev = -1;
        for (int64_t q = cp[c]; q < cp[c + 1]; ++q) {
          int32_t r = row[q];
          int kind = 0;
          if (r < 0 || r >= m) kind = 1;
          else if (r <= prev) kind = 2;
          else if (!std::isfinite(val[q])) kind = 3;
          if (kind) {
            bad = kind;
            bad_col = c;
            return;
          }
          prev = r;
        }
      }
    });
  for (auto& x : th) x.join();
  (void)nnz;
  if (bad == 1) return fail(MACE_E_MATRIX, "row index out of range in column %lld", (long long)bad_col.load());
  if (bad == 2) return fail(MACE_E_MATRIX, "rows not strictly ascending in column %lld", (long long)bad_col.load());
  if (bad == 3) return fail(MACE_E_MATRIX, "non-finite value in column %lld", (long long)bad_col.load());
  return MACE_OK;
}

// Footprint of one column in one view: first channel d0 and the values on
// channels d0 and d0 + 1 (d0 + 1 < n_ch always).
struct Foot {
  int d0;
  float a0, a1;
  bool any;
};

// Host image of the device layout of the matrix.
struct HostPack {
  std::vector<float2> aval;
  std::vector<__half2> hval;
  std::vector<float> hscale;
  std::vector<uint16_t> aoff;
  std::vector<BandEnt> band;
  std::vector<int> brows;
  std::vector<int> row_src;
};

static int repack(mace_system* s, const int64_t* cp, const int32_t* row, const float* val,
                  HostPack& hp) {
  const int N = s->N, n = s->n, kpad = s->kpad, S = s->S;
  s->gx = (s->nx + S - 1) / S;
  s->gy = (s->ny + S - 1) / S;
  s->n_sv = s->gx * s->gy;
  s->sv_pix0.assign(s->n_sv + 1, 0);
  for (int sv = 0; sv < s->n_sv; ++sv) {
    int sy = sv / s->gx, sx = sv % s->gx;
    int sh = std::min(S, s->ny - sy * S), sw = std::min(S, s->nx - sx * S);
    s->sv_pix0[sv + 1] = s->sv_pix0[sv] + sh * sw;
  }
  // agent-local view index of every view
  std::vector<int> local(s->n_views);
  for (int a = 0; a < N; ++a)
    for (size_t k = 0; k < s->views[a].size(); ++k) local[s->views[a][k]] = (int)k;

  const size_t nrec = (size_t)N * n * kpad;
  std::vector<float2>& h_aval = hp.aval;
  std::vector<__half2>& h_hval = hp.hval;
  std::vector<float>& h_hscale = hp.hscale;
  if (s->precision == 0 || s->fp32_tail > 0) h_aval.resize(nrec);
  if (s->precision == 1) {
    h_hval.resize(nrec);
    h_hscale.resize((size_t)N * n);
  }
  std::vector<uint16_t>& h_aoff = hp.aoff;
  h_aoff.resize(nrec);
  std::vector<BandEnt>& h_band = hp.band;
  h_band.resize((size_t)N * s->n_sv * kpad);
  std::vector<int>& h_brows = hp.brows;
  h_brows.resize((size_t)N * s->n_sv);
  std::atomic<int> err{0};
  std::atomic<int> bmax{0};
  std::atomic<int> wmaxa{0};
  std::atomic<int64_t> err_col{-1};

  const int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t] {
      std::vector<Foot> foot;         // [npix][n_views]
      std::vector<int> cmin(s->n_views), cmax(s->n_views);
      std::vector<int> lrow(s->n_views);
      for (int sv = t; sv < s->n_sv && !err; sv += nth) {
        const int sy = sv / s->gx, sx = sv % s->gx;
        const int y0 = sy * S, x0 = sx * S;
        const int sh = std::min(S, s->ny - y0), sw = std::min(S, s->nx - x0);
        const int npix = sh * sw;
        foot.assign((size_t)npix * s->n_views, Foot{0, 0.f, 0.f, false});
        for (int j = 0; j < npix; ++j) {
          const int64_t col = (int64_t)(y0 + j / sw) * s->nx + x0 + j % sw;
          for (int64_t q = cp[col]; q < cp[col + 1]; ++q) {
            const int k = row[q] / s->n_ch, d = row[q] % s->n_ch;
            Foot& f = foot[(size_t)j * s->n_views + k];
            if (!f.any) {
              f.any = true;
              if (d + 1 < s->n_ch) {
                f.d0 = d;
                f.a0 = val[q];
                f.a1 = 0.f;
              } else if (d > 0) {
                f.d0 = d - 1;
                f.a0 = 0.f;
                f.a1 = val[q];
              } else {
                err = 1;
                err_col = col;
                return;
              }
            } else {
              // second entry of this view: must be the channel right after the first
              const int first = (f.a0 != 0.f || f.a1 == 0.f) ? f.d0 : f.d0 + 1;
              if (d != first + 1 || f.a1 != 0.f || d >= s->n_ch) {
                err = 2;
                err_col = col;
                return;
              }
              f.d0 = first;
              f.a1 = val[q];
            }
          }
        }
        for (int a = 0; a < N; ++a) {
          const auto& vw = s->views[a];
          const int K = (int)vw.size();
          int B = 0;
          const size_t asv = (size_t)a * s->n_sv + sv;
          for (int kl = 0; kl < K; ++kl) {
            const int k = vw[kl];
            int lo = 1 << 30, hi = -1;
            for (int j = 0; j < npix; ++j) {
              const Foot& f = foot[(size_t)j * s->n_views + k];
              if (!f.any) continue;
              lo = std::min(lo, f.d0);
              hi = std::max(hi, f.d0);
            }
            BandEnt b{0, 0, 0};
            if (hi >= 0) {
              b.gstart = (uint32_t)((int64_t)kl * s->n_ch + lo);
              b.width = (uint16_t)(hi - lo + 2);
              b.lds_row = (uint16_t)B;
              B += b.width;
              int cw = wmaxa.load();
              while (b.width > cw && !wmaxa.compare_exchange_weak(cw, b.width)) {
              }
            }
            cmin[k] = lo;
            lrow[k] = b.lds_row;
            h_band[asv * kpad + kl] = b;
          }
          for (int kl = K; kl < kpad; ++kl) h_band[asv * kpad + kl] = BandEnt{0, 0, 0};
          if (B + 2 > 65535) {
            err = 3;
            return;
          }
          h_brows[asv] = B;
          int cur = bmax.load();
          while (B + 2 > cur && !bmax.compare_exchange_weak(cur, B + 2)) {
          }
          for (int j = 0; j < npix; ++j) {
            const size_t rec = (size_t)a * n + s->sv_pix0[sv] + j;
            float mx = 0.f;
            for (int kl = 0; kl < K; ++kl) {
              const Foot& f = foot[(size_t)j * s->n_views + vw[kl]];
              mx = std::max(mx, std::max(std::fabs(f.a0), std::fabs(f.a1)));
            }
            const float scale = mx > 0.f ? mx : 1.f;
            if (!h_hscale.empty()) h_hscale[rec] = scale;
            for (int kl = 0; kl < kpad; ++kl) {
              const size_t idx = rec * kpad + kl;
              float a0 = 0.f, a1 = 0.f;
              int off = B;  // dummy rows
              if (kl < K) {
                const int k = vw[kl];
                const Foot& f = foot[(size_t)j * s->n_views + k];
                if (f.any) {
                  a0 = f.a0;
                  a1 = f.a1;
                  off = lrow[k] + (f.d0 - cmin[k]);
                }
              }
              if (!h_aval.empty()) h_aval[idx] = make_float2(a0, a1);
              if (!h_hval.empty()) h_hval[idx] = __floats2half2_rn(a0 / scale, a1 / scale);
              h_aoff[idx] = (uint16_t)off;
            }
          }
        }
      }
    });
  for (auto& x : th) x.join();
  if (err == 1) return fail(MACE_E_MATRIX, "column %lld: a view with a single channel detector", (long long)err_col.load());
  if (err == 2)
    return fail(MACE_E_MATRIX,
                "column %lld: more than two nonzeros, or non-adjacent channels, in one view",
                (long long)err_col.load());
  if (err == 3) return fail(MACE_E_MATRIX, "super-voxel band exceeds 65533 rows; use a smaller sv_size");
  s->bmax = (bmax.load() + 1) & ~1;
  s->wmax = wmaxa.load();
  if (s->bmax < 2) s->bmax = 2;

  // agent-block row -> global sinogram row
  hp.row_src.assign((size_t)N * s->estride, -1);
  for (int a = 0; a < N; ++a)
    for (size_t kl = 0; kl < s->views[a].size(); ++kl)
      for (int d = 0; d < s->n_ch; ++d)
        hp.row_src[(size_t)a * s->estride + kl * s->n_ch + d] = s->views[a][kl] * s->n_ch + d;

  // colour lists: SVs of colour c = (sx mod 2) + 2 (sy mod 2), in a seeded
  // random order so that the SVs processed together are spread over the image
  for (int c = 0; c < 4; ++c) s->colour_svs[c].clear();
  for (int sv = 0; sv < s->n_sv; ++sv) {
    int sy = sv / s->gx, sx = sv % s->gx;
    s->colour_svs[(sx & 1) + 2 * (sy & 1)].push_back(sv);
  }
  for (int c = 0; c < 4; ++c) {
    std::mt19937_64 rng(0x9e3779b97f4a7c15ULL + c);
    std::shuffle(s->colour_svs[c].begin(), s->colour_svs[c].end(), rng);
  }
  return MACE_OK;
}

static int upload_pack(mace_system* s, const HostPack& hp) {
  HIP_OK(s->aoff.upload(hp.aoff.data(), hp.aoff.size()));
  if (!hp.aval.empty()) HIP_OK(s->aval.upload(hp.aval.data(), hp.aval.size()));
  if (!hp.hval.empty()) {
    HIP_OK(s->hval.upload(hp.hval.data(), hp.hval.size()));
    HIP_OK(s->hscale.upload(hp.hscale.data(), hp.hscale.size()));
  }
  HIP_OK(s->band.upload(hp.band.data(), hp.band.size()));
  HIP_OK(s->band_rows.upload(hp.brows.data(), hp.brows.size()));
  HIP_OK(s->d_sv_pix0.upload(s->sv_pix0.data(), s->sv_pix0.size()));
  HIP_OK(s->row_src.upload(hp.row_src.data(), hp.row_src.size()));
  s->matrix_bytes = (int64_t)(s->aval.bytes() + s->hval.bytes() + s->hscale.bytes() +
                              s->aoff.bytes() + s->band.bytes() + s->band_rows.bytes());
  return MACE_OK;
}

// Every index the kernels form from the tables stays inside its buffer.
static int check_pack(const mace_system* s, const HostPack& hp) {
  const int N = s->N, kpad = s->kpad;
  for (int a = 0; a < N; ++a) {
    const int64_t K = (int64_t)s->views[a].size();
    for (int sv = 0; sv < s->n_sv; ++sv) {
      const size_t asv = (size_t)a * s->n_sv + sv;
      const int B = hp.brows[asv];
      if (B < 0 || B + 2 > s->bmax) return fail(MACE_E_MATRIX, "check: band rows %d exceed bmax %d", B, s->bmax);
      int rows = 0;
      for (int kl = 0; kl < kpad; ++kl) {
        const BandEnt& b = hp.band[asv * kpad + kl];
        if (b.width == 0) continue;
        if (kl >= K) return fail(MACE_E_MATRIX, "check: band entry on a padding view");
        if ((int)b.lds_row + b.width > B) return fail(MACE_E_MATRIX, "check: band overruns its rows");
        if ((int64_t)b.gstart + b.width > K * s->n_ch) return fail(MACE_E_MATRIX, "check: band leaves the agent block");
        if ((int64_t)b.gstart / s->n_ch != kl ||
            ((int64_t)b.gstart + b.width - 1) / s->n_ch != kl)
          return fail(MACE_E_MATRIX, "check: band crosses a view boundary");
        rows += b.width;
      }
      if (rows != B) return fail(MACE_E_MATRIX, "check: band rows do not add up");
      const int npix = s->sv_pix0[sv + 1] - s->sv_pix0[sv];
      if (npix < 1 || npix > s->S * s->S) return fail(MACE_E_MATRIX, "check: bad SV pixel count");
      for (int j = 0; j < npix; ++j) {
        const size_t rec = (size_t)a * s->n + s->sv_pix0[sv] + j;
        for (int kl = 0; kl < kpad; ++kl) {
          const int off = hp.aoff[rec * kpad + kl];
          if (off > B) return fail(MACE_E_MATRIX, "check: record row %d beyond band (%d)", off, B);
          if (kl < K && off < B) {
            const BandEnt& b = hp.band[asv * kpad + kl];
            if (off < b.lds_row || off + 1 >= b.lds_row + b.width)
              return fail(MACE_E_MATRIX, "check: record row outside its view's band");
          }
        }
      }
    }
  }
  if (s->sv_pix0[s->n_sv] != s->n) return fail(MACE_E_MATRIX, "check: SVs do not tile the image");
  return MACE_OK;
}

// ---------------------------------------------------------------- schedules
// Rows of 16 lanes are grouped 16 to a workgroup; workgroups are dispatched
// round-robin over the 8 XCDs, so the rows serving one agent are placed in
// workgroups of one XCD where possible (its e/Lambda then live in one L2).
struct HostSchedule {
  int grid = 0, R = 0, T[4] = {0, 0, 0, 0};
  std::vector<int> tab[4];
};

static void build_schedule(const mace_system* s, int only_agent, int P, HostSchedule& hs) {
  std::vector<int> agents;
  if (only_agent >= 0)
    agents.push_back(only_agent);
  else
    for (int a = 0; a < s->N; ++a) agents.push_back(a);
  const int nxcd = 8;
  std::vector<std::vector<std::pair<int, int>>> xrows(nxcd);  // (agent, rank within agent)
  for (size_t i = 0; i < agents.size(); ++i) {
    const int x = (int)(i % nxcd);
    for (int r = 0; r < P; ++r) xrows[x].push_back({agents[i], r});
  }
  int wg_per_xcd = 0;
  for (int x = 0; x < nxcd; ++x)
    wg_per_xcd = std::max<int>(wg_per_xcd, (int)((xrows[x].size() + kRowsPerBlock - 1) / kRowsPerBlock));
  std::vector<std::pair<int, int>> row_of;  // global row -> (agent, rank) or (-1, -1)
  if (agents.size() >= (size_t)nxcd) {
    hs.grid = wg_per_xcd * nxcd;
    row_of.assign((size_t)hs.grid * kRowsPerBlock, {-1, -1});
    for (int x = 0; x < nxcd; ++x)
      for (size_t q = 0; q < xrows[x].size(); ++q) {
        const int u = (int)(q / kRowsPerBlock), j = (int)(q % kRowsPerBlock);
        row_of[(size_t)(u * nxcd + x) * kRowsPerBlock + j] = xrows[x][q];
      }
  } else {
    // fewer agents than XCDs: pack the rows densely
    std::vector<std::pair<int, int>> all;
    for (int a : agents)
      for (int r = 0; r < P; ++r) all.push_back({a, r});
    hs.grid = (int)((all.size() + kRowsPerBlock - 1) / kRowsPerBlock);
    row_of.assign((size_t)hs.grid * kRowsPerBlock, {-1, -1});
    for (size_t q = 0; q < all.size(); ++q) row_of[q] = all[q];
  }
  hs.R = hs.grid * kRowsPerBlock;
  for (int c = 0; c < 4; ++c) {
    const auto& L = s->colour_svs[c];
    const int T = (int)((L.size() + P - 1) / P);
    hs.T[c] = T;
    hs.tab[c].assign((size_t)hs.R * std::max(T, 1), -1);
    for (int r = 0; r < hs.R; ++r) {
      const int a = row_of[r].first, rank = row_of[r].second;
      if (a < 0) continue;
      for (int t = 0; t < T; ++t) {
        const size_t q = (size_t)t * P + rank;
        if (q < L.size()) hs.tab[c][(size_t)r * T + t] = a * s->n_sv + L[q];
      }
    }
  }
}

// Every (agent, SV) of the scheduled agents appears exactly once per pass,
// in the phase of its colour, and every task id is in range.
static int check_schedule(const mace_system* s, int only_agent, const HostSchedule& hs) {
  std::vector<int> seen((size_t)s->N * s->n_sv, 0);
  for (int c = 0; c < 4; ++c)
    for (int t : hs.tab[c]) {
      if (t < 0) continue;
      if (t >= s->N * s->n_sv) return fail(MACE_E_ARG, "check: task id out of range");
      const int sv = t % s->n_sv;
      if (((sv % s->gx) & 1) + 2 * ((sv / s->gx) & 1) != c) return fail(MACE_E_ARG, "check: task in the wrong colour phase");
      seen[t]++;
    }
  for (int a = 0; a < s->N; ++a)
    for (int sv = 0; sv < s->n_sv; ++sv) {
      const int want = (only_agent < 0 || only_agent == a) ? 1 : 0;
      if (seen[(size_t)a * s->n_sv + sv] != want) return fail(MACE_E_ARG, "check: task visited %d times", seen[(size_t)a * s->n_sv + sv]);
    }
  return MACE_OK;
}

static Schedule* get_schedule(mace_system* s, int only_agent, int P) {
  const int64_t key = ((int64_t)(only_agent + 1) << 32) | (uint32_t)P;
  auto it = s->schedules.find(key);
  if (it != s->schedules.end()) return it->second.get();
  HostSchedule hs;
  build_schedule(s, only_agent, P, hs);
  if (check_schedule(s, only_agent, hs)) return nullptr;
  auto sch = std::make_unique<Schedule>();
  sch->grid = hs.grid;
  sch->R = hs.R;
  for (int c = 0; c < 4; ++c) {
    sch->T[c] = hs.T[c];
    if (sch->tasks[c].upload(hs.tab[c].data(), hs.tab[c].size()) != hipSuccess) return nullptr;
  }
  Schedule* out = sch.get();
  s->schedules[key] = std::move(sch);
  return out;
}

// Concurrent super-voxels per agent: enough 16-lane rows in total (about
// 4096, i.e. 1024 waves) to keep every CU busy, but at most a quarter of the
// SVs of one colour (updating a whole colour at once is block Jacobi, which
// loses stability on small images).
static int default_rows_per_agent(const mace_system* s) {
  if (s->rows_per_agent > 0) return s->rows_per_agent;
  const int per_colour = (s->n_sv + 3) / 4;
  const int P = (4096 + s->N - 1) / s->N;
  return std::max(1, std::min(P, per_colour / 4));
}

// ---------------------------------------------------------------- workspace
static int ensure_workspace(mace_system* s, int max_iters, int R) {
  const size_t nimg = (size_t)s->N * s->n;
  const size_t nrow = (size_t)s->N * s->estride;
  if (s->e.count != nrow) {
    HIP_OK(s->e.alloc(nrow));
    HIP_OK(s->lam.alloc(nrow));
    HIP_OK(s->yb.alloc(nrow));
    HIP_OK(s->X.alloc(nimg));
    HIP_OK(s->w.alloc(nimg));
    HIP_OK(s->th2.alloc(nimg));
    HIP_OK(s->wbar.alloc(s->n));
    HIP_OK(s->counter.alloc(1));
  }
  const int pc = 4 * R;
  if (s->part_cap < pc) {
    HIP_OK(s->part.alloc((size_t)pc * 4));
    s->part_cap = pc;
  }
  if (s->resid_cap < max_iters) {
    HIP_OK(s->resid.alloc((size_t)std::max(1, max_iters)));
    s->resid_cap = std::max(1, max_iters);
  }
  return MACE_OK;
}

static void fill_args(const mace_system* s, SvArgs& a, const mace_prior* pr, double rho,
                      double sigma, bool fp16) {
  memset(&a, 0, sizeof a);
  a.nx = s->nx;
  a.ny = s->ny;
  a.n = s->n;
  a.S = s->S;
  a.gx = s->gx;
  a.n_sv = s->n_sv;
  a.kpad = s->kpad;
  a.bmax = s->bmax;
  a.wmax = s->wmax;
  a.sv_pix0 = s->d_sv_pix0.p;
  a.aval = s->aval.p;
  a.hval = s->hval.p;
  a.hscale = s->hscale.p;
  a.fp16 = fp16 ? 1 : 0;
  a.aoff = s->aoff.p;
  a.band = s->band.p;
  a.band_rows = s->band_rows.p;
  a.estride = s->estride;
  a.e = s->e.p;
  a.lam = s->lam.p;
  a.X = s->X.p;
  a.w = s->w.p;
  a.wbar = s->wbar.p;
  a.th2 = s->th2.p;
  a.invN = (float)(1.0 / s->N);
  a.relax = (float)(s->relax > 0.0 ? s->relax : (default_rows_per_agent(s) == 1 ? 1.0 : 0.5));
  a.rho = (float)rho;
  a.is2 = sigma > 0 ? (float)(1.0 / (sigma * sigma)) : 0.f;
  if (pr) {
    const double be = (pr->b_edge == 0 && pr->b_diag == 0) ? 1.0 / (4.0 + 2.0 * std::sqrt(2.0)) : pr->b_edge;
    const double bd = (pr->b_edge == 0 && pr->b_diag == 0) ? 1.0 / (4.0 * std::sqrt(2.0) + 4.0) : pr->b_diag;
    a.kind = pr->kind;
    a.bedge = (float)be;
    a.bdiag = (float)bd;
    a.c0 = (float)(1.0 / (pr->sigma_x * pr->sigma_x));
    a.inv_tsx = pr->kind == 1 ? (float)(1.0 / (pr->T * pr->sigma_x)) : 0.f;
    a.qexp = pr->kind == 1 ? (float)(2.0 - pr->q) : 0.f;
    a.qhalf = pr->kind == 1 ? (float)(pr->q / 2.0) : 0.f;
  }
}

static int check_prior(const mace_prior* pr) {
  if (!pr) return fail(MACE_E_ARG, "prior is NULL");
  if (pr->kind != 0 && pr->kind != 1) return fail(MACE_E_ARG, "prior kind %d unknown", pr->kind);
  if (!(pr->sigma_x > 0) || !std::isfinite(pr->sigma_x)) return fail(MACE_E_ARG, "sigma_x must be > 0");
  if (pr->kind == 1) {
    if (pr->p != 2.0) return fail(MACE_E_ARG, "q-GGMRF: the GPU path needs p = 2 (got %g)", pr->p);
    if (!(pr->q >= 1.0 && pr->q <= pr->p)) return fail(MACE_E_ARG, "q-GGMRF: need 1 <= q <= p");
    if (!(pr->T > 0) || !std::isfinite(pr->T)) return fail(MACE_E_ARG, "q-GGMRF: T must be > 0");
  }
  if (pr->b_edge < 0 || pr->b_diag < 0) return fail(MACE_E_ARG, "negative neighbour weight");
  return MACE_OK;
}

// ---------------------------------------------------------------- ABI
extern "C" int mace_load_system(const mace_geom* geom, const int64_t* col_ptr,
                                const int32_t* row_idx, const float* val, int32_t n_agents,
                                const int32_t* view_to_agent, const mace_opts* opts,
                                mace_system** out) {
  if (!out) return fail(MACE_E_ARG, "out is NULL");
  *out = nullptr;
  if (!geom || !col_ptr || !row_idx || !val) return fail(MACE_E_ARG, "NULL argument");
  if (geom->nx <= 0 || geom->ny <= 0 || geom->n_views <= 0 || geom->n_channels < 2)
    return fail(MACE_E_ARG, "bad geometry (need sizes > 0 and >= 2 channels)");
  if ((int64_t)geom->nx * geom->ny > (1LL << 30)) return fail(MACE_E_ARG, "image too large");
  if ((int64_t)geom->n_views * geom->n_channels >= (1LL << 31)) return fail(MACE_E_ARG, "sinogram too large");
  if (n_agents <= 0) return fail(MACE_E_ARG, "n_agents must be > 0");
  auto s = std::make_unique<mace_system>();
  s->nx = geom->nx;
  s->ny = geom->ny;
  s->n = geom->nx * geom->ny;
  s->n_views = geom->n_views;
  s->n_ch = geom->n_channels;
  s->N = n_agents;
  if (opts) {
    if (opts->precision != 0 && opts->precision != 1) return fail(MACE_E_ARG, "precision must be 0 or 1");
    if (opts->sv_size != 0 && opts->sv_size != 4 && opts->sv_size != 8)
      return fail(MACE_E_ARG, "sv_size must be 0 (default 4), 4 or 8");
    if (opts->rows_per_agent < 0) return fail(MACE_E_ARG, "rows_per_agent must be >= 0");
    if (opts->fp32_tail_iters < 0) return fail(MACE_E_ARG, "fp32_tail_iters must be >= 0");
    s->precision = opts->precision;
    s->S = opts->sv_size;
    s->rows_per_agent = opts->rows_per_agent;
    s->fp32_tail = opts->precision == 1 ? opts->fp32_tail_iters : 0;
    if (opts->refresh_every < 0) return fail(MACE_E_ARG, "refresh_every must be >= 0");
    s->refresh_every = opts->refresh_every;
  }
  if (s->S == 0) s->S = std::min(s->nx, s->ny) >= 256 ? 8 : 4;
  int rc = build_partition(s.get(), view_to_agent);
  if (rc) return rc;
  rc = check_matrix(s.get(), col_ptr, row_idx, val);
  if (rc) return rc;
  {
    HostPack hp;
    rc = repack(s.get(), col_ptr, row_idx, val, hp);
    if (rc) return rc;
    rc = check_pack(s.get(), hp);
    if (rc) return rc;
    rc = upload_pack(s.get(), hp);
    if (rc) return rc;
  }
  if (sv_lds_bytes(s->bmax, s->S, s->kpad) > 160 * 1024)
    return fail(MACE_E_ARG, "super-voxel band needs %zu bytes of LDS per workgroup; use a smaller sv_size",
                sv_lds_bytes(s->bmax, s->S, s->kpad));
  *out = s.release();
  g_err.clear();
  return MACE_OK;
}

// Host-only dry run of mace_load_system plus the schedules: builds every
// table and checks all the indices the kernels will form, without a device.
extern "C" int mace_check_layout(const mace_geom* geom, const int64_t* col_ptr,
                                 const int32_t* row_idx, const float* val, int32_t n_agents,
                                 const int32_t* view_to_agent, const mace_opts* opts,
                                 int64_t* lds_bytes) {
  if (!geom || !col_ptr || !row_idx || !val || n_agents <= 0) return fail(MACE_E_ARG, "bad argument");
  if (geom->nx <= 0 || geom->ny <= 0 || geom->n_views <= 0 || geom->n_channels < 2)
    return fail(MACE_E_ARG, "bad geometry");
  mace_system s;
  s.nx = geom->nx;
  s.ny = geom->ny;
  s.n = geom->nx * geom->ny;
  s.n_views = geom->n_views;
  s.n_ch = geom->n_channels;
  s.N = n_agents;
  if (opts) {
    if (opts->sv_size != 0 && opts->sv_size != 4 && opts->sv_size != 8)
      return fail(MACE_E_ARG, "sv_size must be 0 (default 4), 4 or 8");
    s.precision = opts->precision;
    s.S = opts->sv_size;
    s.rows_per_agent = opts->rows_per_agent;
    s.fp32_tail = opts->precision == 1 ? opts->fp32_tail_iters : 0;
  }
  if (s.S == 0) s.S = std::min(s.nx, s.ny) >= 256 ? 8 : 4;
  int rc = build_partition(&s, view_to_agent);
  if (rc) return rc;
  rc = check_matrix(&s, col_ptr, row_idx, val);
  if (rc) return rc;
  HostPack hp;
  rc = repack(&s, col_ptr, row_idx, val, hp);
  if (rc) return rc;
  rc = check_pack(&s, hp);
  if (rc) return rc;
  const int P = default_rows_per_agent(&s);
  for (int only = -1; only < s.N; ++only) {
    for (int PP : {1, P}) {
      HostSchedule hs;
      build_schedule(&s, only, PP, hs);
      rc = check_schedule(&s, only, hs);
      if (rc) return rc;
    }
    if (only >= 2) break;
  }
  if (lds_bytes) *lds_bytes = (int64_t)sv_lds_bytes(s.bmax, s.S, s.kpad);
  if (sv_lds_bytes(s.bmax, s.S, s.kpad) > 160 * 1024) return fail(MACE_E_ARG, "LDS per workgroup exceeds 160 KiB");
  return MACE_OK;
}

extern "C" void mace_free_system(mace_system* s) { delete s; }

extern "C" int64_t mace_system_bytes(const mace_system* s) { return s ? s->matrix_bytes : 0; }

extern "C" int mace_set_relaxation(mace_system* s, double relax) {
  if (!s) return fail(MACE_E_ARG, "NULL system");
  if (!(relax > 0.0 && relax <= 1.0)) return fail(MACE_E_ARG, "relaxation must be in (0, 1]");
  s->relax = relax;
  return MACE_OK;
}

extern "C" int mace_set_timing(mace_system* s, int32_t enable) {
  if (!s) return fail(MACE_E_ARG, "NULL system");
  s->timing = enable != 0;
  return MACE_OK;
}

extern "C" int mace_visit_order(const mace_system* s, int64_t* order) {
  if (!s || !order) return fail(MACE_E_ARG, "NULL argument");
  int64_t q = 0;
  for (int c = 0; c < 4; ++c)
    for (int sv : s->colour_svs[c]) {
      const int sy = sv / s->gx, sx = sv % s->gx;
      const int y0 = sy * s->S, x0 = sx * s->S;
      const int sh = std::min(s->S, s->ny - y0), sw = std::min(s->S, s->nx - x0);
      for (int j = 0; j < sh * sw; ++j) order[q++] = (int64_t)(y0 + j / sw) * s->nx + x0 + j % sw;
    }
  return MACE_OK;
}

extern "C" int mace_get_state(const mace_system* s, float* w, float* X) {
  if (!s) return fail(MACE_E_ARG, "NULL system");
  if (!s->w.p) return fail(MACE_E_ARG, "no solve has run on this system");
  const size_t bytes = (size_t)s->N * s->n * sizeof(float);
  if (w) HIP_OK(hipMemcpy(w, s->w.p, bytes, hipMemcpyDeviceToHost));
  if (X) HIP_OK(hipMemcpy(X, s->X.p, bytes, hipMemcpyDeviceToHost));
  return MACE_OK;
}

extern "C" int mace_get_error_sinogram(const mace_system* s, float* e) {
  if (!s || !e) return fail(MACE_E_ARG, "NULL argument");
  if (!s->e.p) return fail(MACE_E_ARG, "no solve has run on this system");
  std::vector<float> blk(s->e.count);
  HIP_OK(hipMemcpy(blk.data(), s->e.p, s->e.bytes(), hipMemcpyDeviceToHost));
  for (int a = 0; a < s->N; ++a)
    for (size_t kl = 0; kl < s->views[a].size(); ++kl)
      memcpy(e + (size_t)s->views[a][kl] * s->n_ch, blk.data() + (size_t)a * s->estride + kl * s->n_ch,
             sizeof(float) * s->n_ch);
  return MACE_OK;
}

// Load y / Lambda (device, global row order) into the agent blocks and set the
// initial state: w = w_init (or 0), X = G(w), e = y - A X, theta2.
static int start_scan(mace_system* s, const float* y, const float* lam, const float* w_init,
                      const mace_prior* pr, double sigma, bool fp16, hipStream_t st) {
  const int64_t nrow = (int64_t)s->N * s->estride;
  HIP_OK(launch_gather_rows(s->yb.p, y, s->row_src.p, nrow, st));
  HIP_OK(launch_copy(s->e.p, s->yb.p, nrow, st));
  HIP_OK(launch_gather_rows(s->lam.p, lam, s->row_src.p, nrow, st));
  const int64_t nimg = (int64_t)s->N * s->n;
  if (w_init)
    HIP_OK(launch_copy(s->w.p, w_init, nimg, st));
  else
    HIP_OK(launch_fill(s->w.p, 0.f, nimg, st));
  HIP_OK(launch_broadcast_mean(s->w.p, s->wbar.p, s->X.p, s->N, s->n, st));
  const int P = default_rows_per_agent(s);
  Schedule* sch = get_schedule(s, -1, P);
  if (!sch) return fail(MACE_E_HIP, "schedule upload failed");
  SvArgs a;
  fill_args(s, a, pr, 0.8, sigma, fp16);
  a.R = sch->R;
  a.strict = P == 1 ? 1 : 0;
  const size_t lds = sv_lds_bytes(s->bmax, s->S, s->kpad);
  for (int c = 0; c < 4; ++c) {
    a.tasks = sch->tasks[c].p;
    a.T = sch->T[c];
    HIP_OK(launch_sv(a, kTheta2, s->slots, sch->grid, lds, st));
    if (w_init) HIP_OK(launch_sv(a, kRefresh, s->slots, sch->grid, lds, st));
  }
  return MACE_OK;
}

static int solve_impl(mace_system* s, const float* y, const float* lam, const mace_prior* pr,
                      double rho, double sigma, int sweeps, int max_iters, double tol,
                      const float* w_init, float* x_out, mace_info* info, hipStream_t st) {
  int rc = check_prior(pr);
  if (rc) return rc;
  if (!(rho > 0 && rho < 1)) return fail(MACE_E_ARG, "rho must be in (0, 1)");
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(MACE_E_ARG, "sigma must be > 0");
  if (sweeps < 1) return fail(MACE_E_ARG, "sweeps must be >= 1");
  if (max_iters < 0) return fail(MACE_E_ARG, "max_iters must be >= 0");
  const int P = default_rows_per_agent(s);
  Schedule* sch = get_schedule(s, -1, P);
  if (!sch) return fail(MACE_E_HIP, "schedule upload failed");
  rc = ensure_workspace(s, max_iters, sch->R);
  if (rc) return rc;
  const bool fp16 = s->precision == 1;
  rc = start_scan(s, y, lam, w_init, pr, sigma, fp16, st);
  if (rc) return rc;
  HIP_OK(hipMemsetAsync(s->counter.p, 0, sizeof(int), st));
  const size_t lds = sv_lds_bytes(s->bmax, s->S, s->kpad);
  SvArgs a;
  fill_args(s, a, pr, rho, sigma, fp16);
  a.R = sch->R;
  a.strict = P == 1 ? 1 : 0;
  std::vector<double> hres(std::max(1, max_iters));
  // timing: one event pair around the sweep launches of each iteration, one
  // pair around the whole loop
  const bool timing = s->timing;
  if (timing && (int)s->ev.size() < 2 * max_iters + 2) {
    for (auto e : s->ev) (void)hipEventDestroy(e);
    s->ev.assign(2 * max_iters + 2, nullptr);
    for (auto& e : s->ev) HIP_OK(hipEventCreate(&e));
  }
  if (timing) HIP_OK(hipEventRecord(s->ev[2 * max_iters], st));
  int it = 0;
  int status = MACE_OK;
  double last = 0.0;
  const int check_every = tol > 0 ? 1 : 0;
  bool refreshed = false;
  for (; it < max_iters; ++it) {
    if (fp16 && s->fp32_tail > 0 && !refreshed && it >= max_iters - s->fp32_tail) {
      // switch to FP32 A values: rebuild e = y - A X and theta2 with them
      a.fp16 = 0;
      refreshed = true;
      HIP_OK(launch_copy(s->e.p, s->yb.p, (int64_t)s->N * s->estride, st));
      for (int c = 0; c < 4; ++c) {
        a.tasks = sch->tasks[c].p;
        a.T = sch->T[c];
        HIP_OK(launch_sv(a, kTheta2, s->slots, sch->grid, lds, st));
        HIP_OK(launch_sv(a, kRefresh, s->slots, sch->grid, lds, st));
      }
    }
    if (s->refresh_every > 0 && it > 0 && it % s->refresh_every == 0 && !refreshed) {
      // rebuild e = y - A X_i from the agent states (FP32 drift of the
      // incrementally updated error sinogram)
      HIP_OK(launch_copy(s->e.p, s->yb.p, (int64_t)s->N * s->estride, st));
      for (int c = 0; c < 4; ++c) {
        a.tasks = sch->tasks[c].p;
        a.T = sch->T[c];
        HIP_OK(launch_sv(a, kRefresh, s->slots, sch->grid, lds, st));
      }
    }
    if (timing) HIP_OK(hipEventRecord(s->ev[2 * it], st));
    for (int sw = 0; sw < sweeps; ++sw) {
      a.mann = (sw == sweeps - 1) ? 1 : 0;
      for (int c = 0; c < 4; ++c) {
        a.tasks = sch->tasks[c].p;
        a.T = sch->T[c];
        a.part = s->part.p + (size_t)c * sch->R * 4;
        HIP_OK(launch_sv(a, kSweep, s->slots, sch->grid, lds, st));
      }
    }
    if (timing) HIP_OK(hipEventRecord(s->ev[2 * it + 1], st));
    HIP_OK(launch_epilogue(s->w.p, s->wbar.p, s->N, s->n, s->part.p, 4 * sch->R, s->resid.p,
                           s->counter.p, max_iters, st));
    if (check_every) {
      HIP_OK(hipMemcpyAsync(&last, s->resid.p + it, sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      if (!std::isfinite(last)) {
        status = MACE_E_NONFINITE;
        ++it;
        break;
      }
      if (last < tol) {
        ++it;
        break;
      }
    }
  }
  if (timing) HIP_OK(hipEventRecord(s->ev[2 * max_iters + 1], st));
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
  if (it > 0) {
    HIP_OK(hipMemcpy(hres.data(), s->resid.p, sizeof(double) * it, hipMemcpyDeviceToHost));
    last = hres[it - 1];
    if (!std::isfinite(last)) status = MACE_E_NONFINITE;
  }
  if (status == MACE_OK && tol > 0 && !(last < tol)) status = MACE_W_MAXITER;
  // x = mean_i w_i: wbar already holds it after the last epilogue
  if (max_iters == 0) HIP_OK(launch_broadcast_mean(s->w.p, s->wbar.p, s->X.p, s->N, s->n, st));
  HIP_OK(launch_copy(x_out, s->wbar.p, s->n, st));
  HIP_OK(hipStreamSynchronize(st));
  if (info) {
    info->iters = it;
    info->residual = last;
    info->equits = (double)sweeps * it;
    info->status = status;
    info->sweep_ms = sweep_ms;
    info->sweep_launches = timing ? it * sweeps * 4 : 0;
    info->iter_ms = iter_ms;
  }
  if (status == MACE_E_NONFINITE) return fail(MACE_E_NONFINITE, "non-finite residual at iteration %d", it);
  return status;
}

extern "C" int mace_solve_dev(mace_system* s, const float* y, const float* lam,
                              const mace_prior* pr, double rho, double sigma, int32_t sweeps,
                              int32_t max_iters, double tol, const float* w_init, float* x_out,
                              mace_info* info, void* stream) {
  if (!s || !y || !lam || !x_out) return fail(MACE_E_ARG, "NULL argument");
  return solve_impl(s, y, lam, pr, rho, sigma, sweeps, max_iters, tol, w_init, x_out, info,
                    (hipStream_t)stream);
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
  int rc = solve_impl(s, dy.p, dl.p, pr, rho, sigma, sweeps, max_iters, tol,
                      w_init ? dw.p : nullptr, dx.p, info, nullptr);
  if (rc < 0 && rc != MACE_E_NONFINITE) return rc;
  HIP_OK(hipMemcpy(x_out, dx.p, sizeof(float) * s->n, hipMemcpyDeviceToHost));
  if (rc == MACE_E_NONFINITE) return fail(MACE_E_NONFINITE, "%s", g_err.c_str());
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
  Schedule* sch = get_schedule(s, agent, P);
  Schedule* full = get_schedule(s, -1, P);
  if (!sch || !full) return fail(MACE_E_HIP, "schedule upload failed");
  rc = ensure_workspace(s, 1, std::max(sch->R, full->R));
  if (rc) return rc;
  const size_t m = (size_t)s->n_views * s->n_ch;
  const int64_t nrow = (int64_t)s->N * s->estride;
  DevBuf<float> dy, dl, dv;
  HIP_OK(dy.upload(y, m));
  HIP_OK(dl.upload(lam, m));
  HIP_OK(dv.upload(v, s->n));
  hipStream_t st = nullptr;
  HIP_OK(launch_gather_rows(s->e.p, dy.p, s->row_src.p, nrow, st));
  HIP_OK(launch_gather_rows(s->lam.p, dl.p, s->row_src.p, nrow, st));
  // every agent's image = x_init, w_agent = wbar = v so that 2 wbar - w = v
  std::vector<float> xi((size_t)s->N * s->n);
  for (int a = 0; a < s->N; ++a) memcpy(xi.data() + (size_t)a * s->n, x_init, sizeof(float) * s->n);
  HIP_OK(hipMemcpy(s->X.p, xi.data(), sizeof(float) * xi.size(), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(s->wbar.p, dv.p, sizeof(float) * s->n, hipMemcpyDeviceToDevice));
  HIP_OK(hipMemcpy(s->w.p + (size_t)agent * s->n, dv.p, sizeof(float) * s->n, hipMemcpyDeviceToDevice));
  const bool fp16 = s->precision == 1;
  const size_t lds = sv_lds_bytes(s->bmax, s->S, s->kpad);
  SvArgs a;
  fill_args(s, a, pr, 0.5, sigma, fp16);
  a.R = sch->R;
  a.strict = P == 1 ? 1 : 0;
  for (int c = 0; c < 4; ++c) {
    a.tasks = sch->tasks[c].p;
    a.T = sch->T[c];
    HIP_OK(launch_sv(a, kTheta2, s->slots, sch->grid, lds, st));
    HIP_OK(launch_sv(a, kRefresh, s->slots, sch->grid, lds, st));
  }
  a.mann = 0;
  for (int sw = 0; sw < sweeps; ++sw)
    for (int c = 0; c < 4; ++c) {
      a.tasks = sch->tasks[c].p;
      a.T = sch->T[c];
      a.part = s->part.p;
      HIP_OK(launch_sv(a, kSweep, s->slots, sch->grid, lds, st));
    }
  HIP_OK(hipMemcpy(x_out, s->X.p + (size_t)agent * s->n, sizeof(float) * s->n, hipMemcpyDeviceToHost));
  return MACE_OK;
}
