// Host runtime of the MACE library, part 1: argument checks, repacking of the
// system matrix into the device layout, super-voxel schedules, and the
// system-level entry points of the C ABI (include/mace.h).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <random>
#include <thread>
#include <tuple>

#include "mace_runtime.h"

using namespace mace;

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

namespace mace {
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
const std::string& last_error_text() { return g_err; }

std::atomic<int>& alloc_fail_countdown() {
  static std::atomic<int> c{-1};
  return c;
}

std::mutex& capture_mutex() {
  static std::mutex mu;
  return mu;
}
}  // namespace mace

extern "C" const char* mace_last_error(void) { return g_err.c_str(); }

extern "C" int mace_test_fail_alloc(int32_t after) {
  alloc_fail_countdown().store(after < 0 ? -1 : after);
  return MACE_OK;
}

mace_system::~mace_system() {
  batch.graphs.clear();
  std::lock_guard<std::mutex> lk(capture_mutex());
  for (auto e : ev) (void)hipEventDestroy(e);
  if (stream) (void)hipStreamDestroy(stream);
}

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
  std::vector<uint32_t> adel;  // packed row deltas, kpad / 8 words per record
  std::vector<BandEnt> band;
  std::vector<int> brows;
  std::vector<int> row_src;
  std::vector<float> gval;     // general records
  std::vector<uint16_t> grow;
};

// Agent-block row map and the super-voxel colour lists (both formats).
static void finish_layout(mace_system* s, HostPack& hp) {
  const int N = s->N;
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
}

static void sv_tiling(mace_system* s) {
  const int S = s->S;
  s->gx = (s->nx + S - 1) / S;
  s->gy = (s->ny + S - 1) / S;
  s->n_sv = s->gx * s->gy;
  s->sv_pix0.assign(s->n_sv + 1, 0);
  for (int sv = 0; sv < s->n_sv; ++sv) {
    int sy = sv / s->gx, sx = sv % s->gx;
    int sh = std::min(S, s->ny - sy * S), sw = std::min(S, s->nx - sx * S);
    s->sv_pix0[sv + 1] = s->sv_pix0[sv] + sh * sw;
  }
}

// General records (any sparsity pattern): for each (agent, super-voxel, view
// of the agent) the band is the channel range the SV's pixels touch in that
// view; a pixel's record lists its nonzeros in the agent's rows as (LDS row
// of the band, value), padded to nzp entries with zero values on the task's
// first dummy row B.
static int repack_general(mace_system* s, const int64_t* cp, const int32_t* row, const float* val,
                          HostPack& hp) {
  const int N = s->N, n = s->n, kpad = s->kpad, S = s->S;
  sv_tiling(s);
  // entries per (agent, column); nzp = the largest, rounded up to 32 (the
  // sweep's lanes take the entries in pairs, 16 lanes)
  int maxc = 0;
  {
    std::vector<int> cnt(N);
    for (int64_t c = 0; c < n; ++c) {
      std::fill(cnt.begin(), cnt.end(), 0);
      for (int64_t q = cp[c]; q < cp[c + 1]; ++q) ++cnt[s->view_agent[row[q] / s->n_ch]];
      for (int a = 0; a < N; ++a) maxc = std::max(maxc, cnt[a]);
    }
  }
  const int pair_row = 2 * kRowLanes;
  s->nzp = std::max(pair_row, (maxc + pair_row - 1) / pair_row * pair_row);
  const size_t nrec = (size_t)N * n;
  hp.gval.assign(nrec * s->nzp, 0.0f);
  hp.grow.assign(nrec * s->nzp, 0);
  hp.band.assign((size_t)N * s->n_sv * kpad, BandEnt{0, 0, 0});
  hp.brows.assign((size_t)N * s->n_sv, 0);
  std::vector<int> local(s->n_views);
  for (int a = 0; a < N; ++a)
    for (size_t k = 0; k < s->views[a].size(); ++k) local[s->views[a][k]] = (int)k;
  std::atomic<int> err{0};
  std::atomic<int> bmax{0};
  std::atomic<int> wmaxa{0};
  const int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t] {
      std::vector<int> lo(s->n_views), hi(s->n_views), ldsr(s->n_views);
      for (int sv = t; sv < s->n_sv && !err; sv += nth) {
        const int sy = sv / s->gx, sx = sv % s->gx;
        const int y0 = sy * S, x0 = sx * S;
        const int sh = std::min(S, s->ny - y0), sw = std::min(S, s->nx - x0);
        const int npix = sh * sw;
        std::fill(lo.begin(), lo.end(), 1 << 30);
        std::fill(hi.begin(), hi.end(), -1);
        for (int j = 0; j < npix; ++j) {
          const int64_t col = (int64_t)(y0 + j / sw) * s->nx + x0 + j % sw;
          for (int64_t q = cp[col]; q < cp[col + 1]; ++q) {
            const int k = row[q] / s->n_ch, d = row[q] % s->n_ch;
            lo[k] = std::min(lo[k], d);
            hi[k] = std::max(hi[k], d);
          }
        }
        std::vector<int> B(N, 0);
        for (int a = 0; a < N; ++a) {
          const size_t asv = (size_t)a * s->n_sv + sv;
          for (size_t kl = 0; kl < s->views[a].size(); ++kl) {
            const int k = s->views[a][kl];
            if (hi[k] < 0) continue;
            BandEnt b;
            b.gstart = (uint32_t)((int64_t)kl * s->n_ch + lo[k]);
            b.width = (uint16_t)(hi[k] - lo[k] + 1);
            b.lds_row = (uint16_t)B[a];
            ldsr[k] = B[a];
            B[a] += b.width;
            if (B[a] + 2 > 65535) {
              err = 3;
              return;
            }
            hp.band[asv * kpad + kl] = b;
            int cw = wmaxa.load();
            while (b.width > cw && !wmaxa.compare_exchange_weak(cw, b.width)) {
            }
          }
          // views that miss the SV, and padding views: width 0 on the dummy rows
          for (int kl = 0; kl < kpad; ++kl)
            if (hp.band[asv * kpad + kl].width == 0) hp.band[asv * kpad + kl] = BandEnt{0, (uint16_t)B[a], 0};
          hp.brows[asv] = B[a];
          int cur = bmax.load();
          while (B[a] + 2 > cur && !bmax.compare_exchange_weak(cur, B[a] + 2)) {
          }
        }
        std::vector<int> fillc(N);
        for (int j = 0; j < npix; ++j) {
          const int64_t col = (int64_t)(y0 + j / sw) * s->nx + x0 + j % sw;
          std::fill(fillc.begin(), fillc.end(), 0);
          for (int a = 0; a < N; ++a) {
            const size_t rec = (size_t)a * n + s->sv_pix0[sv] + j;
            for (int q = 0; q < s->nzp; ++q) hp.grow[rec * s->nzp + q] = (uint16_t)B[a];
          }
          for (int64_t q = cp[col]; q < cp[col + 1]; ++q) {
            const int k = row[q] / s->n_ch, d = row[q] % s->n_ch;
            const int a = s->view_agent[k];
            const size_t rec = (size_t)a * n + s->sv_pix0[sv] + j;
            const size_t e = rec * s->nzp + fillc[a]++;
            hp.gval[e] = val[q];
            hp.grow[e] = (uint16_t)(ldsr[k] + d - lo[k]);
          }
        }
      }
    });
  for (auto& x : th) x.join();
  if (err == 3) return fail(MACE_E_MATRIX, "super-voxel band exceeds 65533 rows; use a smaller sv_size");
  s->bmax = (bmax.load() + 1) & ~1;
  if (s->bmax < 2) s->bmax = 2;
  s->wmax = wmaxa.load();
  finish_layout(s, hp);
  return MACE_OK;
}

// Every index the general kernel forms stays inside its buffer.
static int check_pack_general(const mace_system* s, const HostPack& hp) {
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
        // the kernel reads entry gstart of an empty band
        if (b.width == 0 && b.gstart != 0) return fail(MACE_E_MATRIX, "check: empty band with gstart %u", b.gstart);
        if (b.width == 0) continue;
        // the kernel keeps the staged e in registers, one chunk per view,
        // when wmax says every band fits 16 lanes
        if (b.width > s->wmax) return fail(MACE_E_MATRIX, "check: band of %d channels above wmax %d", b.width, s->wmax);
        if (kl >= K) return fail(MACE_E_MATRIX, "check: band entry on a padding view");
        if ((int)b.lds_row + b.width > B) return fail(MACE_E_MATRIX, "check: band overruns its rows");
        if ((int64_t)b.gstart / s->n_ch != kl || ((int64_t)b.gstart + b.width - 1) / s->n_ch != kl)
          return fail(MACE_E_MATRIX, "check: band crosses a view boundary");
        rows += b.width;
      }
      if (rows != B) return fail(MACE_E_MATRIX, "check: band rows do not add up");
      const int npix = s->sv_pix0[sv + 1] - s->sv_pix0[sv];
      if (npix < 1 || npix > s->S * s->S) return fail(MACE_E_MATRIX, "check: bad SV pixel count");
      for (int j = 0; j < npix; ++j) {
        const size_t rec = (size_t)a * s->n + s->sv_pix0[sv] + j;
        for (int q = 0; q < s->nzp; ++q) {
          const int r = hp.grow[rec * s->nzp + q];
          if (r > B || (r == B && hp.gval[rec * s->nzp + q] != 0.0f))
            return fail(MACE_E_MATRIX, "check: record row %d outside its band (%d rows)", r, B);
        }
      }
    }
  }
  if (s->sv_pix0[s->n_sv] != s->n) return fail(MACE_E_MATRIX, "check: SVs do not tile the image");
  return MACE_OK;
}

static int repack(mace_system* s, const int64_t* cp, const int32_t* row, const float* val,
                  HostPack& hp) {
  const int N = s->N, n = s->n, kpad = s->kpad, S = s->S;
  sv_tiling(s);
  // agent-local view index of every view
  std::vector<int> local(s->n_views);
  for (int a = 0; a < N; ++a)
    for (size_t k = 0; k < s->views[a].size(); ++k) local[s->views[a][k]] = (int)k;

  const size_t nrec = (size_t)N * n * kpad;
  // values at stride Kmax per record, plus a tail pad of one slot group that
  // the lanes past Kmax of the last record read (and zero)
  const int kstr = s->Kmax;
  const size_t nval = (size_t)N * n * kstr + kRowLanes;
  std::vector<float2>& h_aval = hp.aval;
  std::vector<__half2>& h_hval = hp.hval;
  std::vector<float>& h_hscale = hp.hscale;
  if (s->precision == 0 || s->fp32_tail > 0) h_aval.assign(nval, make_float2(0.f, 0.f));
  if (s->precision == 1) {
    h_hval.assign(nval, __floats2half2_rn(0.f, 0.f));
    h_hscale.resize((size_t)N * n);
  }
  std::vector<uint32_t>& h_adel = hp.adel;
  h_adel.assign(nrec / 8, 0u);
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
            h_band[asv * kpad + kl] = b;
          }
          // views that miss the SV, and padding views, point at the dummy rows
          for (int kl = 0; kl < K; ++kl)
            if (h_band[asv * kpad + kl].width == 0) h_band[asv * kpad + kl].lds_row = (uint16_t)B;
          for (int kl = K; kl < kpad; ++kl) h_band[asv * kpad + kl] = BandEnt{0, (uint16_t)B, 0};
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
              const size_t idx = rec * kstr + kl;  // used for kl < kstr only
              float a0 = 0.f, a1 = 0.f;
              uint32_t del = 0;  // a view the pixel misses: row 0 of its band, a0 = a1 = 0
              if (kl < K) {
                const int k = vw[kl];
                const Foot& f = foot[(size_t)j * s->n_views + k];
                if (f.any) {
                  a0 = f.a0;
                  a1 = f.a1;
                  del = (uint32_t)(f.d0 - cmin[k]);
                }
              }
              if (kl < kstr) {
                if (!h_aval.empty()) h_aval[idx] = make_float2(a0, a1);
                if (!h_hval.empty()) h_hval[idx] = __floats2half2_rn(a0 / scale, a1 / scale);
              }
              // slot kl = 16 s + l: word 2 s + l / 8, nibble l mod 8
              h_adel[rec * (kpad / 8) + (kl / 16) * 2 + (kl % 16) / 8] |= (del & 15u) << (4 * (kl % 8));
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

  finish_layout(s, hp);
  return MACE_OK;
}

static int upload_pack(mace_system* s, const HostPack& hp) {
  if (!hp.adel.empty()) HIP_OK(s->adel.upload(hp.adel.data(), hp.adel.size()));
  if (!hp.gval.empty()) {
    HIP_OK(s->gval.upload(hp.gval.data(), hp.gval.size()));
    HIP_OK(s->grow.upload(hp.grow.data(), hp.grow.size()));
  }
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
                              s->adel.bytes() + s->band.bytes() + s->band_rows.bytes() +
                              s->gval.bytes() + s->grow.bytes());
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
        if (b.width == 0) {
          // the kernel reads entry gstart of an empty band, and its records
          // address the dummy rows B, B + 1
          if (b.gstart != 0) return fail(MACE_E_MATRIX, "check: empty band with gstart %u", b.gstart);
          if (b.lds_row != B) return fail(MACE_E_MATRIX, "check: empty band off the dummy rows");
          continue;
        }
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
          // the kernel reads and writes band rows lds_row + del and the next one
          const int del = (int)((hp.adel[rec * (kpad / 8) + (kl / 16) * 2 + (kl % 16) / 8] >> (4 * (kl % 8))) & 15u);
          const BandEnt& b = hp.band[asv * kpad + kl];
          if (b.width == 0) {
            if (b.lds_row != B || del != 0) return fail(MACE_E_MATRIX, "check: empty view not on the dummy rows");
          } else if (del + 1 >= b.width) {
            return fail(MACE_E_MATRIX, "check: record row %d outside its view's band (%d rows)", del, b.width);
          }
        }
      }
    }
  }
  if (s->sv_pix0[s->n_sv] != s->n) return fail(MACE_E_MATRIX, "check: SVs do not tile the image");
  const int wm = s->S <= 4 ? 8 : 16;
  if (s->wmax > wm)
    return fail(MACE_E_MATRIX, "a super-voxel's band spans %d channels of one view (at most %d); use sv_size 4",
                s->wmax, wm);
  return MACE_OK;
}

// Rows per workgroup of the sweep kernel: 16 (two workgroups per CU at
// 79 KB each for the 45-view workloads), fewer when a row's band, halo and
// scratch would not fit 16 to the 160 KiB of LDS (many views per agent).
static int pick_rows_per_block(mace_system* s) {
  s->rpb = sv_rows_per_block(s->bmax, s->S, s->kpad, s->format, s->wmax, s->nzp);
  if (s->rpb == 0)  // rows of 16 lanes: at least 4 per workgroup (compact), 1 (general)
    return fail(MACE_E_ARG,
                "a super-voxel band of %d rows needs more than %d KiB of LDS per row; %s", s->bmax,
                (int)(kMaxLdsBytes / 1024 / (s->format == 1 ? 1 : 4)),
                s->S > 4 ? "use a smaller sv_size" : "use more agents (fewer views per agent)");
  return MACE_OK;
}

// ---------------------------------------------------------------- schedules
struct HostSchedule {
  int grid = 0, R = 0, T[4] = {0, 0, 0, 0};
  std::vector<int> tab[4];
};

// Rows of 16 lanes are grouped s->rpb to a workgroup (16 unless a row's LDS
// is too large for that); workgroups are dispatched
// round-robin over the 8 XCDs. The rows serving agent a (of every slot) are
// placed in workgroups of XCD a mod 8, so the agent's sinogram blocks and its
// matrix records stay in one L2; all slots walk the SVs in the same order, so
// the same records are read by several slots at about the same time.
// Slot sl takes part in a schedule of this parity (-1: every slot; else the
// slots whose group of `group` consecutive slots has that parity -- the
// even / odd slices of a volume, or its even / odd slice groups).
static bool slot_in(int sl, int parity, int group) {
  return parity < 0 || ((sl / group) & 1) == parity;
}

// group > 1 (a volume's slice groups): a row holds one group of that many
// consecutive slots for one (agent, rank) and sweeps each of its super-voxels
// through the group's slices in order before the next super-voxel.
static void build_schedule(const mace_system* s, int n_slots, int only_agent, int P, int parity,
                           int group, HostSchedule& hs) {
  std::vector<int> agents;
  if (only_agent >= 0)
    agents.push_back(only_agent);
  else
    for (int a = 0; a < s->N; ++a) agents.push_back(a);
  struct RowId {
    int slot, agent, rank;
  };
  const int nxcd = 8;
  std::vector<std::vector<RowId>> xrows(nxcd);
  // rank-major: the rows that run at the same time (consecutive workgroups)
  // hold the same rank of every slot and agent, so the slots of a batch
  // walk the super-voxels in step and share the matrix records in L2
  // (parity 0 / 1: only the even / odd slots -- the slices of a volume)
  // (with slice groups, a row's slot is its group's first slot)
  for (int r = 0; r < P; ++r)
    for (int sl = 0; sl < n_slots; sl += group) {
      if (!slot_in(sl, parity, group)) continue;
      for (size_t i = 0; i < agents.size(); ++i) xrows[agents[i] % nxcd].push_back({sl, agents[i], r});
    }
  int wg_per_xcd = 0, used = 0;
  for (int x = 0; x < nxcd; ++x) {
    wg_per_xcd = std::max<int>(wg_per_xcd, (int)((xrows[x].size() + s->rpb - 1) / s->rpb));
    used += !xrows[x].empty();
  }
  std::vector<RowId> row_of;
  if (used == nxcd) {
    hs.grid = wg_per_xcd * nxcd;
    row_of.assign((size_t)hs.grid * s->rpb, {-1, -1, -1});
    for (int x = 0; x < nxcd; ++x)
      for (size_t q = 0; q < xrows[x].size(); ++q) {
        const int u = (int)(q / s->rpb), j = (int)(q % s->rpb);
        row_of[(size_t)(u * nxcd + x) * s->rpb + j] = xrows[x][q];
      }
  } else {
    // some XCDs would stay idle: pack the rows densely instead
    std::vector<RowId> all;
    for (int x = 0; x < nxcd; ++x) all.insert(all.end(), xrows[x].begin(), xrows[x].end());
    hs.grid = (int)((all.size() + s->rpb - 1) / s->rpb);
    row_of.assign((size_t)hs.grid * s->rpb, {-1, -1, -1});
    for (size_t q = 0; q < all.size(); ++q) row_of[q] = all[q];
  }
  hs.R = hs.grid * s->rpb;
  for (int c = 0; c < 4; ++c) {
    const auto& L = s->colour_svs[c];
    const int Tsv = (int)((L.size() + P - 1) / P);  // super-voxels per row
    const int T = Tsv * group;
    hs.T[c] = T;
    hs.tab[c].assign((size_t)hs.R * std::max(T, 1), -1);
    for (int r = 0; r < hs.R; ++r) {
      const RowId id = row_of[r];
      if (id.agent < 0) continue;
      for (int t = 0; t < Tsv; ++t) {
        const size_t q = (size_t)t * P + id.rank;
        if (q >= L.size()) continue;
        for (int z = 0; z < group && id.slot + z < n_slots; ++z)
          hs.tab[c][(size_t)r * T + (size_t)t * group + z] =
              ((id.slot + z) << kSlotShift) | (id.agent * s->n_sv + L[q]);
      }
    }
  }
}

// Every (slot, agent, SV) of the scheduled agents and slots appears exactly
// once per pass, in the phase of its colour, and every task id is in range.
static int check_schedule(const mace_system* s, int n_slots, int only_agent, int parity,
                          int group, const HostSchedule& hs) {
  const size_t per_slot = (size_t)s->N * s->n_sv;
  if (per_slot >= ((size_t)1 << kSlotShift)) return fail(MACE_E_ARG, "check: too many (agent, SV) pairs");
  if (n_slots > kMaxScanSlots) return fail(MACE_E_ARG, "check: too many slots");
  std::vector<int> seen(per_slot * n_slots, 0);
  for (int c = 0; c < 4; ++c)
    for (int t : hs.tab[c]) {
      if (t < 0) continue;
      const int slot = t >> kSlotShift, local = t & ((1 << kSlotShift) - 1);
      if (slot >= n_slots || (size_t)local >= per_slot) return fail(MACE_E_ARG, "check: task id out of range");
      const int sv = local % s->n_sv;
      if (((sv % s->gx) & 1) + 2 * ((sv / s->gx) & 1) != c) return fail(MACE_E_ARG, "check: task in the wrong colour phase");
      seen[(size_t)slot * per_slot + local]++;
    }
  for (int sl = 0; sl < n_slots; ++sl)
    for (int a = 0; a < s->N; ++a)
      for (int sv = 0; sv < s->n_sv; ++sv) {
        const int want = (only_agent < 0 || only_agent == a) && slot_in(sl, parity, group) ? 1 : 0;
        const int got = seen[(size_t)sl * per_slot + (size_t)a * s->n_sv + sv];
        if (got != want) return fail(MACE_E_ARG, "check: task visited %d times", got);
      }
  return MACE_OK;
}

namespace mace {
Schedule* get_schedule(mace_system* s, int n_slots, int only_agent, int P, int parity, int group) {
  const auto key = std::make_tuple(n_slots, only_agent, P, parity, group);
  auto it = s->schedules.find(key);
  if (it != s->schedules.end()) return it->second.get();
  HostSchedule hs;
  build_schedule(s, n_slots, only_agent, P, parity, group, hs);
  if (check_schedule(s, n_slots, only_agent, parity, group, hs)) return nullptr;
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
// 8192, two waves per SIMD) to keep every CU busy, and enough that a row
// runs at most kMaxTasksPerRow super-voxels per phase (short workgroups let
// the launches of other streams in between), but at most half of the SVs of
// one colour -- a quarter on small images (fewer than 256 SVs per colour),
// where updating most of a colour at once (block Jacobi) loses stability.
constexpr int kMaxTasksPerRow = 4;
int default_rows_per_agent(const mace_system* s) {
  if (s->rows_per_agent > 0) return s->rows_per_agent;
  const int per_colour = (s->n_sv + 3) / 4;
  const int P = std::max((8192 + s->N - 1) / s->N, (per_colour + kMaxTasksPerRow - 1) / kMaxTasksPerRow);
  const int cap = per_colour >= 256 ? per_colour / 2 : per_colour / 4;
  return std::max(1, std::min(P, cap));
}
}  // namespace mace

// ---------------------------------------------------------------- kernel arguments
void mace::fill_args(const mace_system* s, SvArgs& a, const mace_prior* pr, double rho,
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
  a.rpb = s->rpb;
  a.kstr = s->Kmax;
  a.sv_pix0 = s->d_sv_pix0.p;
  a.aval = s->aval.p;
  a.hval = s->hval.p;
  a.hscale = s->hscale.p;
  a.fp16 = fp16 ? 1 : 0;
  a.adel = s->adel.p;
  a.format = s->format;
  a.gval = s->gval.p;
  a.grow = s->grow.p;
  a.nzp = s->nzp;
  a.band = s->band.p;
  a.band_rows = s->band_rows.p;
  a.estride = s->estride;
  a.slots = s->batch.table.p;
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

int mace::check_prior(const mace_prior* pr) {
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

// ---------------------------------------------------------------- layout choice
// Builds the device tables in hp for the record format the options ask for
// (0: compact when the matrix and options allow it, else general; 1:
// compact; 2: general), checks every index the kernels form, and picks the
// rows per workgroup.  The compact records need super-voxel sides 4 or 8, at
// most 128 views per agent, at most two nonzeros per (column, view) on
// adjacent channels and bands of at most 16 (S = 8) or 8 (S = 4) channels;
// the general records take any matrix, FP32 values only.
static int build_layout(mace_system* s, const int64_t* cp, const int32_t* row, const float* val,
                        int fmt_req, HostPack& hp) {
  const bool small_s = s->S == 4 || s->S == 8;
  const bool compact_ok = small_s && s->Kmax <= kRowLanes * kMaxSlots;
  if (fmt_req == 1 && !compact_ok)
    return fail(MACE_E_ARG, "the compact record format needs sv_size 4 or 8 and at most %d views "
                            "per agent", kRowLanes * kMaxSlots);
  int rc;
  if (fmt_req != 2 && compact_ok) {
    s->format = 0;
    rc = repack(s, cp, row, val, hp);
    if (rc == MACE_OK) rc = check_pack(s, hp);
    if (rc == MACE_OK) rc = pick_rows_per_block(s);
    if (rc != MACE_E_MATRIX || fmt_req == 1) return rc;
    if (s->precision == 1)
      return fail(MACE_E_MATRIX, "FP16 matrix values need the compact records, and %s",
                  std::string(last_error_text()).c_str());
    hp = HostPack{};  // not representable in the compact records
  }
  if (s->precision == 1)
    return fail(MACE_E_ARG, "FP16 matrix values need the compact record format (sv_size 4 or 8, "
                            "at most %d views per agent, at most two adjacent nonzeros per view)",
                kRowLanes * kMaxSlots);
  s->format = 1;
  s->kpad = (s->Kmax + kRowLanes - 1) / kRowLanes * kRowLanes;
  rc = repack_general(s, cp, row, val, hp);
  if (rc == MACE_OK) rc = check_pack_general(s, hp);
  if (rc == MACE_OK) rc = pick_rows_per_block(s);
  return rc;
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
  if (opts && opts->sv_size == -1) {
    // autotuned S and rows per agent (cached per geometry for the process)
    mace_opts tuned{};
    int rc = mace_autotune(geom, col_ptr, row_idx, val, n_agents, view_to_agent, opts, 6, &tuned,
                           nullptr, nullptr, 0, nullptr);
    if (rc) return rc;
    return mace_load_system(geom, col_ptr, row_idx, val, n_agents, view_to_agent, &tuned, out);
  }
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
    if (opts->sv_size != 0 && opts->sv_size != 4 && opts->sv_size != 8 && opts->sv_size != 16 &&
        opts->sv_size != 32)
      return fail(MACE_E_ARG, "sv_size must be -1 (autotune), 0 (automatic), 4, 8, 16 or 32");
    if (opts->format < 0 || opts->format > 2) return fail(MACE_E_ARG, "format must be 0, 1 or 2");
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
    rc = build_layout(s.get(), col_ptr, row_idx, val, opts ? opts->format : 0, hp);
    if (rc) return rc;
    rc = upload_pack(s.get(), hp);
    if (rc) return rc;
  }
  HIP_OK(hipGetDevice(&s->device));
  {
    std::lock_guard<std::mutex> lk(capture_mutex());
    HIP_OK(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
  }
  // what the allocation-free solve needs: its workspace's address on this
  // device and the one-scan schedule
  rc = noalloc_prepare(s->device);
  if (rc) return rc;
  if (!get_schedule(s.get(), 1, -1, default_rows_per_agent(s.get())))
    return fail(MACE_E_HIP, "schedule upload failed");
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
    if (opts->sv_size != 0 && opts->sv_size != 4 && opts->sv_size != 8 && opts->sv_size != 16 &&
        opts->sv_size != 32)
      return fail(MACE_E_ARG,
                  "sv_size must be 0 (automatic: 8 from 256 x 256 pixels on, else 4), 4, 8, 16 or 32");
    if (opts->format < 0 || opts->format > 2) return fail(MACE_E_ARG, "format must be 0, 1 or 2");
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
  rc = build_layout(&s, col_ptr, row_idx, val, opts ? opts->format : 0, hp);
  if (rc) return rc;
  const int P = default_rows_per_agent(&s);
  for (int only = -1; only < s.N; ++only) {
    for (int PP : {1, P}) {
      for (int ns : {1, 3})
        for (int par : {-1, 0, 1})  // all slots; the even / odd slices (groups) of a volume
          for (int grp : {1, 2}) {
            if (par < 0 && grp > 1) continue;
            HostSchedule hs;
            build_schedule(&s, ns, only, PP, par, grp, hs);
            rc = check_schedule(&s, ns, only, par, grp, hs);
            if (rc) return rc;
          }
    }
    if (only >= 2) break;
  }
  if (lds_bytes) *lds_bytes = (int64_t)sv_lds_bytes(s.bmax, s.S, s.kpad, s.format, s.wmax, s.nzp, false);
  return MACE_OK;
}

extern "C" void mace_free_system(mace_system* s) { delete s; }

extern "C" int64_t mace_system_bytes(const mace_system* s) { return s ? s->matrix_bytes : 0; }

extern "C" int mace_get_config(const mace_system* s, mace_opts* out) {
  if (!s || !out) return fail(MACE_E_ARG, "NULL argument");
  *out = mace_opts{};
  out->precision = s->precision;
  out->sv_size = s->S;
  out->rows_per_agent = default_rows_per_agent(s);
  out->fp32_tail_iters = s->fp32_tail;
  out->refresh_every = s->refresh_every;
  out->format = s->format == 1 ? 2 : 1;
  return MACE_OK;
}

extern "C" int mace_set_relaxation(mace_system* s, double relax) {
  if (!s) return fail(MACE_E_ARG, "NULL system");
  if (!(relax > 0.0 && relax <= 1.0)) return fail(MACE_E_ARG, "relaxation must be in (0, 1]");
  s->relax = relax;
  return MACE_OK;
}

extern "C" int mace_set_slice_group(mace_system* s, int32_t slices) {
  if (!s) return fail(MACE_E_ARG, "NULL system");
  if (slices < 1 || slices > kMaxScanSlots)
    return fail(MACE_E_ARG, "slices per group must be in [1, %d]", kMaxScanSlots);
  s->slice_group = slices;
  return MACE_OK;
}

extern "C" int mace_set_fp32_tail(mace_system* s, int32_t iters) {
  if (!s) return fail(MACE_E_ARG, "NULL system");
  if (iters < 0) return fail(MACE_E_ARG, "iters must be >= 0");
  if (s->precision != 1) return fail(MACE_E_ARG, "the system's matrix values are FP32 already");
  if (iters > 0 && !s->aval.p)
    return fail(MACE_E_ARG, "the system holds no FP32 values: load it with fp32_tail_iters > 0");
  s->fp32_tail = iters;
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

