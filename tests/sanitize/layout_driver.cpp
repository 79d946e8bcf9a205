// Sanitizer driver for the library's host runtime: builds the device tables
// and schedules of several matrices in host memory (mace_check_layout, which
// repacks the matrix into the compact or the general records, checks every
// index the kernels form and builds the super-voxel schedules) under
// AddressSanitizer and UndefinedBehaviorSanitizer, and checks the argument
// validation of the load call.  No device is used.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/mace.h"

extern "C" {
typedef struct {
  int32_t nx, ny, n_views, n_ch;
  double pix, chan;
} mi_geom;
int64_t mi_sysmat_colptr(const mi_geom* g, int64_t* col_ptr);
int mi_sysmat_fill(const mi_geom* g, const int64_t* col_ptr, int32_t* row, float* val);
}

static int check(int nx, int ny, int nv, int nc, double chan, int N, int S, int fmt, int prec) {
  mi_geom g{nx, ny, nv, nc, 1.0, chan};
  std::vector<int64_t> cp((size_t)nx * ny + 1);
  const int64_t nnz = mi_sysmat_colptr(&g, cp.data());
  std::vector<int32_t> row((size_t)nnz);
  std::vector<float> val((size_t)nnz);
  mi_sysmat_fill(&g, cp.data(), row.data(), val.data());
  mace_geom mg{nx, ny, nv, nc};
  mace_opts o{};
  o.sv_size = S;
  o.format = fmt;
  o.precision = prec;
  o.fp32_tail_iters = prec ? 2 : 0;
  int64_t lds = 0;
  const int rc = mace_check_layout(&mg, cp.data(), row.data(), val.data(), N, nullptr, &o, &lds);
  std::printf("%dx%d views %d channels %d (%.1f mm) N %d S %d format %d precision %d: rc %d lds %lld %s\n",
              nx, ny, nv, nc, chan, N, S, fmt, prec, rc, (long long)lds, rc ? mace_last_error() : "");
  return rc;
}

int main() {
  int bad = 0;
  bad |= check(32, 32, 64, 48, 1.0, 4, 4, 0, 0) != MACE_OK;
  bad |= check(42, 38, 180, 64, 1.0, 4, 8, 0, 1) != MACE_OK;   // ragged, FP16
  bad |= check(26, 26, 200, 40, 1.0, 2, 4, 0, 0) != MACE_OK;   // 100 views per agent
  bad |= check(24, 24, 4, 8, 1.0, 4, 8, 0, 0) != MACE_OK;      // empty columns
  bad |= check(32, 32, 48, 113, 0.4, 2, 4, 0, 0) != MACE_OK;   // general (0.4 mm)
  bad |= check(16, 16, 720, 24, 1.0, 1, 4, 0, 0) != MACE_OK;   // general (720 views)
  bad |= check(40, 33, 48, 60, 1.0, 2, 16, 0, 0) != MACE_OK;   // general, S = 16
  bad |= check(48, 40, 96, 72, 1.0, 4, 32, 2, 0) != MACE_OK;   // general, S = 32
  // rejected: FP16 values (compact records only) for 0.4 mm channels or 720
  // views per agent, and compact records for 0.4 mm channels
  bad |= check(32, 32, 48, 113, 0.4, 2, 4, 0, 1) != MACE_E_MATRIX;
  bad |= check(16, 16, 720, 24, 1.0, 1, 4, 0, 1) != MACE_E_ARG;
  bad |= check(32, 32, 48, 113, 0.4, 2, 4, 1, 0) != MACE_E_MATRIX;
  // argument checks of the load call (rejected before any device work)
  mace_system* sys = nullptr;
  mace_geom mg{8, 8, 4, 8};
  bad |= mace_load_system(&mg, nullptr, nullptr, nullptr, 1, nullptr, nullptr, &sys) != MACE_E_ARG;
  mace_geom neg{-1, 8, 4, 8};
  int64_t cp0 = 0;
  int32_t r0 = 0;
  float v0 = 0.f;
  bad |= mace_load_system(&neg, &cp0, &r0, &v0, 1, nullptr, nullptr, &sys) != MACE_E_ARG;
  std::printf(bad ? "FAILED\n" : "OK\n");
  return bad;
}
