// HIP kernels (gfx950) of partial-update MACE: launch dispatch of the
// super-voxel sweep (mace_sweep.h), the consensus / residual epilogue and
// small helpers.
#include <hip/hip_runtime.h>

#include "mace_internal.h"
#include "mace_sweep.h"
#include "mace_sweep_gen.h"

namespace mace {

static size_t row_bytes(int bmax, int S, int kpad, int format, int wmax, int nzp, bool vol) {
  return format == 1 ? gen_row_lds_bytes(bmax, S, gen_e0_in_regs(kpad, wmax, nzp), vol)
                     : row_lds_bytes(bmax, S, kpad);
}

int sv_rows_per_block(int bmax, int S, int kpad, int format, int wmax, int nzp) {
  // sized for a volume's launches, the larger rows (a slice's launches then
  // take less LDS per workgroup with the same rows)
  const size_t row = row_bytes(bmax, S, kpad, format, wmax, nzp, true);
  // whole waves (16, 8 or 4 rows): the size that keeps the most rows of a
  // CU's LDS resident (the larger one on a tie)
  int best = 0;
  size_t best_rows = 0;
  for (int rpb = kMaxRowsPerBlock; rpb >= 4; rpb /= 2) {
    if ((size_t)rpb * row > kMaxLdsBytes) continue;
    const size_t resident = kMaxLdsBytes / ((size_t)rpb * row) * rpb;
    if (resident > best_rows) {
      best = rpb;
      best_rows = resident;
    }
  }
  if (best > 0 || format != 1) return best;
  // general records: rows too large for four to a workgroup
  for (int rpb = 2; rpb >= 1; rpb /= 2)
    if ((size_t)rpb * row <= kMaxLdsBytes) return rpb;
  return 0;
}

size_t sv_lds_bytes(int bmax, int S, int kpad, int format, int wmax, int nzp, bool vol) {
  const int rpb = sv_rows_per_block(bmax, S, kpad, format, wmax, nzp);
  return (size_t)(rpb > 0 ? rpb : 1) * row_bytes(bmax, S, kpad, format, wmax, nzp, vol);
}

hipError_t launch_sv(const SvArgs& a, int mode, int slots, int grid, size_t lds, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  if (a.format == 1) return launch_sv_gen(a, mode, grid, lds, st);
  if (a.S == 4) return a.fp16 ? launch_sv_s4f16(a, mode, slots, grid, lds, st)
                              : launch_sv_s4f32(a, mode, slots, grid, lds, st);
  if (a.S == 8) return a.fp16 ? launch_sv_s8f16(a, mode, slots, grid, lds, st)
                              : launch_sv_s8f32(a, mode, slots, grid, lds, st);
  return hipErrorInvalidValue;
}

// ---------------- consensus / residual epilogue ----------------

// For every active slot (blockIdx.y): wbar[s] = mean_i w[i][s], and the
// slot's residual r_k = sqrt(num) / sqrt(den > 0 ? den : ||X||^2) from the
// per-task FP64 partials (NaN when a partial sum is not finite).  The
// first blocks average the agents' w; kEpiRedBlocks more blocks, running
// beside them, sum the partials in a fixed order whatever the timing: each
// sums a fixed chunk and stores its sums after the task partials, and the
// one that arrives last (ticket in counter[1]) adds the block sums in block
// order, stores r_k at iteration k = counter[0] and resets the ticket.
constexpr int kEpiBlocks = 1024;    // at most this many averaging blocks per slot
constexpr int kEpiRedBlocks = 64;   // blocks that sum the residual partials

__host__ __device__ inline int epi_mean_blocks(int n) {
  const int gx = (n + 255) / 256;
  return gx < kEpiBlocks ? gx : kEpiBlocks;
}

__device__ __forceinline__ double load_l2(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum over a 64-lane wave (butterfly, the same order on every call).
__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums of three values over a block of 256 threads (four waves): each wave
// reduces its lanes, then thread 0 adds the four wave sums in wave order.
__device__ void block_sum3(double s0, double s1, double s2, double* out) {
  __shared__ double red[3][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  s0 = wave_sum64(s0);
  s1 = wave_sum64(s1);
  s2 = wave_sum64(s2);
  if (lane == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
    red[2][wave] = s2;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = (red[c][0] + red[c][1]) + (red[c][2] + red[c][3]);
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void epilogue_kernel(const SlotDesc* __restrict__ slots, int N,
                                                       int n, int nparts, double* sums) {
  const SlotDesc d = slots[blockIdx.y];
  if (!d.active) return;
  const int tid = threadIdx.x;
  const int gm = epi_mean_blocks(n);
  if ((int)blockIdx.x < gm) {  // an averaging block
    for (int s = blockIdx.x * blockDim.x + tid; s < n; s += gm * blockDim.x) {
      // sixteen (then eight) agents' loads in flight before they are added,
      // in agent order
      float m = 0.0f;
      int i = 0;
      for (; i + 16 <= N; i += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = d.w[(size_t)(i + u) * n + s];
#pragma unroll
        for (int u = 0; u < 16; ++u) m += v[u];
      }
      for (; i + 8 <= N; i += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = d.w[(size_t)(i + u) * n + s];
#pragma unroll
        for (int u = 0; u < 8; ++u) m += v[u];
      }
      for (; i < N; ++i) m += d.w[(size_t)i * n + s];
      d.wbar[s] = m / (float)N;
    }
    return;
  }
  // a reduction block: its fixed chunk of the task partials
  const int nb = kEpiRedBlocks, rb = (int)blockIdx.x - gm;
  const int chunk = (nparts + nb - 1) / nb;
  const int p0 = rb * chunk, p1 = min(nparts, p0 + chunk);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
  for (int p = p0 + tid; p < p1; p += 256) {
    s0 += d.part[(size_t)p * 4 + 0];
    s1 += d.part[(size_t)p * 4 + 1];
    s2 += d.part[(size_t)p * 4 + 2];
  }
  __shared__ double bs[3];
  __shared__ int last;
  block_sum3(s0, s1, s2, bs);
  double* bpart = d.part + (size_t)nparts * 4;
  if (tid == 0) {
    bpart[rb * 4 + 0] = bs[0];
    bpart[rb * 4 + 1] = bs[1];
    bpart[rb * 4 + 2] = bs[2];
    __threadfence();
    last = atomicAdd(&d.counter[1], 1) == nb - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  s0 = s1 = s2 = 0.0;
  for (int b = tid; b < nb; b += 256) {
    s0 += load_l2(bpart + b * 4 + 0);
    s1 += load_l2(bpart + b * 4 + 1);
    s2 += load_l2(bpart + b * 4 + 2);
  }
  block_sum3(s0, s1, s2, bs);
  if (tid == 0) {
    const int k = d.counter[0];
    const double den = bs[1] > 0.0 ? bs[1] : bs[2];
    // a non-finite state (a diverging iteration) makes r non-finite too, so
    // the stopping test can never take it for convergence
    const bool finite = isfinite(bs[0]) && isfinite(bs[1]) && isfinite(bs[2]);
    const double r = !finite ? __builtin_nan("") : den > 0.0 ? sqrt(bs[0]) / sqrt(den) : 0.0;
    if (k < d.resid_cap) d.resid[k] = r;
    *d.last = r;
    if (sums) {  // the slot's sums, for statistics over several slots (volumes)
      sums[blockIdx.y * 4 + 0] = bs[0];
      sums[blockIdx.y * 4 + 1] = bs[1];
      sums[blockIdx.y * 4 + 2] = bs[2];
    }
    d.counter[0] = k + 1;
    d.counter[1] = 0;
  }
}

hipError_t launch_epilogue(const SlotDesc* slots, int n_slots, int N, int n, int nparts,
                           hipStream_t st, double* sums) {
  if (n_slots <= 0) return hipSuccess;
  const int gx = epi_mean_blocks(n) + kEpiRedBlocks;
  hipLaunchKernelGGL(epilogue_kernel, dim3(gx, n_slots), dim3(256), 0, st, slots, N, n, nparts,
                     sums);
  return hipGetLastError();
}

size_t epilogue_scratch_doubles() { return (size_t)kEpiRedBlocks * 4; }

// ---------------- MACE-PnP consensus: G_H(w) = H(mean w) ----------------

// One axis of the binomial smoother (1/4, 1/2, 1/4) with zero values outside
// the image: along rows wbar -> aux (COLS = false), along columns aux -> wbar.
template <bool COLS>
__global__ __launch_bounds__(256) void smooth_kernel(const SlotDesc* __restrict__ slots, int nx,
                                                     int ny) {
  const SlotDesc d = slots[blockIdx.y];
  if (!d.active) return;
  const float* src = COLS ? d.aux : d.wbar;
  float* dst = COLS ? d.wbar : d.aux;
  const int n = nx * ny;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    const int i = s / nx, j = s - (s / nx) * nx;
    const int step = COLS ? nx : 1;
    const bool lo = COLS ? i > 0 : j > 0;
    const bool hi = COLS ? i < ny - 1 : j < nx - 1;
    const float a = lo ? src[s - step] : 0.0f;
    const float c = hi ? src[s + step] : 0.0f;
    dst[s] = 0.25f * a + 0.5f * src[s] + 0.25f * c;
  }
}

hipError_t launch_smooth(const SlotDesc* slots, int n_slots, int nx, int ny, int passes,
                         hipStream_t st) {
  if (n_slots <= 0 || passes <= 0) return hipSuccess;
  int gx = (nx * ny + 255) / 256;
  if (gx > kEpiBlocks) gx = kEpiBlocks;
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(smooth_kernel<false>, dim3(gx, n_slots), dim3(256), 0, st, slots, nx, ny);
    hipLaunchKernelGGL(smooth_kernel<true>, dim3(gx, n_slots), dim3(256), 0, st, slots, nx, ny);
  }
  return hipGetLastError();
}

// ---------------- small helpers ----------------

__global__ void gather_rows_kernel(float* __restrict__ dst, const float* __restrict__ src,
                                   const int* __restrict__ row_src, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = row_src[i];
    dst[i] = r >= 0 ? src[r] : 0.0f;
  }
}

hipError_t launch_gather_rows(float* dst, const float* src, const int* row_src, int64_t count,
                              hipStream_t st) {
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((int)g), dim3(256), 0, st, dst, src, row_src, count);
  return hipGetLastError();
}

__global__ void fill_kernel(float* __restrict__ dst, float v, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

hipError_t launch_fill(float* dst, float v, int64_t count, hipStream_t st) {
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(fill_kernel, dim3((int)g), dim3(256), 0, st, dst, v, count);
  return hipGetLastError();
}

__global__ void copy_kernel(float* __restrict__ dst, const float* __restrict__ src, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

hipError_t launch_copy(float* dst, const float* src, int64_t count, hipStream_t st) {
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(copy_kernel, dim3((int)g), dim3(256), 0, st, dst, src, count);
  return hipGetLastError();
}

// wbar = mean_i w_i and X_i = wbar for every agent (X^0 = G(w^0)).
__global__ void broadcast_mean_kernel(const float* __restrict__ w, float* __restrict__ wbar,
                                      float* __restrict__ X, int N, int n) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    float m = 0.0f;
    for (int i = 0; i < N; ++i) m += w[(size_t)i * n + s];
    m /= (float)N;
    wbar[s] = m;
    for (int i = 0; i < N; ++i) X[(size_t)i * n + s] = m;
  }
}

hipError_t launch_broadcast_mean(const float* w, float* wbar, float* X, int N, int n,
                                 hipStream_t st) {
  int grid = (n + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(broadcast_mean_kernel, dim3(grid), dim3(256), 0, st, w, wbar, X, N, n);
  return hipGetLastError();
}

__global__ void write_slot_kernel(SlotDesc* table, int i, SlotDesc d) {
  if (threadIdx.x == 0) table[i] = d;
}

hipError_t launch_write_slot(SlotDesc* table, int i, SlotDesc d, hipStream_t st) {
  hipLaunchKernelGGL(write_slot_kernel, dim3(1), dim3(64), 0, st, table, i, d);
  return hipGetLastError();
}

}  // namespace mace
