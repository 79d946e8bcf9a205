// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mace {

// One row of 16 lanes works on one super-voxel; a workgroup holds up to
// 4 waves x 4 rows (fewer when a row's LDS is large: 16, 8 or 4 rows).
constexpr int kRowLanes = 16;
constexpr int kMaxRowsPerBlock = 16;
constexpr int kBlockThreads = kMaxRowsPerBlock * kRowLanes;
constexpr size_t kMaxLdsBytes = 160 * 1024;
constexpr int kMaxSlots = 8;  // views per agent <= 16 * kMaxSlots

// Band of one (agent, super-voxel, agent-local view): channels
// [cmin, cmin + width) of that view, staged in LDS from row lds_row on.
struct BandEnt {
  uint32_t gstart;   // index of (view, cmin) in the agent's sinogram block
  uint16_t lds_row;  // first LDS row of the band (the dummy rows B when width is 0)
  uint16_t width;    // channels in the band (0: the view misses the SV)
};

enum KernelMode { kSweep = 0, kTheta2 = 1, kRefresh = 2 };

// Tasks: slot << kSlotShift | (agent * n_sv + sv); -1 = none.
constexpr int kSlotShift = 24;
constexpr int kMaxScanSlots = 128;  // scans per batch (slot field of a task)

// Per-scan state of one slot of a batch (device table entry).
struct SlotDesc {
  float* e;           // error sinogram y - A X_i, agent blocks
  const float* lam;   // inverse-variance weights, agent blocks
  float* X;           // [N][n] agent states
  float* w;           // [N][n] Mann state
  float* wbar;        // [n] mean of w (updated by the epilogue); with a PnP
                      // denoiser H, H(mean of w)
  float* aux;         // [n] scratch of the denoiser passes
  float* th2;         // [N][n] theta2 = sum_r A_rs^2 Lambda_r
  double* part;       // [N * n_sv][4] FP64 residual partials per task, then
                      // the epilogue's per-block sums
  double* resid;      // [resid_cap] residual trace
  double* last;       // latest residual (one double)
  int* counter;       // [0] Mann iterations done, [1] epilogue ticket (0 between launches)
  int resid_cap;
  int active;         // 0: the slot's tasks and epilogue are skipped
  int prec;           // matrix values the slot's sweeps read: 0 FP32, 1 FP16
                      // (a sweep launch runs only the slots of its precision)
};

struct SvArgs {
  int nx, ny, n;        // image
  int S, gx, n_sv;      // super-voxel side, grid width, count
  int kpad;             // record entries per pixel (slots * 16)
  int bmax;             // LDS rows reserved per super-voxel (even)
  int wmax;             // widest band of one view (channels)
  const int* tasks;     // [R][T] task = agent * n_sv + sv, or -1
  int T, R;
  const int* sv_pix0;   // [n_sv + 1] first record of each super-voxel
  const float2* aval;   // FP32 records: (a0, a1) per (agent, pixel, view < kstr)
  const __half2* hval;  // FP16 records (precision 1), scaled by hscale
  const float* hscale;  // [N * n] per (agent, pixel) scale of the FP16 values
  const uint32_t* adel; // row of d0 in its view's band, 4 bits per (agent, pixel, view slot)
  const BandEnt* band;  // [(agent * n_sv + sv) * kpad + view]
  const int* band_rows; // [agent * n_sv + sv] rows B of the band (dummy rows at B, B+1)
  int64_t estride;      // per-agent stride of e / lam blocks
  const SlotDesc* slots; // per-scan state, indexed by the task's slot
  int kind;             // 0 quadratic, 1 q-GGMRF (p = 2)
  float invN, is2, rho;
  float relax;          // scale of each coordinate step (1 = exact minimiser)
  float bedge, bdiag;
  float c0;             // 1 / sigma_x^2
  float inv_tsx;        // 1 / (T sigma_x)
  float qexp;           // p - q = 2 - q
  float qhalf;          // q / p = q / 2
  int mann;             // apply the reflection + Mann update at the end
  int fp16;             // read the FP16 records
  int strict;           // one SV of an agent at a time: stage e after the previous flush
  int rpb;              // rows per workgroup (16, 8 or 4); the block has rpb * 16 threads
  int kstr;             // record values per (agent, pixel): the largest view count of an agent
  int hpass;            // MACE-PnP: passes of the denoiser H after each epilogue (0: plain MACE)
  int format;           // 0: compact records (sv_kernel); 1: general records (sv_kernel_gen)
  const float* gval;    // general records: values [N * n][nzp]
  const uint16_t* grow; // general records: LDS rows of the task's band [N * n][nzp]
  int nzp;              // general records: entries per (agent, pixel), a multiple of 16
  int vol_nz;           // volume of vol_nz slices, slice z in slot z (0: independent scans)
  float baxial;         // weight of the axial cliques of a volume
};

// Per-variant sweep launchers (mace_sweep_*.hip); general records for
// super-voxel sides 4, 8, 16, 32 (mace_sweep_gen.hip).
hipError_t launch_sv_gen(const SvArgs& a, int mode, int grid, size_t lds, hipStream_t st);
hipError_t launch_sv_s4f32(const SvArgs& a, int mode, int slots, int grid, size_t lds, hipStream_t st);
hipError_t launch_sv_s4f16(const SvArgs& a, int mode, int slots, int grid, size_t lds, hipStream_t st);
hipError_t launch_sv_s8f32(const SvArgs& a, int mode, int slots, int grid, size_t lds, hipStream_t st);
hipError_t launch_sv_s8f16(const SvArgs& a, int mode, int slots, int grid, size_t lds, hipStream_t st);

// Launchers (defined in mace_kernels.hip).
hipError_t launch_sv(const SvArgs& a, int mode, int slots, int grid, size_t lds, hipStream_t st);
// Rows per workgroup: of 16, 8 and 4, the one that keeps the most rows of a
// CU's 160 KiB of LDS resident (general records: down to 1 when not even 4
// fit; 0 if none does), and the LDS bytes of such a workgroup.
int sv_rows_per_block(int bmax, int S, int kpad, int format, int wmax, int nzp);
// vol: a volume's launches (the general records stage the axial neighbours)
size_t sv_lds_bytes(int bmax, int S, int kpad, int format, int wmax, int nzp, bool vol);
// Doubles the epilogue needs after a slot's task partials.
size_t epilogue_scratch_doubles();
// The epilogue of each slot: consensus w-bar and the FP64 residual; with
// `sums`, also each slot's (numerator, denominator, ||X||^2) at sums[slot * 4].
hipError_t launch_epilogue(const SlotDesc* slots, int n_slots, int N, int n, int nparts,
                           hipStream_t st, double* sums = nullptr);
// MACE-PnP consensus G_H: `passes` applications of the 3x3 binomial smoother
// to every active slot's wbar (through its aux buffer).
hipError_t launch_smooth(const SlotDesc* slots, int n_slots, int nx, int ny, int passes,
                         hipStream_t st);
hipError_t launch_gather_rows(float* dst, const float* src, const int* row_src, int64_t count,
                              hipStream_t st);
hipError_t launch_fill(float* dst, float v, int64_t count, hipStream_t st);
hipError_t launch_broadcast_mean(const float* w, float* wbar, float* X, int N, int n,
                                 hipStream_t st);
hipError_t launch_copy(float* dst, const float* src, int64_t count, hipStream_t st);
// table[i] = d, ordered on the stream (the descriptor travels as a kernel argument).
hipError_t launch_write_slot(SlotDesc* table, int i, SlotDesc d, hipStream_t st);

}  // namespace mace
