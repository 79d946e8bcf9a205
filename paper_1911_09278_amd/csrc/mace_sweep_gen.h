#pragma once
// Super-voxel ICD sweep for matrices of any sparsity pattern (general
// records).  Same algorithm and task structure as sv_kernel (mace_sweep.h):
// one 16-lane row per (agent, super-voxel) task, the task's error-sinogram
// band staged in LDS, per pixel theta1 / theta2 / the prior's majoriser /
// the prox term summed over the row, the coordinate step, the band update,
// the band's change added to the agent's error sinogram with atomics, and
// the reflection + Mann update with FP64 residual partials.  What differs:
//   * a record is the list of the pixel's nonzeros in the agent's rows, as
//     (LDS row of the band, value) pairs padded to nzp entries (a multiple
//     of 32) with zero values on the task's dummy row; a column may have any
//     number of nonzeros per view, on any channels;
//   * a view's band may be wider than 16 channels, and an agent may own any
//     number of views: the band is staged and written back view by view in
//     chunks of 16 channels;
//   * the staged copy of e that the write-back subtracts lives in
//     registers when every band fits 16 channels and the view slots fit
//     beside the record registers, else in LDS;
//   * super-voxel sides 4, 8, 16 and 32;
//   * volumes: slice z of a stack lives in slot z, and lanes 9 and 10 add
//     the axial cliques to the voxels of slices z - 1 and z + 1 of the same
//     agent (the 3-D prior's ten-voxel neighbourhood).  Even and odd slices
//     sweep in separate launches, so the axial neighbours a task stages do
//     not change while it runs.
// Records of up to 256 entries (the common case: 1 mm channels and tens of
// views per agent) are held in registers in the sweep, two entries per
// load, loaded two pixels ahead; longer ones are read in the pixel loop.
// The pixel loop is not unrolled, nor the loops over views unless the
// staged e is in registers.  FP32 values only.
#include <hip/hip_runtime.h>

#include "mace_internal.h"
#include "mace_sweep.h"

namespace mace {

// The staged copy of e stays in registers (one per view slot and lane) when
// every view's band fits one 16-lane chunk and the view slots fit what the
// record registers leave (at most 256 VGPRs, no spill): 48 slots with records
// of up to 128 entries, 32 with up to 256, 64 with records read in the loop.
// Otherwise it lives in LDS.
__host__ __device__ inline bool gen_e0_in_regs(int kpad, int wmax, int nzp) {
  const int max_slots = nzp <= 8 * kRowLanes ? 3 * kRowLanes
                        : nzp <= 16 * kRowLanes ? 2 * kRowLanes : 4 * kRowLanes;
  return kpad <= max_slots && wmax <= kRowLanes;
}

// LDS bytes of one row of the general kernel: band (e, Lambda), the staged
// e (unless it stays in registers), the halo tile, v / theta2 and, in a
// volume's launches, the axial neighbours below and above of the
// super-voxel's pixels.
__host__ __device__ inline size_t gen_row_lds_bytes(int bmax, int S, bool e0_regs, bool vol) {
  size_t per_row = (size_t)bmax * (e0_regs ? 8 : 12) + (size_t)halo_cells(S) * 4 +
                   (size_t)S * S * (vol ? 16 : 8);
  per_row = (per_row + 7) & ~(size_t)7;
  const size_t red = kRowLanes * 3 * sizeof(double);
  return per_row > red ? per_row : red;
}

// Value of lane l of the lane's DPP row (16 lanes), for every lane of the row
// (every lane of the row must be active).
template <int L>
__device__ __forceinline__ uint32_t row_bcast_c(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 | L, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t row_bcast(uint32_t v, int l) {
  switch (l) {  // l is a constant in the unrolled loops that call this
    case 0: return row_bcast_c<0>(v);
    case 1: return row_bcast_c<1>(v);
    case 2: return row_bcast_c<2>(v);
    case 3: return row_bcast_c<3>(v);
    case 4: return row_bcast_c<4>(v);
    case 5: return row_bcast_c<5>(v);
    case 6: return row_bcast_c<6>(v);
    case 7: return row_bcast_c<7>(v);
    case 8: return row_bcast_c<8>(v);
    case 9: return row_bcast_c<9>(v);
    case 10: return row_bcast_c<10>(v);
    case 11: return row_bcast_c<11>(v);
    case 12: return row_bcast_c<12>(v);
    case 13: return row_bcast_c<13>(v);
    case 14: return row_bcast_c<14>(v);
    default: return row_bcast_c<15>(v);
  }
}

// The lane's share of a general record in the register path: entry pairs
// (2p, 2p + 1) for p = lr, lr + 16, ..., nzp / 32 <= NZL / 2 of them, each
// pair one 8-byte value load and one 4-byte load of its two 16-bit rows
// (the list's own padding holds 0 on the task's dummy row).
template <int NZL>
struct GenRec {
  float2 val[NZL / 2];
  uint32_t row2[NZL / 2];  // rows of the pair: low and high 16 bits
};

template <int NZL>
__device__ __forceinline__ void load_gen(const SvArgs& a, size_t rec0, int j, int lr,
                                         GenRec<NZL>& g) {
  const size_t base = (rec0 + j) * (size_t)a.nzp;  // even: nzp is a multiple of 32
  const float2* gv = reinterpret_cast<const float2*>(a.gval + base) + lr;
  const uint32_t* gr = reinterpret_cast<const uint32_t*>(a.grow + base) + lr;
  const int np = a.nzp / (2 * kRowLanes);  // pairs per lane, the same for every lane
#pragma unroll
  for (int u = 0; u < NZL / 2; ++u)
    if (u < np) {  // slots past np are never read
      g.val[u] = gv[u * kRowLanes];
      g.row2[u] = gr[u * kRowLanes];
    }
}

// NZL > 0 (sweep mode only): records of at most 16 NZL entries, held in
// registers and loaded two pixels ahead; NZL = 0: any length, read in the
// pixel loop.
// E0N > 0 (sweep mode only, when gen_e0_in_regs): the staged e in E0N
// registers per lane (E0N >= kpad).
template <int MODE, int S, int NZL, int E0N>
__global__ __launch_bounds__(kBlockThreads) void sv_kernel_gen(SvArgs a) {
  constexpr int HS = S + 2;
  constexpr int NHC = halo_cells(S);
  extern __shared__ __align__(16) char smem[];
  const int lane64 = threadIdx.x & 63;
  const int lr = lane64 & 15;
  const int rib = threadIdx.x >> 4;  // row in block
  const int row = blockIdx.x * a.rpb + rib;
  const bool e0_regs = gen_e0_in_regs(a.kpad, a.wmax, a.nzp);
  const size_t per_row = gen_row_lds_bytes(a.bmax, S, e0_regs, a.vol_nz > 0);
  char* base = smem + rib * per_row;
  float2* band = reinterpret_cast<float2*>(base);
  float* e0l = reinterpret_cast<float*>(base + (size_t)a.bmax * 8);  // when !e0_regs
  float* halo = e0l + (e0_regs ? 0 : a.bmax);
  float* vv = halo + NHC;
  float* t2 = vv + S * S;
  float* xlo = t2 + S * S;  // volumes: the agent's voxels in slices z - 1, z + 1
  float* xhi = xlo + S * S;

  const int ndi = (lr < 3) ? -1 : (lr < 5 ? 0 : 1);
  const int ndj = (lr == 0 || lr == 3 || lr == 5) ? -1 : ((lr == 1 || lr == 6) ? 0 : 1);
  // lanes 9 and 10: the axial neighbours below and above (volumes)
  const bool axial = a.vol_nz > 0 && (lr == 9 || lr == 10);
  const float nbw = lr < 8 ? ((ndi != 0 && ndj != 0) ? a.bdiag : a.bedge) * a.invN
                           : (axial ? a.baxial * a.invN : 0.0f);
  const int noff = lr < 8 ? ndi * HS + ndj : 0;
  const int ndi8 = lr < 8 ? ndi : 0, ndj8 = lr < 8 ? ndj : 0;
  const float proxw = lr == 8 ? a.is2 : 0.0f;
  const bool row_ok = row < a.R;
  const int* my_tasks = a.tasks + (size_t)(row_ok ? row : 0) * a.T;

  for (int t = 0; t < a.T; ++t) {
    const int raw = row_ok ? my_tasks[t] : -1;
    if (raw < 0) continue;
    const int task = raw & ((1 << kSlotShift) - 1);
    const SlotDesc* sd = a.slots + (raw >> kSlotShift);
    if (!sd->active || sd->prec != 0) continue;
    const int agent = task / a.n_sv;
    const int sv = task - agent * a.n_sv;
    const size_t asv = (size_t)agent * a.n_sv + sv;
    const int sy = sv / a.gx, sx = sv - sy * a.gx;
    const int y0 = sy * S, x0 = sx * S;
    const int sh = min(S, a.ny - y0), sw = min(S, a.nx - x0);
    const int npix = sh * sw;
    const size_t img = (size_t)agent * a.n;
    gptr<float> eag = glb(sd->e) + (size_t)agent * a.estride;
    gptr<const float> lam = glb(sd->lam) + (size_t)agent * a.estride;
    gptr<float> cX = glb(sd->X);
    gptr<float> cw = glb(sd->w);
    gptr<const float> cwbar = glb(sd->wbar);
    gptr<float> cth2 = glb(sd->th2);
    gptr<double> cpart = glb(sd->part);
    const BandEnt* be = a.band + asv * a.kpad;
    const int B = a.band_rows[asv];
    const int z = raw >> kSlotShift;  // volumes: the task's slice
    const bool has_lo = a.vol_nz > 0 && z > 0, has_hi = a.vol_nz > 0 && z + 1 < a.vol_nz;

    // ---- 1. stage the band, 16 views at a time: each lane loads one
    //         view's band entry, every view's entry is broadcast over the
    //         row, and the 16 views' first 16 channels are loaded before
    //         any is written (channels past 16 of a wide view follow); e as
    //         staged goes to e0 (registers or LDS) for the write-back ----
    // one batch of 16 views from view slot kb; ev receives the lane's
    // staged e of each of them (its channel lr)
    auto stage_batch = [&](int kb, float* ev) {
      uint2 mine = make_uint2(0u, 0u);  // (gstart, lds_row | width << 16); 0: no view
      if (kb + lr < a.kpad) mine = *reinterpret_cast<const uint2*>(be + kb + lr);
      float lv[kRowLanes];
      uint32_t lw[kRowLanes], gs[kRowLanes];
#pragma unroll
      for (int k = 0; k < kRowLanes; ++k) {
        gs[k] = row_bcast(mine.x, k);
        lw[k] = row_bcast(mine.y, k);
        const int wd = (int)(lw[k] >> 16);
        // lanes past the band (and views past kpad: gstart 0) read a valid
        // entry of the agent's block and write nothing
        const uint32_t gi = gs[k] + (uint32_t)min(lr, max(wd - 1, 0));
        ev[k] = MODE == kSweep ? load_e(eag + gi) : 0.0f;
        lv[k] = MODE != kRefresh ? lam[gi] : 0.0f;
      }
#pragma unroll
      for (int k = 0; k < kRowLanes; ++k) {
        const int wd = (int)(lw[k] >> 16), lrow = (int)(lw[k] & 0xFFFFu);
        if (lr < wd) {
          band[lrow + lr] = make_float2(ev[k], lv[k]);
          if (MODE == kSweep && E0N == 0) e0l[lrow + lr] = ev[k];
        }
        if constexpr (E0N == 0) {  // bands wider than 16 channels
          for (int c = lr + kRowLanes; c < wd; c += kRowLanes) {
            const uint32_t gi = gs[k] + (uint32_t)c;
            const float e2 = MODE == kSweep ? load_e(eag + gi) : 0.0f;
            const float l2 = MODE != kRefresh ? lam[gi] : 0.0f;
            band[lrow + c] = make_float2(e2, l2);
            if (MODE == kSweep) e0l[lrow + c] = e2;
          }
        }
      }
    };
    float e0r[E0N > 0 ? E0N : 1];
    if constexpr (E0N > 0) {
#pragma unroll
      for (int kb = 0; kb < E0N; kb += kRowLanes) {
        if (kb < a.kpad) {
          float evb[kRowLanes];
          stage_batch(kb, evb);
#pragma unroll
          for (int k = 0; k < kRowLanes; ++k) e0r[kb + k] = evb[k];
        }
      }
    } else {
      for (int kb = 0; kb < a.kpad; kb += kRowLanes) {
        float evb[kRowLanes];
        stage_batch(kb, evb);
      }
    }
    if (lr < 2) band[B + lr] = make_float2(0.0f, 0.0f);
    // halo, v, theta2 (and the axial neighbours): fixed trip counts per
    // lane, unrolled so that several loads are in flight before the writes
    if (MODE != kTheta2) {
#pragma unroll 8
      for (int u = 0; u < NHC / kRowLanes; ++u) {
        const int c = u * kRowLanes + lr;  // cells past HS * HS are padding
        const int hi = c / HS, hj = c - hi * HS;
        const int iy = y0 - 1 + hi, ix = x0 - 1 + hj;
        const bool in = c < HS * HS && iy >= 0 && iy < a.ny && ix >= 0 && ix < a.nx;
        const int iyc = min(max(iy, 0), a.ny - 1), ixc = min(max(ix, 0), a.nx - 1);
        const float xv = cX[img + (size_t)iyc * a.nx + ixc];
        halo[c] = in ? xv : 0.0f;
      }
    }
    if (MODE == kSweep) {
      gptr<const float> Xlo = glb((const float*)a.slots[has_lo ? z - 1 : z].X);
      gptr<const float> Xhi = glb((const float*)a.slots[has_hi ? z + 1 : z].X);
#pragma unroll 8
      for (int u = 0; u < S * S / kRowLanes; ++u) {
        // S * S is a multiple of 16; entries past npix (ragged SVs) repeat
        // the last pixel and are never read
        const int p = u * kRowLanes + lr;
        const int pc = min(p, npix - 1);
        const int pi = pc / sw, pj = pc - (pc / sw) * sw;
        const size_t pix = (size_t)(y0 + pi) * a.nx + x0 + pj;
        vv[p] = 2.0f * cwbar[pix] - cw[img + pix];
        t2[p] = cth2[img + pix];
        if (a.vol_nz > 0) {
          // agent scope, past the L1: with slice groups the row itself
          // updated slice z - 1 in its previous task
          xlo[p] = has_lo ? load_e(Xlo + img + pix) : 0.0f;
          xhi[p] = has_hi ? load_e(Xhi + img + pix) : 0.0f;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();

    // ---- 2. pixel loop ----
    const size_t rec0 = (size_t)agent * a.n + (size_t)a.sv_pix0[sv];
    // The coordinate step of pixel j (sweep mode) from the lane's share of
    // theta1's sum: alpha, with z_s updated in the halo.  The caller gathers
    // `part` and applies alpha to the band.
    auto step_alpha = [&](int j, float part) {
      const int pi = j / sw, pj = j - (j / sw) * sw;
      const int cidx = (pi + 1) * HS + pj + 1;
      const float zs = halo[cidx];
      float nbv = halo[cidx + noff];
      const float vj = vv[j], tj = t2[j];
      const int iy = y0 + pi + ndi8, ix = x0 + pj + ndj8;
      // the clique's weight, 0 for a neighbour outside the image (volume)
      float nbwin = ((unsigned)iy < (unsigned)a.ny && (unsigned)ix < (unsigned)a.nx) ? nbw : 0.0f;
      if (axial) {
        nbv = lr == 9 ? xlo[j] : xhi[j];
        nbwin = (lr == 9 ? has_lo : has_hi) ? nbw : 0.0f;
      }
      const float d = zs - nbv;
      const float wgt = nbwin * prior_curv(a, d);
      const float gl = wgt * d + proxw * (zs - vj) - part;
      const float G = row_sum16(gl);
      const float H = row_sum16(wgt);
      const float alpha = -a.relax * G * __builtin_amdgcn_rcpf(tj + H + a.is2);
      if (lr == 0) halo[cidx] = zs + alpha;
      return alpha;
    };
    // entries per lane, and entry pairs per lane in the register path: nzp
    // is a multiple of 32, the same for every lane
    const int nu = a.nzp / kRowLanes;
    const int np = a.nzp / (2 * kRowLanes);
    if constexpr (MODE == kSweep && NZL > 0) {
      // records of at most 16 NZL entries: the lane's share in registers,
      // loaded two pixels ahead
      GenRec<NZL> buf[3];
      load_gen<NZL>(a, rec0, 0, lr, buf[0]);
      if (npix > 1) load_gen<NZL>(a, rec0, 1, lr, buf[1]);
      for (int jb = 0; jb < npix; jb += 3) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int j = jb + q;
          if (j < npix) {
            if (j + 2 < npix) load_gen<NZL>(a, rec0, j + 2, lr, buf[(q + 2) % 3]);
            const GenRec<NZL>& r = buf[q];
            float pa = 0.0f, pb = 0.0f;  // first and second entries of the pairs
            float ea[NZL / 2], eb[NZL / 2];  // their e, kept for the update
#pragma unroll
            for (int u = 0; u < NZL / 2; ++u)
              if (u < np) {
                const float2 p0 = band[r.row2[u] & 0xFFFFu], p1 = band[r.row2[u] >> 16];
                ea[u] = p0.x;
                eb[u] = p1.x;
                pa = __builtin_fmaf(r.val[u].x, p0.y * p0.x, pa);
                pb = __builtin_fmaf(r.val[u].y, p1.y * p1.x, pb);
              }
            const float alpha = step_alpha(j, pa + pb);
            // the rows of one column are distinct, so no other lane changes
            // them meanwhile; padding entries write back the dummy row's
            // value unchanged
#pragma unroll
            for (int u = 0; u < NZL / 2; ++u)
              if (u < np) {
                band[r.row2[u] & 0xFFFFu].x = ea[u] - r.val[u].x * alpha;
                band[r.row2[u] >> 16].x = eb[u] - r.val[u].y * alpha;
              }
            __builtin_amdgcn_wave_barrier();
          }
        }
      }
    } else {
      for (int j = 0; j < npix; ++j) {
        const int pi = j / sw, pj = j - (j / sw) * sw;
        const int cidx = (pi + 1) * HS + pj + 1;
        const float* gv = a.gval + (rec0 + j) * (size_t)a.nzp + lr;
        const uint16_t* gr = a.grow + (rec0 + j) * (size_t)a.nzp + lr;
        if (MODE == kSweep) {
          float part = 0.0f;
          for (int u = 0; u < nu; ++u) {
            const float2 p = band[gr[u * kRowLanes]];
            part = __builtin_fmaf(gv[u * kRowLanes], p.y * p.x, part);
          }
          const float alpha = step_alpha(j, part);
          for (int u = 0; u < nu; ++u) band[gr[u * kRowLanes]].x -= gv[u * kRowLanes] * alpha;
        } else if (MODE == kTheta2) {
          float part = 0.0f;
          for (int u = 0; u < nu; ++u) {
            const float av = gv[u * kRowLanes];
            part += av * av * band[gr[u * kRowLanes]].y;
          }
          const float th = row_sum16(part);
          if (lr == 0) cth2[img + (size_t)(y0 + pi) * a.nx + x0 + pj] = th;
        } else {
          const float xs = halo[cidx];
          for (int u = 0; u < nu; ++u) band[gr[u * kRowLanes]].x -= gv[u * kRowLanes] * xs;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }

    // ---- 3. write back, 16 views at a time (entries broadcast as in the
    //         staging) ----
    if (MODE != kTheta2) {
      auto flush_batch = [&](int kb, const float* e0b) {
        uint2 mine = make_uint2(0u, 0u);
        if (kb + lr < a.kpad) mine = *reinterpret_cast<const uint2*>(be + kb + lr);
#pragma unroll
        for (int k = 0; k < kRowLanes; ++k) {
          const uint32_t g0 = row_bcast(mine.x, k), lw = row_bcast(mine.y, k);
          const int wd = (int)(lw >> 16), lrow = (int)(lw & 0xFFFFu);
          if constexpr (E0N > 0) {  // every band fits one chunk
            if (lr < wd) {
              float d = band[lrow + lr].x;
              if (MODE == kSweep) d -= e0b[k];
              add_e(eag + g0 + lr, d);
            }
          } else {
            for (int c = lr; c < wd; c += kRowLanes) {
              float d = band[lrow + c].x;
              if (MODE == kSweep) d -= e0l[lrow + c];
              add_e(eag + g0 + c, d);
            }
          }
        }
      };
      if constexpr (E0N > 0) {
#pragma unroll
        for (int kb = 0; kb < E0N; kb += kRowLanes)
          if (kb < a.kpad) flush_batch(kb, e0r + kb);
      } else {
        for (int kb = 0; kb < a.kpad; kb += kRowLanes) flush_batch(kb, nullptr);
      }
    }
    if (MODE == kSweep) {
      double pn = 0.0, pd = 0.0, px = 0.0;
      for (int p = lr; p < npix; p += kRowLanes) {
        const int pi = p / sw, pj = p - (p / sw) * sw;
        const size_t pix = (size_t)(y0 + pi) * a.nx + x0 + pj;
        const float xn = halo[(pi + 1) * HS + pj + 1];
        cX[img + pix] = xn;
        if (a.mann) {
          const float wo = cw[img + pix], wb = cwbar[pix];
          const float v = 2.0f * wb - wo;
          cw[img + pix] = a.rho * (2.0f * xn - v) + (1.0f - a.rho) * wo;
          const double dd = (double)xn - (double)wb;
          pn += dd * dd;
          pd += (double)wo * (double)wo;
          px += (double)xn * (double)xn;
        }
      }
      if (a.mann) {
        double* red = reinterpret_cast<double*>(base);
        __builtin_amdgcn_wave_barrier();
        red[lr * 3 + 0] = pn;
        red[lr * 3 + 1] = pd;
        red[lr * 3 + 2] = px;
        __builtin_amdgcn_wave_barrier();
        if (lr == 0) {
          double s0 = 0.0, s1 = 0.0, s2 = 0.0;
          for (int l = 0; l < kRowLanes; ++l) {
            s0 += red[l * 3 + 0];
            s1 += red[l * 3 + 1];
            s2 += red[l * 3 + 2];
          }
          cpart[(size_t)task * 4 + 0] = s0;
          cpart[(size_t)task * 4 + 1] = s1;
          cpart[(size_t)task * 4 + 2] = s2;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (a.strict) __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
}

template <int MODE, int SV, int NZL, int E0N>
inline hipError_t launch_gen_mode(const SvArgs& a, int grid, size_t lds, hipStream_t st) {
  static std::atomic<bool> attr_set{false};
  if (!attr_set.load(std::memory_order_acquire)) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sv_kernel_gen<MODE, SV, NZL, E0N>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kMaxLdsBytes);
    if (e != hipSuccess) return e;
    attr_set.store(true, std::memory_order_release);
  }
  hipLaunchKernelGGL((sv_kernel_gen<MODE, SV, NZL, E0N>), dim3(grid), dim3(a.rpb * kRowLanes), lds,
                     st, a);
  return hipGetLastError();
}

// The staged e in registers takes the smallest of 32, 48 and 64 slots that
// holds kpad (only the sizes gen_e0_in_regs admits with these records).
template <int SV, int NZL>
inline hipError_t launch_gen_sweep(const SvArgs& a, int grid, size_t lds, hipStream_t st) {
  if (!gen_e0_in_regs(a.kpad, a.wmax, a.nzp)) return launch_gen_mode<kSweep, SV, NZL, 0>(a, grid, lds, st);
  if (a.kpad <= 2 * kRowLanes) return launch_gen_mode<kSweep, SV, NZL, 2 * kRowLanes>(a, grid, lds, st);
  if constexpr (NZL != 16) {
    if (a.kpad <= 3 * kRowLanes) return launch_gen_mode<kSweep, SV, NZL, 3 * kRowLanes>(a, grid, lds, st);
  }
  if constexpr (NZL == 0) return launch_gen_mode<kSweep, SV, NZL, 4 * kRowLanes>(a, grid, lds, st);
  return hipErrorInvalidValue;  // not reached: gen_e0_in_regs bounds kpad
}

template <int SV>
inline hipError_t launch_gen_s(const SvArgs& a, int mode, int grid, size_t lds, hipStream_t st) {
  if (mode == kSweep) {
    if (a.nzp <= 8 * kRowLanes) return launch_gen_sweep<SV, 8>(a, grid, lds, st);
    if (a.nzp <= 16 * kRowLanes) return launch_gen_sweep<SV, 16>(a, grid, lds, st);
    return launch_gen_sweep<SV, 0>(a, grid, lds, st);
  }
  if (mode == kTheta2) return launch_gen_mode<kTheta2, SV, 0, 0>(a, grid, lds, st);
  return launch_gen_mode<kRefresh, SV, 0, 0>(a, grid, lds, st);
}

}  // namespace mace
