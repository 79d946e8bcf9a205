#pragma once
// Super-voxel ICD sweep kernel (gfx950) of partial-update MACE: templates,
// instantiated per (super-voxel size, record precision) in mace_sweep_*.hip.
//
// sv_kernel: one launch processes one colour phase of the super-voxel (SV)
// tiling for all agents at once.  Each 16-lane row of a wave owns one
// (agent, SV) task at a time:
//   1. stage the agent's error-sinogram band of the SV (and Lambda) in LDS,
//      together with the SV's pixels plus a one-pixel halo of the agent image;
//   2. visit the SV's pixels in raster order; for each pixel (Algorithm 2):
//        theta1 = -sum_r A_rs Lambda_r e_r   (lanes over the agent's views,
//                                             two adjacent channels per view)
//        prior terms of the 8 neighbours     (lanes 0-7)
//        prox term (z_s - v_s)/sigma^2       (lane 8)
//      reduce over the 16 lanes (DPP butterfly), take the coordinate step
//        alpha = -(theta1 + P1 + (z_s - v_s)/sigma^2) / (theta2 + P2 + 1/sigma^2)
//      (P1, P2: the prior's gradient and curvature terms of the symmetric
//      quadratic majoriser, exact for the quadratic prior), and update the
//      band e_r -= A_rs alpha and z_s += alpha;
//   3. add the band's change to the agent's error sinogram with atomics and
//      write the pixels back; in the last sweep of a Mann iteration also apply
//      the reflection and Mann update w <- rho (2X - v) + (1 - rho) w for the
//      SV's pixels (Algorithm 1) and accumulate the FP64 residual partials.
// Same-colour SVs never touch each other's 8-neighbourhoods, so the prior
// reads no pixel that is changing.  SVs of one agent that run at the same
// time share sinogram rows: each works on the band as staged when it started
// (it may or may not see changes of SVs running beside it) and adds only its
// own change back with atomics, so e = y - A X holds exactly after every
// launch.  Kernel boundaries make all changes of a phase visible to the next.
// The coordinate step is scaled by `relax` (1: the exact minimiser of the
// surrogate; below 1: an under-relaxed step with the same fixed points).
#include <atomic>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "mace_internal.h"

namespace mace {

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 16 lanes of a DPP row; every lane receives the total.
__device__ __forceinline__ float row_sum16(float v) {
  // no contraction: each step stays one DPP add instead of an FMA that
  // recomputes the caller's product beside a separate DPP move
#pragma clang fp contract(off)
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return v;
}

// Curvature of the symmetric quadratic majoriser of the prior potential,
// c(d) = rho'(d)/d.  q-GGMRF with p = 2:
//   c(d) = (1/sigma_x^2) (1 + (q/2) s) / (1 + s)^2,  s = (|d| / (T sigma_x))^(2-q).
__device__ __forceinline__ float prior_curv(const SvArgs& a, float d) {
  if (a.kind == 0) return a.c0;
  float s;
  if (a.qexp == 0.0f) {
    s = 1.0f;
  } else {
    float u = fabsf(d) * a.inv_tsx;
    s = __builtin_amdgcn_exp2f(a.qexp * __builtin_amdgcn_logf(u));
  }
  float den = 1.0f + s;
  return a.c0 * (1.0f + a.qhalf * s) * __builtin_amdgcn_rcpf(den * den);
}

template <bool F16>
__device__ __forceinline__ float2 load_vals(const SvArgs& a, size_t idx, float scale) {
  if constexpr (F16) {
    const float2 f = __half22float2(a.hval[idx]);
    return make_float2(f.x * scale, f.y * scale);
  } else {
    return a.aval[idx];
  }
}

// Record of one pixel for the lane's view slots: (a0, a1) on channels d0,
// d0 + 1, and the row of d0 within its view's band (4 bits; 0 for a view the
// pixel misses, whose a0 = a1 = 0).  The row deltas of a pixel are packed
// eight to a 32-bit word: slot s * 16 + lr sits in word 2 s + lr / 8, bits
// 4 (lr mod 8) .. 4 (lr mod 8) + 3.
constexpr int kPrefetch = 3;
constexpr int kFlushGroup = 16;  // views per group in the band write-back

template <int SL>
struct Rec {
  float2 val[SL];
  int off[SL];  // row delta within the view's band
  float ax;     // volumes: the axial neighbour of lanes 9 and 10
};

__device__ __forceinline__ int row_delta(uint32_t word, int lr) {
  return (int)__builtin_amdgcn_ubfe(word, 4u * (uint32_t)(lr & 7), 4u);
}

// The values of a record are stored for the agents' largest view count
// kstr (not the padded 16 SL slots); a lane past it reads the next record
// (or the array's tail pad) and zeroes what it read.
template <int SL, bool F16>
__device__ __forceinline__ void load_rec(const SvArgs& a, size_t rec, int lr, Rec<SL>& r) {
  float scale = 1.0f;
  if constexpr (F16) scale = a.hscale[rec];
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    const size_t idx = rec * a.kstr + s * kRowLanes + lr;
    const float2 v = load_vals<F16>(a, idx, scale);
    const bool ok = s * kRowLanes + lr < a.kstr;
    r.val[s] = make_float2(ok ? v.x : 0.0f, ok ? v.y : 0.0f);
    r.off[s] = row_delta(a.adel[rec * (SL * 2) + s * 2 + (lr >> 3)], lr);
  }
}

// Record j of a super-voxel from per-SV base pointers (the lane's first slot
// of the SV's first pixel; values at stride kstr, row deltas at 2 SL words).
// Only the last slot group can run past kstr: last_ok says whether this
// lane's slot there is a view.
template <int SL, bool F16>
__device__ __forceinline__ void load_rec_at(const float2* vb, const __half2* hb, const float* sb,
                                            const uint32_t* db, int kstr, bool last_ok, int lr,
                                            int j, Rec<SL>& r) {
  float scale = 1.0f;
  if constexpr (F16) scale = sb[j];
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    float2 v;
    if constexpr (F16) {
      const float2 f = __half22float2(hb[(size_t)j * kstr + s * kRowLanes]);
      v = make_float2(f.x * scale, f.y * scale);
    } else {
      v = vb[(size_t)j * kstr + s * kRowLanes];
    }
    if (s == SL - 1) v = make_float2(last_ok ? v.x : 0.0f, last_ok ? v.y : 0.0f);
    r.val[s] = v;
    r.off[s] = row_delta(db[j * (SL * 2) + s * 2], lr);
  }
}

// The staged copy of e that the write-back subtracts lives in registers for
// up to 64 views per agent, in LDS beyond that.
__host__ __device__ constexpr bool e0_in_lds(int kpad) { return kpad > 4 * kRowLanes; }

// Halo cells of an S x S super-voxel, padded to whole 16-lane groups.
__host__ __device__ constexpr int halo_cells(int S) {
  return ((S + 2) * (S + 2) + kRowLanes - 1) / kRowLanes * kRowLanes;
}

// LDS bytes of one row: band (e, Lambda) over bmax rows, the staged copy of e
// when it does not stay in registers, the halo tile of the agent image, and a
// scratch area that holds the task's band entries while its band is staged,
// then v and theta2 of the SV's pixels.
__host__ __device__ inline size_t row_lds_bytes(int bmax, int S, int kpad) {
  const size_t scratch = (size_t)S * S * 8 > (size_t)kpad * 8 ? (size_t)S * S * 8 : (size_t)kpad * 8;
  size_t per_row = (size_t)bmax * 8 + (e0_in_lds(kpad) ? (size_t)bmax * 4 : 0) +
                   (size_t)halo_cells(S) * 4 + scratch;
  per_row = (per_row + 7) & ~(size_t)7;
  const size_t red = kRowLanes * 3 * sizeof(double);  // per-task FP64 reduction
  return per_row > red ? per_row : red;
}

// Per-scan buffers reached through the slot table are global memory; saying
// so keeps their accesses off the flat path (whose loads also count as LDS
// operations and would stall the LDS waits of the pixel loop).
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> glb(T* p) {
  return (gptr<T>)p;
}

// Error-sinogram entries are read at agent scope (from L2): other rows add
// their changes there with atomics during the launch.
__device__ __forceinline__ float load_e(gptr<const float> p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_e(gptr<float> p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Two waves per SIMD when the register budget allows it: the second wave's
// instructions fill the first one's LDS and dependency stalls.
template <int SL>
struct Occupancy {
  static constexpr int waves = SL <= 3 ? 2 : 1;
};

// VOL: the slots are the slices of a volume, and lanes 9 and 10 add the
// axial cliques to the agent's voxels of slices z - 1 and z + 1 (read with
// the records, a pixel step ahead; the other parity's slices do not change
// during the launch).
template <int SL, int MODE, int S, bool F16, bool VOL = false>
__global__ __launch_bounds__(kBlockThreads, Occupancy<SL>::waves) void sv_kernel(SvArgs a) {
  constexpr int HS = S + 2;
  constexpr int KP = SL * kRowLanes;                                 // view slots
  constexpr int HC = halo_cells(S) / kRowLanes;                     // halo cells per lane
  constexpr int PPL = (S * S + kRowLanes - 1) / kRowLanes;          // pixels per lane
  static_assert(PPL * kRowLanes == S * S, "a row covers the SV's pixels in whole lane groups");
  constexpr bool kE0Lds = e0_in_lds(KP);
  constexpr bool kE0Reg = MODE == kSweep && !kE0Lds;
  extern __shared__ __align__(16) char smem[];
  const int lane64 = threadIdx.x & 63;
  const int lr = lane64 & 15;
  const int rib = ((threadIdx.x >> 6) << 2) | (lane64 >> 4);  // row in block
  const int row = blockIdx.x * a.rpb + rib;
  const size_t per_row = row_lds_bytes(a.bmax, S, KP);
  char* base = smem + rib * per_row;
  float2* band = reinterpret_cast<float2*>(base);
  float* e0l = reinterpret_cast<float*>(base + (size_t)a.bmax * 8);  // kE0Lds only
  float* halo = reinterpret_cast<float*>(base + (size_t)a.bmax * (kE0Lds ? 12 : 8));
  float* vv = halo + halo_cells(S);
  float* t2 = vv + S * S;
  BandEnt* bents = reinterpret_cast<BandEnt*>(vv);  // while the band is staged

  // neighbour of lanes 0-7: (di, dj) in raster order of the 3x3 block
  const int ndi = (lr < 3) ? -1 : (lr < 5 ? 0 : 1);
  const int ndj = (lr == 0 || lr == 3 || lr == 5) ? -1 : ((lr == 1 || lr == 6) ? 0 : 1);
  // lanes 8-15 carry no neighbour: zero weight, offset 0 (their own cell)
  // lanes 9 and 10 of a volume: the axial neighbours below and above
  const bool axial = VOL && (lr == 9 || lr == 10);
  const float nbw = lr < 8 ? ((ndi != 0 && ndj != 0) ? a.bdiag : a.bedge) * a.invN
                           : (axial ? a.baxial * a.invN : 0.0f);
  const int noff = lr < 8 ? ndi * HS + ndj : 0;
  const int ndi8 = lr < 8 ? ndi : 0, ndj8 = lr < 8 ? ndj : 0;
  const float proxw = lr == 8 ? a.is2 : 0.0f;  // lane 8 adds the prox term

  const bool row_ok = row < a.R;
  const bool strict = a.strict != 0;
  const int* my_tasks = a.tasks + (size_t)(row_ok ? row : 0) * a.T;

  // Header of a task: everything its id determines (issued one task ahead).
  struct Hdr {
    int task;  // agent * n_sv + sv, or -1
    int slot;  // the task's slot (the slice of a volume)
    gptr<float> e;
    gptr<const float> lam;
    gptr<float> X, w, th2;
    gptr<const float> wbar;
    gptr<double> part;
    int B, pix0;
    BandEnt cb[SL];  // the lane's band entries (view slots lr, lr + 16, ...)
  };
  auto load_hdr = [&](int raw, Hdr& h) {
    h.task = -1;
    if (raw < 0) return;
    const int task = raw & ((1 << kSlotShift) - 1);
    h.slot = raw >> kSlotShift;
    const SlotDesc* sd = a.slots + h.slot;
    const int agent = task / a.n_sv;
    const int sv = task - agent * a.n_sv;
    const size_t agent_sv = (size_t)agent * a.n_sv + sv;
    const BandEnt* be = a.band + agent_sv * KP;
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) h.cb[sl] = be[sl * kRowLanes + lr];
    h.B = a.band_rows[agent_sv];
    h.pix0 = a.sv_pix0[sv];
    h.e = glb(sd->e) + (size_t)agent * a.estride;
    h.lam = glb(sd->lam) + (size_t)agent * a.estride;
    h.X = glb(sd->X);
    h.w = glb(sd->w);
    h.wbar = glb(sd->wbar);
    h.th2 = glb(sd->th2);
    h.part = glb(sd->part);
    if (sd->active && sd->prec == (F16 ? 1 : 0)) h.task = task;
  };
  // Stage task h in LDS: its band (e, Lambda) with the 16 lanes on
  // consecutive channels of one view at a time, the halo tile of the agent
  // image, v = 2 w-bar - w and theta2 of its pixels; e as staged stays in e0
  // (registers or LDS) for the write-back, w and w-bar in wo / wb.
  auto stage = [&](const Hdr& h, float* e0r, float* wo, float* wb) {
    if (h.task < 0) return;
    const int agent = h.task / a.n_sv;
    const int sv = h.task - agent * a.n_sv;
    const int sy = sv / a.gx, sx = sv - sy * a.gx;
    const int y0 = sy * S, x0 = sx * S;
    const int sw = min(S, a.nx - x0);
    const int npix = min(S, a.ny - y0) * sw;
    const size_t img = (size_t)agent * a.n;
    float ev[KP], lv[KP];
    float hv[HC], t2v[PPL];
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) bents[sl * kRowLanes + lr] = h.cb[sl];
    __builtin_amdgcn_wave_barrier();
    // No branches: lanes past a view's band re-read its last channel (an
    // empty band has gstart 0), so every address is valid whatever the lane
    // and the entry's fields are used unconditionally.
    const uint2* bent2 = reinterpret_cast<const uint2*>(bents);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const uint2 b = bent2[k];  // (gstart, lds_row | width << 16)
      const int wd = (int)(b.y >> 16);
      const uint32_t gi = b.x + (uint32_t)min(lr, max(wd - 1, 0));
      // values of lanes past the band go to the throw-away cell below and
      // are never subtracted in the write-back
      ev[k] = MODE == kSweep ? load_e(h.e + gi) : 0.0f;
      lv[k] = MODE != kRefresh ? h.lam[gi] : 0.0f;
    }
    if (MODE != kTheta2) {
#pragma unroll
      for (int u = 0; u < HC; ++u) {
        // cells past HS * HS are padding; every load reads a pixel inside
        // the image and out-of-image cells are zeroed
        const int c = u * kRowLanes + lr;
        const int hi = c / HS, hj = c - (c / HS) * HS;
        const int iy = y0 - 1 + hi, ix = x0 - 1 + hj;
        const bool in = iy >= 0 && iy < a.ny && ix >= 0 && ix < a.nx;
        const int iyc = min(max(iy, 0), a.ny - 1), ixc = min(max(ix, 0), a.nx - 1);
        const float xv = h.X[img + (size_t)iyc * a.nx + ixc];
        hv[u] = in ? xv : 0.0f;
      }
    }
    if (MODE == kSweep) {
#pragma unroll
      for (int u = 0; u < PPL; ++u) {
        // PPL * 16 == S * S; entries past npix (ragged SVs) repeat the last
        // pixel and are never read
        const int p = u * kRowLanes + lr;
        const int pc = min(p, npix - 1);
        const int pi = pc / sw, pj = pc - (pc / sw) * sw;
        const size_t pix = (size_t)(y0 + pi) * a.nx + x0 + pj;
        wb[u] = h.wbar[pix];
        wo[u] = h.w[img + pix];
        t2v[u] = h.th2[img + pix];
      }
    }
    // LDS writes; lanes past a view's band write to a throw-away cell (the
    // halo, written last).  The band entries are read again rather than
    // kept in registers (the empty asm keeps the compiler from reusing the
    // first reads).
    asm volatile("" ::: "memory");
    float2* trash2 = reinterpret_cast<float2*>(halo);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const uint2 b = bent2[k];
      const int wd = (int)(b.y >> 16), lrow = (int)(b.y & 0xFFFFu);
      float2* dst = lr < wd ? band + lrow + lr : trash2;
      *dst = make_float2(ev[k], lv[k]);
      if constexpr (kE0Lds && MODE == kSweep) {
        float* d0 = lr < wd ? e0l + lrow + lr : reinterpret_cast<float*>(trash2);
        *d0 = ev[k];
      }
      if constexpr (kE0Reg) e0r[k] = ev[k];
    }
    if (lr < 2) band[h.B + lr] = make_float2(0.0f, 0.0f);
    if (MODE != kTheta2) {
#pragma unroll
      for (int u = 0; u < HC; ++u) halo[u * kRowLanes + lr] = hv[u];
    }
    if (MODE == kSweep) {
      __builtin_amdgcn_wave_barrier();  // v / theta2 overwrite the band entries
#pragma unroll
      for (int u = 0; u < PPL; ++u) {
        const int p = u * kRowLanes + lr;
        vv[p] = 2.0f * wb[u] - wo[u];
        t2[p] = t2v[u];
      }
    }
  };

  Hdr h;
  load_hdr((row_ok && a.T > 0) ? my_tasks[0] : -1, h);
  int raw_next = (row_ok && a.T > 1) ? my_tasks[1] : -1;
  for (int t = 0; t < a.T; ++t) {
    const Hdr cur = h;
    // ---- 1. stage the task ----
    float e0r[kE0Reg ? KP : 1];
    float cwo[PPL], cwb[PPL];
    stage(cur, e0r, cwo, cwb);
    __builtin_amdgcn_wave_barrier();
    // header of the next task, loaded behind this task's pixel loop
    load_hdr(raw_next, h);
    raw_next = (row_ok && t + 2 < a.T) ? my_tasks[t + 2] : -1;
    if (cur.task < 0) continue;
    const int task = cur.task;
    const int agent = task / a.n_sv;
    const int sv = task - agent * a.n_sv;
    const int sy = sv / a.gx, sx = sv - sy * a.gx;
    const int y0 = sy * S, x0 = sx * S;
    const int sh = min(S, a.ny - y0), sw = min(S, a.nx - x0);
    const int npix = sh * sw;
    const size_t img = (size_t)agent * a.n;
    const int pix0 = cur.pix0;
    gptr<float> eag = cur.e;
    gptr<float> cX = cur.X;
    gptr<float> cw = cur.w;
    gptr<float> cth2 = cur.th2;
    gptr<double> cpart = cur.part;
    // volumes: the slices below and above (own slice where there is none;
    // those lanes' weight is then 0)
    const bool has_lo = VOL && cur.slot > 0, has_hi = VOL && cur.slot + 1 < a.vol_nz;
    const int zn = lr == 9 ? (has_lo ? cur.slot - 1 : cur.slot)
                           : (lr == 10 && has_hi ? cur.slot + 1 : cur.slot);
    // (read at agent scope, past the L1: with slice groups the row itself
    // updated slice z - 1 in its previous task)
    gptr<const float> axp = nullptr;
    if constexpr (VOL) axp = glb((const float*)a.slots[zn].X) + img;
    const float ax_in = (lr == 9 ? has_lo : has_hi) ? 1.0f : 0.0f;

    // ---- 2. pixel loop: records prefetched kPrefetch pixels ahead ----
    const size_t rec0 = (size_t)agent * a.n + pix0;
    // first LDS row of each of the lane's views in this task's band (the
    // dummy rows of the task for a view that misses the super-voxel)
    float2* bl[SL];
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) bl[sl] = band + cur.cb[sl].lds_row;
    auto update = [&](const Rec<SL>& cur, int j, int pi, int pj) {
      const int cidx = (pi + 1) * HS + pj + 1;
      // the pixel's two band rows in each of the lane's views
      float2* o[SL];
#pragma unroll
      for (int s2 = 0; s2 < SL; ++s2) o[s2] = bl[s2] + cur.off[s2];
      if (MODE == kSweep) {
        // every LDS read of this pixel first, then the arithmetic
        float2 p0[SL], p1[SL];
#pragma unroll
        for (int s2 = 0; s2 < SL; ++s2) {
          p0[s2] = o[s2][0];
          p1[s2] = o[s2][1];
        }
        const float zs = halo[cidx];
        float nbv = halo[cidx + noff];
        const float vj = vv[j], tj = t2[j];
        // the neighbour lies in the image (lanes 8-15: weight 0 anyway)
        const int iy = y0 + pi + ndi8, ix = x0 + pj + ndj8;
        // the clique's weight, 0 for a neighbour outside the image
        float nbwin = ((unsigned)iy < (unsigned)a.ny && (unsigned)ix < (unsigned)a.nx) ? nbw : 0.0f;
        if constexpr (VOL) {
          if (axial) {
            nbv = cur.ax;
            nbwin = nbw * ax_in;
          }
        }
        // the lane's share of theta1's sum: two FMA chains over the slots
        // (first and second channel), joined at the end
        float pa = cur.val[0].x * (p0[0].y * p0[0].x);
        float pb = cur.val[0].y * (p1[0].y * p1[0].x);
#pragma unroll
        for (int s2 = 1; s2 < SL; ++s2) {
          pa = __builtin_fmaf(cur.val[s2].x, p0[s2].y * p0[s2].x, pa);
          pb = __builtin_fmaf(cur.val[s2].y, p1[s2].y * p1[s2].x, pb);
        }
        const float part = pa + pb;
        const float d = zs - nbv;
        const float wgt = nbwin * prior_curv(a, d);
        const float gl = wgt * d + proxw * (zs - vj) - part;
        const float H = row_sum16(wgt);
        const float G = row_sum16(gl);
        const float alpha = -a.relax * G * __builtin_amdgcn_rcpf(tj + H + a.is2);
#pragma unroll
        for (int s2 = 0; s2 < SL; ++s2) {
          o[s2][0].x = p0[s2].x - cur.val[s2].x * alpha;
          o[s2][1].x = p1[s2].x - cur.val[s2].y * alpha;
        }
        if (lr == 0) halo[cidx] = zs + alpha;
      } else if (MODE == kTheta2) {
        float part = 0.0f;
#pragma unroll
        for (int s2 = 0; s2 < SL; ++s2) {
          const float l0 = o[s2][0].y, l1 = o[s2][1].y;
          part += cur.val[s2].x * cur.val[s2].x * l0 + cur.val[s2].y * cur.val[s2].y * l1;
        }
        const float th = row_sum16(part);
        if (lr == 0) {
          const size_t pix = (size_t)(y0 + pi) * a.nx + x0 + pj;
          cth2[img + pix] = th;
        }
      } else {  // kRefresh: accumulate -A x into the band
        const float xs = halo[cidx];
#pragma unroll
        for (int s2 = 0; s2 < SL; ++s2) {
          o[s2][0].x -= cur.val[s2].x * xs;
          o[s2][1].x -= cur.val[s2].y * xs;
        }
      }
      __builtin_amdgcn_wave_barrier();
    };
    if (npix == S * S) {
      // full super-voxel: straight-line code, every record in its own
      // registers, so each wait covers exactly the record it needs
      const int kstr = a.kstr;
      const bool last_ok = (SL - 1) * kRowLanes + lr < kstr;
      const size_t rb = rec0 * kstr + lr;
      const float2* vb = F16 ? nullptr : a.aval + rb;
      const __half2* hb = F16 ? a.hval + rb : nullptr;
      const float* sb = F16 ? a.hscale + rec0 : nullptr;
      const uint32_t* db = a.adel + rec0 * (SL * 2) + (lr >> 3);
      Rec<SL> buf[S * S];
#pragma unroll
      for (int q = 0; q < kPrefetch; ++q) {
        load_rec_at<SL, F16>(vb, hb, sb, db, kstr, last_ok, lr, q, buf[q]);
        if constexpr (VOL) buf[q].ax = load_e(axp + (size_t)(y0 + q / S) * a.nx + x0 + q % S);
      }
#pragma unroll
      for (int j = 0; j < S * S; ++j) {
        if (j + kPrefetch < S * S) {
          load_rec_at<SL, F16>(vb, hb, sb, db, kstr, last_ok, lr, j + kPrefetch, buf[j + kPrefetch]);
          if constexpr (VOL) {
            const int q = j + kPrefetch;
            buf[q].ax = load_e(axp + (size_t)(y0 + q / S) * a.nx + x0 + q % S);
          }
        }
        update(buf[j], j, j / S, j % S);
      }
    } else {
      // ragged super-voxel at the image border
      for (int j = 0; j < npix; ++j) {
        Rec<SL> cur;
        load_rec<SL, F16>(a, rec0 + j, lr, cur);
        if constexpr (VOL) cur.ax = load_e(axp + (size_t)(y0 + j / sw) * a.nx + x0 + j - (j / sw) * sw);
        update(cur, j, j / sw, j - (j / sw) * sw);
      }
    }

    // ---- 3. write back: the band's change goes to the agent's error
    //         sinogram with atomics, one view per instruction, the 16 lanes
    //         on consecutive channels (one or two cache lines each; a band
    //         is at most 16 channels wide).  Views go in groups of
    //         kFlushGroup so that their LDS reads overlap. ----
    if (MODE != kTheta2) {
      // v / theta2 are done: the scratch area holds the band entries again
#pragma unroll
      for (int sl = 0; sl < SL; ++sl) bents[sl * kRowLanes + lr] = cur.cb[sl];
      __builtin_amdgcn_wave_barrier();
      const uint2* bent2 = reinterpret_cast<const uint2*>(bents);
#pragma unroll
      for (int kb = 0; kb < KP; kb += kFlushGroup) {
        uint2 b[kFlushGroup];
        float d[kFlushGroup];
#pragma unroll
        for (int u = 0; u < kFlushGroup; ++u) b[u] = bent2[kb + u];
#pragma unroll
        for (int u = 0; u < kFlushGroup; ++u) {
          // lanes past the band read its last row (any valid row) and add
          // nothing
          const int wd = (int)(b[u].y >> 16), lrow = (int)(b[u].y & 0xFFFFu);
          const int r = lrow + min(lr, max(wd - 1, 0));
          d[u] = band[r].x;
          if constexpr (MODE == kSweep) {
            if constexpr (kE0Reg) d[u] -= e0r[kb + u];
            else d[u] -= e0l[r];
          }
        }
#pragma unroll
        for (int u = 0; u < kFlushGroup; ++u)
          if (lr < (int)(b[u].y >> 16)) add_e(eag + b[u].x + lr, d[u]);
      }
    }
    if (MODE == kSweep) {
      double pn = 0.0, pd = 0.0, px = 0.0;
#pragma unroll
      for (int u = 0; u < PPL; ++u) {
        const int p = u * kRowLanes + lr;
        if (p < npix) {
          const int pi = p / sw, pj = p - (p / sw) * sw;
          const size_t pix = (size_t)(y0 + pi) * a.nx + x0 + pj;
          const float xn = halo[(pi + 1) * HS + pj + 1];
          cX[img + pix] = xn;
          if (a.mann) {
            const float wo = cwo[u], wb = cwb[u];
            const float v = 2.0f * wb - wo;
            cw[img + pix] = a.rho * (2.0f * xn - v) + (1.0f - a.rho) * wo;
            const double dd = (double)xn - (double)wb;
            pn += dd * dd;
            pd += (double)wo * (double)wo;
            px += (double)xn * (double)xn;
          }
        }
      }
      if (a.mann) {
        // the task's FP64 partials, summed over the row in a fixed order
        // through LDS (the band is free after the write-back)
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
    // sequential schedule: this row's atomics complete before it stages its
    // next band
    if (strict) __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
}


template <int MODE, int SV, bool F16V, bool VOL = false>
inline hipError_t launch_mode(const SvArgs& a, int slots, int grid, size_t lds, hipStream_t st) {
  switch (slots) {
#define MACE_CASE(SLV)                                                                   \
  case SLV: {                                                                            \
    static std::atomic<bool> attr_set{false};                                            \
    if (!attr_set.load(std::memory_order_acquire)) {                                     \
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sv_kernel<SLV, MODE, SV, F16V, VOL>), \
                                         hipFuncAttributeMaxDynamicSharedMemorySize,     \
                                         (int)kMaxLdsBytes);                              \
      if (e != hipSuccess) return e;                                                     \
      attr_set.store(true, std::memory_order_release);                                   \
    }                                                                                    \
    hipLaunchKernelGGL((sv_kernel<SLV, MODE, SV, F16V, VOL>), dim3(grid), dim3(a.rpb * kRowLanes), lds, st, a); \
    break;                                                                               \
  }
    MACE_CASE(1)
    MACE_CASE(2)
    MACE_CASE(3)
    MACE_CASE(4)
    MACE_CASE(5)
    MACE_CASE(6)
    MACE_CASE(7)
    MACE_CASE(8)
#undef MACE_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int SV, bool F16V>
inline hipError_t launch_s(const SvArgs& a, int mode, int slots, int grid, size_t lds,
                           hipStream_t st) {
  if constexpr (!F16V) {  // volumes run with FP32 values
    if (mode == kSweep && a.vol_nz > 0) return launch_mode<kSweep, SV, false, true>(a, slots, grid, lds, st);
  }
  if (mode == kSweep) return launch_mode<kSweep, SV, F16V>(a, slots, grid, lds, st);
  if (mode == kTheta2) return launch_mode<kTheta2, SV, F16V>(a, slots, grid, lds, st);
  return launch_mode<kRefresh, SV, F16V>(a, slots, grid, lds, st);
}

}  // namespace mace
