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
// d0 + 1 and the LDS row of d0.
constexpr int kPrefetch = 4;

template <int SL>
struct Rec {
  float2 val[SL];
  int off[SL];
};

template <int SL, bool F16>
__device__ __forceinline__ void load_rec(const SvArgs& a, size_t rec, int lr, Rec<SL>& r) {
  float scale = 1.0f;
  if constexpr (F16) scale = a.hscale[rec];
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    const size_t idx = rec * (SL * kRowLanes) + s * kRowLanes + lr;
    r.val[s] = load_vals<F16>(a, idx, scale);
    r.off[s] = a.aoff[idx];
  }
}

// Record j of a super-voxel from per-SV base pointers (the lane's first slot
// of the SV's first pixel): the offsets are compile-time constants.
template <int SL, bool F16>
__device__ __forceinline__ void load_rec_at(const float2* vb, const __half2* hb, const float* sb,
                                            const uint16_t* ob, int j, Rec<SL>& r) {
  constexpr int KP = SL * kRowLanes;
  float scale = 1.0f;
  if constexpr (F16) scale = sb[j];
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    if constexpr (F16) {
      const float2 f = __half22float2(hb[j * KP + s * kRowLanes]);
      r.val[s] = make_float2(f.x * scale, f.y * scale);
    } else {
      r.val[s] = vb[j * KP + s * kRowLanes];
    }
    r.off[s] = ob[j * KP + s * kRowLanes];
  }
}

// LDS bytes of one row: band (e, Lambda) and the staged copy of e over bmax
// rows, the halo tile (value, inside-image flag), v and theta2 of the SV.
__host__ __device__ inline size_t row_lds_bytes(int bmax, int S, int kpad) {
  const size_t HS = S + 2;
  const size_t per_row = (size_t)bmax * 12 + HS * HS * 8 + (size_t)S * S * 8 + (size_t)kpad * 8;
  const size_t red = kRowLanes * 3 * sizeof(double);  // per-task FP64 reduction
  return per_row > red ? per_row : red;
}

// Everything a row needs to start its next task, loaded into registers while
// the current task's pixels are being updated.
template <int SL, int S, int WM>
struct Stage {
  static constexpr int HS = S + 2;
  static constexpr int HC = (HS * HS + kRowLanes - 1) / kRowLanes;  // halo cells per lane
  static constexpr int PPL = (S * S + kRowLanes - 1) / kRowLanes;   // pixels per lane
  int task;   // agent * n_sv + sv, or -1
  int B;
  int pix0;
  float* e;   // the task's slot: error sinogram, agent state, Mann state,
  float* X;   // theta2 and residual partials
  float* w;
  float* th2;
  double* part;
  BandEnt be[SL];
  float ev[SL][WM];
  float lv[SL][WM];
  float hv[HC];
  float wo[PPL];  // w of the agent before the update
  float wb[PPL];  // consensus average w-bar
  float t2[PPL];
};

template <int SL, int MODE, int S, bool F16>
__global__ __launch_bounds__(kBlockThreads) void sv_kernel(SvArgs a) {
  constexpr int WM = (S <= 4) ? 8 : 16;
  constexpr int HS = S + 2;
  using St = Stage<SL, S, WM>;
  extern __shared__ __align__(16) char smem[];
  const int lane64 = threadIdx.x & 63;
  const int lr = lane64 & 15;
  const int rib = ((threadIdx.x >> 6) << 2) | (lane64 >> 4);  // row in block
  const int row = blockIdx.x * kRowsPerBlock + rib;
  const size_t per_row = row_lds_bytes(a.bmax, S, a.kpad);
  char* base = smem + rib * per_row;
  float2* band = reinterpret_cast<float2*>(base);
  float* e0 = reinterpret_cast<float*>(base + (size_t)a.bmax * 8);
  float2* halo = reinterpret_cast<float2*>(base + (size_t)a.bmax * 12);
  float* vv = reinterpret_cast<float*>(base + (size_t)a.bmax * 12 + (size_t)HS * HS * 8);
  float* t2 = vv + S * S;
  BandEnt* bents = reinterpret_cast<BandEnt*>(t2 + S * S);  // [kpad]

  // neighbour of lanes 0-7: (di, dj) in raster order of the 3x3 block
  const int ndi = (lr < 3) ? -1 : (lr < 5 ? 0 : 1);
  const int ndj = (lr == 0 || lr == 3 || lr == 5) ? -1 : ((lr == 1 || lr == 6) ? 0 : 1);
  // lanes 8-15 carry no neighbour: zero weight, offset 0 (their own cell)
  const float nbw = lr < 8 ? ((ndi != 0 && ndj != 0) ? a.bdiag : a.bedge) * a.invN : 0.0f;
  const int noff = lr < 8 ? ndi * HS + ndj : 0;
  const float proxw = lr == 8 ? a.is2 : 0.0f;  // lane 8 adds the prox term

  const bool row_ok = row < a.R;
  // strict: this row sees every earlier task's changes (one SV of an agent
  // at a time); otherwise the next band may be staged before the current
  // task's changes land
  const bool strict = a.strict != 0;

  // ---- staging of task t into registers ----
  auto stage_load = [&](int t, St& st) {
    const int raw = (row_ok && t < a.T) ? a.tasks[(size_t)row * a.T + t] : -1;
    st.task = -1;
    if (raw < 0) return;
    const int local = raw & ((1 << kSlotShift) - 1);
    const SlotDesc* sd = a.slots + (raw >> kSlotShift);
    const int agent = local / a.n_sv;
    const int sv = local - agent * a.n_sv;
    const int sy = sv / a.gx, sx = sv - sy * a.gx;
    const int y0 = sy * S, x0 = sx * S;
    const int sh = min(S, a.ny - y0), sw = min(S, a.nx - x0);
    const size_t agent_sv = (size_t)agent * a.n_sv + sv;
    const BandEnt* be = a.band + agent_sv * a.kpad;
    const size_t img = (size_t)agent * a.n;
    // slot pointers and the task's tables are independent loads
    float* se = sd->e;
    const float* slam = sd->lam;
    float* sX = sd->X;
    float* sw_ = sd->w;
    const float* swb = sd->wbar;
    float* sth2 = sd->th2;
    double* spart = sd->part;
    const int sactive = sd->active;
    st.B = a.band_rows[agent_sv];
    st.pix0 = a.sv_pix0[sv];
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) st.be[sl] = be[sl * kRowLanes + lr];
    if (!sactive) return;
    st.task = local;
    st.e = se;
    st.X = sX;
    st.w = sw_;
    st.th2 = sth2;
    st.part = spart;
    const float* eag = se + (size_t)agent * a.estride;
    const float* lag = slam + (size_t)agent * a.estride;
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int wdt = min((int)st.be[sl].width, WM);
#pragma unroll
      for (int c = 0; c < WM; ++c) {
        st.ev[sl][c] = 0.0f;
        st.lv[sl][c] = 0.0f;
        if (c < wdt) {
          if (MODE == kSweep && !strict) st.ev[sl][c] = eag[st.be[sl].gstart + c];
          if (MODE != kRefresh) st.lv[sl][c] = lag[st.be[sl].gstart + c];
        }
      }
    }
    if (MODE != kTheta2) {
#pragma unroll
      for (int u = 0; u < St::HC; ++u) {
        const int c = u * kRowLanes + lr;
        const int hi = c / HS, hj = c - (c / HS) * HS;
        const int iy = y0 - 1 + hi, ix = x0 - 1 + hj;
        const bool in = c < HS * HS && iy >= 0 && iy < a.ny && ix >= 0 && ix < a.nx;
        st.hv[u] = in ? sX[img + (size_t)iy * a.nx + ix] : 0.0f;
      }
    }
    if (MODE == kSweep) {
#pragma unroll
      for (int u = 0; u < St::PPL; ++u) {
        const int p = u * kRowLanes + lr;
        st.wo[u] = 0.0f;
        st.wb[u] = 0.0f;
        st.t2[u] = 0.0f;
        if (p < sh * sw) {
          const int pi = p / sw, pj = p - (p / sw) * sw;
          const size_t pix = (size_t)(y0 + pi) * a.nx + x0 + pj;
          st.wb[u] = swb[pix];
          st.wo[u] = sw_[img + pix];
          st.t2[u] = sth2[img + pix];
        }
      }
    }
  };

  St st;
  stage_load(0, st);
  for (int t = 0; t < a.T; ++t) {
    // current task from the stage
    const int task = st.task;
    if (task >= 0) {
      const int agent = task / a.n_sv;
      const int sv = task - agent * a.n_sv;
      const int sy = sv / a.gx, sx = sv - sy * a.gx;
      const int y0 = sy * S, x0 = sx * S;
      const int sh = min(S, a.ny - y0), sw = min(S, a.nx - x0);
      const int npix = sh * sw;
      const size_t agent_sv = (size_t)agent * a.n_sv + sv;
      const BandEnt* be = a.band + agent_sv * a.kpad;
      const int B = st.B;
      float* eag = st.e + (size_t)agent * a.estride;
      float* cX = st.X;
      float* cw = st.w;
      float* cth2 = st.th2;
      double* cpart = st.part;
      const size_t img = (size_t)agent * a.n;
      BandEnt cb[SL];

      // ---- 1. commit the staged task to LDS ----
#pragma unroll
      for (int sl = 0; sl < SL; ++sl) {
        cb[sl] = st.be[sl];
        const int wdt = (int)cb[sl].width;
        float ev[WM];
#pragma unroll
        for (int c = 0; c < WM; ++c) ev[c] = st.ev[sl][c];
        if (MODE == kSweep && strict) {
#pragma unroll
          for (int c = 0; c < WM; ++c)
            if (c < wdt) ev[c] = eag[cb[sl].gstart + c];
        }
#pragma unroll
        for (int c = 0; c < WM; ++c)
          if (c < wdt) {
            band[cb[sl].lds_row + c] = make_float2(ev[c], st.lv[sl][c]);
            if (MODE == kSweep) e0[cb[sl].lds_row + c] = ev[c];
          }
      }
      if (lr < 2) band[B + lr] = make_float2(0.0f, 0.0f);
      if (MODE != kTheta2) {
#pragma unroll
        for (int u = 0; u < St::HC; ++u) {
          const int c = u * kRowLanes + lr;
          if (c < HS * HS) {
            const int hi = c / HS, hj = c - (c / HS) * HS;
            const int iy = y0 - 1 + hi, ix = x0 - 1 + hj;
            const bool in = iy >= 0 && iy < a.ny && ix >= 0 && ix < a.nx;
            halo[c] = make_float2(st.hv[u], in ? 1.0f : 0.0f);
          }
        }
      }
      float cwo[St::PPL], cwb[St::PPL];
      if (MODE == kSweep) {
#pragma unroll
        for (int u = 0; u < St::PPL; ++u) {
          const int p = u * kRowLanes + lr;
          cwo[u] = st.wo[u];
          cwb[u] = st.wb[u];
          if (p < npix) {
            vv[p] = 2.0f * cwb[u] - cwo[u];
            t2[p] = st.t2[u];
          }
        }
      }
      const int pix0 = st.pix0;
      __builtin_amdgcn_wave_barrier();

      // ---- 2. pixel loop: records prefetched kPrefetch pixels ahead; the
      //         next task is staged right after the first pixel ----
      const size_t rec0 = (size_t)agent * a.n + pix0;
      auto update = [&](const Rec<SL>& cur, int j, int pi, int pj) {
        const int cidx = (pi + 1) * HS + pj + 1;
        if (MODE == kSweep) {
          // every LDS read of this pixel first, then the arithmetic
          float2 p0[SL], p1[SL];
#pragma unroll
          for (int s2 = 0; s2 < SL; ++s2) {
            p0[s2] = band[cur.off[s2]];
            p1[s2] = band[cur.off[s2] + 1];
          }
          const float zs = halo[cidx].x;
          const float2 nb = halo[cidx + noff];
          const float vj = vv[j], tj = t2[j];
          float part = 0.0f;
#pragma unroll
          for (int s2 = 0; s2 < SL; ++s2)
            part += cur.val[s2].x * p0[s2].y * p0[s2].x + cur.val[s2].y * p1[s2].y * p1[s2].x;
          const float d = zs - nb.x;
          const float wgt = nbw * nb.y * prior_curv(a, d);
          const float gl = wgt * d + proxw * (zs - vj) - part;
          const float G = row_sum16(gl);
          const float H = row_sum16(wgt);
          const float alpha = -a.relax * G * __builtin_amdgcn_rcpf(tj + H + a.is2);
#pragma unroll
          for (int s2 = 0; s2 < SL; ++s2) {
            band[cur.off[s2]].x = p0[s2].x - cur.val[s2].x * alpha;
            band[cur.off[s2] + 1].x = p1[s2].x - cur.val[s2].y * alpha;
          }
          if (lr == 0) halo[cidx].x = zs + alpha;
        } else if (MODE == kTheta2) {
          float part = 0.0f;
#pragma unroll
          for (int s2 = 0; s2 < SL; ++s2) {
            const float l0 = band[cur.off[s2]].y, l1 = band[cur.off[s2] + 1].y;
            part += cur.val[s2].x * cur.val[s2].x * l0 + cur.val[s2].y * cur.val[s2].y * l1;
          }
          const float th = row_sum16(part);
          if (lr == 0) {
            const size_t pix = (size_t)(y0 + pi) * a.nx + x0 + pj;
            cth2[img + pix] = th;
          }
        } else {  // kRefresh: accumulate -A x into the band
          const float xs = halo[cidx].x;
#pragma unroll
          for (int s2 = 0; s2 < SL; ++s2) {
            band[cur.off[s2]].x -= cur.val[s2].x * xs;
            band[cur.off[s2] + 1].x -= cur.val[s2].y * xs;
          }
        }
        __builtin_amdgcn_wave_barrier();
      };
      if (npix == S * S) {
        // full super-voxel: straight-line code, every record in its own
        // registers, so each wait covers exactly the record it needs
        constexpr int KP = SL * kRowLanes;
        const size_t rb = rec0 * KP + lr;
        const float2* vb = F16 ? nullptr : a.aval + rb;
        const __half2* hb = F16 ? a.hval + rb : nullptr;
        const float* sb = F16 ? a.hscale + rec0 : nullptr;
        const uint16_t* ob = a.aoff + rb;
        Rec<SL> buf[S * S];
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q) load_rec_at<SL, F16>(vb, hb, sb, ob, q, buf[q]);
#pragma unroll
        for (int j = 0; j < S * S; ++j) {
          if (j + kPrefetch < S * S)
            load_rec_at<SL, F16>(vb, hb, sb, ob, j + kPrefetch, buf[j + kPrefetch]);
          if (j == 0) stage_load(t + 1, st);
          update(buf[j], j, j / S, j % S);
        }
      } else {
        // ragged super-voxel at the image border
        for (int j = 0; j < npix; ++j) {
          Rec<SL> cur;
          load_rec<SL, F16>(a, rec0 + j, lr, cur);
          if (j == 0) stage_load(t + 1, st);
          update(cur, j, j / sw, j - (j / sw) * sw);
        }
      }

      // ---- 3. write back: the band's change goes to the agent's error
      //         sinogram with atomics, one view per instruction, the 16 lanes
      //         on consecutive channels (one or two cache lines each) ----
      if (MODE != kTheta2) {
#pragma unroll
        for (int sl = 0; sl < SL; ++sl) bents[sl * kRowLanes + lr] = cb[sl];
        __builtin_amdgcn_wave_barrier();
        for (int kl = 0; kl < a.kpad; ++kl) {
          const BandEnt b = bents[kl];
          for (int c = lr; c < (int)b.width; c += kRowLanes) {
            float d = band[b.lds_row + c].x;
            if (MODE == kSweep) d -= e0[b.lds_row + c];
            atomicAdd(eag + b.gstart + c, d);
          }
        }
      }
      if (MODE == kSweep) {
        double pn = 0.0, pd = 0.0, px = 0.0;
#pragma unroll
        for (int u = 0; u < St::PPL; ++u) {
          const int p = u * kRowLanes + lr;
          if (p < npix) {
            const int pi = p / sw, pj = p - (p / sw) * sw;
            const size_t pix = (size_t)(y0 + pi) * a.nx + x0 + pj;
            const float xn = halo[(pi + 1) * HS + pj + 1].x;
            cX[img + pix] = xn;
            if (a.mann) {
              const float wo = cwo[u], wb = cwb[u];
              const float v = 2.0f * wb - wo;
              cw[img + pix] = a.rho * (2.0f * xn - v) + (1.0f - a.rho) * wo;
              const double d = (double)xn - (double)wb;
              pn += d * d;
              pd += (double)wo * (double)wo;
              px += (double)xn * (double)xn;
            }
          }
        }
        if (a.mann) {
          // the task's FP64 partials, summed over the row in a fixed order
          // through LDS (the band is free after the flush)
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
      // in strict mode this row's atomics complete before it stages its
      // next band
      if (strict) __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    } else {
      stage_load(t + 1, st);
    }
  }

}

template <int MODE, int SV, bool F16V>
inline hipError_t launch_mode(const SvArgs& a, int slots, int grid, size_t lds, hipStream_t st) {
  switch (slots) {
#define MACE_CASE(SLV)                                                                   \
  case SLV: {                                                                            \
    static std::atomic<bool> attr_set{false};                                            \
    if (!attr_set.load(std::memory_order_acquire)) {                                     \
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sv_kernel<SLV, MODE, SV, F16V>), \
                                         hipFuncAttributeMaxDynamicSharedMemorySize,     \
                                         160 * 1024);                                    \
      if (e != hipSuccess) return e;                                                     \
      attr_set.store(true, std::memory_order_release);                                   \
    }                                                                                    \
    hipLaunchKernelGGL((sv_kernel<SLV, MODE, SV, F16V>), dim3(grid), dim3(kBlockThreads), lds, st, a); \
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
  if (mode == kSweep) return launch_mode<kSweep, SV, F16V>(a, slots, grid, lds, st);
  if (mode == kTheta2) return launch_mode<kTheta2, SV, F16V>(a, slots, grid, lds, st);
  return launch_mode<kRefresh, SV, F16V>(a, slots, grid, lds, st);
}

}  // namespace mace
