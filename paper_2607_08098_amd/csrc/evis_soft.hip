// Smooth event-count surrogate and its hand-written backward (gfx950): the
// same splat, gather and blend as the fused tile kernel, scored per
// substep by a logistic of the distance to the crossing threshold.
#include "evis_internal.h"
#include "evis_warp.h"

namespace evis {

// ---------------------------------------------------------------------------
// smooth event-count surrogate and its backward
// ---------------------------------------------------------------------------

// One workgroup per target tile.  For j = 1..K the sub-frame L_j is built as
// in the fused kernel (splat, gather, blend), then
//   S += sigma((|L_j - R| - C) / tau)
// with R the hard reference level of Eq. 4 (threshold C both ways), which is
// then moved by p n C with an integer count n.  The backward pass rebuilds
// the same sub-frames and sends dLoss/dL_j = gS sigma' sign(L_j - R) / tau
// through the blend: to the winner's L_A (atomically: the winner may belong
// to another tile), to the four B taps (atomically) and to m_B(q) through
// the gather position (d s / d m_B = -(1 - f)); the splat value does not
// depend on m_A, so its gradient is zero.  R does not move with L where the
// counts stay put, but it does move with C: dR/dC accumulates p n per
// substep, and dS/dC = -sigma' (1 + sign(L_j - R) dR/dC) / tau (or only
// -sigma' / tau with hold_ref, R a constant).
template <int TW, int TH, bool BWD>
__global__ __launch_bounds__(kBlock) void k_soft(const SoftArgs a) {
  constexpr int NPX = TW * TH;
  constexpr int PPT = NPX / kBlock;
  constexpr int ZN = zcells<TW, TH>();
  __shared__ unsigned long long zbuf[ZN];
  __shared__ uint32_t list[kListCapMax];
  __shared__ uint32_t s_wl[kWavesPerBlock][kWave];
  __shared__ int s_lcnt;
  __shared__ float s_red[kWavesPerBlock];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  for (int i = tid; i < ZN; i += kBlock) zbuf[i] = kEmptyKey;
  if (tid == 0) s_lcnt = 0;
  const int item = (int)blockIdx.x;
  int lo = 0, hi = a.n_envs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.item_prefix[mid] <= item) lo = mid; else hi = mid - 1;
  }
  const int env = __builtin_amdgcn_readfirstlane(lo);
  const EnvDesc d = a.envs[env];
  const EnvDyn dy = a.dyn[env];
  const SoftPtrs P = a.ptrs[env];
  const float C = a.C[env];
  const int K = a.K;
  const int H = d.H, W = d.W;
  const int ntx = (W + TW - 1) / TW;
  const int tile = item - a.item_prefix[env];
  const int Tx0 = (tile % ntx) * TW, Ty0 = (tile / ntx) * TH;
  const int Tx1 = min(Tx0 + TW, W) - 1, Ty1 = min(Ty0 + TH, H) - 1;
  __syncthreads();

  float LAq[PPT], LBq[PPT], R[PPT], acc[PPT], gSq[PPT], regA[PPT], regB[PPT], dRdC[PPT];
  float2 mBq[PPT], regm[PPT];
  uint32_t okbits = 0;
  auto pix_x = [&](int k) { return Tx0 + (tid + k * kBlock) % TW; };
  auto pix_y = [&](int k) { return Ty0 + (tid + k * kBlock) / TW; };
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int x = pix_x(k), y = pix_y(k);
    const bool ok = (x <= Tx1) && (y <= Ty1);
    const int q = ok ? (y * W + x) : 0;
    okbits |= (ok ? 1u : 0u) << k;
    LAq[k] = ok ? ldg(d.LA, q) : 0.0f;
    LBq[k] = ok ? ldg(d.LB, q) : 0.0f;
    mBq[k] = ok ? ldg(d.mB, q) : make_float2(0.0f, 0.0f);
    R[k] = ok ? ldg(P.Lref, q) : 0.0f;
    gSq[k] = (BWD && ok) ? ldg(P.gS, q) : 0.0f;
    acc[k] = 0.0f;
    regA[k] = regB[k] = dRdC[k] = 0.0f;
    regm[k] = make_float2(0.0f, 0.0f);
  }
  Window win{};
  int nlist = 0;
  bool overflow = false;
  if (K > 1) {
    nlist = build_candidates(d, dy, K, Tx0, Tx1, Ty0, Ty1, list, &s_lcnt, a.list_cap, win);
    overflow = nlist > a.list_cap;
  }
  float gCacc = 0.0f;
  for (int j = 1; j <= K; ++j) {
    const float f = (float)j / (float)K;
    const float g = 1.0f - f;
    const float alpha = (d.blend == EVIS_BLEND_TIME) ? f : 1.0f;
    if (j < K) {
      const float fs[1] = {f};
      unsigned long long* const zs[1] = {zbuf};
      splat_candidates<TW, 1>(d, list, nlist, overflow, win, K, j, 1, fs, Tx0, Tx1, Ty0, Ty1,
                              s_wl[wave], zs);
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (!((okbits >> k) & 1u)) continue;
      const int x = pix_x(k), y = pix_y(k);
      float L;
      bool vA = false, vB = false;
      int widx = 0;
      float Ah = 0.0f;
      BTaps bt;
      if (j < K) {
        const int i = tid + k * kBlock;
        const int zi = zcell<TW>(i % TW, i / TW);
        const unsigned long long key = zbuf[zi];
        zbuf[zi] = kEmptyKey;
        vA = key != kEmptyKey;
        widx = (int)(key & 0xFFFFFFFFull);
        if (vA) Ah = ldg(d.LA, widx);
        bt = b_taps(d, x, y, mBq[k], g, true);
        vB = bt.v;
        const float Bh = vB ? b_value(bt) : 0.0f;
        if (vA && vB) L = lerp32(Ah, Bh, alpha);
        else if (vA) L = Ah;
        else if (vB) L = Bh;
        else L = lerp32(LAq[k], LBq[k], alpha);
      } else {
        L = LBq[k];
      }
      const float dl = L - R[k];
      const float u = (fabsf(dl) - C) * a.inv_tau;
      // sigma(u) and sigma(u) (1 - sigma(u)) from e = exp(-|u|) <= 1, so
      // that neither loses digits to 1 - sigma when sigma is close to 1:
      // sigma = 1 / (1 + e) for u >= 0, e / (1 + e) below, and
      // sigma (1 - sigma) = e / (1 + e)^2 either way
      const float e = expf(-fabsf(u));
      const float inv = 1.0f / (1.0f + e);
      const float sg = (u >= 0.0f) ? inv : e * inv;
      if (!BWD) {
        acc[k] += sg;
      } else {
        const float dS = e * inv * inv * a.inv_tau;
        const float sgn = (dl > 0.0f) ? 1.0f : ((dl < 0.0f) ? -1.0f : 0.0f);
        const float gL = gSq[k] * dS * sgn;
        gCacc -= gSq[k] * dS * (a.hold_ref ? 1.0f : (1.0f + sgn * dRdC[k]));
        if (j == K) {
          regB[k] += gL;
        } else if (vA || vB) {
          const float gAh = vA ? (vB ? (1.0f - alpha) * gL : gL) : 0.0f;
          const float gBh = vB ? (vA ? alpha * gL : gL) : 0.0f;
          if (vA && gAh != 0.0f) unsafeAtomicAdd(&P.gLA[widx], gAh);
          if (vB && gBh != 0.0f) {
            const float fx0 = floorf((float)x - g * mBq[k].x), fy0 = floorf((float)y - g * mBq[k].y);
            const int x0 = (int)fx0, y0 = (int)fy0;
            const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
            const float wx = bt.wx, wy = bt.wy;
            unsafeAtomicAdd(&P.gLB[y0 * W + x0], gBh * ((1.0f - wx) * (1.0f - wy)));
            unsafeAtomicAdd(&P.gLB[y0 * W + x1], gBh * (wx * (1.0f - wy)));
            unsafeAtomicAdd(&P.gLB[y1 * W + x0], gBh * ((1.0f - wx) * wy));
            unsafeAtomicAdd(&P.gLB[y1 * W + x1], gBh * (wx * wy));
            const float top = lerp32(bt.a, bt.b, wx), bot = lerp32(bt.c, bt.d, wx);
            const float dBdwx = (1.0f - wy) * (bt.b - bt.a) + wy * (bt.d - bt.c);
            const float dBdwy = bot - top;
            regm[k].x -= gBh * dBdwx * g;
            regm[k].y -= gBh * dBdwy * g;
          }
        } else {
          regA[k] += (1.0f - alpha) * gL;
          regB[k] += alpha * gL;
        }
      }
      // hard reference update (Eq. 4, threshold C both ways)
      const float aa = fabsf(dl);
      if (aa >= C && C > 0.0f) {
        const float n = (float)crossing_count(aa, C);
        const float nc = n * C;
        R[k] = (dl > 0.0f) ? (R[k] + nc) : (R[k] - nc);
        if (BWD) dRdC[k] += (dl > 0.0f) ? n : -n;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    if (!((okbits >> k) & 1u)) continue;
    const int q = pix_y(k) * W + pix_x(k);
    if (!BWD) {
      stg(P.S, q, acc[k]);
    } else {
      if (regA[k] != 0.0f) unsafeAtomicAdd(&P.gLA[q], regA[k]);
      if (regB[k] != 0.0f) unsafeAtomicAdd(&P.gLB[q], regB[k]);
      stg(P.gmB, q, regm[k]);
      stg(P.gmA, q, make_float2(0.0f, 0.0f));
    }
  }
  if (BWD) {
    const float w = wave_sum(gCacc);
    if (lane == 0) s_red[wave] = w;
    __syncthreads();
    if (tid == 0) {
      float t = 0.0f;
      for (int i = 0; i < kWavesPerBlock; ++i) t += s_red[i];
      unsafeAtomicAdd(&a.gC[env], t);
    }
  }
}

// Zero the accumulated outputs of the backward pass (one workgroup per env).
__global__ __launch_bounds__(kBlock) void k_soft_zero(const SoftPtrs* ptrs, const EnvDesc* envs,
                                                      float* gC) {
  const int e = blockIdx.x;
  const SoftPtrs P = ptrs[e];
  const int n = envs[e].H * envs[e].W;
  for (int i = threadIdx.x; i < n; i += kBlock) {
    stg(P.gLA, i, 0.0f);
    stg(P.gLB, i, 0.0f);
  }
  if (threadIdx.x == 0) gC[e] = 0.0f;
}

hipError_t launch_soft(bool backward, const SoftArgs& a, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (backward)
    hipLaunchKernelGGL((k_soft<kSoftTW, kSoftTH, true>), dim3(n_items), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_soft<kSoftTW, kSoftTH, false>), dim3(n_items), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_soft_zero(const SoftPtrs* ptrs, const EnvDesc* envs, int n_envs, float* gC,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_soft_zero, dim3(n_envs), dim3(kBlock), 0, s, ptrs, envs, gC);
  return hipGetLastError();
}

}  // namespace evis
