// Fused warp + emit path: per-pair preparation, the per-step work queue and
// the persistent tile kernel (gfx950).
//
// One work item = one target tile (TW x TH pixels) of one environment.  A
// workgroup holds the tile's per-pixel state (reference level, last event
// time, thresholds, the previous sample, its own L_A, L_B and m_B) in
// registers for the whole keyframe gap and loops over the K substeps:
//   splat   every source that can land in the tile at fraction f = j/K is
//           splatted into an LDS z-buffer of 64-bit (depth bits << 32 |
//           source index) keys with ds_min_u64 (Eq. 5 q_A, bilinear
//           footprint, Eq. 6, Eq. 7);
//   resolve the winner's L_A, the bilinear L_B at s = q - (1-f) m_B(q) and
//           the hole-aware blend give the sub-frame in registers;
//   emit    Eq. 4 crossings with exact counts, interpolated timestamps,
//           Eq. 8 thresholds and the refractory period; events are
//           compacted by wave prefix sums into an LDS buffer that is
//           appended to the global stream with one atomic per flush.
// The sources that can reach a tile are found once per pair: the env's
// 8x8 source tiles carry motion bounds (from the prep kernel), and each
// candidate's interval of substeps [j_lo, j_hi] during which its footprint
// can touch the tile is kept in an LDS list.
#include "evis_internal.h"
#include "evis_sink.h"

namespace evis {

// ---------------------------------------------------------------------------
// per-step reset and per-pair preparation
// ---------------------------------------------------------------------------

__global__ void k_reset(EnvDyn* dyn, int n_envs, unsigned int* queue,
                        unsigned long long* cursor) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_envs) dyn[i].msq_bits = 0ull;
  if (i == 0) {
    queue[0] = 0u;
    if (cursor) *cursor = 0ull;
  }
}

// One wave per 8x8 source tile: endpoint depth (Eq. 7, p_B = p - m_A(p),
// Z_B edge-clamped) stored as Zend - Z_A, the tile's bounds of m_A over
// sources with a finite motion vector, and the env's largest finite |m|^2.
__global__ __launch_bounds__(kBlock) void k_prep(const EnvDesc* __restrict__ envs, EnvDyn* dyn,
                                                 const int32_t* __restrict__ src_prefix,
                                                 int n_envs, int total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int gt = blockIdx.x * kWavesPerBlock + (threadIdx.x / kWave);
  if (gt >= total) return;   // wave-uniform
  int lo = 0, hi = n_envs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (src_prefix[mid] <= gt) lo = mid; else hi = mid - 1;
  }
  const int e = lo;
  const EnvDesc& d = envs[e];
  const int t = gt - src_prefix[e];
  const int tx = t % d.ntx_src, ty = t / d.ntx_src;
  const int x = tx * kSrcTile + (lane & 7), y = ty * kSrcTile + (lane >> 3);
  const float inf = __int_as_float(0x7f800000);
  float mnx = inf, mxx = -inf, mny = inf, mxy = -inf;
  double msq = 0.0;
  if (x < d.W && y < d.H) {
    const int p = y * d.W + x;
    const float2 a = d.mA[p];
    const float2 b = d.mB[p];
    const float sx = clamp_into((float)x - a.x, (float)(d.W - 1));
    const float sy = clamp_into((float)y - a.y, (float)(d.H - 1));
    const float zend = bilinear(d.ZB, d.H, d.W, sx, sy);
    d.dZ[p] = zend - d.ZA[p];
    if (finite32(a.x) && finite32(a.y)) {
      mnx = mxx = a.x;
      mny = mxy = a.y;
    }
    const double ma = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
    const double mb = (double)b.x * (double)b.x + (double)b.y * (double)b.y;
    if (ma <= 1.7976931348623157e308) msq = ma;
    if (mb <= 1.7976931348623157e308 && mb > msq) msq = mb;
  }
  mnx = wave_min(mnx);
  mxx = wave_max(mxx);
  mny = wave_min(mny);
  mxy = wave_max(mxy);
  msq = wave_max_d(msq);
  if (lane == 0) {
    d.tb[t] = make_float4(mnx, mxx, mny, mxy);
    if (msq > 0.0) {
      unsigned long long* slot = &dyn[e].msq_bits;
      const unsigned long long bits = (unsigned long long)__double_as_longlong(msq);
      if (bits > __atomic_load_n(slot, __ATOMIC_RELAXED)) atomicMax(slot, bits);
    }
  }
}

// Single workgroup: each env's K (fixed or the exact adaptive count), its
// substep length Dt = fl(fl(t1 - t0) / K), its tile grid, and the work
// queue order: envs by descending K (longest items first), items numbered
// consecutively in that order.
__global__ __launch_bounds__(EVIS_MAX_ENVS) void k_queue(const EnvDesc* __restrict__ envs,
                                                          EnvDyn* dyn, int n_envs, int TW, int TH,
                                                          int32_t* rank_begin, int32_t* env_order,
                                                          int32_t* n_items, int32_t* K_used) {
  __shared__ int sK[EVIS_MAX_ENVS];
  __shared__ int sN[EVIS_MAX_ENVS];
  __shared__ int sOrder[EVIS_MAX_ENVS];
  __shared__ int sScan[EVIS_MAX_ENVS];
  const int e = threadIdx.x;
  int K = 0;
  if (e < n_envs) {
    const EnvDesc& d = envs[e];
    const double M = __longlong_as_double((long long)dyn[e].msq_bits);
    K = (d.K_fixed > 0) ? d.K_fixed : exact_k(M, d.K_max);
    const float Dt = (float)d.span / (float)K;
    const int ntx = (d.W + TW - 1) / TW, nty = (d.H + TH - 1) / TH;
    dyn[e].K = K;
    dyn[e].Dt = Dt;
    dyn[e].ntx = ntx;
    dyn[e].nty = nty;
    if (K_used) K_used[e] = K;
    sK[e] = K;
    sN[e] = ntx * nty;
  }
  __syncthreads();
  if (e < n_envs) {
    int r = 0;
    for (int o = 0; o < n_envs; ++o) {
      const int Ko = sK[o];
      r += (Ko > K) || (Ko == K && o < e);
    }
    sOrder[r] = e;
  }
  __syncthreads();
  const int v = (e < n_envs) ? sN[sOrder[e]] : 0;
  sScan[e] = v;
  __syncthreads();
  for (int dd = 1; dd < EVIS_MAX_ENVS; dd <<= 1) {
    const int t = (e >= dd) ? sScan[e - dd] : 0;
    __syncthreads();
    sScan[e] += t;
    __syncthreads();
  }
  if (e < n_envs) {
    const int env = sOrder[e];
    rank_begin[e] = sScan[e] - v;
    env_order[e] = env;
    dyn[env].item_begin = sScan[e] - v;
  }
  if (e == n_envs - 1) {
    rank_begin[n_envs] = sScan[e];
    *n_items = sScan[e];
  }
}

// ---------------------------------------------------------------------------
// candidate source tiles
// ---------------------------------------------------------------------------

// Conservative interval of substeps during which some source of the 8x8
// tile [Sx0,Sx1]x[Sy0,Sy1] with motion bounds b can put a footprint corner
// into the target tile [Tx0,Tx1]x[Ty0,Ty1].  A corner lies in [Tx0,Tx1]
// only if q_x = p_x - f m_x is in [Tx0 - 1, Tx1 + 1); over the tile q_x lies
// in [Sx0 - f max m_x, Sx1 - f min m_x].  One pixel of slack covers
// rounding; the substep range is widened by one on each side.
__device__ __forceinline__ void lin_le(double a, double bnd, double& flo, double& fhi) {
  if (a > 0.0) fhi = fmin(fhi, bnd / a);        // a f <= bnd
  else if (a < 0.0) flo = fmax(flo, bnd / a);
  else if (bnd < 0.0) flo = 2.0;
}
__device__ __forceinline__ void lin_ge(double a, double bnd, double& flo, double& fhi) {
  if (a > 0.0) flo = fmax(flo, bnd / a);        // a f >= bnd
  else if (a < 0.0) fhi = fmin(fhi, bnd / a);
  else if (bnd > 0.0) flo = 2.0;
}

__device__ __forceinline__ bool substep_range(float4 b, int Sx0, int Sx1, int Sy0, int Sy1,
                                              int Tx0, int Tx1, int Ty0, int Ty1, int K,
                                              int& jlo, int& jhi) {
  if (!(b.x <= b.y) || !(b.z <= b.w)) return false;   // no finite source
  double flo = 0.0, fhi = 1.0;
  const double slack = 1.0;
  lin_le((double)b.x, (double)(Sx1 - Tx0 + 1) + slack, flo, fhi);
  lin_ge((double)b.y, (double)(Sx0 - Tx1 - 1) - slack, flo, fhi);
  lin_le((double)b.z, (double)(Sy1 - Ty0 + 1) + slack, flo, fhi);
  lin_ge((double)b.w, (double)(Sy0 - Ty1 - 1) - slack, flo, fhi);
  if (!(flo <= fhi)) return false;
  const int lo = max(1, (int)floor(flo * (double)K));
  const int hi = min(K - 1, (int)ceil(fhi * (double)K));
  if (lo > hi) return false;
  jlo = lo;
  jhi = hi;
  return true;
}

// Splat the 64 sources of source tile st (one per lane) at fraction f into
// the LDS z-buffer of target tile [Tx0,Tx1]x[Ty0,Ty1].
template <int TW>
__device__ __forceinline__ void splat_src_tile(const EnvDesc& d, int st, float f, int Tx0, int Tx1,
                                               int Ty0, int Ty1, unsigned long long* zbuf) {
  const int lane = threadIdx.x & (kWave - 1);
  const int sxt = st % d.ntx_src, syt = st / d.ntx_src;
  const int sx = sxt * kSrcTile + (lane & 7), sy = syt * kSrcTile + (lane >> 3);
  if (sx >= d.W || sy >= d.H) return;
  const int p = sy * d.W + sx;
  const float2 m = d.mA[p];
  const float za = d.ZA[p];
  const float dz = d.dZ[p];
  const float qx = (float)sx - f * m.x;
  const float qy = (float)sy - f * m.y;
  const float zt = za + f * dz;
  if (!(zt > 0.0f)) return;
  if (!(qx >= (float)(Tx0 - 1) && qx < (float)(Tx1 + 1) && qy >= (float)(Ty0 - 1) &&
        qy < (float)(Ty1 + 1)))
    return;
  const float fx0 = floorf(qx), fy0 = floorf(qy);
  const int x0 = (int)fx0, y0 = (int)fy0;
  const bool bx = (qx - fx0) > 0.0f, by = (qy - fy0) > 0.0f;
  const unsigned long long key = ((unsigned long long)__float_as_uint(zt) << 32) | (unsigned)p;
  const int lx = x0 - Tx0, ly = y0 - Ty0;
  const bool in_x0 = x0 >= Tx0, in_x1 = bx && (x0 + 1 <= Tx1);
  const bool in_y0 = y0 >= Ty0, in_y1 = by && (y0 + 1 <= Ty1);
  if (in_x0 && in_y0) atomicMin(&zbuf[ly * TW + lx], key);
  if (in_x1 && in_y0) atomicMin(&zbuf[ly * TW + lx + 1], key);
  if (in_x0 && in_y1) atomicMin(&zbuf[(ly + 1) * TW + lx], key);
  if (in_x1 && in_y1) atomicMin(&zbuf[(ly + 1) * TW + lx + 1], key);
}

// ---------------------------------------------------------------------------
// the persistent tile kernel
// ---------------------------------------------------------------------------

template <int TW, int TH, int MODE>
__global__ __launch_bounds__(kBlock) void k_tile(const TileArgs a) {
  constexpr int NPX = TW * TH;
  constexpr int PPT = NPX / kBlock;
  static_assert(PPT * kBlock == NPX, "tile must be a multiple of the workgroup");
  constexpr int EVB = (MODE == MODE_STEP) ? kEventBuf : 1;
  __shared__ unsigned long long zbuf[NPX];
  __shared__ uint32_t list[kListCapMax];
  __shared__ uint2 evbuf[EVB];
  __shared__ int s_wtot[2][kWavesPerBlock];
  __shared__ unsigned long long s_gbase;
  __shared__ int s_item, s_rank, s_lcnt;

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
#pragma unroll
  for (int k = 0; k < PPT; ++k) zbuf[tid + k * kBlock] = kEmptyKey;
  const SinkShared sh{evbuf, s_wtot, &s_gbase, EVB};
  const SinkOut so{a.out, a.capacity, a.cursor};
  int ev_count = 0, round = 0;
  const int n_items = *a.n_items;

  for (;;) {
    __syncthreads();
    if (tid == 0) {
      const int item = (int)atomicAdd(a.queue, 1u);
      int r = 0;
      if (item < n_items) {
        int lo = 0, hi = a.n_envs - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (a.rank_begin[mid] <= item) lo = mid; else hi = mid - 1;
        }
        r = lo;
      }
      s_item = item;
      s_rank = r;
      s_lcnt = 0;
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= n_items) break;
    const int rank = __builtin_amdgcn_readfirstlane(s_rank);
    const int env = __builtin_amdgcn_readfirstlane(a.env_order[rank]);
    const EnvDesc d = a.envs[env];
    const EnvDyn dy = a.dyn[env];
    const int tile = item - a.rank_begin[rank];
    const int H = d.H, W = d.W, K = dy.K;
    const int tx = tile % dy.ntx, ty = tile / dy.ntx;
    const int Tx0 = tx * TW, Ty0 = ty * TH;
    const int Tx1 = min(Tx0 + TW, W) - 1, Ty1 = min(Ty0 + TH, H) - 1;

    // per-pixel registers
    float LAq[PPT], LBq[PPT], Lp[PPT], R[PPT], con[PPT], coff[PPT];
    float2 mBq[PPT];
    int tl[PPT];
    uint32_t xy[PPT];
    int qi[PPT];
    uint32_t okbits = 0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int i = tid + k * kBlock;
      const int x = Tx0 + i % TW, y = Ty0 + i / TW;
      const bool ok = (x <= Tx1) && (y <= Ty1);
      const int q = ok ? (y * W + x) : 0;
      okbits |= (ok ? 1u : 0u) << k;
      qi[k] = q;
      xy[k] = (uint32_t)x | ((uint32_t)y << 11);
      LAq[k] = ok ? d.LA[q] : 0.0f;
      LBq[k] = ok ? d.LB[q] : 0.0f;
      mBq[k] = ok ? d.mB[q] : make_float2(0.0f, 0.0f);
      Lp[k] = LAq[k];
      R[k] = 0.0f;
      tl[k] = EVIS_T_LAST_INIT;
      con[k] = d.C_on;
      coff[k] = d.C_off;
      if (MODE == MODE_STEP) {
        R[k] = ok ? d.Lref[q] : 0.0f;
        if (ok && d.tlast) tl[k] = d.tlast[q];
        if (ok && d.th_on) con[k] = d.th_on[q];
        if (ok && d.th_off) coff[k] = d.th_off[q];
      }
    }

    // Candidate source tiles and their substep intervals.
    int nlist = 0, wx0 = 0, wy0 = 0, nwx = 0, nwin = 0;
    bool overflow = false;
    if (K > 1) {
      const double M = __longlong_as_double((long long)dy.msq_bits);
      const int Rw = (M > 1.0e12) ? (1 << 20) : ((int)ceil(sqrt(M)) + 3);
      wx0 = max(0, Tx0 - Rw) / kSrcTile;
      wy0 = max(0, Ty0 - Rw) / kSrcTile;
      const int wx1 = min(d.ntx_src - 1, min(Tx1 + Rw, W - 1) / kSrcTile);
      const int wy1 = min(d.nty_src - 1, min(Ty1 + Rw, H - 1) / kSrcTile);
      nwx = wx1 - wx0 + 1;
      nwin = nwx * (wy1 - wy0 + 1);
      for (int w = tid; w < nwin; w += kBlock) {
        const int sxt = wx0 + w % nwx, syt = wy0 + w / nwx;
        const int st = syt * d.ntx_src + sxt;
        int jlo, jhi;
        if (substep_range(d.tb[st], sxt * kSrcTile, min(sxt * kSrcTile + 7, W - 1),
                          syt * kSrcTile, min(syt * kSrcTile + 7, H - 1), Tx0, Tx1, Ty0, Ty1,
                          K, jlo, jhi)) {
          const int slot = atomicAdd(&s_lcnt, 1);
          if (slot < a.list_cap) list[slot] = ((uint32_t)st << 16) | ((uint32_t)jlo << 8) | (uint32_t)jhi;
        }
      }
      __syncthreads();
      nlist = __builtin_amdgcn_readfirstlane(s_lcnt);
      overflow = nlist > a.list_cap;
    }

    // Static tile: every source that can reach it does not move, it does not
    // move in B and L_A == L_B on it, so every sub-frame equals L_A.
    bool is_static = false;
    if (MODE == MODE_STEP && a.static_tiles && K > 1 && !overflow) {
      bool okst = true;
      for (int e2 = tid; e2 < nlist; e2 += kBlock) {
        const float4 b = d.tb[list[e2] >> 16];
        okst = okst && b.x == 0.0f && b.y == 0.0f && b.z == 0.0f && b.w == 0.0f;
      }
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if ((okbits >> k) & 1u) {
          const int q = qi[k];
          const int x = q % W, y = q / W;
          const int x1 = min(x + 1, W - 1), y1 = min(y + 1, H - 1);
          const float t1 = d.LB[y * W + x1], t2 = d.LB[y1 * W + x], t3 = d.LB[y1 * W + x1];
          okst = okst && mBq[k].x == 0.0f && mBq[k].y == 0.0f && LAq[k] == LBq[k] &&
                 fabsf(LBq[k]) < 1e30f && fabsf(t1) < 1e30f && fabsf(t2) < 1e30f &&
                 fabsf(t3) < 1e30f;
        }
      }
      is_static = __syncthreads_and(okst ? 1 : 0) != 0;
    }

    int j_first = 1, j_last = K;
    if (MODE == MODE_INTERP) {
      if (a.j_begin == 0) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          if ((okbits >> k) & 1u) {
            a.L_out[qi[k]] = LAq[k];
            if (a.hole) a.hole[qi[k]] = 0;
          }
        }
      }
      j_first = max(1, a.j_begin);
      j_last = min(K, a.j_end - 1);
    }

    for (int j = j_first; j <= j_last; ++j) {
      float Lj[PPT];
      uint32_t hb[PPT];
      if (j < K) {
        const float f = (float)j / (float)K;
        const float g = 1.0f - f;
        const float alpha = (d.blend == EVIS_BLEND_TIME) ? f : 1.0f;
        if (!is_static) {
          if (!overflow) {
            for (int base = 0; base < nlist; base += kBlock) {
              const int e2 = base + lane * kWavesPerBlock + wave;
              uint32_t ent = 0u;
              bool act = false;
              if (e2 < nlist) {
                ent = list[e2];
                const int jlo = (int)((ent >> 8) & 0xFFu), jhi = (int)(ent & 0xFFu);
                act = (j >= jlo) && (j <= jhi);
              }
              unsigned long long mask = __ballot(act);
              while (mask) {
                const int b = __ffsll((long long)mask) - 1;
                mask &= mask - 1ull;
                const int st = (int)((uint32_t)__builtin_amdgcn_readlane((int)ent, b) >> 16);
                splat_src_tile<TW>(d, st, f, Tx0, Tx1, Ty0, Ty1, zbuf);
              }
            }
          } else {
            // Window scan: the candidate list did not fit.
            for (int w = wave; w < nwin; w += kWavesPerBlock) {
              const int sxt = wx0 + w % nwx, syt = wy0 + w / nwx;
              const int st = syt * d.ntx_src + sxt;
              int jlo, jhi;
              if (substep_range(d.tb[st], sxt * kSrcTile, min(sxt * kSrcTile + 7, W - 1),
                                syt * kSrcTile, min(syt * kSrcTile + 7, H - 1), Tx0, Tx1, Ty0,
                                Ty1, K, jlo, jhi) &&
                  j >= jlo && j <= jhi)
                splat_src_tile<TW>(d, st, f, Tx0, Tx1, Ty0, Ty1, zbuf);
            }
          }
          __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          hb[k] = 0u;
          Lj[k] = LAq[k];
          if (((okbits >> k) & 1u) && !is_static) {
            const int i = tid + k * kBlock;
            const unsigned long long key = zbuf[i];
            zbuf[i] = kEmptyKey;
            const bool vA = key != kEmptyKey;
            const float Ah = vA ? d.LA[(int)(key & 0xFFFFFFFFull)] : 0.0f;
            const int q = qi[k];
            const float sx = (float)(q % W) - g * mBq[k].x;
            const float sy = (float)(q / W) - g * mBq[k].y;
            const bool vB = sx >= 0.0f && sx <= (float)(W - 1) && sy >= 0.0f && sy <= (float)(H - 1);
            const float Bh = vB ? bilinear(d.LB, H, W, sx, sy) : 0.0f;
            float v;
            if (vA && vB) v = lerp32(Ah, Bh, alpha);
            else if (vA) v = Ah;
            else if (vB) v = Bh;
            else v = lerp32(LAq[k], LBq[k], alpha);
            Lj[k] = v;
            hb[k] = (vA ? 0u : 1u) | (vB ? 0u : 2u);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          Lj[k] = LBq[k];
          hb[k] = 0u;
        }
      }

      if (MODE == MODE_STEP) {
        emit_substep<PPT>(j, Lj, Lp, R, tl, con, coff, xy, okbits, d.t0, d.span, dy.Dt, d.refr,
                          d.env_bits, sh, so, ev_count, round);
      } else if (MODE == MODE_INTERP) {
        const long long plane = (long long)H * W;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          if ((okbits >> k) & 1u) {
            const long long o = (long long)(j - a.j_begin) * plane + qi[k];
            a.L_out[o] = Lj[k];
            if (a.hole) a.hole[o] = (uint8_t)hb[k];
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int k = 0; k < PPT; ++k) Lp[k] = Lj[k];
    }

    if (MODE == MODE_STEP) {
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if ((okbits >> k) & 1u) {
          d.Lref[qi[k]] = R[k];
          if (d.tlast) d.tlast[qi[k]] = tl[k];
        }
      }
    }
  }
  if (MODE == MODE_STEP) sink_flush(sh, so, ev_count);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_reset(EnvDyn* dyn, int n_envs, unsigned int* queue, unsigned long long* cursor,
                        hipStream_t s) {
  const int n = max(n_envs, 1);
  hipLaunchKernelGGL(k_reset, dim3((n + 255) / 256), dim3(256), 0, s, dyn, n_envs, queue, cursor);
  return hipGetLastError();
}

hipError_t launch_prep(const EnvDesc* envs, EnvDyn* dyn, const int32_t* src_prefix, int n_envs,
                       int total_src_tiles, hipStream_t s) {
  if (total_src_tiles <= 0) return hipSuccess;
  const int blocks = (total_src_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(kBlock), 0, s, envs, dyn, src_prefix, n_envs,
                     total_src_tiles);
  return hipGetLastError();
}

hipError_t launch_queue(const EnvDesc* envs, EnvDyn* dyn, int n_envs, int tile_w, int tile_h,
                        int32_t* rank_begin, int32_t* env_order, int32_t* n_items,
                        int32_t* K_used, hipStream_t s) {
  hipLaunchKernelGGL(k_queue, dim3(1), dim3(EVIS_MAX_ENVS), 0, s, envs, dyn, n_envs, tile_w,
                     tile_h, rank_begin, env_order, n_items, K_used);
  return hipGetLastError();
}

template <int TW, int TH>
static hipError_t launch_tile_shape(int mode, const TileArgs& a, int grid, hipStream_t s) {
  switch (mode) {
    case MODE_STEP:
      hipLaunchKernelGGL((k_tile<TW, TH, MODE_STEP>), dim3(grid), dim3(kBlock), 0, s, a);
      break;
    case MODE_INTERP:
      hipLaunchKernelGGL((k_tile<TW, TH, MODE_INTERP>), dim3(grid), dim3(kBlock), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TW, int TH>
static int occupancy_shape(int mode) {
  int nb = 0;
  hipError_t err = hipErrorInvalidValue;
  if (mode == MODE_STEP)
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile<TW, TH, MODE_STEP>, kBlock, 0);
  else if (mode == MODE_INTERP)
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile<TW, TH, MODE_INTERP>, kBlock, 0);
  return (err == hipSuccess && nb > 0) ? nb : 1;
}

#define EVIS_TILE_SHAPES(X) X(16, 16) X(32, 16) X(32, 32) X(64, 16) X(64, 32)

bool tile_shape_supported(int tw, int th) {
#define X(W_, H_) if (tw == W_ && th == H_) return true;
  EVIS_TILE_SHAPES(X)
#undef X
  return false;
}

hipError_t launch_tile(int tw, int th, int mode, const TileArgs& a, int grid, hipStream_t s) {
#define X(W_, H_) if (tw == W_ && th == H_) return launch_tile_shape<W_, H_>(mode, a, grid, s);
  EVIS_TILE_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

int tile_occupancy(int tw, int th, int mode) {
  // Queried once per (shape, mode) and cached: no runtime query happens while
  // a launch sequence is being captured into a graph.
  static int cache[5][4] = {};
  int idx = 0;
#define X(W_, H_)                                                         \
  if (tw == W_ && th == H_) {                                             \
    if (mode >= 0 && mode < 4 && cache[idx][mode] == 0)                   \
      cache[idx][mode] = occupancy_shape<W_, H_>(mode);                   \
    return (mode >= 0 && mode < 4) ? cache[idx][mode] : 1;                \
  }                                                                       \
  ++idx;
  EVIS_TILE_SHAPES(X)
#undef X
  return 1;
}

}  // namespace evis
