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
  if (i < kXcd) queue[i] = 0u;
  if (i == 0 && cursor) *cursor = 0ull;
}

// One wave per 8x8 source tile: endpoint depth (Eq. 7, p_B = p - m_A(p),
// Z_B edge-clamped) stored as Zend - Z_A, the tile's bounds of m_A over
// sources with a finite motion vector, and the env's largest finite |m|^2.
__global__ __launch_bounds__(kBlock) void k_prep(const EnvDesc* __restrict__ envs, EnvDyn* dyn,
                                                 const int32_t* __restrict__ src_prefix,
                                                 int n_envs, int total) {
  __shared__ int s_prefix[EVIS_MAX_ENVS + 1];
  for (int i = threadIdx.x; i <= n_envs; i += kBlock) s_prefix[i] = src_prefix[i];
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int gt = blockIdx.x * kWavesPerBlock + (threadIdx.x / kWave);
  if (gt >= total) return;   // wave-uniform
  int lo = 0, hi = n_envs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_prefix[mid] <= gt) lo = mid; else hi = mid - 1;
  }
  const int e = lo;
  const EnvDesc& d = envs[e];
  const int t = gt - s_prefix[e];
  const int tx = t % d.ntx_src, ty = t / d.ntx_src;
  const int x = tx * kSrcTile + (lane & 7), y = ty * kSrcTile + (lane >> 3);
  const float inf = __int_as_float(0x7f800000);
  float mnx = inf, mxx = -inf, mny = inf, mxy = -inf;
  double msq = 0.0;
  if (x < d.W && y < d.H) {
    const int p = y * d.W + x;
    const float2 a = ldg(d.mA, p);
    const float2 b = ldg(d.mB, p);
    const float sx = clamp_into((float)x - a.x, (float)(d.W - 1));
    const float sy = clamp_into((float)y - a.y, (float)(d.H - 1));
    const float zend = bilinear(d.ZB, d.H, d.W, sx, sy);
    stg(d.dZ, p, zend - ldg(d.ZA, p));
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
    stg(d.tb, t, make_float4(mnx, mxx, mny, mxy));
    if (msq > 0.0) {
      unsigned long long* slot = &dyn[e].msq_bits;
      const unsigned long long bits = (unsigned long long)__double_as_longlong(msq);
      if (bits > __atomic_load_n(slot, __ATOMIC_RELAXED)) atomicMax(slot, bits);
    }
  }
}

// Single workgroup: each env's K (fixed or the exact adaptive count), its
// substep length Dt = fl(fl(t1 - t0) / K) and tile grid, and the work
// queues.  Envs are ranked by descending K (longest items first).  Queue x
// holds horizontal band x of every env (tile rows [x*nty/8, (x+1)*nty/8)),
// rank by rank, so that the workgroups of one XCD work on neighbouring
// tiles and share their sources in that XCD's L2.
__global__ __launch_bounds__(EVIS_MAX_ENVS) void k_queue(const EnvDesc* __restrict__ envs,
                                                          EnvDyn* dyn, int n_envs, int TW, int TH,
                                                          int32_t* xbegin, int32_t* env_order,
                                                          int32_t* n_items, int32_t* K_used) {
  __shared__ int sK[EVIS_MAX_ENVS];
  __shared__ int sOrder[EVIS_MAX_ENVS];
  __shared__ int sScan[EVIS_MAX_ENVS];
  const int e = threadIdx.x;
  int K = 0;
  if (e < n_envs) {
    const EnvDesc& d = envs[e];
    const double M = __longlong_as_double((long long)dyn[e].msq_bits);
    K = (d.K_fixed > 0) ? d.K_fixed : exact_k(M, d.K_max);
    const float Dt = (float)d.span / (float)K;
    dyn[e].K = K;
    dyn[e].Dt = Dt;
    dyn[e].ntx = (d.W + TW - 1) / TW;
    dyn[e].nty = (d.H + TH - 1) / TH;
    if (K_used) K_used[e] = K;
    sK[e] = K;
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
  if (e < n_envs) env_order[e] = sOrder[e];
  for (int x = 0; x < kXcd; ++x) {
    int v = 0;
    if (e < n_envs) {
      const int env = sOrder[e];
      const int nty = (envs[env].H + TH - 1) / TH, ntx = (envs[env].W + TW - 1) / TW;
      v = ntx * ((x + 1) * nty / kXcd - x * nty / kXcd);
    }
    sScan[e] = v;
    __syncthreads();
    for (int dd = 1; dd < EVIS_MAX_ENVS; dd <<= 1) {
      const int t = (e >= dd) ? sScan[e - dd] : 0;
      __syncthreads();
      sScan[e] += t;
      __syncthreads();
    }
    if (e < n_envs) xbegin[x * (n_envs + 1) + e] = sScan[e] - v;
    if (e == n_envs - 1) {
      xbegin[x * (n_envs + 1) + n_envs] = sScan[e];
      n_items[x] = sScan[e];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// candidate source tiles
// ---------------------------------------------------------------------------

// Conservative interval of substeps during which some source of the 8x8
// tile [Sx0,Sx1]x[Sy0,Sy1] with motion bounds b can put a footprint corner
// into the target tile [Tx0,Tx1]x[Ty0,Ty1].  A corner lies in [Tx0,Tx1]
// only if q_x = p_x - f m_x is in [Tx0 - 1, Tx1 + 1); over the tile q_x lies
// in [Sx0 - f max m_x, Sx1 - f min m_x].
__device__ __forceinline__ void lin_le(float a, float bnd, float& flo, float& fhi) {
  if (a > 0.0f) fhi = fminf(fhi, __fdividef(bnd, a));        // a f <= bnd
  else if (a < 0.0f) flo = fmaxf(flo, __fdividef(bnd, a));
  else if (bnd < 0.0f) flo = 2.0f;
}
__device__ __forceinline__ void lin_ge(float a, float bnd, float& flo, float& fhi) {
  if (a > 0.0f) flo = fmaxf(flo, __fdividef(bnd, a));        // a f >= bnd
  else if (a < 0.0f) fhi = fminf(fhi, __fdividef(bnd, a));
  else if (bnd > 0.0f) flo = 2.0f;
}

// The footprint test is conservative by 1/64 px (far above the rounding of
// q = p - f m for |q| < 4096 and |m| < 2^20) and the substep bounds by
// 1/256 of a substep (above the error of the fast division), so no source
// that can land in the tile at substep j is ever left out.
__device__ __forceinline__ bool substep_range(float4 b, int Sx0, int Sx1, int Sy0, int Sy1,
                                              int Tx0, int Tx1, int Ty0, int Ty1, int K,
                                              int& jlo, int& jhi) {
  if (!(b.x <= b.y) || !(b.z <= b.w)) return false;   // no finite source
  float flo = 0.0f, fhi = 1.0f;
  const float slack = 1.0f / 64.0f;
  lin_le(b.x, (float)(Sx1 - Tx0 + 1) + slack, flo, fhi);
  lin_ge(b.y, (float)(Sx0 - Tx1 - 1) - slack, flo, fhi);
  lin_le(b.z, (float)(Sy1 - Ty0 + 1) + slack, flo, fhi);
  lin_ge(b.w, (float)(Sy0 - Ty1 - 1) - slack, flo, fhi);
  if (!(flo <= fhi)) return false;
  const float Kf = (float)K;
  const int lo = max(1, (int)ceilf(flo * Kf - (1.0f / 256.0f)));
  const int hi = min(K - 1, (int)floorf(fhi * Kf + (1.0f / 256.0f)));
  if (lo > hi) return false;
  jlo = lo;
  jhi = hi;
  return true;
}

// The LDS z-buffer of a TW x TH target tile has rows of ZS(TW) = TW + 8
// keys: consecutive rows then start 64 bytes apart in the 32 banks, so the
// 8 rows touched by one source tile's footprint spread over all banks.
template <int TW>
__device__ __forceinline__ constexpr int zrow() { return TW + 8; }

// Splat up to kChunk source tiles (one source per lane and tile) at fraction
// f into the LDS z-buffer of target tile [Tx0,Tx1]x[Ty0,Ty1].  The loads of
// all tiles of the chunk are issued before any of them is used.
constexpr int kChunk = 4;

template <int TW>
__device__ __forceinline__ void splat_chunk(const EnvDesc& d, const int (&st)[kChunk], int nb,
                                            float f, int Tx0, int Tx1, int Ty0, int Ty1,
                                            unsigned long long* zbuf) {
  const int lane = threadIdx.x & (kWave - 1);
  float2 m[kChunk];
  float za[kChunk], dz[kChunk];
  int sxs[kChunk], sys[kChunk];
  bool ok[kChunk];
#pragma unroll
  for (int c = 0; c < kChunk; ++c) {
    ok[c] = false;
    sxs[c] = 0;
    sys[c] = 0;
    if (c < nb) {
      const int sxt = st[c] >> 8, syt = st[c] & 0xFF;   // wave-uniform
      sxs[c] = sxt * kSrcTile + (lane & 7);
      sys[c] = syt * kSrcTile + (lane >> 3);
      ok[c] = (sxs[c] < d.W) && (sys[c] < d.H);
    }
    if (ok[c]) {
      const int p = sys[c] * d.W + sxs[c];
      m[c] = ldg(d.mA, p);
      za[c] = ldg(d.ZA, p);
      dz[c] = ldg(d.dZ, p);
    }
  }
#pragma unroll
  for (int c = 0; c < kChunk; ++c) {
    if (!ok[c]) continue;
    const float qx = (float)sxs[c] - f * m[c].x;
    const float qy = (float)sys[c] - f * m[c].y;
    const float zt = za[c] + f * dz[c];
    if (!(zt > 0.0f)) continue;
    if (!(qx >= (float)(Tx0 - 1) && qx < (float)(Tx1 + 1) && qy >= (float)(Ty0 - 1) &&
          qy < (float)(Ty1 + 1)))
      continue;
    const float fx0 = floorf(qx), fy0 = floorf(qy);
    const int x0 = (int)fx0, y0 = (int)fy0;
    const bool bx = (qx - fx0) > 0.0f, by = (qy - fy0) > 0.0f;
    const unsigned p = (unsigned)(sys[c] * d.W + sxs[c]);
    const unsigned long long key = ((unsigned long long)__float_as_uint(zt) << 32) | p;
    const int lx = x0 - Tx0, ly = y0 - Ty0;
    const bool in_x0 = x0 >= Tx0, in_x1 = bx && (x0 + 1 <= Tx1);
    const bool in_y0 = y0 >= Ty0, in_y1 = by && (y0 + 1 <= Ty1);
    constexpr int ZS = zrow<TW>();
    unsigned long long* zr = zbuf + ly * ZS + lx;
    if (in_x0 && in_y0) atomicMin(zr, key);
    if (in_x1 && in_y0) atomicMin(zr + 1, key);
    if (in_x0 && in_y1) atomicMin(zr + ZS, key);
    if (in_x1 && in_y1) atomicMin(zr + ZS + 1, key);
  }
}

// B gather at fraction g = 1 - f for one target pixel (x, y): the sample
// position s = (x, y) - g m_B, its validity and the four taps of its cell.
struct BTaps {
  float a, b, c, d, wx, wy;
  bool v;
};

__device__ __forceinline__ BTaps b_taps(const EnvDesc& d, int x, int y, float2 mB, float g,
                                        bool pixel_ok) {
  BTaps t;
  const float sx = (float)x - g * mB.x;
  const float sy = (float)y - g * mB.y;
  t.v = pixel_ok && sx >= 0.0f && sx <= (float)(d.W - 1) && sy >= 0.0f && sy <= (float)(d.H - 1);
  const float sxc = t.v ? sx : 0.0f, syc = t.v ? sy : 0.0f;
  const float fx0 = floorf(sxc), fy0 = floorf(syc);
  t.wx = sxc - fx0;
  t.wy = syc - fy0;
  const int x0 = (int)fx0, y0 = (int)fy0;
  const int x1 = min(x0 + 1, d.W - 1), y1 = min(y0 + 1, d.H - 1);
  t.a = t.b = t.c = t.d = 0.0f;
  if (t.v) {
    t.a = ldg(d.LB, y0 * d.W + x0);
    t.b = ldg(d.LB, y0 * d.W + x1);
    t.c = ldg(d.LB, y1 * d.W + x0);
    t.d = ldg(d.LB, y1 * d.W + x1);
  }
  return t;
}

__device__ __forceinline__ float b_value(const BTaps& t) {
  return lerp32(lerp32(t.a, t.b, t.wx), lerp32(t.c, t.d, t.wx), t.wy);
}

// Window of 8x8 source tiles that can reach a target tile: source tile
// columns [wx0, wx0 + nwx), nwin tiles in all.
struct Window {
  int wx0, wy0, nwx, nwin;
};

// Candidate source tiles of target tile [Tx0,Tx1]x[Ty0,Ty1] and the substeps
// during which each can reach it, appended to the LDS list (at most cap
// entries: x-tile << 24 | y-tile << 16 | j_lo << 8 | j_hi).  *count must be
// zero on entry; returns the number of candidates (uniform; more than cap
// means the list overflowed).  Holds a barrier.
__device__ __forceinline__ int build_candidates(const EnvDesc& d, const EnvDyn& dy, int K,
                                                int Tx0, int Tx1, int Ty0, int Ty1,
                                                uint32_t* list, int* count, int cap, Window& w) {
  const int tid = threadIdx.x;
  const int W = d.W, H = d.H;
  const double M = __longlong_as_double((long long)dy.msq_bits);
  const int Rw = (M > 1.0e12) ? (1 << 20) : ((int)ceil(sqrt(M)) + 3);
  w.wx0 = max(0, Tx0 - Rw) / kSrcTile;
  w.wy0 = max(0, Ty0 - Rw) / kSrcTile;
  const int wx1 = min(d.ntx_src - 1, min(Tx1 + Rw, W - 1) / kSrcTile);
  const int wy1 = min(d.nty_src - 1, min(Ty1 + Rw, H - 1) / kSrcTile);
  w.nwx = wx1 - w.wx0 + 1;
  w.nwin = w.nwx * (wy1 - w.wy0 + 1);
  for (int i = tid; i < w.nwin; i += kBlock) {
    const int sxt = w.wx0 + i % w.nwx, syt = w.wy0 + i / w.nwx;
    const int st = syt * d.ntx_src + sxt;
    int jlo, jhi;
    if (substep_range(ldg(d.tb, st), sxt * kSrcTile, min(sxt * kSrcTile + 7, W - 1),
                      syt * kSrcTile, min(syt * kSrcTile + 7, H - 1), Tx0, Tx1, Ty0, Ty1, K,
                      jlo, jhi)) {
      const int slot = atomicAdd(count, 1);
      if (slot < cap)
        list[slot] = ((uint32_t)sxt << 24) | ((uint32_t)syt << 16) | ((uint32_t)jlo << 8) | (uint32_t)jhi;
    }
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*count);
}

// Splat every source that can reach the target tile at substep j (fraction
// f): the active entries of the candidate list, or, if the list overflowed,
// the active tiles of the whole window; each wave takes every fourth entry
// and splats its active tiles in chunks.
template <int TW>
__device__ __forceinline__ void splat_candidates(const EnvDesc& d, const uint32_t* list, int nlist,
                                                 bool overflow, const Window& w, int K, int j,
                                                 float f, int Tx0, int Tx1, int Ty0, int Ty1,
                                                 unsigned long long* zbuf) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int W = d.W, H = d.H;
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
        int st[kChunk];
        int nb = 0;
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
          st[c] = 0;
          if (mask) {
            const int b = __ffsll((long long)mask) - 1;
            mask &= mask - 1ull;
            st[c] = (int)((uint32_t)__builtin_amdgcn_readlane((int)ent, b) >> 16);   // sxt<<8 | syt
            ++nb;
          }
        }
        splat_chunk<TW>(d, st, nb, f, Tx0, Tx1, Ty0, Ty1, zbuf);
      }
    }
  } else {
    // Window scan: the candidate list did not fit.
    for (int i = wave; i < w.nwin; i += kWavesPerBlock) {
      const int sxt = w.wx0 + i % w.nwx, syt = w.wy0 + i / w.nwx;
      const int st0 = syt * d.ntx_src + sxt;
      int jlo, jhi;
      if (substep_range(ldg(d.tb, st0), sxt * kSrcTile, min(sxt * kSrcTile + 7, W - 1),
                        syt * kSrcTile, min(syt * kSrcTile + 7, H - 1), Tx0, Tx1, Ty0, Ty1, K,
                        jlo, jhi) &&
          j >= jlo && j <= jhi) {
        int st[kChunk] = {};
        st[0] = (sxt << 8) | syt;
        splat_chunk<TW>(d, st, 1, f, Tx0, Tx1, Ty0, Ty1, zbuf);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// the persistent tile kernel
// ---------------------------------------------------------------------------

// Per substep j of an item: (1) issue the B-gather loads of j, (2) splat j
// into the LDS z-buffer, (3) read the winners of j and issue the loads of
// their L_A, (4) blend and emit substep j - 1, whose loads were issued one
// substep earlier.  The z-buffer is cleared by its readers in (3); the
// barrier of (4) orders that before the next splat.
template <int TW, int TH, int MODE>
__global__ __launch_bounds__(kBlock, 4) void k_tile(const TileArgs a) {
  constexpr int NPX = TW * TH;
  constexpr int PPT = NPX / kBlock;
  static_assert(PPT * kBlock == NPX, "tile must be a multiple of the workgroup");
  constexpr int EVB = (MODE == MODE_STEP) ? kEventBuf : 1;
  constexpr int ZS = zrow<TW>();
  __shared__ unsigned long long zbuf[ZS * TH];
  __shared__ uint32_t list[kListCapMax];
  __shared__ uint2 evbuf[EVB];
  __shared__ int s_wtot[2][kWavesPerBlock];
  __shared__ unsigned long long s_gbase;
  __shared__ int s_item, s_rank, s_q, s_lcnt;
  constexpr int AUXN = (MODE == MODE_STEP) ? NPX : 1;
  __shared__ float s_con[AUXN], s_coff[AUXN];
  __shared__ int s_tl[AUXN];

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  for (int i = tid; i < ZS * TH; i += kBlock) zbuf[i] = kEmptyKey;
  const SinkShared sh{evbuf, s_wtot, &s_gbase, EVB};
  const SinkOut so{a.out, a.capacity, a.cursor};
  int ev_count = 0, round = 0;
  const int home = (int)(blockIdx.x % kXcd);
  int qsel = 0;   // 0..kXcd-1: queues tried so far (own queue first, then stealing)
  int rcur = 0;   // rank of the last item taken from the current queue

  for (;;) {
    __syncthreads();
    if (tid == 0) {
      int item = -1, r = 0, q = -1;
      while (qsel < kXcd) {
        const int qq = (home + qsel) % kXcd;
        const int it = (int)atomicAdd(&a.queue[qq], 1u);
        if (it < a.n_items[qq]) {
          item = it;
          q = qq;
          break;
        }
        ++qsel;
        rcur = 0;
      }
      if (item >= 0) {
        // items of a queue are taken in increasing order: walk ranks forward
        const int32_t* xb = a.xbegin + q * (a.n_envs + 1);
        r = rcur;
        while (r + 1 < a.n_envs && xb[r + 1] <= item) ++r;
        rcur = r;
      }
      s_item = item;
      s_rank = r;
      s_q = q;
      s_lcnt = 0;
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item < 0) break;
    const int rank = __builtin_amdgcn_readfirstlane(s_rank);
    const int q = __builtin_amdgcn_readfirstlane(s_q);
    const int env = __builtin_amdgcn_readfirstlane(a.env_order[rank]);
    const EnvDesc d = a.envs[env];
    const EnvDyn dy = a.dyn[env];
    const int li = item - a.xbegin[q * (a.n_envs + 1) + rank];
    const int H = d.H, W = d.W, K = dy.K;
    const int row0 = q * dy.nty / kXcd;
    const int tx = li % dy.ntx, ty = row0 + li / dy.ntx;
    const int Tx0 = tx * TW, Ty0 = ty * TH;
    const int Tx1 = min(Tx0 + TW, W) - 1, Ty1 = min(Ty0 + TH, H) - 1;

    // per-pixel registers; pixel k of this thread is i = tid + k * kBlock,
    // at (Tx0 + i % TW, Ty0 + i / TW)
    float LAq[PPT], LBq[PPT], Lp[PPT], R[PPT];
    float2 mBq[PPT];
    uint32_t okbits = 0;
    auto pix_x = [&](int k) { return Tx0 + (tid + k * kBlock) % TW; };
    auto pix_y = [&](int k) { return Ty0 + (tid + k * kBlock) / TW; };
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int x = pix_x(k), y = pix_y(k);
      const bool ok = (x <= Tx1) && (y <= Ty1);
      const int qq = ok ? (y * W + x) : 0;
      okbits |= (ok ? 1u : 0u) << k;
      LAq[k] = ok ? ldg(d.LA, qq) : 0.0f;
      LBq[k] = ok ? ldg(d.LB, qq) : 0.0f;
      mBq[k] = ok ? ldg(d.mB, qq) : make_float2(0.0f, 0.0f);
      Lp[k] = LAq[k];
      R[k] = 0.0f;
      if (MODE == MODE_STEP) {
        const int i = tid + k * kBlock;
        R[k] = ok ? ldg(d.Lref, qq) : 0.0f;
        s_tl[i] = (ok && d.tlast) ? ldg(d.tlast, qq) : EVIS_T_LAST_INIT;
        if (d.th_on) s_con[i] = ok ? ldg(d.th_on, qq) : 1.0f;
        if (d.th_off) s_coff[i] = ok ? ldg(d.th_off, qq) : 1.0f;
      }
    }
    const PixAux aux{(MODE == MODE_STEP && d.th_on) ? s_con : nullptr,
                     (MODE == MODE_STEP && d.th_off) ? s_coff : nullptr, s_tl, d.C_on, d.C_off,
                     Tx0, Ty0, TW, __builtin_ctz(TW), -1};

    // Candidate source tiles and their substep intervals.
    Window win{};
    int nlist = 0;
    bool overflow = false;
    if (K > 1) {
      nlist = build_candidates(d, dy, K, Tx0, Tx1, Ty0, Ty1, list, &s_lcnt, a.list_cap, win);
      overflow = nlist > a.list_cap;
    }

    // Static tile: every source that can reach it does not move, it does not
    // move in B and L_A == L_B on it, so every sub-frame equals L_A.
    bool is_static = false;
    if (MODE == MODE_STEP && a.static_tiles && K > 1 && !overflow) {
      bool okst = true;
      for (int e2 = tid; e2 < nlist; e2 += kBlock) {
        const uint32_t ent = list[e2];
        const float4 b = ldg(d.tb, (int)((ent >> 16) & 0xFFu) * d.ntx_src + (int)(ent >> 24));
        okst = okst && b.x == 0.0f && b.y == 0.0f && b.z == 0.0f && b.w == 0.0f;
      }
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if ((okbits >> k) & 1u) {
          const int x = pix_x(k), y = pix_y(k);
          const int x1 = min(x + 1, W - 1), y1 = min(y + 1, H - 1);
          const float t1 = ldg(d.LB, y * W + x1), t2 = ldg(d.LB, y1 * W + x);
          const float t3 = ldg(d.LB, y1 * W + x1);
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
            const int qq = pix_y(k) * W + pix_x(k);
            a.L_out[qq] = LAq[k];
            if (a.hole) a.hole[qq] = 0;
          }
        }
      }
      j_first = max(1, a.j_begin);
      j_last = min(K, a.j_end - 1);
    }

    // Consumers of a finished sub-frame (substep jj, values Lj, holes hb).
    auto consume = [&](int jj, const float (&Lj)[PPT], const uint32_t (&hb)[PPT]) {
      if (MODE == MODE_STEP) {
        emit_substep<PPT>(jj, Lj, Lp, R, aux, okbits, d.t0, d.span, dy.Dt, d.refr, d.env_bits,
                          sh, so, ev_count, round);
      } else if (MODE == MODE_INTERP) {
        const long long plane = (long long)H * W;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          if ((okbits >> k) & 1u) {
            const long long o = (long long)(jj - a.j_begin) * plane + (pix_y(k) * W + pix_x(k));
            a.L_out[o] = Lj[k];
            if (a.hole) a.hole[o] = (uint8_t)hb[k];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < PPT; ++k) Lp[k] = Lj[k];
    };

    // pending interior substep (values whose loads were issued last iteration)
    float pAh[PPT], pBh[PPT];
    uint32_t phb[PPT];
    float palpha = 0.0f;
    bool pending = false;
    int pj = 0;

    auto finish_pending = [&]() {
      float Lj[PPT];
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const bool vA = !(phb[k] & 1u), vB = !(phb[k] & 2u);
        float v;
        if (is_static) v = LAq[k];
        else if (vA && vB) v = lerp32(pAh[k], pBh[k], palpha);
        else if (vA) v = pAh[k];
        else if (vB) v = pBh[k];
        else v = lerp32(LAq[k], LBq[k], palpha);
        Lj[k] = v;
      }
      consume(pj, Lj, phb);
      pending = false;
    };

    const int j_int_last = min(j_last, K - 1);   // last interior substep to build
    for (int j = j_first; j <= j_int_last; ++j) {
      const float f = (float)j / (float)K;
      const float g = 1.0f - f;
      const float alpha = (d.blend == EVIS_BLEND_TIME) ? f : 1.0f;
      float cAh[PPT], cBh[PPT];
      uint32_t chb[PPT];
      if (!is_static) {
        // (1) B-gather loads of substep j
        BTaps bt[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) bt[k] = b_taps(d, pix_x(k), pix_y(k), mBq[k], g, (okbits >> k) & 1u);
        // (2) splat substep j
        splat_candidates<TW>(d, list, nlist, overflow, win, K, j, f, Tx0, Tx1, Ty0, Ty1, zbuf);
        __syncthreads();
        // (3) winners of substep j: issue their L_A loads; B values
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          const int i = tid + k * kBlock;
          const int zi = (i / TW) * ZS + (i % TW);
          bool vA = false;
          cAh[k] = 0.0f;
          if ((okbits >> k) & 1u) {
            const unsigned long long key = zbuf[zi];
            zbuf[zi] = kEmptyKey;
            vA = key != kEmptyKey;
            if (vA) cAh[k] = ldg(d.LA, (int)(key & 0xFFFFFFFFull));
          }
          cBh[k] = bt[k].v ? b_value(bt[k]) : 0.0f;
          chb[k] = (vA ? 0u : 1u) | (bt[k].v ? 0u : 2u);
        }
      } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          cAh[k] = 0.0f;
          cBh[k] = 0.0f;
          chb[k] = 0u;
        }
      }
      // (4) substep j - 1.  In MODE_STEP its emission holds a barrier that
      // orders (3) before the next splat; otherwise take one here.
      const bool had_pending = pending;
      if (pending) finish_pending();
      if (!(MODE == MODE_STEP && had_pending)) __syncthreads();
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        pAh[k] = cAh[k];
        pBh[k] = cBh[k];
        phb[k] = chb[k];
      }
      palpha = alpha;
      pj = j;
      pending = true;
    }
    if (pending) finish_pending();
    if (j_last == K) {
      float Lj[PPT];
      uint32_t hb[PPT];
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        Lj[k] = LBq[k];
        hb[k] = 0u;
      }
      consume(K, Lj, hb);
    }
    if (MODE == MODE_INTERP) __syncthreads();

    if (MODE == MODE_STEP) {
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if ((okbits >> k) & 1u) {
          const int qq = pix_y(k) * W + pix_x(k);
          stg(d.Lref, qq, R[k]);
          if (d.tlast) stg(d.tlast, qq, s_tl[tid + k * kBlock]);
        }
      }
    }
  }
  if (MODE == MODE_STEP) sink_flush(sh, so, ev_count);
}

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
  constexpr int ZS = zrow<TW>();
  __shared__ unsigned long long zbuf[ZS * TH];
  __shared__ uint32_t list[kListCapMax];
  __shared__ int s_lcnt;
  __shared__ float s_red[kWavesPerBlock];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  for (int i = tid; i < ZS * TH; i += kBlock) zbuf[i] = kEmptyKey;
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
      splat_candidates<TW>(d, list, nlist, overflow, win, K, j, f, Tx0, Tx1, Ty0, Ty1, zbuf);
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
        const int zi = (i / TW) * ZS + (i % TW);
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
      const float sg = 1.0f / (1.0f + expf(-u));
      if (!BWD) {
        acc[k] += sg;
      } else {
        const float dS = sg * (1.0f - sg) * a.inv_tau;
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_reset(EnvDyn* dyn, int n_envs, unsigned int* queue, unsigned long long* cursor,
                        hipStream_t s) {
  const int n = max(n_envs, kXcd);
  hipLaunchKernelGGL(k_reset, dim3((n + 255) / 256), dim3(256), 0, s, dyn, n_envs, queue, cursor);
  return hipGetLastError();
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

hipError_t launch_prep(const EnvDesc* envs, EnvDyn* dyn, const int32_t* src_prefix, int n_envs,
                       int total_src_tiles, hipStream_t s) {
  if (total_src_tiles <= 0) return hipSuccess;
  const int blocks = (total_src_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(kBlock), 0, s, envs, dyn, src_prefix, n_envs,
                     total_src_tiles);
  return hipGetLastError();
}

hipError_t launch_queue(const EnvDesc* envs, EnvDyn* dyn, int n_envs, int tile_w, int tile_h,
                        int32_t* xbegin, int32_t* env_order, int32_t* n_items,
                        int32_t* K_used, hipStream_t s) {
  hipLaunchKernelGGL(k_queue, dim3(1), dim3(EVIS_MAX_ENVS), 0, s, envs, dyn, n_envs, tile_w,
                     tile_h, xbegin, env_order, n_items, K_used);
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
