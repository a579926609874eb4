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
#include "evis_warp.h"

namespace evis {

// ---------------------------------------------------------------------------
// per-step reset and per-pair preparation
// ---------------------------------------------------------------------------

__global__ void k_reset(EnvDyn* dyn, int n_envs, unsigned int* queue,
                        unsigned long long* cursor) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_envs) dyn[i].msq_bits = 0ull;
  if (i < kXcd) queue[i * kQueueStride] = 0u;
  if (i == 0 && cursor) *cursor = 0ull;
}

// Per 4x4 source block (a row of 16 lanes; a wave takes four consecutive
// blocks of one env): the endpoint depth (Eq. 7, p_B = p - m_A(p), Z_B
// edge-clamped), stored with m_A and Z_A as the source's splat record
// (m_A.x, m_A.y, Z_A, Zend - Z_A), block-major, so that the splat reads one
// 16-byte value per source and a block's 16 records are contiguous; the
// block's bounds of m_A over sources with a finite motion vector; and the
// env's largest finite |m|^2.
__global__ __launch_bounds__(kBlock) void k_prep(const EnvDesc* __restrict__ envs, EnvDyn* dyn,
                                                 const int32_t* __restrict__ src_prefix,
                                                 int n_envs, int total) {
  __shared__ int s_prefix[EVIS_MAX_ENVS + 1];
  for (int i = threadIdx.x; i <= n_envs; i += kBlock) s_prefix[i] = src_prefix[i];
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int g = lane >> 4, r = lane & (kBlkPx - 1);   // block of the group, lane in the block
  const int nwaves = (int)gridDim.x * kWavesPerBlock;
  const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x / kWave);
  const int chunk = (total + nwaves - 1) / nwaves;
  const int c0 = min(total, wid * chunk), c1 = min(total, c0 + chunk);
  constexpr int U = 2;   // groups in flight per wave
  const float inf = __int_as_float(0x7f800000);
  // the env's largest |m|^2 seen by this wave, published when the env changes
  int run_env = -1;
  double run_msq = 0.0;
  auto publish = [&]() {
    if (run_env >= 0 && run_msq > 0.0 && lane == 0)
      atomicMax(&dyn[run_env].msq_bits, (unsigned long long)__double_as_longlong(run_msq));
  };
  // each wave walks a contiguous run of block groups (wave-uniform loop), U
  // groups at a time so that their loads overlap
  for (int g0 = c0; g0 < c1; g0 += U) {
    int e[U], blk[U], x[U], y[U], p[U];
    bool has[U], in[U];
    float2 ma[U], mb[U];
    float za[U], zend[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int gt = min(g0 + u, c1 - 1);   // a duplicate of the last group is harmless
      int lo = 0, hi = n_envs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_prefix[mid] <= gt) lo = mid; else hi = mid - 1;
      }
      e[u] = lo;
      const EnvDesc& d = envs[lo];
      blk[u] = (gt - s_prefix[lo]) * 4 + g;
      has[u] = blk[u] < d.ntx_src * d.nty_src;
      const int bx = has[u] ? blk[u] % d.ntx_src : 0, by = has[u] ? blk[u] / d.ntx_src : 0;
      x[u] = bx * kSrcBlk + (r & 3);
      y[u] = by * kSrcBlk + (r >> 2);
      in[u] = has[u] && x[u] < d.W && y[u] < d.H;
      p[u] = in[u] ? y[u] * d.W + x[u] : 0;
      ma[u] = ldg(d.mA, p[u]);
      mb[u] = ldg(d.mB, p[u]);
      za[u] = ldg(d.ZA, p[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const EnvDesc& d = envs[e[u]];
      const float sx = clamp_into((float)x[u] - ma[u].x, (float)(d.W - 1));
      const float sy = clamp_into((float)y[u] - ma[u].y, (float)(d.H - 1));
      zend[u] = bilinear(d.ZB, d.H, d.W, sx, sy);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const EnvDesc& d = envs[e[u]];
      float mnx = inf, mxx = -inf, mny = inf, mxy = -inf;
      double msq = 0.0;
      if (in[u]) {
        const float2 a = ma[u], b = mb[u];
        if (finite32(a.x) && finite32(a.y)) {
          mnx = mxx = a.x;
          mny = mxy = a.y;
        }
        const double mda = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
        const double mdb = (double)b.x * (double)b.x + (double)b.y * (double)b.y;
        if (mda <= 1.7976931348623157e308) msq = mda;
        if (mdb <= 1.7976931348623157e308 && mdb > msq) msq = mdb;
      }
      if (has[u])
        stg(d.src, blk[u] * kBlkPx + r,
            in[u] ? make_float4(ma[u].x, ma[u].y, za[u], zend[u] - za[u]) : make_float4(0.f, 0.f, 0.f, 0.f));
      mnx = row16_min(mnx);
      mxx = row16_max(mxx);
      mny = row16_min(mny);
      mxy = row16_max(mxy);
      msq = wave_max_d(msq);
      if (r == 0 && has[u]) stg(d.tb, blk[u], make_float4(mnx, mxx, mny, mxy));
      if (e[u] != run_env) {   // wave-uniform
        publish();
        run_env = e[u];
        run_msq = 0.0;
      }
      run_msq = fmax(run_msq, msq);
    }
  }
  publish();
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
// the persistent tile kernel
// ---------------------------------------------------------------------------

// Substeps go in pairs (j, j + 1) that share one splat pass (each source's
// record is loaded once for both).  Per substep j: (1) issue the B-gather
// loads of j; (2) at the first substep of a pair, splat j and j + 1 into LDS
// z-buffers j & 3 and (j + 1) & 3, barrier; (3) read the winners of j
// (clearing their cells) and issue the loads of their L_A; (4) blend and emit
// substep j - 1, whose loads were issued one substep earlier.  The next pair
// splats into the other two buffers, and the pair after it comes after the
// next pair's barrier, so one barrier per pair suffices; emission takes none.
template <int TW, int TH, int MODE>
__global__ __launch_bounds__(kBlock, 4) void k_tile(const TileArgs a) {
  constexpr int NPX = TW * TH;
  constexpr int PPT = NPX / kBlock;
  static_assert(PPT * kBlock == NPX, "tile must be a multiple of the workgroup");
  constexpr int EVB = (MODE == MODE_STEP) ? kEventBuf : 1;
  constexpr int ZN = zcells<TW, TH>();
  __shared__ unsigned long long zbuf[4 * ZN];
  __shared__ uint32_t list[kListCapMax];
  __shared__ uint32_t s_wl[kWavesPerBlock][kWave];   // per-wave packed active candidates
  __shared__ uint2 evbuf[EVB];
  __shared__ int s_evn, s_req[4];
  __shared__ unsigned long long s_gbase;
  __shared__ int s_item, s_rank, s_q, s_lcnt;
  constexpr int AUXN = (MODE == MODE_STEP) ? NPX : 1;
  __shared__ float s_con[AUXN], s_coff[AUXN];
  __shared__ int s_tl[AUXN];

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const SinkShared sh{evbuf, &s_evn, s_req, &s_gbase, EVB};
  const SinkOut so{a.out, a.capacity, a.cursor};
  SinkRound sr;
  sink_init(sh);
  const int home = (int)(blockIdx.x % kXcd);
  int qsel = 0;   // 0..kXcd-1: queues tried so far (own queue first, then stealing)
  int rcur = 0;   // rank of the last item taken from the current queue

  for (;;) {
    __syncthreads();
    if (MODE == MODE_STEP) sink_check(sh, so, sr);
    // Readers clear the cells they read; apron cells and those of pixels
    // outside the image are cleared here, once per item.
    for (int i = tid; i < 4 * ZN; i += kBlock) zbuf[i] = kEmptyKey;
    if (tid == 0) {
      int item = -1, r = 0, q = -1;
      while (qsel < kXcd) {
        const int qq = (home + qsel) % kXcd;
        const int it = (int)atomicAdd(&a.queue[qq * kQueueStride], 1u);
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
        const float4 b = ldg(d.tb, cand_by(ent) * d.ntx_src + cand_bx(ent));
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
                          sh, so, sr);
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
        if (is_static) v = Lp[k];   // every sample of a static tile is L_A
        else if (vA && vB) v = lerp32(pAh[k], pBh[k], palpha);
        else if (vA) v = pAh[k];
        else if (vB) v = pBh[k];
        else {   // neither side: the pixel's own values (rare; read again, not kept in registers)
          const int qq = ((okbits >> k) & 1u) ? pix_y(k) * W + pix_x(k) : 0;
          v = lerp32(ldg(d.LA, qq), ldg(d.LB, qq), palpha);
        }
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
      unsigned long long* zb = zbuf + (j & 3) * ZN;
      const bool pair_start = ((j - j_first) & 1) == 0;   // uniform
      if (!is_static) {
        // (1) B-gather loads of substep j
        BTaps bt[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) bt[k] = b_taps(d, pix_x(k), pix_y(k), mBq[k], g, (okbits >> k) & 1u);
        // (2) splat substeps j and j + 1
        if (pair_start) {
          const int nf = (j + 1 <= j_int_last) ? 2 : 1;
          const float fs[2] = {f, (float)(j + 1) / (float)K};
          unsigned long long* const zs[2] = {zb, zbuf + ((j + 1) & 3) * ZN};
          splat_candidates<TW, 2>(d, list, nlist, overflow, win, K, j, nf, fs, Tx0, Tx1, Ty0,
                                  Ty1, s_wl[wave], zs);
          __syncthreads();
          if (MODE == MODE_STEP) sink_check(sh, so, sr);
        }
        // (3) winners of substep j: issue their L_A loads; B values
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          const int i = tid + k * kBlock;
          const int zi = zcell<TW>(i % TW, i / TW);
          bool vA = false;
          cAh[k] = 0.0f;
          if ((okbits >> k) & 1u) {
            const unsigned long long key = zb[zi];
            zb[zi] = kEmptyKey;
            vA = key != kEmptyKey;
            if (vA) cAh[k] = ldg(d.LA, (int)(key & 0xFFFFFFFFull));
          }
          cBh[k] = bt[k].v ? b_value(bt[k]) : 0.0f;
          chb[k] = (vA ? 0u : 1u) | (bt[k].v ? 0u : 2u);
        }
      } else {
        if (pair_start) {
          __syncthreads();
          if (MODE == MODE_STEP) sink_check(sh, so, sr);
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          cAh[k] = 0.0f;
          cBh[k] = 0.0f;
          chb[k] = 0u;
        }
      }
      // (4) substep j - 1
      if (pending) finish_pending();
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
        Lj[k] = ((okbits >> k) & 1u) ? ldg(d.LB, pix_y(k) * W + pix_x(k)) : 0.0f;
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
  if (MODE == MODE_STEP) sink_flush(sh, so);
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

hipError_t launch_prep(const EnvDesc* envs, EnvDyn* dyn, const int32_t* src_prefix, int n_envs,
                       int total_src_tiles, hipStream_t s) {
  if (total_src_tiles <= 0) return hipSuccess;
  // a run of block groups per wave: 256 CUs x 8 workgroups at most
  const int blocks = std::min((total_src_tiles + kWavesPerBlock - 1) / kWavesPerBlock, 256 * 8);
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
