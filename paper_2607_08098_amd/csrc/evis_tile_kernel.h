// The persistent fused tile kernel k_tile<TW, TH, MODE, WARP> (gfx950):
// instantiated for the gather warp in evis_tile.hip and for the two
// splat warps in evis_tile_splat.hip.
#pragma once

#include "evis_internal.h"
#include "evis_sink.h"
#include "evis_warp.h"

namespace evis {

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
//
// The two-splat warps (WARP = EVIS_WARP_SPLAT or EVIS_WARP_JOINT) replace
// the B gather by B's backward splat: both directions' candidates share
// one list, both are splatted, and the winners give A^ and B^.  JOINT
// splats pairs into one z-buffer set as above (the winner's tag tells A
// from B); SPLAT needs a z-buffer per direction, so it splats each pair
// into two buffers per direction (A: j & 1, B: 2 + (j & 1)) and takes a
// second barrier after the pair's second resolve, before the next pair's
// splat reuses them (two barriers per pair, as many as substeps).
//
// NOISE = 1 (fused step only) adds the sensor-noise events of every env that
// has noise after each substep's crossings.
// Waves per SIMD each tile shape is compiled for: with one or two pixels
// per thread the kernel fits 128 VGPRs (4 waves per SIMD, four workgroups
// per CU); four pixels per thread need up to 256 (2 waves), eight 1.
template <int TW, int TH>
constexpr int tile_waves() {
  return (TW * TH / kBlock) <= 2 ? 4 : ((TW * TH / kBlock) == 4 ? 2 : 1);
}

template <int TW, int TH, int MODE, int WARP = EVIS_WARP_GATHER, int NOISE = 0>
__global__ __launch_bounds__(kBlock, (tile_waves<TW, TH>())) void k_tile(const TileArgs a) {
  constexpr int NPX = TW * TH;
  constexpr int PPT = NPX / kBlock;
  static_assert(PPT * kBlock == NPX, "tile must be a multiple of the workgroup");
  constexpr bool kGather = WARP == EVIS_WARP_GATHER;
  // The two-splat warps hold both directions' candidates in a list twice as
  // long, paid for by half the event buffer (LDS stays within 4 workgroups
  // per CU for the 32 x 16 tile).
  constexpr int LCAP = kGather ? kListCapMax : 2 * kListCapMax;
  // The gather warp's crossing queues (4 KB) are paid for by half the
  // event buffer; the two-splat warps, whose LDS is full, and the noise
  // path, whose registers are, emit at once.
  constexpr bool kQueue = MODE == MODE_STEP && kGather && NOISE == 0;
  constexpr int EVB = (MODE != MODE_STEP) ? 1 : ((kGather && !kQueue) ? kEventBuf : kEventBuf / 2);
  constexpr int CQN = kQueue ? kWavesPerBlock * kCrossQ : 1;
  constexpr int ZN = zcells<TW, TH>();
  constexpr bool kOwnB = WARP == EVIS_WARP_SPLAT;   // B has z-buffers of its own
  constexpr int NZB = 4;
  __shared__ unsigned long long zbuf[NZB * ZN];
  __shared__ uint32_t list[LCAP];
  __shared__ uint32_t s_wl[kWavesPerBlock][kWave];   // per-wave packed active candidates
  __shared__ uint2 evbuf[EVB];
  __shared__ float4 s_cq[CQN];   // crossing queues of the waves (no refractory period)
  __shared__ int s_evn, s_req[4];
  __shared__ unsigned long long s_gbase;
  __shared__ int s_item, s_rank, s_q, s_lcnt, s_sbn;
  __shared__ unsigned long long s_lcnt2;   // two-splat warps: A's and B's candidate counts
  constexpr int AUXN = (MODE == MODE_STEP) ? NPX : 1;
  __shared__ float s_con[AUXN], s_coff[AUXN];
  __shared__ int s_tl[AUXN];

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int lcap = kGather ? a.list_cap : 2 * a.list_cap;   // entries the list may hold
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
    for (int i = tid; i < NZB * ZN; i += kBlock) zbuf[i] = kEmptyKey;
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
      s_sbn = 0;
      if (!kGather) s_lcnt2 = 0ull;
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
      // the fused step's event model covers only the pixels inside the crop
      // margin (0 unless the env was rendered with one)
      const int mg = (MODE == MODE_STEP) ? d.margin : 0;
      const bool ok = (x <= Tx1) && (y <= Ty1) && x >= mg && y >= mg && x < W - mg && y < H - mg;
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
        // without a refractory period t_last is only written: the item
        // keeps the largest event time of each pixel (INT_MIN: none)
        s_tl[i] = (kQueue && d.refr == 0)
                      ? INT_MIN : ((ok && d.tlast) ? ldg(d.tlast, qq) : EVIS_T_LAST_INIT);
        if (d.th_on) s_con[i] = ok ? ldg(d.th_on, qq) : 1.0f;
        if (d.th_off) s_coff[i] = ok ? ldg(d.th_off, qq) : 1.0f;
      }
    }
    const PixAux aux{(MODE == MODE_STEP && d.th_on) ? s_con : nullptr,
                     (MODE == MODE_STEP && d.th_off) ? s_coff : nullptr, s_tl, d.C_on, d.C_off,
                     Tx0 - (MODE == MODE_STEP ? d.margin : 0), Ty0 - (MODE == MODE_STEP ? d.margin : 0),
                     TW, __builtin_ctz(TW), -1};   // event coordinates are the cropped frame's
    NoiseCfg ncfg{};
    uint32_t hotb = 0;
    if constexpr (NOISE != 0 && MODE == MODE_STEP) {
      if (d.noise_on) {   // uniform
        ncfg = noise_cfg(d, dy.Dt);
        hotb = hot_bits<PPT>(ncfg, aux, okbits);
      }
    }

    // Candidate source blocks and their substep intervals.
    Window win{};
    int nlist = 0, nlistB = 0;
    bool overflow = false;
    if (K > 1) {
      if (kGather) {
        // the splat's per-wave slices are free until the splat: they hold
        // the list of superblocks meanwhile (kBlock entries)
        nlist = build_candidates(d, dy, K, Tx0, Tx1, Ty0, Ty1, list, &s_lcnt, a.list_cap, win,
                                 reinterpret_cast<int*>(&s_wl[0][0]), &s_sbn);
        overflow = nlist > a.list_cap;
      } else {
        build_candidates_two(d, dy, K, Tx0, Tx1, Ty0, Ty1, list, &s_lcnt2, lcap, win, nlist,
                             nlistB);
        overflow = nlist + nlistB > lcap;
      }
    }

    // Static tile: every source that can reach it does not move, it does not
    // move in B and L_A == L_B on it, so every sub-frame equals L_A.  (The
    // test costs a round of loads and a barrier; with one or two warped
    // substeps it is not worth them, and the full path gives the same
    // sub-frames.)
    bool is_static = false;
    if (MODE == MODE_STEP && kGather && a.static_tiles && K > 3 && !overflow) {
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
    CrossQueue cq{s_cq};
    auto consume = [&](int jj, const float (&Lj)[PPT], const uint32_t (&hb)[PPT]) {
      if (MODE == MODE_STEP) {
        if (kQueue && d.refr == 0)   // uniform
          emit_queued<PPT>(jj, jj == K, Lj, Lp, R, aux, okbits, d.t0, d.span, dy.Dt, d.env_bits,
                           sh, so, sr, cq);
        else
          emit_substep<PPT>(jj, Lj, Lp, R, aux, okbits, d.t0, d.span, dy.Dt, d.refr, d.env_bits,
                            sh, so, sr);
        if constexpr (NOISE != 0) {
          if (d.noise_on)
            emit_noise<PPT>(jj, Lj, aux, okbits, hotb, ncfg, d.t0, d.span, dy.Dt, d.env_bits, sh,
                            so, sr);
        }
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

    // A static tile's samples are all L_A (and L_B = L_A): once a substep
    // leaves every pixel within its thresholds of the reference, no later
    // substep can emit (the reference moves only with a crossing), so the
    // interior substeps stop there and the last one (which drains the
    // crossing queue) follows.  Noise draws per substep: the noise kernel
    // runs them all.
    bool static_done = false;
    if (MODE == MODE_STEP && NOISE == 0 && is_static) {   // uniform
      uint32_t hb0[PPT];
      float Lj[PPT];
#pragma unroll
      for (int k = 0; k < PPT; ++k) hb0[k] = 0u;
      for (int j = 1; j <= K - 1; ++j) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) Lj[k] = LAq[k];
        consume(j, Lj, hb0);
        int quiet = 1;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          if ((okbits >> k) & 1u) {
            const float dd = LAq[k] - R[k];
            const float c = aux.c(k, dd > 0.0f);
            if (fabsf(dd) >= c && c > 0.0f) quiet = 0;
          }
        }
        if (__syncthreads_and(quiet) != 0) break;   // uniform
      }
#pragma unroll
      for (int k = 0; k < PPT; ++k) Lj[k] = LAq[k];
      consume(K, Lj, hb0);
      static_done = true;
    }
    const int j_int_last = static_done ? 0 : min(j_last, K - 1);   // last interior substep to build
    for (int j = j_first; j <= j_int_last; ++j) {
      const float f = (float)j / (float)K;
      const float g = 1.0f - f;
      const float alpha = (d.blend == EVIS_BLEND_TIME) ? f : 1.0f;
      float cAh[PPT], cBh[PPT];
      uint32_t chb[PPT];
      unsigned long long* zb = zbuf + (kOwnB ? (j & 1) : (j & 3)) * ZN;
      const bool pair_start = ((j - j_first) & 1) == 0;   // uniform
      if constexpr (!kGather) {
        // two-splat warps: (2) splat A forward and B backward for j and j + 1
        unsigned long long* const zbB = kOwnB ? zbuf + (2 + (j & 1)) * ZN : zb;
        if (kOwnB && pair_start) {
          const int nf = (j + 1 <= j_int_last) ? 2 : 1;
          const float fs[2] = {f, (float)(j + 1) / (float)K};
          unsigned long long* const zs[2] = {zb, zbuf + ((j + 1) & 1) * ZN};
          unsigned long long* const zsB[2] = {zbB, zbuf + (2 + ((j + 1) & 1)) * ZN};
          splat_candidates<TW, 2, DIR_A>(d, list, nlist, overflow, win, K, j, nf, fs, Tx0, Tx1,
                                         Ty0, Ty1, s_wl[wave], zs);
          splat_candidates<TW, 2, DIR_B>(d, list, nlistB, overflow, win, K, j, nf, fs, Tx0, Tx1,
                                         Ty0, Ty1, s_wl[wave], zsB, lcap - 1, -1);
          __syncthreads();
          if (MODE == MODE_STEP) sink_check(sh, so, sr);
        } else if (!kOwnB && pair_start) {
          const int nf = (j + 1 <= j_int_last) ? 2 : 1;
          const float fs[2] = {f, (float)(j + 1) / (float)K};
          unsigned long long* const zs[2] = {zb, zbuf + ((j + 1) & 3) * ZN};
          splat_candidates<TW, 2, DIR_A_TAGGED>(d, list, nlist, overflow, win, K, j, nf, fs, Tx0,
                                                Tx1, Ty0, Ty1, s_wl[wave], zs);
          splat_candidates<TW, 2, DIR_B>(d, list, nlistB, overflow, win, K, j, nf, fs, Tx0, Tx1,
                                         Ty0, Ty1, s_wl[wave], zs, lcap - 1, -1);
          __syncthreads();
          if (MODE == MODE_STEP) sink_check(sh, so, sr);
        }
        // (3) winners of substep j: issue the loads of their L_A / L_B
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          const int i = tid + k * kBlock;
          const int zi = zcell<TW>(i % TW, i / TW);
          bool vA = false, vB = false;
          cAh[k] = 0.0f;
          cBh[k] = 0.0f;
          if ((okbits >> k) & 1u) {
            const unsigned long long key = zb[zi];
            zb[zi] = kEmptyKey;
            const uint32_t low = (uint32_t)(key & 0xFFFFFFFFull);
            if (kOwnB) {
              const unsigned long long keyB = zbB[zi];
              zbB[zi] = kEmptyKey;
              vA = key != kEmptyKey;
              vB = keyB != kEmptyKey;
              if (vA) cAh[k] = ldg(d.LA, (int)low);
              if (vB) cBh[k] = ldg(d.LB, (int)(keyB & 0xFFFFFFFFull));
            } else {
              const bool hit = key != kEmptyKey;
              vA = hit && (low & kATag) != 0u;
              vB = hit && (low & kATag) == 0u;
              if (vA) cAh[k] = ldg(d.LA, (int)(low & ~kATag));
              if (vB) cBh[k] = ldg(d.LB, (int)low);
            }
          }
          chb[k] = (vA ? 0u : 1u) | (vB ? 0u : 2u);
        }
        if (kOwnB && !pair_start) {   // both buffer pairs read and cleared
          __syncthreads();
          if (MODE == MODE_STEP) sink_check(sh, so, sr);
        }
      } else if (!is_static) {
        // (1) B-gather loads of substep j
        BTaps bt[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) bt[k] = b_taps(d, pix_x(k), pix_y(k), mBq[k], g, (okbits >> k) & 1u);
        // (2) splat substeps j and j + 1
        if (pair_start) {
          const int nf = (j + 1 <= j_int_last) ? 2 : 1;
          const float fs[2] = {f, (float)(j + 1) / (float)K};
          unsigned long long* const zs[2] = {zb, zbuf + ((j + 1) & 3) * ZN};
          // (three blocks per lane group per window-scan pass in the plain
          // step; the noise kernel, at its register limit, scans one)
          splat_candidates<TW, 2, DIR_A, (NOISE == 0 ? kChunk : 1)>(
              d, list, nlist, overflow, win, K, j, nf, fs, Tx0, Tx1, Ty0, Ty1, s_wl[wave], zs);
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
    if (j_last == K && !static_done) {
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
          const int tl = s_tl[tid + k * kBlock];
          if (d.tlast && (!kQueue || d.refr != 0 || tl != INT_MIN)) stg(d.tlast, qq, tl);
        }
      }
    }
  }
  if (MODE == MODE_STEP) sink_flush(sh, so);
}

}  // namespace evis
