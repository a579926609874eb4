// Event emission (Eq. 4 with Eq. 8 thresholds and the refractory period)
// and wave-ballot / prefix-sum compaction into a workgroup-local LDS buffer
// that is appended to the global event stream with one atomic per flush.
//
// Emission takes no barrier: each wave reserves its slots in the LDS buffer
// with one atomic add on the buffer's count; slots past the end of the
// buffer go straight to the stream after one global atomic (the count may
// then exceed the buffer, whose every slot is still filled); the wave
// raises a flush request once the buffer is three quarters full.  Requests
// are read after
// the next workgroup barrier, where every wave sees the same values: round r
// writes request slot r & 3, at most two rounds run between two checks, and
// round r + 4 cannot start before the barrier that follows the check of
// round r, by which time every wave has read slot r & 3.  So that this holds
// whatever the caller does, an emission that finds two rounds unchecked
// takes the barrier and the check itself.
#pragma once

#include "evis_common.h"

namespace evis {

struct SinkShared {
  uint2* buf;                   // LDS [cap] staged events
  int* cnt;                     // LDS: events staged
  int* req;                     // LDS [4]: flush requests by round, modulo 4
  unsigned long long* gbase;    // LDS: global slot of the current flush
  int cap;
};

struct SinkOut {
  evis_event* out;
  long long capacity;
  unsigned long long* cursor;
};

// Workgroup-uniform sink state kept in registers.
struct SinkRound {
  int round = 0;          // emissions so far
  int unchecked = 0;      // emissions whose requests have not been read yet (<= 2)
};

// Clear the LDS state; a barrier must follow before the first emission.
__device__ __forceinline__ void sink_init(const SinkShared& sh) {
  if (threadIdx.x == 0) {
    *sh.cnt = 0;
    sh.req[0] = sh.req[1] = sh.req[2] = sh.req[3] = 0;
  }
}

// Append the staged events to the stream.  Every thread calls it, right
// after a barrier that follows the last emission, and no wave emits until
// it returns.  Thread 0 alone reads and resets the count (and hands the
// number over with the global slot); the flush requests, which every wave
// reads before calling, are cleared only after the second barrier.
__device__ __forceinline__ void sink_drain(const SinkShared& sh, const SinkOut& so) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    const int n0 = min(lds_ld(sh.cnt, 0), sh.cap);
    *sh.cnt = 0;
    *sh.gbase = ((unsigned long long)(n0 > 0 ? atomicAdd(so.cursor, (unsigned long long)n0) : 0ull)
                 << 16) | (unsigned long long)n0;
  }
  __syncthreads();
  const unsigned long long hb = *sh.gbase;
  const int n = (int)(hb & 0xFFFFull);
  const unsigned long long gb = hb >> 16;
  for (int i = tid; i < n; i += kBlock) {
    if ((long long)(gb + i) < so.capacity) {
      const uint2 r = lds_ld(sh.buf, i);
      stg64(so.out, gb + (unsigned long long)i, evis_event{r.x, (int32_t)r.y});
    }
  }
  __syncthreads();         // copies done (and gbase read) before the buffer is reused
  if (tid == 0) sh.req[0] = sh.req[1] = sh.req[2] = sh.req[3] = 0;
}

// Read the flush requests of the emissions since the last check and flush
// if one is set.  Call it right after a workgroup barrier (every thread).
__device__ __forceinline__ void sink_check(const SinkShared& sh, const SinkOut& so,
                                           SinkRound& sr) {
  if (sr.unchecked == 0) return;
  int want = lds_ld(sh.req, (sr.round - 1) & 3);
  if (sr.unchecked > 1) want |= lds_ld(sh.req, (sr.round - 2) & 3);
  sr.unchecked = 0;
  if (__builtin_amdgcn_readfirstlane(want)) sink_drain(sh, so);
}

// Per-pixel state that only a crossing pixel reads: thresholds, last event
// time, coordinates.  Kept in LDS (index tid + k * kBlock) so that it costs
// no registers across the substep loop.  Pixel (x, y) of slot k is
// (x0 + i % row, y0 + i / row) with i = tid + k * kBlock and `row` pixels
// per row of the workgroup's pixel block (row = W for a flat pixel range).
struct PixAux {
  float* con;       // LDS, or null: C_on everywhere
  float* coff;      // LDS, or null: C_off everywhere
  int* tl;          // LDS
  float C_on, C_off;
  int x0, y0, row;
  int row_shift;    // log2(row) for a tile (row a power of two); unused for a flat range
  long long flat0;  // first pixel of the block when row == W (flat range), else -1
  __device__ __forceinline__ float c_at(int i, bool pos) const {
    if (pos) return con ? lds_ld(con, i) : C_on;
    return coff ? lds_ld(coff, i) : C_off;
  }
  __device__ __forceinline__ float c(int k, bool pos) const { return c_at(threadIdx.x + k * kBlock, pos); }
  __device__ __forceinline__ int tlast(int k) const { return lds_ld(tl, (int)threadIdx.x + k * kBlock); }
  __device__ __forceinline__ void set_tlast_at(int i, int t) const { lds_st(tl, i, t); }
  __device__ __forceinline__ uint32_t xy_at(int i) const {
    long long x, y;
    if (flat0 >= 0) {
      const long long q = flat0 + i;
      x = q % row;
      y = q / row;
    } else {
      x = x0 + (i & (row - 1));
      y = y0 + (i >> row_shift);
    }
    return (uint32_t)x | ((uint32_t)y << 11);
  }
};

// One substep of the event model for the PPT pixels of this thread and the
// wave's compaction.  Every thread of the workgroup must call it (it takes a
// barrier only when two rounds are unchecked).
template <int PPT>
__device__ __forceinline__ void emit_substep(
    int j, const float (&Lj)[PPT], const float (&Lp)[PPT], float (&R)[PPT], const PixAux& aux,
    uint32_t okbits, long long t0, int span, float Dt, int refr, uint32_t env_bits,
    const SinkShared& sh, const SinkOut& so, SinkRound& sr) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  if (sr.unchecked >= 2) {
    __syncthreads();
    sink_check(sh, so, sr);
  }
  int nn[PPT];
  uint32_t posbits = 0;
  int m = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    nn[k] = 0;
    if ((okbits >> k) & 1u) {
      const float d = Lj[k] - R[k];
      const bool pos = d > 0.0f;
      const float c = aux.c(k, pos);
      const float a = fabsf(d);
      if (a >= c && c > 0.0f) {
        // c <= a < 2c (2c is exact) is one crossing: the common case skips
        // the general count
        const int n = (a < c + c) ? 1 : crossing_count(a, c);
        nn[k] = n;
        posbits |= (pos ? 1u : 0u) << k;
        if (refr == 0) {
          m += n;
        } else {
          long long tlk = aux.tlast(k);
          for (int kk = 1; kk <= n; ++kk) {
            const long long t = t0 + crossing_offset(j, kk, R[k], c, pos, Lp[k], Lj[k], Dt, span);
            if (t - tlk >= refr) {
              ++m;
              tlk = t;
            }
          }
        }
      }
    }
  }
  // Wave offsets by prefix sum (skipped when no lane has an event); the
  // wave's slots by one reservation.
  int incl = 0, excl = 0, wtot = 0;
  if (__ballot(m > 0) != 0ull) {   // wave-uniform
    incl = wave_inclusive_scan(m);
    excl = incl - m;
    wtot = __builtin_amdgcn_readlane(incl, kWave - 1);
  }
  const int slot_req = sr.round & 3;
  ++sr.round;
  ++sr.unchecked;
  if (wtot > 0) {   // wave-uniform
    int lb = 0;
    if (lane == kWave - 1) lb = atomicAdd(sh.cnt, wtot);
    lb = __builtin_amdgcn_readlane(lb, kWave - 1);
    // slots [0, n_lds) of the wave go to the buffer, the rest to the stream
    const int n_lds = max(0, min(wtot, sh.cap - lb));
    unsigned long long gbase_w = 0;
    if (n_lds < wtot) {   // wave-uniform
      unsigned long long g = 0;
      if (lane == kWave - 1) g = atomicAdd(so.cursor, (unsigned long long)(wtot - n_lds));
      gbase_w = __shfl(g, kWave - 1, kWave);
    }
    if (lane == kWave - 1 && lb + wtot > sh.cap - sh.cap / 4) lds_st(sh.req, slot_req, 1);
    auto put = [&](int slot, uint32_t word, int t) {
      if (slot < n_lds) {
        lds_st(sh.buf, lb + slot, make_uint2(word, (uint32_t)t));
      } else {
        const unsigned long long idx = gbase_w + (unsigned long long)(slot - n_lds);
        if ((long long)idx < so.capacity) stg64(so.out, idx, evis_event{word, (int32_t)t});
      }
    };
    if (refr == 0 && __ballot(m > 4) == 0ull) {   // no lane has more than four
      // Few events per lane: each lane writes its own, in order.
      int widx = excl;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int n = nn[k];
        if (n > 0) {
          const bool pos = (posbits >> k) & 1u;
          const float c = aux.c(k, pos);
          const int io = tid + k * kBlock;
          const uint32_t word = aux.xy_at(io) | ((pos ? 1u : 0u) << 22) | env_bits;
          int t = 0;
          for (int kk = 1; kk <= n; ++kk) {
            t = (int)(t0 + crossing_offset(j, kk, R[k], c, pos, Lp[k], Lj[k], Dt, span));
            put(widx, word, t);
            ++widx;
          }
          aux.set_tlast_at(io, t);   // the pixel's last event
        }
      }
    } else if (refr == 0) {
      // Expansion: lane l writes events l, l + 64, ... of the wave.  Event e
      // belongs to the lane whose exclusive prefix is the largest <= e; its
      // rank within that lane's events picks the pixel slot and crossing.
      for (int e = lane; e - lane < wtot; e += kWave) {
        int o = 0;
#pragma unroll
        for (int step = kWave / 2; step >= 1; step >>= 1) {
          const int ex = __shfl(excl, o + step, kWave);
          if (ex <= e) o += step;
        }
        const int r = e - __shfl(excl, o, kWave);
        int k = PPT - 1, before = 0;
        bool found = false;
        int cnt_k = 0;
        float Rk = 0.0f, Lpk = 0.0f, Ljk = 0.0f;
        const uint32_t pb = (uint32_t)__shfl((int)posbits, o, kWave);
#pragma unroll
        for (int sl = 0; sl < PPT; ++sl) {
          const int cs = __shfl(nn[sl], o, kWave);
          const float rs = __shfl(R[sl], o, kWave);
          const float ps = __shfl(Lp[sl], o, kWave);
          const float js = __shfl(Lj[sl], o, kWave);
          if (!found && r < before + cs) {
            found = true;
            k = sl;
            cnt_k = cs;
            Rk = rs;
            Lpk = ps;
            Ljk = js;
          } else if (!found) {
            before += cs;
          }
        }
        if (e < wtot) {
          const int kk = r - before + 1;
          const bool pos = (pb >> k) & 1u;
          const int io = wave * kWave + o + k * kBlock;
          const float c = aux.c_at(io, pos);
          const long long t = t0 + crossing_offset(j, kk, Rk, c, pos, Lpk, Ljk, Dt, span);
          put(e, aux.xy_at(io) | ((pos ? 1u : 0u) << 22) | env_bits, (int)t);
          if (kk == cnt_k) aux.set_tlast_at(io, (int)t);   // the pixel's last event
        }
      }
    } else if (m > 0) {
      // Refractory period: a pixel's crossings are filtered in order.
      int widx = excl;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int n = nn[k];
        if (n > 0) {
          const bool pos = (posbits >> k) & 1u;
          const float c = aux.c(k, pos);
          const int io = tid + k * kBlock;
          const uint32_t word = aux.xy_at(io) | ((pos ? 1u : 0u) << 22) | env_bits;
          for (int kk = 1; kk <= n; ++kk) {
            const long long t = t0 + crossing_offset(j, kk, R[k], c, pos, Lp[k], Lj[k], Dt, span);
            if (t - (long long)aux.tlast(k) >= refr) {
              put(widx, word, (int)t);
              ++widx;
              aux.set_tlast_at(io, (int)t);
            }
          }
        }
      }
    }
  }
  // The reference moves by n*c for every crossing, emitted or suppressed.
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    if (nn[k] > 0) {
      const bool pos = (posbits >> k) & 1u;
      const float c = aux.c(k, pos);
      const float nc = (float)nn[k] * c;
      R[k] = pos ? (R[k] + nc) : (R[k] - nc);
    }
  }
}

// ---------------------------------------------------------------------------
// Deferred emission (no refractory period): the crossing pixels of each
// substep are appended to a queue of the wave in LDS, and their events are
// timed and written when the queue is full and after the last substep, one
// queue entry per lane.  A substep then costs every pixel only its count
// and the reference update; the timestamp (a correctly rounded division
// among other things) runs with nearly every lane busy, instead of once per
// pixel slot whenever any lane of the wave crosses.  Without a refractory
// period the crossings of a pixel are independent of each other, so their
// order does not matter; the pixel's last event time, kept for the next
// pair, is the largest (times grow with the substep and the crossing), so
// it is taken with an atomic maximum over an array that starts at INT_MIN
// for every item (unchanged pixels keep the caller's value).
// ---------------------------------------------------------------------------

constexpr int kCrossQ = 64;   // queue entries per wave

// Entry: (reference before the substep, previous sample, current sample,
// pixel index | substep << 11 | polarity << 19).
struct CrossQueue {
  float4* q;   // LDS [kWavesPerBlock * kCrossQ]
  int n = 0;   // entries this wave holds (wave-uniform)
};

__device__ __forceinline__ void lds_atomic_max(int* p, int idx, int v) {
#if defined(__HIP_DEVICE_COMPILE__)
  __hip_atomic_fetch_max(((__attribute__((address_space(3))) int*)p) + idx, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
#else
  p[idx] = v > p[idx] ? v : p[idx];
#endif
}

// Time and write the events of every queued entry (the wave's lanes take
// one entry each) and empty the queue.  Wave-level: no barrier.
__device__ __forceinline__ void cq_drain(CrossQueue& cq, const PixAux& aux, long long t0, int span,
                                         float Dt, uint32_t env_bits, const SinkShared& sh,
                                         const SinkOut& so, int slot_req) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const bool v = lane < cq.n;
  const float4 e = v ? lds_ld(cq.q, wave * kCrossQ + lane) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  cq.n = 0;
  const uint32_t meta = __float_as_uint(e.w);
  const int io = (int)(meta & 0x7FFu), j = (int)((meta >> 11) & 0xFFu);
  const bool pos = ((meta >> 19) & 1u) != 0u;
  const float R = e.x, Lp = e.y, Lj = e.z;
  const float c = aux.c_at(io, pos);
  int n = 0;
  if (v) {   // the same count the substep took (same values, same operations)
    const float a = fabsf(Lj - R);
    n = (a < c + c) ? 1 : crossing_count(a, c);
  }
  const int incl = wave_inclusive_scan(n);
  const int excl = incl - n;
  const int wtot = __builtin_amdgcn_readlane(incl, kWave - 1);
  int lb = 0;
  if (lane == kWave - 1) lb = atomicAdd(sh.cnt, wtot);
  lb = __builtin_amdgcn_readlane(lb, kWave - 1);
  // slots [0, n_lds) of the wave go to the buffer, the rest to the stream
  const int n_lds = max(0, min(wtot, sh.cap - lb));
  unsigned long long gbase_w = 0;
  if (n_lds < wtot) {   // wave-uniform
    unsigned long long g = 0;
    if (lane == kWave - 1) g = atomicAdd(so.cursor, (unsigned long long)(wtot - n_lds));
    gbase_w = __shfl(g, kWave - 1, kWave);
  }
  if (lane == kWave - 1 && lb + wtot > sh.cap - sh.cap / 4) lds_st(sh.req, slot_req, 1);
  auto put = [&](int slot, uint32_t word, int t) {
    if (slot < n_lds) {
      lds_st(sh.buf, lb + slot, make_uint2(word, (uint32_t)t));
    } else {
      const unsigned long long idx = gbase_w + (unsigned long long)(slot - n_lds);
      if ((long long)idx < so.capacity) stg64(so.out, idx, evis_event{word, (int32_t)t});
    }
  };
  if (__ballot(n > 4) == 0ull) {   // wave-uniform: few events per entry
    const uint32_t word = aux.xy_at(io) | ((pos ? 1u : 0u) << 22) | env_bits;
    int t = 0;
    for (int kk = 1; kk <= n; ++kk) {
      t = (int)(t0 + crossing_offset(j, kk, R, c, pos, Lp, Lj, Dt, span));
      put(excl + kk - 1, word, t);
    }
    if (n > 0) lds_atomic_max(aux.tl, io, t);
  } else {
    // Expansion: lane l writes events l, l + 64, ... of the wave.  Event s
    // belongs to the lane whose exclusive prefix is the largest <= s.
    for (int s = lane; s - lane < wtot; s += kWave) {
      int o = 0;
#pragma unroll
      for (int step = kWave / 2; step >= 1; step >>= 1) {
        const int ex = __shfl(excl, o + step, kWave);
        if (ex <= s) o += step;
      }
      const int kk = s - __shfl(excl, o, kWave) + 1;
      const float Ro = __shfl(R, o, kWave), Lpo = __shfl(Lp, o, kWave), Ljo = __shfl(Lj, o, kWave);
      const float co = __shfl(c, o, kWave);
      const uint32_t mo = (uint32_t)__shfl((int)meta, o, kWave);
      const int no = __shfl(n, o, kWave);
      if (s < wtot) {
        const int ioo = (int)(mo & 0x7FFu), jo = (int)((mo >> 11) & 0xFFu);
        const bool po = ((mo >> 19) & 1u) != 0u;
        const int t = (int)(t0 + crossing_offset(jo, kk, Ro, co, po, Lpo, Ljo, Dt, span));
        put(s, aux.xy_at(ioo) | ((po ? 1u : 0u) << 22) | env_bits, t);
        if (kk == no) lds_atomic_max(aux.tl, ioo, t);
      }
    }
  }
}

// One substep of the event model without a refractory period: counts and
// reference updates now, the crossing pixels queued (see above); `last`
// (the pair's final substep) drains the queue.  Every thread of the
// workgroup must call it, like emit_substep.
template <int PPT>
__device__ __forceinline__ void emit_queued(
    int j, bool last, const float (&Lj)[PPT], const float (&Lp)[PPT], float (&R)[PPT],
    const PixAux& aux, uint32_t okbits, long long t0, int span, float Dt, uint32_t env_bits,
    const SinkShared& sh, const SinkOut& so, SinkRound& sr, CrossQueue& cq) {
  const int tid = threadIdx.x, wave = tid / kWave;
  if (sr.unchecked >= 2) {
    __syncthreads();
    sink_check(sh, so, sr);
  }
  const int slot_req = sr.round & 3;
  ++sr.round;
  ++sr.unchecked;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    int n = 0;
    bool pos = false;
    float c = 0.0f;
    if ((okbits >> k) & 1u) {
      const float d = Lj[k] - R[k];
      pos = d > 0.0f;
      c = aux.c(k, pos);
      const float a = fabsf(d);
      // c <= a < 2c (2c is exact) is one crossing: the common case skips
      // the general count
      if (a >= c && c > 0.0f) n = (a < c + c) ? 1 : crossing_count(a, c);
    }
    const unsigned long long bal = __ballot(n > 0);
    if (bal != 0ull) {   // wave-uniform
      const int cnt = (int)__popcll(bal);
      if (cq.n + cnt > kCrossQ) cq_drain(cq, aux, t0, span, Dt, env_bits, sh, so, slot_req);
      if (n > 0) {
        const int rank = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        const uint32_t meta = (uint32_t)(tid + k * kBlock) | ((uint32_t)j << 11) |
                              ((pos ? 1u : 0u) << 19);
        lds_st(cq.q, wave * kCrossQ + cq.n + rank, make_float4(R[k], Lp[k], Lj[k], __uint_as_float(meta)));
        // the reference moves by n*c for every crossing
        const float nc = (float)n * c;
        R[k] = pos ? (R[k] + nc) : (R[k] - nc);
      }
      cq.n += cnt;
    }
  }
  if (last && cq.n > 0) cq_drain(cq, aux, t0, span, Dt, env_bits, sh, so, slot_req);
}

__device__ __forceinline__ NoiseCfg noise_cfg(const EnvDesc& d, float Dt) {
  const float dts = Dt * 1e-6f;
  return NoiseCfg{d.leak_hz * dts, d.shot_hz * dts, d.hot_hz * dts, d.shot_L0, d.shot_inv,
                  d.hot_frac, d.seed_lo, d.seed_hi, d.pair_index};
}

// Hot-pixel membership of this thread's pixels (bit k for slot k).
template <int PPT>
__device__ __forceinline__ uint32_t hot_bits(const NoiseCfg& nc, const PixAux& aux, uint32_t okbits) {
  uint32_t hb = 0;
  if (nc.p_hot > 0.0f) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const uint4 w = philox4x32_10(make_uint4(aux.xy_at(threadIdx.x + k * kBlock), 0u, 0u, 4u),
                                    nc.k0, nc.k1);
      hb |= (((okbits >> k) & 1u) && uniform24(w.x) < nc.hot_frac ? 1u : 0u) << k;
    }
  }
  return hb;
}

// Leak, shot and hot-pixel events of substep j (Lj the current samples).
// Call right after emit_substep of the same substep (every thread): the
// events are staged like the crossings and share that emission's flush
// request slot, so the sink's round accounting does not change.
template <int PPT>
__device__ __forceinline__ void emit_noise(int j, const float (&Lj)[PPT], const PixAux& aux,
                                           uint32_t okbits, uint32_t hotbits, const NoiseCfg& nc,
                                           long long t0, int span, float Dt, uint32_t env_bits,
                                           const SinkShared& sh, const SinkOut& so,
                                           const SinkRound& sr) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  uint32_t fired = 0;   // 3 bits per slot: leak, shot, hot
  int m = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    if ((okbits >> k) & 1u) {
      const uint4 w = philox4x32_10(
          make_uint4(aux.xy_at(tid + k * kBlock), (uint32_t)j, nc.pair, 0u), nc.k0, nc.k1);
      float ib = (Lj[k] - nc.shot_L0) * nc.shot_inv;
      ib = (ib > 0.0f) ? ib : 0.0f;
      ib = (ib < 1.0f) ? ib : 1.0f;
      const float p_shot = nc.shot_scale * (1.0f - ib);
      const uint32_t f = (uniform24(w.x) < nc.p_leak ? 1u : 0u) |
                         (uniform24(w.y) < p_shot ? 2u : 0u) |
                         (((hotbits >> k) & 1u) && uniform24(w.z) < nc.p_hot ? 4u : 0u);
      fired |= f << (3 * k);
      m += __builtin_popcount(f);
    }
  }
  if (__ballot(m > 0) == 0ull) return;   // wave-uniform
  const int incl = wave_inclusive_scan(m);
  const int wtot = __builtin_amdgcn_readlane(incl, kWave - 1);
  int lb = 0;
  if (lane == kWave - 1) lb = atomicAdd(sh.cnt, wtot);
  lb = __builtin_amdgcn_readlane(lb, kWave - 1);
  const int n_lds = max(0, min(wtot, sh.cap - lb));
  unsigned long long gbase_w = 0;
  if (n_lds < wtot) {   // wave-uniform
    unsigned long long g = 0;
    if (lane == kWave - 1) g = atomicAdd(so.cursor, (unsigned long long)(wtot - n_lds));
    gbase_w = __shfl(g, kWave - 1, kWave);
  }
  if (lane == kWave - 1 && lb + wtot > sh.cap - sh.cap / 4) lds_st(sh.req, (sr.round - 1) & 3, 1);
  int widx = incl - m;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const uint32_t f = (fired >> (3 * k)) & 7u;
    if (f) {
      const uint32_t xy = aux.xy_at(tid + k * kBlock);
      for (uint32_t kind = 1; kind <= 3; ++kind) {
        if (!((f >> (kind - 1)) & 1u)) continue;
        const uint4 e = philox4x32_10(make_uint4(xy, (uint32_t)j, nc.pair, kind), nc.k0, nc.k1);
        const float v = ((float)(j - 1) + uniform24(e.x)) * Dt;
        const int t = (int)(t0 + min((int)floorf(v), span));
        const uint32_t pol = (kind == 1u) ? 1u : (e.y & 1u);
        const uint32_t word = xy | (pol << 22) | env_bits;
        if (widx < n_lds) {
          lds_st(sh.buf, lb + widx, make_uint2(word, (uint32_t)t));
        } else {
          const unsigned long long idx = gbase_w + (unsigned long long)(widx - n_lds);
          if ((long long)idx < so.capacity) stg64(so.out, idx, evis_event{word, (int32_t)t});
        }
        ++widx;
      }
    }
  }
}

// Write out whatever is still staged.  Every thread must call it.
__device__ __forceinline__ void sink_flush(const SinkShared& sh, const SinkOut& so) {
  __syncthreads();
  sink_drain(sh, so);
}

}  // namespace evis
