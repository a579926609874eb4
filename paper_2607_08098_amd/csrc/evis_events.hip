// Elementwise front end, state initialisation, the substep count of one
// pair, and the event model over caller-supplied frames (gfx950).
#include "evis_internal.h"
#include "evis_sink.h"
#include "evis_stream.h"

namespace evis {

static int grid_for(long long n, int per_block) {
  long long g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 65535LL * 16) g = 65535LL * 16;
  return (int)g;
}


// Log intensity: Eq. 3 luminance, then ln(Y + eps).
__global__ __launch_bounds__(kBlock) void k_log_luminance(const float* __restrict__ x, int channels,
                                                          long long n, float eps,
                                                          float* __restrict__ L) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float Y;
    if (channels == 3) {
      const float r = x[3 * i], g = x[3 * i + 1], b = x[3 * i + 2];
      Y = 0.2126f * r + 0.7152f * g + 0.0722f * b;
    } else {
      Y = x[i];
    }
    L[i] = logf(Y + eps);
  }
}

// Colour events: each channel's own log, channel-major output.
__global__ __launch_bounds__(kBlock) void k_log_channels(const float* __restrict__ x, long long n,
                                                         float eps, float* __restrict__ L) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float r = x[3 * i], g = x[3 * i + 1], b = x[3 * i + 2];
    L[i] = logf(r + eps);
    L[n + i] = logf(g + eps);
    L[2 * n + i] = logf(b + eps);
  }
}

__global__ __launch_bounds__(kBlock) void k_state_init(const float* __restrict__ L, long long n,
                                                       float* __restrict__ Lref,
                                                       int32_t* __restrict__ tlast) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    Lref[i] = L[i];
    if (tlast) tlast[i] = EVIS_T_LAST_INIT;
  }
}

// Substep count of one pair: largest finite |m|^2 (float64) over both fields.
__global__ __launch_bounds__(kBlock) void k_msq(const float2* __restrict__ mA,
                                                const float2* __restrict__ mB, long long n,
                                                unsigned long long* msq_bits) {
  double best = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float2 a = mA[i], b = mB[i];
    const double ma = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
    const double mb = (double)b.x * (double)b.x + (double)b.y * (double)b.y;
    if (ma <= 1.7976931348623157e308 && ma > best) best = ma;
    if (mb <= 1.7976931348623157e308 && mb > best) best = mb;
  }
  best = wave_max_d(best);
  if ((threadIdx.x & (kWave - 1)) == 0 && best > 0.0)
    atomicMax(msq_bits, (unsigned long long)__double_as_longlong(best));
}

__global__ void k_k_from_msq(const unsigned long long* msq_bits, int K_max, int32_t* K_out) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    *K_out = exact_k(__longlong_as_double((long long)*msq_bits), K_max);
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

// ---------------------------------------------------------------------------
// The event model over caller frames (Eq. 4 crossings with Eq. 8 thresholds,
// interpolated timestamps, the refractory period), in two forms:
//
// * wave form (no refractory period, no noise): the waves of a workgroup do
//   not wait for each other.  Lane l's pixel slot k is pixel
//   wbase + k * kWave + l of its wave's kWave * PPT consecutive pixels.
//   Crossings are queued per wave, as in the fused step, and timed when the
//   queue fills; their events are staged in the wave's own LDS buffer, which
//   the wave appends to the stream with one atomic whenever it would
//   overflow, and once at the end.
// * workgroup form (refractory period or noise): the fused step's shared
//   sink (evis_sink.h), whose flush checks take a workgroup barrier every
//   two substeps.
//
// Both read each of the K + 1 frames once, AHEAD substeps ahead of their
// use, so that enough loads are in flight to keep HBM busy.
// ---------------------------------------------------------------------------

constexpr int kWaveEv = 256;   // events staged per wave

// Crossing ring of a wave: room for the kWave - 1 entries left over from
// the last drain plus one substep's kWave * PPT, rounded up to a power of two.
template <int PPT>
constexpr int wave_ring() { return PPT == 1 ? 128 : (PPT == 2 ? 256 : 512); }

template <int PPT>
struct WaveLds {
  float4 cq[wave_ring<PPT>()];   // crossing ring
  uint2 ev[kWaveEv];             // staged events
  int tl[kWave * PPT];           // largest event time of each pixel (INT_MIN: none)
  float con[kWave * PPT], coff[kWave * PPT];   // per-pixel thresholds (Eq. 8), if any
};

template <int PPT>
struct BlockLds {
  uint2 ev[kEventBuf];
  float4 cq[kWavesPerBlock * kCrossQ];
  float con[kBlock * PPT], coff[kBlock * PPT];
  int tl[kBlock * PPT];
  unsigned long long gbase;
  int evn, req[4];
};

// Where the wave form's events go: the sharded stream of the call
// (evis_stream.h); each wave reserves on stream `s`.
struct WaveOut {
  StreamState st;
  long long base;   // cursor at the start of the call
  int gmax;
  int s;
  evis_event* out;
  long long capacity;
};

__device__ __forceinline__ WaveOut wave_out(const StreamState& st, evis_event* out,
                                            long long capacity) {
  const int wave_id = (int)blockIdx.x * kWavesPerBlock + (int)(threadIdx.x / kWave);
  return WaveOut{st, st.hdr->base, st.hdr->gmax, wave_id % kStreams, out, capacity};
}

// Reserve n stream slots for the whole wave (one lane reserves, every lane
// gets the first slot).  Wave-uniform control flow.
__device__ __forceinline__ unsigned long long wave_reserve(const WaveOut& wo, unsigned long long n) {
  unsigned long long i0 = 0;
  if ((threadIdx.x & (kWave - 1)) == 0) i0 = stream_reserve_lane(wo.st, wo.gmax, wo.s, n);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)i0, 0);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(i0 >> 32), 0);
  return ((unsigned long long)hi << 32) | lo;
}

// Events a wave has staged in LDS (n is wave-uniform).
struct WaveSink {
  uint2* ev;
  int n;
};

// Wait until every vector memory access of the wave has completed
// (s_waitcnt vmcnt(0), the other counters left alone; gfx9 encoding).  On
// gfx950 one counter covers loads and stores, and the compiler cannot tell
// how far a load is in that counter while a store is pending, so it waits
// for everything before the next use of any loaded value; a wait right
// after the (rare) event stores ends that state at once.
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Append the wave's n <= kStreamChunk staged events to the stream: they span at
// most two blocks of the wave's stream.
__device__ __forceinline__ void wave_flush(WaveSink& ws, const WaveOut& wo) {
  if (ws.n == 0) return;
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned long long i0 = wave_reserve(wo, (unsigned long long)ws.n);
  const long long k0 = (long long)(i0 >> kStreamChunkLog);
  const long long k1 = (long long)((i0 + ws.n - 1) >> kStreamChunkLog);
  const int g0 = stream_chunk(wo.st, wo.s, k0);
  const int g1 = (k1 != k0) ? stream_chunk(wo.st, wo.s, k1) : g0;
  for (int i = lane; i < ws.n; i += kWave) {
    const unsigned long long slot = i0 + (unsigned long long)i;
    const int g = ((long long)(slot >> kStreamChunkLog) == k0) ? g0 : g1;
    evis_event* p = stream_slot_ptr(wo.st, wo.base, g, slot, wo.out, wo.capacity);
    if (p) {
      const uint2 r = lds_ld(ws.ev, i);
      stg64(p, 0ull, evis_event{r.x, (int32_t)r.y});
    }
  }
  wait_vm_all();
  ws.n = 0;
}

// Store event `e` at stream slot `slot` of a reservation that may span
// many blocks (each lane finds its own chunk; rare).
__device__ __forceinline__ void wave_put_direct(const WaveOut& wo, unsigned long long slot,
                                                evis_event e) {
  const int g = stream_chunk(wo.st, wo.s, (long long)(slot >> kStreamChunkLog));
  evis_event* p = stream_slot_ptr(wo.st, wo.base, g, slot, wo.out, wo.capacity);
  if (p) stg64(p, 0ull, e);
}

// What the wave form's crossing timer needs besides the queue entries.
struct WaveCtx {
  float C_on, C_off;
  const float* con;    // LDS per-pixel thresholds, or null: C_on everywhere
  const float* coff;
  int* tl;             // LDS
  int wbase, W;
  int x0, y0;          // column and row of pixel wbase
  long long t0;
  int span;
  float Dt;
  uint32_t env_bits;
};

// Time the events of the ntake <= kWave queued crossings from ring slot
// head (lane l takes entry head + l) and stage them.  Wave-uniform control
// flow.
template <int QR>
__device__ __forceinline__ void wave_drain(int head, int ntake, const float4* cq, const WaveCtx& w,
                                           WaveSink& ws, const WaveOut& wo) {
  const int lane = threadIdx.x & (kWave - 1);
  const bool v = lane < ntake;
  const float4 e = v ? lds_ld(cq, (head + lane) & (QR - 1)) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const uint32_t meta = __float_as_uint(e.w);
  const int io = (int)(meta & 0x7FFu), j = (int)((meta >> 11) & 0xFFu);
  const bool pos = ((meta >> 19) & 1u) != 0u;
  const float R = e.x, Lp = e.y, Lj = e.z;
  // no global load here: a load would make this wait for every frame
  // load in flight
  const float c = pos ? (w.con ? lds_ld(w.con, io) : w.C_on) : (w.coff ? lds_ld(w.coff, io) : w.C_off);
  int n = 0;
  if (v) {   // the count the substep took (same values, same operations)
    const float a = fabsf(Lj - R);
    n = (a < c + c) ? 1 : crossing_count(a, c);
  }
  const int incl = wave_inclusive_scan(n);
  const int excl = incl - n;
  const int wtot = __builtin_amdgcn_readlane(incl, kWave - 1);
  if (ws.n + wtot > kWaveEv) wave_flush(ws, wo);
  const bool direct = wtot > kWaveEv;   // uniform: more than the buffer holds
  const unsigned long long g = direct ? wave_reserve(wo, (unsigned long long)wtot) : 0ull;
  const int sb = ws.n;
  auto put = [&](int slot, uint32_t word, int t) {
    if (!direct)
      lds_st(ws.ev, sb + slot, make_uint2(word, (uint32_t)t));
    else
      wave_put_direct(wo, g + (unsigned long long)slot, evis_event{word, (int32_t)t});
  };
  // event word of wave pixel i: x | y << 11 | polarity << 22 | env << 23
  // (the wave's first pixel is (x0, y0); pixel i is i columns on, wrapped)
  auto word_of = [&](int i, bool p) {
    uint32_t x = (uint32_t)(w.x0 + i), y = (uint32_t)w.y0;
    while (x >= (uint32_t)w.W) {
      x -= (uint32_t)w.W;
      ++y;
    }
    return x | (y << 11) | ((p ? 1u : 0u) << 22) | w.env_bits;
  };
  if (__ballot(n > 4) == 0ull) {   // wave-uniform: few events per entry
    const uint32_t word = word_of(io, pos);
    int t = 0;
    for (int kk = 1; kk <= n; ++kk) {
      t = (int)(w.t0 + crossing_offset(j, kk, R, c, pos, Lp, Lj, w.Dt, w.span));
      put(excl + kk - 1, word, t);
    }
    if (n > 0) lds_atomic_max(w.tl, io, t);
  } else {
    // Expansion: lane l times events l, l + 64, ... of the wave.  Event s
    // belongs to the entry whose exclusive prefix is the largest <= s.
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
        const int t = (int)(w.t0 + crossing_offset(jo, kk, Ro, co, po, Lpo, Ljo, w.Dt, w.span));
        put(s, word_of(ioo, po), t);
        if (kk == no) lds_atomic_max(w.tl, ioo, t);
      }
    }
  }
  if (direct) wait_vm_all();
  else ws.n += wtot;
}

// Wave form over the kWave * PPT pixels of one env from wbase (every lane
// of the wave calls it; no lane waits for another wave).  Substeps go in
// blocks of U: while a block is processed from registers (frames j0 - 1 ..
// j0 + U - 1), the loads of the next block's U frames are in flight, so
// each wave keeps U loads per pixel outstanding and waits once per block,
// for loads issued a whole block earlier.  A frame's base address is
// wave-uniform and each lane adds a 32-bit offset.  Crossing pixels are
// appended to the wave's ring, which is drained kWave entries at a time
// after each substep while it holds that many.
template <int PPT, int U>
__device__ __forceinline__ void events_wave(const EventArgs& a, const StreamState& st, int wbase,
                                            WaveLds<PPT>& L) {
  constexpr int QR = wave_ring<PPT>();
  const int lane = threadIdx.x & (kWave - 1);
  const int plane = a.H * a.W;
  const int K = a.K;
  const WaveOut so = wave_out(st, a.out, a.capacity);
  float R[PPT], con[PPT], coff[PPT], cur[U + 1][PPT], nxt[U][PPT];
  int off[PPT];
  uint32_t okbits = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int i = k * kWave + lane;
    const int q = wbase + i;
    const bool ok = q < plane;
    okbits |= (ok ? 1u : 0u) << k;
    off[k] = ok ? q : 0;   // a slot past the end reads pixel 0 and never crosses
    R[k] = ok ? ldg(a.Lref, q) : 0.0f;
    // a per-pixel threshold that is not > 0 never crosses: NaN fails every
    // comparison, so the substep needs no test of its own for it
    con[k] = a.th_on ? ldg(a.th_on, off[k]) : a.C_on;
    coff[k] = a.th_off ? ldg(a.th_off, off[k]) : a.C_off;
    con[k] = con[k] > 0.0f ? con[k] : __builtin_nanf("");
    coff[k] = coff[k] > 0.0f ? coff[k] : __builtin_nanf("");
    if (a.th_on) lds_st(L.con, i, con[k]);
    if (a.th_off) lds_st(L.coff, i, coff[k]);
    lds_st(L.tl, i, INT_MIN);
  }
  // the first block: frames 0 .. U (those past K are never used)
#pragma unroll
  for (int v = 0; v <= U; ++v) {
    const float* fr = a.L_seq + (long long)min(v, K) * plane;
#pragma unroll
    for (int k = 0; k < PPT; ++k) cur[v][k] = ldg(fr, off[k]);
  }
  const WaveCtx w{a.C_on, a.C_off, a.th_on ? L.con : nullptr, a.th_off ? L.coff : nullptr, L.tl,
                  wbase, a.W, wbase % a.W, wbase / a.W, a.t0, a.span, a.Dt, a.env_bits};
  WaveSink ws{L.ev, 0};
  int head = 0, qn = 0;   // ring: entries [head, head + qn) (mod QR)
  for (int j0 = 1; j0 <= K; j0 += U) {
    // the next block's frames j0 + U .. j0 + 2U - 1 (those that exist)
#pragma unroll
    for (int v = 0; v < U; ++v) {
      if (j0 + U + v <= K) {   // uniform
        const float* fr = a.L_seq + (long long)(j0 + U + v) * plane;
#pragma unroll
        for (int k = 0; k < PPT; ++k) nxt[v][k] = ldg(fr, off[k]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u;
      if (j > K) break;   // uniform
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const float Lj = cur[u + 1][k], Lp = cur[u][k];
        const float d = Lj - R[k];
        const bool pos = d > 0.0f;
        const float c = pos ? con[k] : coff[k];
        const float ad = fabsf(d);
        const bool hit = ((okbits >> k) & 1u) && ad >= c;
        const unsigned long long bal = __ballot(hit);
        if (hit) {
          // c <= |d| < 2c (2c is exact) is one crossing: the common case
          // skips the general count
          const int n = (ad < c + c) ? 1 : crossing_count(ad, c);
          const int rank = (int)__builtin_amdgcn_mbcnt_hi(
              (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
          const uint32_t meta = (uint32_t)(k * kWave + lane) | ((uint32_t)j << 11) |
                                ((pos ? 1u : 0u) << 19);
          lds_st(L.cq, (head + qn + rank) & (QR - 1),
                 make_float4(R[k], Lp, Lj, __uint_as_float(meta)));
          // the reference moves by n c for every crossing
          const float nc = (float)n * c;
          R[k] = pos ? (R[k] + nc) : (R[k] - nc);
        }
        qn += (int)__popcll(bal);
      }
      while (qn >= kWave) {   // uniform
        wave_drain<QR>(head, kWave, L.cq, w, ws, so);
        head = (head + kWave) & (QR - 1);
        qn -= kWave;
      }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      cur[0][k] = cur[U][k];
#pragma unroll
      for (int v = 0; v < U; ++v) cur[v + 1][k] = nxt[v][k];
    }
  }
  if (qn > 0) wave_drain<QR>(head, qn, L.cq, w, ws, so);
  wave_flush(ws, so);
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    if ((okbits >> k) & 1u) {
      const int q = wbase + k * kWave + lane;
      stg(a.Lref, q, R[k]);
      const int tl = lds_ld(L.tl, k * kWave + lane);
      if (a.tlast && tl != INT_MIN) stg(a.tlast, q, tl);
    }
  }
}

// Workgroup form over the kBlock * PPT consecutive pixels from `base` of
// one env's frames (pixel slot k of thread t: base + t + k * kBlock; every
// thread of the workgroup calls it).
template <int PPT, int NOISE, int AHEAD>
__device__ __forceinline__ void events_block(const EventArgs& a, long long base, BlockLds<PPT>& L) {
  const SinkShared sh{L.ev, &L.evn, L.req, &L.gbase, kEventBuf};
  const SinkOut so{a.out, a.capacity, a.cursor};
  const int tid = threadIdx.x;
  const long long plane = (long long)a.H * a.W;
  // Frames are read AHEAD substeps ahead of their use (a ring of registers
  // shifted by one each substep).
  float R[PPT], Lp[PPT], Lj[PPT], Ln[AHEAD][PPT];
  uint32_t okbits = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int i = tid + k * kBlock;
    const long long q = base + i;
    const bool ok = q < plane;
    okbits |= (ok ? 1u : 0u) << k;
    R[k] = ok ? ldg(a.Lref, (int)q) : 0.0f;
    // without a refractory period t_last is only written: keep the largest
    // event time of each pixel (INT_MIN: none)
    L.tl[i] = (a.refr == 0) ? INT_MIN : ((ok && a.tlast) ? ldg(a.tlast, (int)q) : EVIS_T_LAST_INIT);
    if (a.th_on) L.con[i] = ok ? ldg(a.th_on, (int)q) : 1.0f;
    if (a.th_off) L.coff[i] = ok ? ldg(a.th_off, (int)q) : 1.0f;
    Lp[k] = ok ? ldg(a.L_seq, (int)q) : 0.0f;
#pragma unroll
    for (int u = 0; u < AHEAD; ++u)
      Ln[u][k] = (ok && u + 1 <= a.K) ? ldg(a.L_seq + (long long)(u + 1) * plane, (int)q) : 0.0f;
  }
  const PixAux aux{a.th_on ? L.con : nullptr, a.th_off ? L.coff : nullptr, L.tl, a.C_on, a.C_off,
                   0, 0, a.W, 0, base};
  uint32_t hotb = 0;
  if constexpr (NOISE != 0) hotb = hot_bits<PPT>(a.noise, aux, okbits);
  SinkRound sr;
  CrossQueue cq{L.cq};
  sink_init(sh);
  __syncthreads();
  for (int j = 1; j <= a.K; ++j) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      Lj[k] = Ln[0][k];
#pragma unroll
      for (int u = 0; u + 1 < AHEAD; ++u) Ln[u][k] = Ln[u + 1][k];
      Ln[AHEAD - 1][k] = (((okbits >> k) & 1u) && j + AHEAD <= a.K)
                             ? ldg(a.L_seq + (long long)(j + AHEAD) * plane, (int)(base + tid + k * kBlock))
                             : 0.0f;
    }
    if (a.refr == 0)   // uniform
      emit_queued<PPT>(j, j == a.K, Lj, Lp, R, aux, okbits, a.t0, a.span, a.Dt, a.env_bits, sh, so,
                       sr, cq);
    else
      emit_substep<PPT>(j, Lj, Lp, R, aux, okbits, a.t0, a.span, a.Dt, a.refr, a.env_bits, sh, so,
                        sr);
    if constexpr (NOISE != 0)
      emit_noise<PPT>(j, Lj, aux, okbits, hotb, a.noise, a.t0, a.span, a.Dt, a.env_bits, sh, so, sr);
#pragma unroll
    for (int k = 0; k < PPT; ++k) Lp[k] = Lj[k];
  }
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    if ((okbits >> k) & 1u) {
      const long long q = base + tid + k * kBlock;
      stg(a.Lref, (int)q, R[k]);
      const int tl = L.tl[tid + k * kBlock];
      if (a.tlast && (a.refr != 0 || tl != INT_MIN)) stg(a.tlast, (int)q, tl);
    }
  }
  sink_flush(sh, so);
}

// The wave form's schedule: pixels per lane, substeps per block (frames in
// flight per pixel), and the waves per SIMD its registers are bounded for
// (eight substeps per block need 69 VGPRs: seven waves); the workgroup
// form is not bounded and loads four frames ahead.  Both forms take
// kEventsPPT pixels per lane in a batched launch, where the workgroups of
// an env are counted before the form is known.
constexpr int kEventsPPT = 1;
constexpr int kEventsWaveU = 8;
constexpr int kEventsWaveOcc = 7;
constexpr int kEventsBlockAhead = 4;

template <int PPT, int NOISE>
__global__ __launch_bounds__(kBlock) void k_events(const EventArgs a) {
  __shared__ BlockLds<PPT> L;
  events_block<PPT, NOISE, 4>(a, (long long)blockIdx.x * (kBlock * PPT), L);
}

template <int PPT, int AHEAD>
__global__ __launch_bounds__(kBlock, kEventsWaveOcc) void k_events_wave(const EventArgs a,
                                                                        const StreamState st) {
  __shared__ WaveLds<PPT> L[kWavesPerBlock];
  const int wave = threadIdx.x / kWave;
  events_wave<PPT, AHEAD>(a, st, (int)blockIdx.x * (kBlock * PPT) + wave * (kWave * PPT), L[wave]);
}

// Env of workgroup b in a batched launch: the last e whose first workgroup
// prefix[e] is <= b (descriptors and prefix in device memory, read through
// the scalar cache).
__device__ __forceinline__ int batch_env(const int32_t* __restrict__ prefix, int n_envs, int b) {
  int lo = 0, hi = n_envs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int PPT, int AHEAD>
__global__ __launch_bounds__(kBlock, kEventsWaveOcc) void k_events_batch_wave(
    const EventArgs* __restrict__ descs, const int32_t* __restrict__ prefix, int n_envs,
    const StreamState st) {
  __shared__ WaveLds<PPT> L[kWavesPerBlock];
  const int b = blockIdx.x;
  const int e = batch_env(prefix, n_envs, b);
  const EventArgs a = descs[e];
  const int wave = threadIdx.x / kWave;
  events_wave<PPT, AHEAD>(a, st, (b - prefix[e]) * (kBlock * PPT) + wave * (kWave * PPT), L[wave]);
}

template <int PPT, int AHEAD>
__global__ __launch_bounds__(kBlock) void k_events_batch(const EventArgs* __restrict__ descs,
                                                         const int32_t* __restrict__ prefix,
                                                         int n_envs) {
  __shared__ BlockLds<PPT> L;
  const int b = blockIdx.x;
  const int e = batch_env(prefix, n_envs, b);
  const EventArgs a = descs[e];
  events_block<PPT, 0, AHEAD>(a, (long long)(b - prefix[e]) * (kBlock * PPT), L);
}

// ---------------------------------------------------------------------------
// The sharded stream of a call (evis_stream.h): set-up and fixup.
// ---------------------------------------------------------------------------

// The chunk table is kept all unpublished between calls: the clean-up
// kernel after each fixup resets the entries the call published, and a
// table that may hold anything else (new, or after a call that did not
// finish its launches) is cleared whole first.
__global__ __launch_bounds__(kBlock) void k_stream_clear(const StreamState st) {
  const long long n = (long long)kStreams * st.kmax;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride)
    st.chunk_of[idx] = kChunkUnpublished;
}

// Set-up (one workgroup): every stream empty, blocks 0 .. kAheadChunks - 1
// of every stream published (chunk s * kAheadChunks + k); the base is the
// cursor (0 with reset).  gmax counts the chunks whose slots all have a
// place: below `capacity` or within the spill buffer after it (the stream
// of a call that fits the output needs at most T + kSpillEvents slots).
__global__ __launch_bounds__(kBlock) void k_stream_init(const StreamState st,
                                                        unsigned long long* cursor, int reset,
                                                        long long capacity) {
  const long long base = reset ? 0 : (long long)*cursor;
  const long long room = capacity > base ? capacity - base + kSpillEvents : 0;
  const int gmax = (int)min(room >> kStreamChunkLog, (long long)0x7FFFFFFF);
  const int t = threadIdx.x;
  if (t < kStreams * kAheadChunks) {
    const int s = t / kAheadChunks, k = t % kAheadChunks;
    const int g = s * kAheadChunks + k;
    if (k < st.kmax) {
      st.chunk_of[(long long)s * st.kmax + k] = g < gmax ? g : kChunkDropped;
      if (g < gmax) st.owner[g] = s | (k << 8);
    }
  }
  if (t < kStreams) st.fill[t * kStreamLine] = 0ull;
  if (t == 0) {
    st.hdr->base = base;
    st.hdr->nchunks = (unsigned int)(kStreams * kAheadChunks);
    st.hdr->gmax = gmax;
  }
}

// Clean-up (after the fixup): stream s published blocks 0 .. e_s +
// kAheadChunks - 1, e_s = ceil(fill_s / kStreamChunk) the blocks it entered.
__global__ __launch_bounds__(kBlock) void k_stream_clean(const StreamState st) {
  const int s = blockIdx.x;
  const long long f = (long long)st.fill[s * kStreamLine];
  const long long e = (f + kStreamChunk - 1) >> kStreamChunkLog;
  const long long kend = min(e + kAheadChunks, (long long)st.kmax);
  for (long long k = threadIdx.x; k < kend; k += blockDim.x)
    st.chunk_of[(long long)s * st.kmax + k] = kChunkUnpublished;
}

// Fixup: move the events stored at or above L = min(base + T, capacity)
// (in the output, or in the spill buffer past `capacity`) into the unfilled
// slots below L, in position order, and set the cursor to base + T.  Every
// workgroup builds the same interval lists (a few hundred entries) and
// moves its own share.
constexpr int kFixupBlocks = 64;
constexpr int kFixupThreads = 1024;
constexpr int kFixupList = kMaxHoleChunks + 2;

__global__ __launch_bounds__(kFixupThreads) void k_stream_fixup(const StreamState st,
                                                                evis_event* __restrict__ out,
                                                                long long capacity,
                                                                unsigned long long* cursor) {
  __shared__ unsigned long long s_fill[kStreams];
  __shared__ long long h_pos[kFixupList], h_len[kFixupList], h_pre[kFixupList + 1];
  __shared__ long long u_pos[kFixupList], u_len[kFixupList], u_pre[kFixupList + 1];
  __shared__ long long hs_pos[kFixupList], hs_len[kFixupList], us_pos[kFixupList], us_len[kFixupList];
  __shared__ int s_nh, s_nu;
  const int tid = threadIdx.x;
  const long long base = st.hdr->base;
  const int gmax = st.hdr->gmax;
  const int G = (int)min((long long)st.hdr->nchunks, (long long)gmax);
  if (tid < kStreams) s_fill[tid] = st.fill[tid * kStreamLine];
  if (tid == 0) {
    s_nh = 0;
    s_nu = 0;
  }
  __syncthreads();
  long long T = 0;
  for (int i = 0; i < kStreams; ++i) T += (long long)s_fill[i];
  const long long L = min(base + T, capacity);
  auto block_fill = [&](int s, long long k) -> long long {
    const long long f = (long long)s_fill[s] - (k << kStreamChunkLog);
    return f < 0 ? 0 : (f > kStreamChunk ? kStreamChunk : f);
  };
  // holes: the blocks of each stream that are not full (the last entered
  // one and the kAheadChunks published after it), clipped to [base, L)
  if (tid < kStreams && L > base) {
    const int s = tid;
    const long long f = (long long)s_fill[s];
    const long long e = (f + kStreamChunk - 1) >> kStreamChunkLog;   // blocks entered
    for (long long k = f >> kStreamChunkLog; k < e + kAheadChunks && k < st.kmax; ++k) {
      const int g = st.chunk_of[(long long)s * st.kmax + k];
      if (g < 0) continue;
      const long long p0 = base + ((long long)g << kStreamChunkLog) + block_fill(s, k);
      const long long p1 = min(base + ((long long)(g + 1) << kStreamChunkLog), L);
      if (p0 < p1) {
        const int slot = atomicAdd(&s_nh, 1);
        if (slot < kFixupList) {
          h_pos[slot] = p0;
          h_len[slot] = p1 - p0;
        }
      }
    }
  }
  // sources: the filled slots of chunks at or above L
  if (L > base) {
    const long long gL = (L - base) >> kStreamChunkLog;
    for (long long g = gL + tid; g < G; g += kFixupThreads) {
      const int ow = st.owner[g];
      const int s = ow & 0xFF;
      const long long k = (long long)(ow >> 8);
      const long long c0 = base + (g << kStreamChunkLog);
      const long long p0 = max(c0, L);
      const long long p1 = c0 + block_fill(s, k);
      if (p0 < p1) {
        const int slot = atomicAdd(&s_nu, 1);
        if (slot < kFixupList) {
          u_pos[slot] = p0;
          u_len[slot] = p1 - p0;
        }
      }
    }
  }
  __syncthreads();
  const int nh = min(s_nh, kFixupList), nu = min(s_nu, kFixupList);
  // order both lists by position (rank sort; positions are distinct)
  if (tid < nh) {
    int r = 0;
    for (int i = 0; i < nh; ++i) r += (h_pos[i] < h_pos[tid]) ? 1 : 0;
    hs_pos[r] = h_pos[tid];
    hs_len[r] = h_len[tid];
  }
  if (tid < nu) {
    int r = 0;
    for (int i = 0; i < nu; ++i) r += (u_pos[i] < u_pos[tid]) ? 1 : 0;
    us_pos[r] = u_pos[tid];
    us_len[r] = u_len[tid];
  }
  __syncthreads();
  if (tid == 0) {
    h_pre[0] = 0;
    for (int i = 0; i < nh; ++i) h_pre[i + 1] = h_pre[i] + hs_len[i];
    u_pre[0] = 0;
    for (int i = 0; i < nu; ++i) u_pre[i + 1] = u_pre[i] + us_len[i];
  }
  __syncthreads();
  const long long M = min(h_pre[nh], u_pre[nu]);
  const long long per = (M + gridDim.x - 1) / gridDim.x;
  const long long m0 = (long long)blockIdx.x * per, m1 = min(M, m0 + per);
  for (long long m = m0 + tid; m < m1; m += kFixupThreads) {
    int lo = 0, hi = nh - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (h_pre[mid] <= m) lo = mid; else hi = mid - 1;
    }
    const long long dst = hs_pos[lo] + (m - h_pre[lo]);
    lo = 0;
    hi = nu - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (u_pre[mid] <= m) lo = mid; else hi = mid - 1;
    }
    const long long src = us_pos[lo] + (m - u_pre[lo]);
    if (src < capacity + kSpillEvents && dst < capacity)
      out[dst] = (src < capacity) ? out[src] : st.spill[src - capacity];
  }
  if (blockIdx.x == 0 && tid == 0) *cursor = (unsigned long long)(base + T);
}

hipError_t launch_zero_u64(unsigned long long* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_stream_init(const StreamState& st, unsigned long long* cursor, int reset,
                              long long capacity, bool clear_table, hipStream_t s) {
  static_assert(kStreams * kAheadChunks <= kBlock, "one workgroup publishes the first blocks");
  if (clear_table) {
    const long long n = (long long)kStreams * st.kmax;
    hipLaunchKernelGGL(k_stream_clear, dim3(grid_for(n, kBlock * 8)), dim3(kBlock), 0, s, st);
  }
  hipLaunchKernelGGL(k_stream_init, dim3(1), dim3(kBlock), 0, s, st, cursor, reset, capacity);
  return hipGetLastError();
}

hipError_t launch_stream_clean(const StreamState& st, hipStream_t s) {
  hipLaunchKernelGGL(k_stream_clean, dim3(kStreams), dim3(kBlock), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_stream_fixup(const StreamState& st, evis_event* out, long long capacity,
                               unsigned long long* cursor, hipStream_t s) {
  hipLaunchKernelGGL(k_stream_fixup, dim3(kFixupBlocks), dim3(kFixupThreads), 0, s, st, out,
                     capacity, cursor);
  return hipGetLastError();
}

// Defocus: one workgroup per 64 x 32 output tile of one channel of one
// image of the batch (many small images fill the chip in one launch).  The
// input tile with an apron of r pixels (edge pixels repeated) goes to LDS,
// then the horizontal pass over all its rows into LDS, then the vertical
// pass to the output; each output sums its 2r + 1 taps in order, k = -r..r,
// with the weights read from LDS.  HBM-bound: one read and one write of
// each image (plus the aprons).
constexpr int kDefTW = 64, kDefTH = 32;

int defocus_tiles(int H, int W, int* tiles_x) {
  *tiles_x = (W + kDefTW - 1) / kDefTW;
  return *tiles_x * ((H + kDefTH - 1) / kDefTH);
}

// R > 0: the radius, fixed at compile time (taps unrolled, weights from the
// kernel arguments in scalar registers); R = 0: any radius, a.r, weights
// from LDS.  Pixel (x, y), channel c is element (y W + x) C + c, below
// 2^26 (H, W <= 4096, C <= 3): 32-bit indices and 24-bit products.
template <int R>
__global__ __launch_bounds__(kBlock) void k_defocus(const DefocusArgs a) {
  extern __shared__ float smem[];
  __shared__ float s_w[R > 0 ? 1 : 2 * kDefocusMaxR + 1];
  const int r = R > 0 ? R : a.r;
  const int C = a.C, c = blockIdx.y;
  // Workgroups go to the XCDs in turn (workgroup b to XCD b % kXcd), and
  // each XCD has its own L2: workgroup b takes tile (b % kXcd) * per +
  // b / kXcd, so that each XCD works through one run of consecutive tiles
  // and the apron lines that neighbouring tiles share come from HBM once,
  // not once per XCD (this halved the reads of a 64-image batch, to the
  // images' own bytes).  The grid is a multiple of kXcd; the few
  // workgroups past the last tile leave.
  const int n_tiles = a.tile_prefix[a.n];
  const int per = (int)gridDim.x / kXcd;
  const int tile = (int)(blockIdx.x % kXcd) * per + (int)(blockIdx.x / kXcd);
  if (tile >= n_tiles) return;
  // image of this tile: the last one whose first tile is <= tile
  int lo = 0, hi = a.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.tile_prefix[mid] <= tile) lo = mid; else hi = mid - 1;
  }
  const DefocusImage im = a.img[lo];
  const int lt = tile - a.tile_prefix[lo];
  const int W = im.W, H = im.H;
  const int inW = kDefTW + 2 * r, inH = kDefTH + 2 * r;
  float* in = smem;                 // [inH][inW]
  float* hb = smem + inW * inH;     // [inH][kDefTW]
  const int x0 = (lt % im.tiles_x) * kDefTW, y0 = (lt / im.tiles_x) * kDefTH;
  const unsigned rowC = (unsigned)(W * C);   // elements per image row
  if (R == 0)
    for (int k = threadIdx.x; k <= 2 * r; k += kBlock) s_w[k] = a.w[k];
  auto wt = [&](int k) { return R > 0 ? a.w[k] : s_w[k]; };
  // Lane l of every wave owns column l of the tile (kDefTW = kWave): its
  // apron columns l and, for l < 2r, kDefTW + l, and output column l.
  static_assert(kDefTW == kWave && kDefTH == kWavesPerBlock * 8, "defocus tile: one column per lane");
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const bool two = lane < 2 * r;   // 2r <= 60 < 64
  const unsigned ca = __umul24((unsigned)min(max(x0 - r + lane, 0), W - 1), (unsigned)C) + (unsigned)c;
  const unsigned cb = __umul24((unsigned)min(max(x0 - r + kDefTW + lane, 0), W - 1), (unsigned)C) + (unsigned)c;
  // The apron: wave w loads rows w, w + 4, ... (a row's source row and
  // offset are uniform), kDefRows rows per pass with all loads in flight
  // (one pass for radii up to 4).
  constexpr int kDefRows = 10;
  for (int row0 = wave; row0 < inH; row0 += kDefRows * kWavesPerBlock) {
    float va[kDefRows], vb[kDefRows];
#pragma unroll
    for (int u = 0; u < kDefRows; ++u) {
      const int row = row0 + u * kWavesPerBlock;
      const unsigned base = __umul24((unsigned)min(max(y0 - r + row, 0), H - 1), rowC);
      va[u] = vb[u] = 0.0f;
      if (row < inH) {   // uniform
        va[u] = ldg(im.x, (int)(base + ca));
        if (two) vb[u] = ldg(im.x, (int)(base + cb));
      }
    }
#pragma unroll
    for (int u = 0; u < kDefRows; ++u) {
      const int row = row0 + u * kWavesPerBlock;
      if (row < inH) {
        in[row * inW + lane] = va[u];
        if (two) in[row * inW + kDefTW + lane] = vb[u];
      }
    }
  }
  __syncthreads();
  // horizontal pass: every apron row, wave w rows w, w + 4, ...
  for (int row = wave; row < inH; row += kWavesPerBlock) {
    const float* src = in + row * inW + lane;
    float acc = 0.0f;
    if constexpr (R > 0) {
#pragma unroll
      for (int k = 0; k <= 2 * R; ++k) acc = acc + wt(k) * src[k];
    } else {
      for (int k = 0; k <= 2 * r; ++k) acc = acc + wt(k) * src[k];
    }
    hb[row * kDefTW + lane] = acc;
  }
  __syncthreads();
  // vertical pass: wave w output rows 8w .. 8w + 7 (uniform row tests)
  const int gx = x0 + lane;
  const unsigned cx = __umul24((unsigned)gx, (unsigned)C) + (unsigned)c;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int row = wave * 8 + j, gy = y0 + row;
    if (gy >= H) break;   // uniform
    const float* src = hb + row * kDefTW + lane;
    float acc = 0.0f;
    if constexpr (R > 0) {
#pragma unroll
      for (int k = 0; k <= 2 * R; ++k) acc = acc + wt(k) * src[k * kDefTW];
    } else {
      for (int k = 0; k <= 2 * r; ++k) acc = acc + wt(k) * src[k * kDefTW];
    }
    if (gx < W) stg(im.out, (int)(__umul24((unsigned)gy, rowC) + cx), acc);
  }
}

hipError_t launch_defocus(const DefocusArgs& a, hipStream_t s) {
  const int inW = kDefTW + 2 * a.r, inH = kDefTH + 2 * a.r;
  const size_t lds = (size_t)(inW * inH + kDefTW * inH) * sizeof(float);
  const dim3 grid((a.tile_prefix[a.n] + kXcd - 1) / kXcd * kXcd, a.C);   // see k_defocus
  switch (a.r) {   // sigma <= 2 (the usual range) unrolled
    case 1: hipLaunchKernelGGL(k_defocus<1>, grid, dim3(kBlock), lds, s, a); break;
    case 2: hipLaunchKernelGGL(k_defocus<2>, grid, dim3(kBlock), lds, s, a); break;
    case 3: hipLaunchKernelGGL(k_defocus<3>, grid, dim3(kBlock), lds, s, a); break;
    case 4: hipLaunchKernelGGL(k_defocus<4>, grid, dim3(kBlock), lds, s, a); break;
    case 5: hipLaunchKernelGGL(k_defocus<5>, grid, dim3(kBlock), lds, s, a); break;
    case 6: hipLaunchKernelGGL(k_defocus<6>, grid, dim3(kBlock), lds, s, a); break;
    default: hipLaunchKernelGGL(k_defocus<0>, grid, dim3(kBlock), lds, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_log_channels(const float* x, long long n, float eps, float* L, hipStream_t s) {
  hipLaunchKernelGGL(k_log_channels, dim3(grid_for(n, kBlock * 4)), dim3(kBlock), 0, s, x, n, eps, L);
  return hipGetLastError();
}

hipError_t launch_log_luminance(const float* x, int channels, long long n, float eps, float* L,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_log_luminance, dim3(grid_for(n, kBlock * 4)), dim3(kBlock), 0, s, x,
                     channels, n, eps, L);
  return hipGetLastError();
}

hipError_t launch_state_init(const float* L_first, long long n, float* L_ref, int32_t* t_last,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(grid_for(n, kBlock * 4)), dim3(kBlock), 0, s, L_first, n,
                     L_ref, t_last);
  return hipGetLastError();
}

hipError_t launch_substep_count(const float2* mA, const float2* mB, long long n, int K_max,
                                unsigned long long* msq_scratch, int32_t* K_out, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, msq_scratch);
  hipLaunchKernelGGL(k_msq, dim3(grid_for(n, kBlock * 8)), dim3(kBlock), 0, s, mA, mB, n,
                     msq_scratch);
  hipLaunchKernelGGL(k_k_from_msq, dim3(1), dim3(64), 0, s, msq_scratch, K_max, K_out);
  return hipGetLastError();
}

hipError_t launch_events(const float* L_seq, int H, int W, int K, long long t0, int span,
                         float Dt, float C_on, float C_off, const float* th_on,
                         const float* th_off, int refr, uint32_t env_bits, float* L_ref,
                         int32_t* t_last, evis_event* out, long long capacity,
                         unsigned long long* cursor, int reset_cursor, const NoiseCfg* noise,
                         const StreamState& st, hipStream_t s) {
  const bool wave = events_wave_form(refr, noise != nullptr);
  if (reset_cursor && !wave) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, cursor);
  EventArgs a{L_seq, H, W, K, t0, span, Dt, C_on, C_off, th_on, th_off, refr, env_bits,
              L_ref, t_last, out, capacity, cursor, noise ? *noise : NoiseCfg{}};
  const long long n = (long long)H * W;
  // Enough workgroups to cover the chip: 4 px per thread on large frames.
  if (noise) {
    if (n >= 4LL * kBlock * 1024)
      hipLaunchKernelGGL((k_events<4, 1>), dim3(grid_for(n, kBlock * 4)), dim3(kBlock), 0, s, a);
    else if (n >= 2LL * kBlock * 512)
      hipLaunchKernelGGL((k_events<2, 1>), dim3(grid_for(n, kBlock * 2)), dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL((k_events<1, 1>), dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, a);
  } else if (wave) {   // one pixel per lane
    hipLaunchKernelGGL((k_events_wave<kEventsPPT, kEventsWaveU>),
                       dim3(grid_for(n, kBlock * kEventsPPT)), dim3(kBlock), 0, s, a, st);
  } else if (n >= 4LL * kBlock * 1024) {
    hipLaunchKernelGGL((k_events<4, 0>), dim3(grid_for(n, kBlock * 4)), dim3(kBlock), 0, s, a);
  } else if (n >= 2LL * kBlock * 512) {
    hipLaunchKernelGGL((k_events<2, 0>), dim3(grid_for(n, kBlock * 2)), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_events<1, 0>), dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

int events_batch_blocks(long long px) { return grid_for(px, kBlock * kEventsPPT); }

hipError_t launch_events_batch(const EventArgs* descs, const int32_t* prefix, int n_envs,
                               int total_blocks, bool wave_form, const StreamState& st,
                               hipStream_t s) {
  if (n_envs == 0 || total_blocks == 0) return hipGetLastError();
  if (wave_form)
    hipLaunchKernelGGL((k_events_batch_wave<kEventsPPT, kEventsWaveU>), dim3(total_blocks),
                       dim3(kBlock), 0, s, descs, prefix, n_envs, st);
  else
    hipLaunchKernelGGL((k_events_batch<kEventsPPT, kEventsBlockAhead>), dim3(total_blocks),
                       dim3(kBlock), 0, s, descs, prefix, n_envs);
  return hipGetLastError();
}

}  // namespace evis
