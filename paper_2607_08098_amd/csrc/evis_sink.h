// Event emission (Eq. 4 with Eq. 8 thresholds and the refractory period)
// and wave-ballot / prefix-sum compaction into a workgroup-local LDS buffer
// that is appended to the global event stream with one atomic per flush.
#pragma once

#include "evis_common.h"

namespace evis {

struct SinkShared {
  uint2* buf;                   // LDS [cap] staged events
  int (*wtot)[kWavesPerBlock];  // LDS [2][4] per-wave event totals (double-buffered)
  unsigned long long* gbase;    // LDS: global slot of the current flush
  int cap;
};

struct SinkOut {
  evis_event* out;
  long long capacity;
  unsigned long long* cursor;
};

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
    if (pos) return con ? con[i] : C_on;
    return coff ? coff[i] : C_off;
  }
  __device__ __forceinline__ float c(int k, bool pos) const { return c_at(threadIdx.x + k * kBlock, pos); }
  __device__ __forceinline__ int tlast(int k) const { return tl[threadIdx.x + k * kBlock]; }
  __device__ __forceinline__ void set_tlast_at(int i, int t) const { tl[i] = t; }
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

// One substep of the event model for the PPT pixels of this thread, followed
// by the workgroup's compaction round.  Every thread of the workgroup must
// call it (it holds a barrier).  ev_count and round are workgroup-uniform.
template <int PPT>
__device__ __forceinline__ void emit_substep(
    int j, const float (&Lj)[PPT], const float (&Lp)[PPT], float (&R)[PPT], const PixAux& aux,
    uint32_t okbits, long long t0, int span, float Dt, int refr, uint32_t env_bits,
    const SinkShared& sh, const SinkOut& so, int& ev_count, int& round) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
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
        const int n = crossing_count(a, c);
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
  // Workgroup offsets: wave prefix sums, then the per-wave totals in LDS.
  const int incl = wave_inclusive_scan(m);
  const int excl = incl - m;
  const int rb = round & 1;
  if (lane == kWave - 1) sh.wtot[rb][wave] = incl;
  __syncthreads();
  int off_w = 0, grand = 0;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) {
    const int v = sh.wtot[rb][w];
    off_w += (w < wave) ? v : 0;
    grand += v;
  }
  ++round;
  if (grand > 0) {   // workgroup-uniform
    bool to_global = false;
    unsigned long long gbase_w = 0;   // this wave's first slot in the stream
    int lbase_w = 0;                  // ... or in the LDS buffer
    if (ev_count + grand <= sh.cap) {
      lbase_w = ev_count + off_w;
      ev_count += grand;
    } else {
      // Flush the staged events and write this round straight to the stream.
      if (tid == 0) *sh.gbase = atomicAdd(so.cursor, (unsigned long long)(ev_count + grand));
      __syncthreads();
      const unsigned long long gb = *sh.gbase;
      for (int i = tid; i < ev_count; i += kBlock) {
        if ((long long)(gb + i) < so.capacity) {
          const uint2 r = sh.buf[i];
          so.out[gb + i] = evis_event{r.x, (int32_t)r.y};
        }
      }
      to_global = true;
      gbase_w = gb + (unsigned long long)(ev_count + off_w);
      ev_count = 0;
    }
    auto put = [&](int slot, uint32_t word, int t) {
      if (to_global) {
        const unsigned long long idx = gbase_w + (unsigned long long)slot;
        if ((long long)idx < so.capacity) so.out[idx] = evis_event{word, (int32_t)t};
      } else {
        sh.buf[lbase_w + slot] = make_uint2(word, (uint32_t)t);
      }
    };
    const int wtot = __shfl(incl, kWave - 1, kWave);
    if (refr == 0) {
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

// Write out whatever is still staged.  Every thread must call it.
__device__ __forceinline__ void sink_flush(const SinkShared& sh, const SinkOut& so, int& ev_count) {
  __syncthreads();
  if (ev_count == 0) return;   // workgroup-uniform
  const int tid = threadIdx.x;
  if (tid == 0) *sh.gbase = atomicAdd(so.cursor, (unsigned long long)ev_count);
  __syncthreads();
  const unsigned long long gb = *sh.gbase;
  for (int i = tid; i < ev_count; i += kBlock) {
    if ((long long)(gb + i) < so.capacity) {
      const uint2 r = sh.buf[i];
      so.out[gb + i] = evis_event{r.x, (int32_t)r.y};
    }
  }
  ev_count = 0;
}

}  // namespace evis
