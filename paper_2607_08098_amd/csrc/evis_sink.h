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

// One substep of the event model for the PPT pixels of this thread, followed
// by the workgroup's compaction round.  Every thread of the workgroup must
// call it (it holds a barrier).  ev_count and round are workgroup-uniform.
template <int PPT>
__device__ __forceinline__ void emit_substep(
    int j, const float (&Lj)[PPT], const float (&Lp)[PPT], float (&R)[PPT], int (&tl)[PPT],
    const float (&con)[PPT], const float (&coff)[PPT], const uint32_t (&xy)[PPT], uint32_t okbits,
    long long t0, int span, float Dt, int refr, uint32_t env_bits, const SinkShared& sh,
    const SinkOut& so, int& ev_count, int& round) {
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
      const float c = pos ? con[k] : coff[k];
      const float a = fabsf(d);
      if (a >= c && c > 0.0f) {
        const int n = crossing_count(a, c);
        nn[k] = n;
        posbits |= (pos ? 1u : 0u) << k;
        if (refr == 0) {
          m += n;
        } else {
          long long tlk = tl[k];
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
    unsigned long long gdst = 0;
    int ldst = 0;
    if (ev_count + grand <= sh.cap) {
      ldst = ev_count + off_w + excl;
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
      gdst = gb + (unsigned long long)(ev_count + off_w + excl);
      ev_count = 0;
    }
    if (m > 0) {
      int widx = 0;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int n = nn[k];
        if (n > 0) {
          const bool pos = (posbits >> k) & 1u;
          const float c = pos ? con[k] : coff[k];
          const uint32_t word = xy[k] | ((pos ? 1u : 0u) << 22) | env_bits;
          for (int kk = 1; kk <= n; ++kk) {
            const long long t = t0 + crossing_offset(j, kk, R[k], c, pos, Lp[k], Lj[k], Dt, span);
            if (refr == 0 || t - (long long)tl[k] >= refr) {
              if (to_global) {
                const unsigned long long idx = gdst + (unsigned long long)widx;
                if ((long long)idx < so.capacity) so.out[idx] = evis_event{word, (int32_t)t};
              } else {
                sh.buf[ldst + widx] = make_uint2(word, (uint32_t)(int32_t)t);
              }
              ++widx;
              tl[k] = (int)t;
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
      const float c = pos ? con[k] : coff[k];
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
