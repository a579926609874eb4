// Elementwise front end, state initialisation, the substep count of one
// pair, and the event model over caller-supplied frames (gfx950).
#include "evis_internal.h"
#include "evis_sink.h"

namespace evis {

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

// Events over materialised frames: PPT pixels per thread, consecutive pixels
// across the workgroup, one pass over the K+1 frames with the state in
// registers and the next frame's values loaded ahead.

// The event model over the kBlock * PPT consecutive pixels from `base` of
// one env's frames (every thread of the workgroup calls it).
template <int PPT, int NOISE, int AHEAD = 4>
__device__ __forceinline__ void events_block(const EventArgs& a, long long base) {
  __shared__ uint2 evbuf[kEventBuf];
  __shared__ float4 s_cq[kWavesPerBlock * kCrossQ];   // crossing queues (no refractory period)
  __shared__ int s_evn, s_req[4];
  __shared__ unsigned long long s_gbase;
  __shared__ float s_con[kBlock * PPT], s_coff[kBlock * PPT];
  __shared__ int s_tl[kBlock * PPT];
  const SinkShared sh{evbuf, &s_evn, s_req, &s_gbase, kEventBuf};
  const SinkOut so{a.out, a.capacity, a.cursor};
  const int tid = threadIdx.x;
  const long long plane = (long long)a.H * a.W;
  // Frames are read kAhead substeps ahead of their use (a ring of registers
  // shifted by one each substep), so that enough loads are in flight to keep
  // HBM busy: the substep loop is otherwise one dependent load per step.
  constexpr int kAhead = AHEAD;
  float R[PPT], Lp[PPT], Lj[PPT], Ln[kAhead][PPT];
  uint32_t okbits = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int i = tid + k * kBlock;
    const long long q = base + i;
    const bool ok = q < plane;
    okbits |= (ok ? 1u : 0u) << k;
    R[k] = ok ? a.Lref[q] : 0.0f;
    // without a refractory period t_last is only written: keep the largest
    // event time of each pixel (INT_MIN: none)
    s_tl[i] = (a.refr == 0) ? INT_MIN : ((ok && a.tlast) ? a.tlast[q] : EVIS_T_LAST_INIT);
    if (a.th_on) s_con[i] = ok ? a.th_on[q] : 1.0f;
    if (a.th_off) s_coff[i] = ok ? a.th_off[q] : 1.0f;
    Lp[k] = ok ? a.L_seq[q] : 0.0f;
#pragma unroll
    for (int u = 0; u < kAhead; ++u)
      Ln[u][k] = (ok && u + 1 <= a.K) ? a.L_seq[(long long)(u + 1) * plane + q] : 0.0f;
  }
  const PixAux aux{a.th_on ? s_con : nullptr, a.th_off ? s_coff : nullptr, s_tl, a.C_on, a.C_off,
                   0, 0, a.W, 0, base};
  uint32_t hotb = 0;
  if constexpr (NOISE != 0) hotb = hot_bits<PPT>(a.noise, aux, okbits);
  SinkRound sr;
  CrossQueue cq{s_cq};
  sink_init(sh);
  __syncthreads();
  for (int j = 1; j <= a.K; ++j) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      Lj[k] = Ln[0][k];
#pragma unroll
      for (int u = 0; u + 1 < kAhead; ++u) Ln[u][k] = Ln[u + 1][k];
      Ln[kAhead - 1][k] = (((okbits >> k) & 1u) && j + kAhead <= a.K)
                              ? a.L_seq[(long long)(j + kAhead) * plane + base + tid + k * kBlock]
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
      a.Lref[q] = R[k];
      const int tl = s_tl[tid + k * kBlock];
      if (a.tlast && (a.refr != 0 || tl != INT_MIN)) a.tlast[q] = tl;
    }
  }
  sink_flush(sh, so);
}

template <int PPT, int NOISE>
__global__ __launch_bounds__(kBlock) void k_events(const EventArgs a) {
  events_block<PPT, NOISE>(a, (long long)blockIdx.x * (kBlock * PPT));
}

// Many envs' frames in one launch: workgroup b works on env e, the last
// whose first workgroup prefix[e] is <= b (descriptors and prefix in device
// memory, read through the scalar cache).
template <int PPT, int AHEAD>
__global__ __launch_bounds__(kBlock) void k_events_batch(const EventArgs* __restrict__ descs,
                                                         const int32_t* __restrict__ prefix,
                                                         int n_envs) {
  const int b = blockIdx.x;
  int lo = 0, hi = n_envs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const EventArgs a = descs[lo];
  events_block<PPT, 0, AHEAD>(a, (long long)(b - prefix[lo]) * (kBlock * PPT));
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

__global__ __launch_bounds__(kBlock) void k_defocus(const DefocusArgs a) {
  extern __shared__ float smem[];
  __shared__ float s_w[2 * kDefocusMaxR + 1];
  const int r = a.r, C = a.C, c = blockIdx.y;
  // image of this tile: the last one whose first tile is <= blockIdx.x
  const int tile = blockIdx.x;
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
  for (int k = threadIdx.x; k <= 2 * r; k += kBlock) s_w[k] = a.w[k];
  // the apron tile, all threads at once, four loads in flight per thread;
  // element i sits at (i % inW, i / inW), stepped by kBlock incrementally
  {
    const int n = inW * inH;
    const int dx = kBlock % inW, dy = kBlock / inW;
    int lx = threadIdx.x % inW, ly = threadIdx.x / inW;
    for (int i0 = threadIdx.x; i0 < n; i0 += 4 * kBlock) {
      float v[4];
      int idx[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        idx[u] = i0 + u * kBlock;
        const int gx = min(max(x0 - r + lx, 0), W - 1);
        const int gy = min(max(y0 - r + ly, 0), H - 1);
        v[u] = (idx[u] < n) ? im.x[((long long)gy * W + gx) * C + c] : 0.0f;
        lx += dx;
        ly += dy;
        if (lx >= inW) {
          lx -= inW;
          ++ly;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (idx[u] < n) in[idx[u]] = v[u];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kDefTW * inH; i += kBlock) {
    const int col = i % kDefTW, row = i / kDefTW;
    const float* src = in + row * inW + col;
    float acc = 0.0f;
    for (int k = 0; k <= 2 * r; ++k) acc = acc + s_w[k] * src[k];
    hb[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kDefTW * kDefTH; i += kBlock) {
    const int col = i % kDefTW, row = i / kDefTW;
    const int gx = x0 + col, gy = y0 + row;
    if (gx >= W || gy >= H) continue;
    const float* src = hb + row * kDefTW + col;
    float acc = 0.0f;
    for (int k = 0; k <= 2 * r; ++k) acc = acc + s_w[k] * src[k * kDefTW];
    im.out[((long long)gy * W + gx) * C + c] = acc;
  }
}

static int grid_for(long long n, int per_block) {
  long long g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 65535LL * 16) g = 65535LL * 16;
  return (int)g;
}

hipError_t launch_defocus(const DefocusArgs& a, hipStream_t s) {
  const int inW = kDefTW + 2 * a.r, inH = kDefTH + 2 * a.r;
  const size_t lds = (size_t)(inW * inH + kDefTW * inH) * sizeof(float);
  hipLaunchKernelGGL(k_defocus, dim3(a.tile_prefix[a.n], a.C), dim3(kBlock), lds, s, a);
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
                         hipStream_t s) {
  if (reset_cursor) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, cursor);
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
  } else if (n >= 4LL * kBlock * 1024) {
    hipLaunchKernelGGL((k_events<4, 0>), dim3(grid_for(n, kBlock * 4)), dim3(kBlock), 0, s, a);
  } else if (n >= 2LL * kBlock * 512) {
    hipLaunchKernelGGL((k_events<2, 0>), dim3(grid_for(n, kBlock * 2)), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_events<1, 0>), dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

constexpr int kEventsBatchPPT = 2;
constexpr int kEventsBatchAhead = 4;

int events_batch_blocks(long long px) { return grid_for(px, kBlock * kEventsBatchPPT); }

hipError_t launch_events_batch(const EventArgs* descs, const int32_t* prefix, int n_envs,
                               int total_blocks, unsigned long long* reset_cursor, hipStream_t s) {
  if (reset_cursor) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, reset_cursor);
  hipLaunchKernelGGL((k_events_batch<kEventsBatchPPT, kEventsBatchAhead>), dim3(total_blocks), dim3(kBlock), 0, s, descs,
                     prefix, n_envs);
  return hipGetLastError();
}

}  // namespace evis
