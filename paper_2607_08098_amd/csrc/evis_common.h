// Device-side building blocks of the EVIS event path (gfx950).
//
// Every floating-point operation here is an IEEE float32 operation rounded to
// nearest, in the order written: the library is compiled with
// -ffp-contract=off and correctly rounded division, so no multiply is fused
// with an add.  The splat winner, the footprint corners and the crossing
// count are discrete decisions taken on these values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "evis.h"

namespace evis {

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // 4 waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kSrcTile = 8;                 // source tiles are 8x8 = one wave
constexpr uint64_t kEmptyKey = 0xFFFFFFFFFFFFFFFFull;
constexpr int kMaxCross = EVIS_MAX_CROSSINGS;

// Per-environment descriptor as the kernels read it (built on the host from
// an evis_env, copied to device memory once per call).
struct EnvDesc {
  const float* LA;
  const float* LB;
  const float2* mA;
  const float2* mB;
  const float* ZA;
  const float* ZB;
  float* Lref;
  int32_t* tlast;          // may be null
  const float* th_on;      // may be null: C_on everywhere
  const float* th_off;     // may be null: C_off everywhere
  float* dZ;               // scratch [H*W]: Zend - Z_A
  float4* tb;              // scratch [n source tiles]: (mx_min, mx_max, my_min, my_max)
  int32_t H, W;
  int32_t ntx_src, nty_src;    // 8x8 source tiles
  int32_t src_tile_base;       // prefix over envs, for the prep kernel
  int32_t K_fixed;             // > 0: fixed K
  int32_t K_max;
  int32_t blend;
  float C_on, C_off;
  int32_t refr;                // refractory period, us
  uint32_t env_bits;           // env_id << 23
  int64_t t0;
  int32_t span;                // t1 - t0 (us)
  int32_t pad0;
};

// Per-environment values computed on the device each step.
struct EnvDyn {
  unsigned long long msq_bits;   // max over finite |m|^2 (float64 bits, >= 0)
  int32_t K;
  float Dt;
  int32_t ntx, nty;              // target tiles of this step's tile shape
  int32_t item_begin;            // first work item of this env
  int32_t pad;
};

__device__ __forceinline__ float lerp32(float a, float b, float w) {
  return a + w * (b - a);
}

// Bilinear sample at (sx, sy) inside [0, W-1] x [0, H-1]: two lerps along x,
// one along y; the right/bottom neighbour is clamped to the last column/row.
__device__ __forceinline__ float bilinear(const float* __restrict__ img, int H, int W, float sx,
                                          float sy) {
  const float fx0 = floorf(sx), fy0 = floorf(sy);
  const float wx = sx - fx0, wy = sy - fy0;
  const int x0 = (int)fx0, y0 = (int)fy0;
  const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
  const float a = img[y0 * W + x0], b = img[y0 * W + x1];
  const float c = img[y1 * W + x0], d = img[y1 * W + x1];
  return lerp32(lerp32(a, b, wx), lerp32(c, d, wx), wy);
}

// Clamp into [0, hi]; NaN becomes 0.
__device__ __forceinline__ float clamp_into(float v, float hi) {
  v = (v > 0.0f) ? v : 0.0f;
  return (v < hi) ? v : hi;
}

__device__ __forceinline__ bool finite32(float v) { return fabsf(v) <= 3.402823466e38f; }

// Exact substep count from the largest squared motion length M (float64):
// the smallest K >= 1 with K*K >= M, at most K_max.
__device__ __forceinline__ int exact_k(double M, int K_max) {
  if (!(M > 0.0)) return 1;
  if (M > (double)K_max * (double)K_max) return K_max;
  int k = (int)ceil(sqrt(M));
  while (k > 1 && (double)(k - 1) * (double)(k - 1) >= M) --k;
  while ((double)k * (double)k < M) ++k;
  return max(1, min(k, K_max));
}

// Eq. 4 crossing count: floor of the exact quotient a / c for a >= c > 0,
// capped at kMaxCross.  The float32 quotient gives a candidate; exact
// float64 products n*c (n < 2^17, c has 24 significant bits) correct it.
__device__ __forceinline__ int crossing_count(float a, float c) {
  if (!(a <= 3.402823466e38f)) return kMaxCross;   // a = +inf
  const float q = a / c;
  int n = (q > 65536.0f) ? 65536 : (int)floorf(q);
  const double ad = (double)a, cd = (double)c;
  if ((double)n * cd > ad)
    n -= 1;
  else if ((double)(n + 1) * cd <= ad)
    n += 1;
  return min(n, kMaxCross);
}

// Integer-microsecond offset from t0 of crossing k of substep j: linear
// interpolation of L between the previous sample and the current one.
__device__ __forceinline__ int crossing_offset(int j, int k, float R, float c, bool pos, float prev,
                                               float cur, float Dt, int span) {
  const float kc = (float)k * c;
  const float lam = pos ? (R + kc) : (R - kc);
  const float den = cur - prev;
  float phi = (den == 0.0f) ? 1.0f : (lam - prev) / den;
  phi = (phi >= 0.0f) ? phi : 0.0f;
  phi = (phi > 1.0f) ? 1.0f : phi;
  const float v = ((float)(j - 1) + phi) * Dt;
  const int off = (int)floorf(v);
  return min(off, span);
}

// float <-> order-preserving int (for atomic min/max on floats)
__device__ __forceinline__ int float_to_ordered(float f) {
  int i = __float_as_int(f);
  return (i >= 0) ? i : (i ^ 0x7FFFFFFF);
}

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int t = __shfl_up(v, d, kWave);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = fminf(v, __shfl_xor(v, d, kWave));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, kWave));
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, kWave));
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

}  // namespace evis
