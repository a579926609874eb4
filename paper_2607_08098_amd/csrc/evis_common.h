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
constexpr int kSrcBlk = 4;                  // source blocks are 4x4 pixels
constexpr int kBlkPx = kSrcBlk * kSrcBlk;   // 16 lanes, one row of a wave
constexpr int kSbBlk = 8;                   // superblocks are 8x8 source blocks (32x32 pixels)
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
  float4* src;             // scratch [blocks * 16]: (m_A.x, m_A.y, Z_A, Zend - Z_A) per
                           // source, block-major (block by * ntx_src + bx, then row-major)
  float4* tb;              // scratch [blocks]: (mx_min, mx_max, my_min, my_max) per block
  float4* sbb;             // scratch [superblocks]: the same bounds over kSbBlk x kSbBlk blocks
  int32_t H, W;
  int32_t ntx_src, nty_src;    // 4x4 source blocks per row / column
  int32_t ntx_sb, nty_sb;      // superblocks per row / column
  int32_t src_tile_base;       // prefix over envs of groups of four blocks (prep work units)
  int32_t K_fixed;             // > 0: fixed K
  int32_t K_max;
  int32_t blend;               // EVIS_BLEND_*
  float C_on, C_off;
  int32_t refr;                // refractory period, us
  uint32_t env_bits;           // env_id << 23
  int64_t t0;
  int32_t span;                // t1 - t0 (us)
  int32_t warp;                // EVIS_WARP_*
  int32_t margin;              // crop margin: only pixels m..W-m-1 x m..H-m-1 emit
  float4* srcB;                // two-splat warps only (else null): (-m_B.x, -m_B.y, Zstart,
                               // Z_B - Zstart) per source, Zstart = Z_A at p + m_B(p), same
                               // layout as src
  float4* tbB;                 // two-splat warps only: bounds of -m_B per block
  // sensor noise (evis_noise); noise_on = 0 when the env has none
  int32_t noise_on;
  float leak_hz, shot_hz, hot_hz, hot_frac, shot_L0, shot_inv;
  uint32_t seed_lo, seed_hi, pair_index;
};

// Noise parameters of one env for one keyframe pair (per substep
// probabilities need the pair's substep length).
struct NoiseCfg {
  float p_leak, shot_scale, p_hot;   // r_l Dt_s, r_s Dt_s, r_h Dt_s
  float shot_L0, shot_inv, hot_frac;
  uint32_t k0, k1, pair;
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

// Loads and stores through a global-address-space pointer with a 32-bit
// element index: the compiler then addresses with the pointer in scalar
// registers plus a 32-bit offset (no 64-bit address arithmetic per access).
// (The host compilation pass of this file only parses these device
// functions; it gets a plain body.)
template <typename T>
__device__ __forceinline__ T ldg(const T* p, int idx) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef const __attribute__((address_space(1))) char* gp;
  return *(const __attribute__((address_space(1))) T*)((gp)p + (unsigned)idx * (unsigned)sizeof(T));
#else
  return p[idx];
#endif
}
// The same with a byte offset (a uniform base plus one 32-bit offset per
// lane, no 64-bit address arithmetic).
template <typename T>
__device__ __forceinline__ T ldg_bytes(const T* p, uint32_t byte_off) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef const __attribute__((address_space(1))) char* gp;
  return *(const __attribute__((address_space(1))) T*)((gp)p + byte_off);
#else
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + byte_off);
#endif
}
template <typename T>
__device__ __forceinline__ void stg(T* p, int idx, T v) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef __attribute__((address_space(1))) char* gp;
  *(__attribute__((address_space(1))) T*)((gp)p + (unsigned)idx * (unsigned)sizeof(T)) = v;
#else
  p[idx] = v;
#endif
}

// A store through a global-address-space pointer with a 64-bit element
// index (the event stream): a pointer read from device memory would
// otherwise be generic, and generic stores also count against the LDS wait
// counter.
template <typename T>
__device__ __forceinline__ void stg64(T* p, unsigned long long idx, T v) {
#if defined(__HIP_DEVICE_COMPILE__)
  ((__attribute__((address_space(1))) T*)p)[idx] = v;
#else
  p[idx] = v;
#endif
}

// Atomic add on a global counter reached through a pointer read from device
// memory (a generic atomic would also wait on outstanding LDS operations).
__device__ __forceinline__ unsigned long long atomic_add_global(unsigned long long* p,
                                                                unsigned long long v) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long*)p, v,
                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#else
  return atomicAdd(p, v);
#endif
}

// Loads and stores of workgroup-shared (LDS) arrays reached through a plain
// pointer: the cast lets the compiler emit LDS instructions instead of
// generic (flat) ones, which would also wait on outstanding global loads.
template <typename T>
__device__ __forceinline__ T lds_ld(const T* p, int idx) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(3))) T*)p)[idx];
#else
  return p[idx];
#endif
}
template <typename T>
__device__ __forceinline__ void lds_st(T* p, int idx, T v) {
#if defined(__HIP_DEVICE_COMPILE__)
  ((__attribute__((address_space(3))) T*)p)[idx] = v;
#else
  p[idx] = v;
#endif
}

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
  const float a = ldg(img, y0 * W + x0), b = ldg(img, y0 * W + x1);
  const float c = ldg(img, y1 * W + x0), d = ldg(img, y1 * W + x1);
  return lerp32(lerp32(a, b, wx), lerp32(c, d, wx), wy);
}

// Clamp into [0, hi]; NaN becomes 0.
__device__ __forceinline__ float clamp_into(float v, float hi) {
  v = (v > 0.0f) ? v : 0.0f;
  return (v < hi) ? v : hi;
}

__device__ __forceinline__ bool finite32(float v) { return fabsf(v) <= 3.402823466e38f; }

// Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
// Shaw (SC 2011): ten rounds of two 32 x 32 -> 64-bit products mixed into
// the counter with the key, the key advanced by the Weyl increments
// between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32 x 32 -> 64-bit product gives both halves (v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// The top 24 bits of a word as a float in [0, 1) (exact).
__device__ __forceinline__ float uniform24(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

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
// capped at kMaxCross.  a * rcp(c) is within 0.02 of the quotient below the
// cap, so one correction step against the exact comparisons n*c <= a <
// (n+1)*c finishes the job.  fma(n, c, -a) rounds the exact n*c - a once,
// and rounding never changes the sign of a nonzero value (every float is a
// multiple of 2^-149, so a nonzero difference never rounds to zero), so the
// sign of the fma is the sign of n*c - a.
__device__ __forceinline__ int crossing_count(float a, float c) {
  if (!(a <= 3.402823466e38f)) return kMaxCross;   // a = +inf
  const float q = a * __builtin_amdgcn_rcpf(c);
  int n = (q >= 65536.0f) ? 65536 : (int)floorf(q);
  if (fmaf((float)n, c, -a) > 0.0f)
    n -= 1;
  else if (fmaf((float)(n + 1), c, -a) <= 0.0f)
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

// Inclusive prefix sum across the 64 lanes of a wave: shifts by 1, 2, 4, 8
// within each row of 16 lanes, then the last lane of row 0 / rows 0-1 is
// broadcast into the rows after it (DPP row_shr and row_bcast; a lane with
// no source lane reads 0).
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31
  return v;
}

// Wave reductions by DPP butterflies within each row of 16 lanes (swap
// neighbours, swap pairs, mirror halves of 8, mirror the row), then the four
// row results read out to scalars.  The result is wave-uniform.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
constexpr int kDppQuadSwap1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

// Minimum / maximum over each row of 16 lanes (every lane of the row gets it).
__device__ __forceinline__ float row16_min(float v) {
  v = fminf(v, dpp_f<kDppQuadSwap1>(v));
  v = fminf(v, dpp_f<kDppQuadSwap2>(v));
  v = fminf(v, dpp_f<kDppHalfMirror>(v));
  return fminf(v, dpp_f<kDppRowMirror>(v));
}
__device__ __forceinline__ float row16_max(float v) {
  v = fmaxf(v, dpp_f<kDppQuadSwap1>(v));
  v = fmaxf(v, dpp_f<kDppQuadSwap2>(v));
  v = fmaxf(v, dpp_f<kDppHalfMirror>(v));
  return fmaxf(v, dpp_f<kDppRowMirror>(v));
}
__device__ __forceinline__ float wave_min(float v) {
  const int b = __float_as_int(row16_min(v));
  return fminf(fminf(__int_as_float(__builtin_amdgcn_readlane(b, 0)),
                     __int_as_float(__builtin_amdgcn_readlane(b, 16))),
               fminf(__int_as_float(__builtin_amdgcn_readlane(b, 32)),
                     __int_as_float(__builtin_amdgcn_readlane(b, 48))));
}
__device__ __forceinline__ float wave_max(float v) {
  const int b = __float_as_int(row16_max(v));
  return fmaxf(fmaxf(__int_as_float(__builtin_amdgcn_readlane(b, 0)),
                     __int_as_float(__builtin_amdgcn_readlane(b, 16))),
               fmaxf(__int_as_float(__builtin_amdgcn_readlane(b, 32)),
                     __int_as_float(__builtin_amdgcn_readlane(b, 48))));
}

// Largest of non-negative doubles (their bit patterns order like their
// values): a 64-bit unsigned max on (hi, lo) halves.
template <int CTRL>
__device__ __forceinline__ void u64_max_step(uint32_t& hi, uint32_t& lo) {
  const uint32_t h2 = (uint32_t)dpp_i<CTRL>((int)hi), l2 = (uint32_t)dpp_i<CTRL>((int)lo);
  const bool take = (h2 > hi) || (h2 == hi && l2 > lo);
  hi = take ? h2 : hi;
  lo = take ? l2 : lo;
}
__device__ __forceinline__ double wave_max_d(double v) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  uint32_t hi = (uint32_t)(bits >> 32), lo = (uint32_t)bits;
  u64_max_step<kDppQuadSwap1>(hi, lo);
  u64_max_step<kDppQuadSwap2>(hi, lo);
  u64_max_step<kDppHalfMirror>(hi, lo);
  u64_max_step<kDppRowMirror>(hi, lo);
  unsigned long long best = 0ull;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned long long w =
        ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)hi, 16 * r) << 32) |
        (uint32_t)__builtin_amdgcn_readlane((int)lo, 16 * r);
    best = (w > best) ? w : best;
  }
  return __longlong_as_double((long long)best);
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

}  // namespace evis
