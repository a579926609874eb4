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
// 4x4 source blocks carry motion bounds (from the prep kernel), and each
// candidate's interval of substeps [j_lo, j_hi] during which its footprint
// can touch the tile is kept in an LDS list.
#include "evis_tile_kernel.h"

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
  // the env's largest |m|^2 seen by this lane; reduced over the wave and
  // published when the env changes (wave-uniform calls)
  int run_env = -1;
  double run_msq = 0.0;
  auto publish = [&]() {
    const double m = wave_max_d(run_msq);
    if (run_env >= 0 && m > 0.0 && lane == 0)
      atomicMax(&dyn[run_env].msq_bits, (unsigned long long)__double_as_longlong(m));
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

// Two-splat warps only: per 4x4 source block (a row of 16 lanes, four
// blocks per wave), B's splat record (-m_B.x, -m_B.y, Zstart, Z_B -
// Zstart), Zstart = Z_A at p + m_B(p) (edge-clamped; Eq. 7 with
// p_A = p + m_B(p), p_B = p), and the block's bounds of -m_B over sources
// with a finite motion vector.
__global__ __launch_bounds__(kBlock) void k_prep_b(const EnvDesc* __restrict__ envs,
                                                   const int32_t* __restrict__ src_prefix,
                                                   int n_envs, int total) {
  __shared__ int s_prefix[EVIS_MAX_ENVS + 1];
  for (int i = threadIdx.x; i <= n_envs; i += kBlock) s_prefix[i] = src_prefix[i];
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int g = lane >> 4, r = lane & (kBlkPx - 1);
  const int nwaves = (int)gridDim.x * kWavesPerBlock;
  const float inf = __int_as_float(0x7f800000);
  for (int gt = blockIdx.x * kWavesPerBlock + (int)(threadIdx.x / kWave); gt < total; gt += nwaves) {
    int lo = 0, hi = n_envs - 1;   // env of block group gt (wave-uniform)
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_prefix[mid] <= gt) lo = mid; else hi = mid - 1;
    }
    const EnvDesc& d = envs[lo];
    if (d.warp == EVIS_WARP_GATHER) continue;
    const int blk = (gt - s_prefix[lo]) * 4 + g;
    const bool has = blk < d.ntx_src * d.nty_src;
    const int bx = has ? blk % d.ntx_src : 0, by = has ? blk / d.ntx_src : 0;
    const int x = bx * kSrcBlk + (r & 3), y = by * kSrcBlk + (r >> 2);
    const bool in = has && x < d.W && y < d.H;
    const int p = in ? y * d.W + x : 0;
    const float2 mb = ldg(d.mB, p);
    const float zb = ldg(d.ZB, p);
    const float sx = clamp_into((float)x + mb.x, (float)(d.W - 1));
    const float sy = clamp_into((float)y + mb.y, (float)(d.H - 1));
    const float zs = bilinear(d.ZA, d.H, d.W, sx, sy);
    float mnx = inf, mxx = -inf, mny = inf, mxy = -inf;
    if (in && finite32(mb.x) && finite32(mb.y)) {
      mnx = mxx = -mb.x;
      mny = mxy = -mb.y;
    }
    if (has)
      stg(d.srcB, blk * kBlkPx + r,
          in ? make_float4(-mb.x, -mb.y, zs, zb - zs) : make_float4(0.f, 0.f, 0.f, 0.f));
    mnx = row16_min(mnx);
    mxx = row16_max(mxx);
    mny = row16_min(mny);
    mxy = row16_max(mxy);
    if (r == 0 && has) stg(d.tbB, blk, make_float4(mnx, mxx, mny, mxy));
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
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_reset(EnvDyn* dyn, int n_envs, unsigned int* queue, unsigned long long* cursor,
                        hipStream_t s) {
  const int n = max(n_envs, kXcd);
  hipLaunchKernelGGL(k_reset, dim3((n + 255) / 256), dim3(256), 0, s, dyn, n_envs, queue, cursor);
  return hipGetLastError();
}

hipError_t launch_prep(const EnvDesc* envs, EnvDyn* dyn, const int32_t* src_prefix, int n_envs,
                       int total_groups, hipStream_t s) {
  if (total_groups <= 0) return hipSuccess;
  // a run of block groups per wave: 256 CUs x 8 workgroups at most
  const int blocks = std::min((total_groups + kWavesPerBlock - 1) / kWavesPerBlock, 256 * 8);
  hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(kBlock), 0, s, envs, dyn, src_prefix, n_envs,
                     total_groups);
  return hipGetLastError();
}

// Motion bounds of each superblock (kSbBlk x kSbBlk source blocks): the
// minima and maxima of its blocks' bounds (a block with no finite source
// holds +inf minima and -inf maxima, which change nothing).  One thread per
// superblock; workgroup row y is env y.
__global__ __launch_bounds__(kBlock) void k_superbounds(const EnvDesc* __restrict__ envs) {
  const EnvDesc& d = envs[blockIdx.y];
  const int sb = blockIdx.x * kBlock + threadIdx.x;
  if (sb >= d.ntx_sb * d.nty_sb) return;
  const int sx = sb % d.ntx_sb, sy = sb / d.ntx_sb;
  const float inf = __int_as_float(0x7f800000);
  float4 m = make_float4(inf, -inf, inf, -inf);
  const int bx1 = min((sx + 1) * kSbBlk, d.ntx_src), by1 = min((sy + 1) * kSbBlk, d.nty_src);
  for (int by = sy * kSbBlk; by < by1; ++by) {
    for (int bx = sx * kSbBlk; bx < bx1; ++bx) {
      const float4 b = ldg(d.tb, by * d.ntx_src + bx);
      m.x = fminf(m.x, b.x);
      m.y = fmaxf(m.y, b.y);
      m.z = fminf(m.z, b.z);
      m.w = fmaxf(m.w, b.w);
    }
  }
  stg(d.sbb, sb, m);
}

hipError_t launch_superbounds(const EnvDesc* envs, int n_envs, int sb_max, hipStream_t s) {
  if (n_envs <= 0 || sb_max <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_superbounds, dim3((sb_max + kBlock - 1) / kBlock, n_envs), dim3(kBlock), 0,
                     s, envs);
  return hipGetLastError();
}

hipError_t launch_prep_b(const EnvDesc* envs, const int32_t* src_prefix, int n_envs,
                         int total_groups, hipStream_t s) {
  if (total_groups <= 0) return hipSuccess;
  const int blocks = std::min((total_groups + kWavesPerBlock - 1) / kWavesPerBlock, 256 * 8);
  hipLaunchKernelGGL(k_prep_b, dim3(blocks), dim3(kBlock), 0, s, envs, src_prefix, n_envs,
                     total_groups);
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

hipError_t launch_tile(int tw, int th, int mode, int warp, bool noise, const TileArgs& a, int grid,
                       hipStream_t s) {
  if (noise && mode == MODE_STEP) return launch_tile_noise(tw, th, warp, a, grid, s);
  if (warp != EVIS_WARP_GATHER) return launch_tile_two(tw, th, mode, warp, a, grid, s);
#define X(W_, H_) if (tw == W_ && th == H_) return launch_tile_shape<W_, H_>(mode, a, grid, s);
  EVIS_TILE_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

int tile_occupancy(int tw, int th, int mode, int warp, bool noise) {
  if (noise && mode == MODE_STEP) return tile_occupancy_noise(tw, th, warp);
  if (warp != EVIS_WARP_GATHER) return tile_occupancy_two(tw, th, mode, warp);
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
