// The fused step with sensor-noise events (leak, shot noise, hot pixels
// drawn from Philox4x32-10) for every warp: instantiations and launchers
// (gfx950).
#include "evis_tile_kernel.h"

namespace evis {

#define EVIS_NOISE_SHAPES(X) X(16, 16) X(32, 16) X(32, 32) X(64, 16) X(64, 32)

template <int TW, int TH, int WARP>
static hipError_t launch_noise_shape(const TileArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_tile<TW, TH, MODE_STEP, WARP, 1>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int TW, int TH, int WARP>
static int occupancy_noise_shape() {
  int nb = 0;
  const hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &nb, k_tile<TW, TH, MODE_STEP, WARP, 1>, kBlock, 0);
  return (err == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_tile_noise(int tw, int th, int warp, const TileArgs& a, int grid, hipStream_t s) {
#define X(W_, H_)                                                                                \
  if (tw == W_ && th == H_) {                                                                    \
    if (warp == EVIS_WARP_GATHER) return launch_noise_shape<W_, H_, EVIS_WARP_GATHER>(a, grid, s); \
    if (warp == EVIS_WARP_SPLAT) return launch_noise_shape<W_, H_, EVIS_WARP_SPLAT>(a, grid, s);   \
    if (warp == EVIS_WARP_JOINT) return launch_noise_shape<W_, H_, EVIS_WARP_JOINT>(a, grid, s);   \
    return hipErrorInvalidValue;                                                                 \
  }
  EVIS_NOISE_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

int tile_occupancy_noise(int tw, int th, int warp) {
  // Cached per (shape, warp): no runtime query while a launch sequence is
  // being captured.
  static int cache[5][3] = {};
  const int wi = (warp == EVIS_WARP_SPLAT) ? 1 : (warp == EVIS_WARP_JOINT) ? 2 : 0;
  int idx = 0;
#define X(W_, H_)                                                                 \
  if (tw == W_ && th == H_) {                                                     \
    if (cache[idx][wi] == 0)                                                      \
      cache[idx][wi] = wi == 0   ? occupancy_noise_shape<W_, H_, EVIS_WARP_GATHER>() \
                       : wi == 1 ? occupancy_noise_shape<W_, H_, EVIS_WARP_SPLAT>()  \
                                 : occupancy_noise_shape<W_, H_, EVIS_WARP_JOINT>(); \
    return cache[idx][wi];                                                        \
  }                                                                               \
  ++idx;
  EVIS_NOISE_SHAPES(X)
#undef X
  return 1;
}

}  // namespace evis
