// The fused tile kernel with the two-splat warps (B splatted backward to
// Eq. 5's q_B; one z-buffer per direction, or one shared by both as in
// Eq. 6): instantiations and launchers (gfx950).
#include "evis_tile_kernel.h"

namespace evis {

template <int TW, int TH, int WARP>
static hipError_t launch_two_shape(int mode, const TileArgs& a, int grid, hipStream_t s) {
  switch (mode) {
    case MODE_STEP:
      hipLaunchKernelGGL((k_tile<TW, TH, MODE_STEP, WARP>), dim3(grid), dim3(kBlock), 0, s, a);
      break;
    case MODE_INTERP:
      hipLaunchKernelGGL((k_tile<TW, TH, MODE_INTERP, WARP>), dim3(grid), dim3(kBlock), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TW, int TH, int WARP>
static int occupancy_two_shape(int mode) {
  int nb = 0;
  hipError_t err = hipErrorInvalidValue;
  if (mode == MODE_STEP)
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile<TW, TH, MODE_STEP, WARP>, kBlock, 0);
  else if (mode == MODE_INTERP)
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile<TW, TH, MODE_INTERP, WARP>, kBlock, 0);
  return (err == hipSuccess && nb > 0) ? nb : 1;
}

#define EVIS_TWO_SHAPES(X) X(16, 16) X(32, 16) X(32, 32) X(64, 16) X(64, 32)

hipError_t launch_tile_two(int tw, int th, int mode, int warp, const TileArgs& a, int grid,
                           hipStream_t s) {
#define X(W_, H_)                                                                        \
  if (tw == W_ && th == H_) {                                                            \
    if (warp == EVIS_WARP_SPLAT) return launch_two_shape<W_, H_, EVIS_WARP_SPLAT>(mode, a, grid, s); \
    if (warp == EVIS_WARP_JOINT) return launch_two_shape<W_, H_, EVIS_WARP_JOINT>(mode, a, grid, s); \
    return hipErrorInvalidValue;                                                         \
  }
  EVIS_TWO_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

int tile_occupancy_two(int tw, int th, int mode, int warp) {
  // Cached per (shape, warp, mode), as for the gather warp: no runtime query
  // while a launch sequence is being captured.
  static int cache[5][2][2] = {};
  const int wi = (warp == EVIS_WARP_JOINT) ? 1 : 0;
  if (mode != MODE_STEP && mode != MODE_INTERP) return 1;
  int idx = 0;
#define X(W_, H_)                                                                   \
  if (tw == W_ && th == H_) {                                                       \
    if (cache[idx][wi][mode] == 0)                                                  \
      cache[idx][wi][mode] = wi ? occupancy_two_shape<W_, H_, EVIS_WARP_JOINT>(mode) \
                                : occupancy_two_shape<W_, H_, EVIS_WARP_SPLAT>(mode); \
    return cache[idx][wi][mode];                                                    \
  }                                                                                 \
  ++idx;
  EVIS_TWO_SHAPES(X)
#undef X
  return 1;
}

}  // namespace evis
