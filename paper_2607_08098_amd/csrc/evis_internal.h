// Host-side interface between the C ABI (evis_api.cpp) and the kernel
// translation units.  Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "evis.h"
#include "evis_common.h"
#include "evis_stream.h"

namespace evis {

enum Mode { MODE_STEP = 0, MODE_INTERP = 1, MODE_SOFT_FWD = 2, MODE_SOFT_BWD = 3 };

constexpr int kListCapMax = 1024;   // per-tile candidate source blocks held in LDS
constexpr int kEventBuf = 1024;     // events staged in LDS per workgroup
constexpr int kXcd = 8;             // work queues: one per accelerator complex die
constexpr int kQueueStride = 64;    // queue counters 256 bytes apart (own cache lines)

// Arguments of the fused tile kernel (all device pointers).
struct TileArgs {
  const EnvDesc* envs;
  EnvDyn* dyn;
  const int32_t* xbegin;       // [kXcd][n_envs + 1] first item of each rank in queue x
  const int32_t* env_order;    // [n_envs] env index of each rank
  int32_t n_envs;
  int32_t list_cap;
  unsigned int* queue;         // [kXcd * kQueueStride] work-queue counters, counter x at
                               // x * kQueueStride (zeroed before the launch)
  const int32_t* n_items;      // [kXcd] items of each queue
  int32_t static_tiles;
  // MODE_STEP
  evis_event* out;
  long long capacity;
  unsigned long long* cursor;
  // MODE_INTERP
  float* L_out;
  uint8_t* hole;
  int32_t j_begin, j_end;
  // MODE_SOFT_*
  const float* C_soft;         // [n_envs] per-env threshold of the surrogate
  float inv_tau;
  float* S_out;                // per env [H*W] via soft_ptrs
  const float* const* soft_S;  // [n_envs] S (fwd out)
  const float* const* soft_gS; // [n_envs] dLoss/dS (bwd in)
  float* const* soft_gLA;      // [n_envs] dL/dL_A (bwd out, accumulated)
  float* const* soft_gLB;
  float* const* soft_gmB;      // [n_envs] [H*W*2]
  float* gC;                   // [n_envs]
};

// Smooth event-count surrogate (evis_soft_count_*): per-env pointers.
struct SoftPtrs {
  const float* Lref;   // [H*W] reference level at the start of the pair
  float* S;            // [H*W] forward out
  const float* gS;     // [H*W] backward in
  float* gLA;          // [H*W] backward out (accumulated; zeroed first)
  float* gLB;
  float2* gmA;         // [H*W] backward out (written)
  float2* gmB;
};

struct SoftArgs {
  const EnvDesc* envs;
  const EnvDyn* dyn;
  const int32_t* item_prefix;   // [n_envs + 1] target tiles of each env
  const SoftPtrs* ptrs;         // [n_envs]
  int32_t n_envs;
  int32_t K;
  float inv_tau;
  int32_t list_cap;
  const float* C;               // [n_envs]
  float* gC;                    // [n_envs] (backward, accumulated; zeroed first)
  int32_t hold_ref;             // 1: the reference trajectory carries no gradient
};

constexpr int kSoftTW = 32, kSoftTH = 16;

// Kernel launchers (defined in evis_tile.hip / evis_events.hip).
hipError_t launch_soft(bool backward, const SoftArgs& a, int n_items, hipStream_t s);
hipError_t launch_soft_zero(const SoftPtrs* ptrs, const EnvDesc* envs, int n_envs, float* gC,
                            hipStream_t s);
hipError_t launch_reset(EnvDyn* dyn, int n_envs, unsigned int* queue,
                        unsigned long long* cursor, hipStream_t s);   // queue: kXcd counters
hipError_t launch_prep(const EnvDesc* envs, EnvDyn* dyn, const int32_t* src_prefix, int n_envs,
                       int total_groups, hipStream_t s);
// Per-superblock motion bounds from the per-block ones (after launch_prep).
hipError_t launch_superbounds(const EnvDesc* envs, int n_envs, int sb_max, hipStream_t s);
hipError_t launch_prep_b(const EnvDesc* envs, const int32_t* src_prefix, int n_envs,
                         int total_groups, hipStream_t s);   // two-splat warps' B records
hipError_t launch_queue(const EnvDesc* envs, EnvDyn* dyn, int n_envs, int tile_w, int tile_h,
                        int32_t* xbegin, int32_t* env_order, int32_t* n_items,
                        int32_t* K_used, hipStream_t s);
// warp: EVIS_WARP_* (the two-splat warps are launched from evis_tile_splat.hip);
// noise: the fused step with sensor-noise events (evis_tile_noise.hip)
hipError_t launch_tile(int tile_w, int tile_h, int mode, int warp, bool noise, const TileArgs& a,
                       int grid, hipStream_t s);
int tile_occupancy(int tile_w, int tile_h, int mode, int warp, bool noise);
hipError_t launch_tile_noise(int tile_w, int tile_h, int warp, const TileArgs& a, int grid,
                             hipStream_t s);
int tile_occupancy_noise(int tile_w, int tile_h, int warp);
hipError_t launch_tile_two(int tile_w, int tile_h, int mode, int warp, const TileArgs& a, int grid,
                           hipStream_t s);
int tile_occupancy_two(int tile_w, int tile_h, int mode, int warp);
bool tile_shape_supported(int tile_w, int tile_h);

hipError_t launch_log_luminance(const float* x, int channels, long long n, float eps, float* L,
                                hipStream_t s);
hipError_t launch_log_channels(const float* x, long long n, float eps, float* L, hipStream_t s);

// Event voxel grid: acc is the output grid [2][bins][H][W], used as uint32
// sums before it is normalised in place.
struct VoxelArgs {
  const evis_event* events;
  const long long* n_events;   // device cursor
  long long capacity;
  uint32_t* acc;
  uint32_t* maxbuf;            // scratch [2 * bins]: per-plane maxima
  long long t0, t1;
  float scale;                 // fl32(fl32(bins - 1) / fl32(t1 - t0))
  int32_t env_id, H, W, bins;
};
hipError_t launch_voxel(const VoxelArgs& a, hipStream_t s);

// Defocus (separable Gaussian blur of linear intensity) of up to
// kDefocusBatch images in one launch: taps w[0..2r]; image i owns output
// tiles [tile_prefix[i], tile_prefix[i + 1]).
constexpr int kDefocusMaxR = 30;
constexpr int kDefocusBatch = 64;
struct DefocusImage {
  const float* x;
  float* out;
  int32_t H, W;
  int32_t tiles_x;   // 64-wide tiles per row
  int32_t pad;
};
struct DefocusArgs {
  DefocusImage img[kDefocusBatch];
  int32_t tile_prefix[kDefocusBatch + 1];
  int32_t n, C, r;
  float w[2 * kDefocusMaxR + 1];
};
hipError_t launch_defocus(const DefocusArgs& a, hipStream_t s);
int defocus_tiles(int H, int W, int* tiles_x);
hipError_t launch_state_init(const float* L_first, long long n, float* L_ref, int32_t* t_last,
                             hipStream_t s);
// The event model over one env's frames.  Without a refractory period and
// noise it runs in the wave form, which writes through the call's sharded
// stream `st` (set up by launch_stream_init before, finished by
// launch_stream_fixup and launch_stream_clean after); otherwise in the
// workgroup form, which
// appends at the cursor (reset first if asked).
inline bool events_wave_form(int refr, bool noise) { return refr == 0 && !noise; }
hipError_t launch_events(const float* L_seq, int H, int W, int K, long long t0, int span,
                         float Dt, float C_on, float C_off, const float* th_on,
                         const float* th_off, int refr, uint32_t env_bits, float* L_ref,
                         int32_t* t_last, evis_event* out, long long capacity,
                         unsigned long long* cursor, int reset_cursor,
                         const NoiseCfg* noise /* host copy, or null: no noise */,
                         const StreamState& st, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, hipStream_t s);   // a kernel, not a memset
hipError_t launch_stream_init(const StreamState& st, unsigned long long* cursor, int reset,
                              long long capacity, bool clear_table, hipStream_t s);
hipError_t launch_stream_clean(const StreamState& st, hipStream_t s);   // after the fixup
hipError_t launch_stream_fixup(const StreamState& st, evis_event* out, long long capacity,
                               unsigned long long* cursor, hipStream_t s);
// The event model over caller frames (k_events): one env's arguments; the
// batched form (k_events_batch) reads an array of them from device memory.
struct EventArgs {
  const float* L_seq;
  int H, W, K;
  long long t0;
  int span;
  float Dt;
  float C_on, C_off;
  const float* th_on;
  const float* th_off;
  int refr;
  uint32_t env_bits;
  float* Lref;
  int32_t* tlast;
  evis_event* out;
  long long capacity;
  unsigned long long* cursor;
  NoiseCfg noise;   // used by the NOISE instantiation only
};

// Workgroups of one env in a batched event-model launch, and the launch
// (descs / prefix: device arrays of n_envs descriptors and n_envs + 1
// workgroup offsets).  wave_form: every env of the launch has no
// refractory period (k_events_batch_wave, through the sharded stream st);
// otherwise the workgroup form (at the cursor).
int events_batch_blocks(long long px);
hipError_t launch_events_batch(const EventArgs* descs, const int32_t* prefix, int n_envs,
                               int total_blocks, bool wave_form, const StreamState& st,
                               hipStream_t s);
hipError_t launch_substep_count(const float2* mA, const float2* mB, long long n, int K_max,
                                unsigned long long* msq_scratch, int32_t* K_out, hipStream_t s);

}  // namespace evis
