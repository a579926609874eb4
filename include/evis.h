/* evis.h -- C ABI of the EVIS event-generation path on AMD Instinct MI355X (gfx950).
 *
 * Paper: "EVIS: Real-Time Event Camera Simulation with Multimodal Supervision
 * in NVIDIA Isaac Sim".  For each environment and keyframe pair A (t0) -> B
 * (t1) the library takes log intensity, backward motion vectors and depth,
 * synthesises K-1 intermediate log frames by bidirectional warping with a
 * depth-tested forward splat (Sec. "Bidirectional Motion Vector Warping",
 * Eq. 5-7) and emits contrast-threshold crossings as (x, y, t, p) events
 * (Sec. "HDR Event Formation Model", Eq. 4; non-idealities Eq. 8 and the
 * refractory period of Sec. "Sensor Calibration and Non-idealities").
 *
 * Conventions shared by every call
 *  - Array arguments are DEVICE pointers owned by the caller; the library
 *    never frees them.  The library owns only the scratch inside evis_ctx.
 *    Float arrays need 4-byte alignment, motion-vector arrays and event
 *    buffers 8-byte alignment.
 *  - Images are row-major [H][W]; pixel centres sit at integer (x, y);
 *    1 <= H, W <= EVIS_MAX_DIM.
 *  - Motion vectors are [H][W][2] float32 (dx, dy) in pixels and point
 *    backward: pixel p of keyframe B sits at p + m_B(p) in keyframe A;
 *    keyframe A's own backward field m_A is reused as its forward velocity.
 *  - Depth is float32 metres; a source whose intermediate depth is not > 0
 *    (NaN included) is invisible to the splat.
 *  - Times are integer microseconds, 0 <= t0 < t1 <= 2^31 - 1 and
 *    t1 - t0 <= EVIS_MAX_SPAN_US.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream); the caller synchronises before reading results.
 *  - An argument error returns a negative status, enqueues nothing and
 *    sets evis_last_error().  One evis_ctx per host thread and stream.
 *  - Event streams are multisets: the order of events in `out` is
 *    unspecified.  `n_total` is a device int64 cursor: events are appended
 *    at out[*n_total ...] and *n_total grows by the number of events of the
 *    call, also past `capacity`; only the events whose index is below
 *    `capacity` are stored (which ones is unspecified) and the state still
 *    advances.  Pass EVIS_FLAG_RESET_CURSOR to start the cursor at 0.
 *  - Non-finite log intensities or motion vectors give unspecified events
 *    but never an access outside the arrays described here.
 */
#ifndef EVIS_H
#define EVIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EVIS_ABI_VERSION 2

#define EVIS_MAX_DIM 2047
#define EVIS_MAX_ENVS 512
#define EVIS_MAX_K 128
#define EVIS_MAX_CROSSINGS 65535       /* library limit: crossings counted per pixel and
                                          substep (Eq. 4 has no bound; an infinite |dL|
                                          counts as this many) */
#define EVIS_MAX_SPAN_US (1 << 24)
#define EVIS_T_LAST_INIT (-1073741824) /* "never fired" refractory state */

enum {
  EVIS_OK = 0,
  EVIS_ERR_INVALID = -1,     /* a bad argument; nothing was enqueued */
  EVIS_ERR_UNSUPPORTED = -2, /* valid but outside the supported range */
  EVIS_ERR_HIP = -3,         /* the HIP runtime reported an error */
  EVIS_ERR_NOMEM = -4        /* scratch allocation failed */
};

/* Blend of the two warped keyframes at fraction f (Sec. "Bidirectional
 * Motion Vector Warping", last paragraph): where both are valid the
 * sub-frame is A^ + alpha (B^ - A^). */
enum {
  EVIS_BLEND_TIME = 0,      /* alpha = f */
  EVIS_BLEND_B_PRIMARY = 1  /* alpha = 1: backward-warped B is the result, A fills B's holes */
};

/* How keyframe B is warped to fraction f (same section, Eq. 5 and Eq. 6),
 * or'ed with an EVIS_BLEND_* value into the mode word that the
 * `blend_mode` arguments and fields carry.
 *  GATHER  B is sampled bilinearly at s = q - (1 - f) m_B(q), with the
 *          motion vector at the target (exact for locally constant flow).
 *  SPLAT   B is splatted backward like A forward: source p of B goes to
 *          q_B = p + (1 - f) m_B(p) over the same footprint, depth from
 *          Eq. 7 with p_A = p + m_B(p), p_B = p (Z_A sampled with edge
 *          clamping), into a z-buffer of its own; B^ is L_B at its winner
 *          (missing where no B source landed) and the blend is as above.
 *          With EVIS_BLEND_B_PRIMARY the backward-warped B is the result
 *          and the forward-warped A fills only B's holes.
 *  JOINT   both splats into one z-buffer (Eq. 6 over both keyframes): the
 *          nearest source wins, B at equal depth, then the smaller index;
 *          the sub-frame is the winner's own intensity, and
 *          lerp(L_A(q), L_B(q), alpha) where nothing landed.
 * The hole mask marks A missing / B missing per side (JOINT: the side
 * that did not win).  The two splat warps are supported by
 * evis_interpolate and evis_step_batch (one warp for all envs of a call),
 * not by the surrogate. */
enum {
  EVIS_WARP_GATHER = 0x00,
  EVIS_WARP_SPLAT = 0x10,
  EVIS_WARP_JOINT = 0x20
};

enum { EVIS_FLAG_RESET_CURSOR = 1 };

/* One event: x in bits 0..10, y in 11..21, polarity in 22 (1 = ON), env id
 * in 23..31; t_us is the absolute time in microseconds. */
typedef struct {
  uint32_t xyp;
  int32_t t_us;
} evis_event;

/* One environment's keyframe pair A -> B (Sec. "Bidirectional Motion Vector
 * Warping").  L_* are log intensities (the output of evis_log_luminance). */
typedef struct {
  int32_t H, W;
  const float *L_A, *L_B;   /* [H*W] */
  const float *m_A, *m_B;   /* [H*W*2] backward motion vectors, px */
  const float *Z_A, *Z_B;   /* [H*W] depth */
  int64_t t0_us, t1_us;
} evis_pair;

/* Per-camera sensor model. */
typedef struct {
  float C_on, C_off;                  /* contrast thresholds (> 0) used where theta_* is NULL */
  const float *theta_on, *theta_off;  /* [H*W] per-pixel thresholds (Eq. 8) or NULL */
  int32_t refractory_us;              /* >= 0; 0 = off */
  int32_t K;                          /* > 0: fixed substep count; <= 0: adaptive */
  int32_t K_max;                      /* 1..EVIS_MAX_K, cap of the adaptive count */
  int32_t blend_mode;                 /* EVIS_BLEND_* | EVIS_WARP_* */
} evis_sensor;

/* Sensor noise (Sec. "Sensor Calibration and Non-idealities": leak events,
 * shot noise, hot pixels), added by evis_step_batch to the events of every
 * substep j = 1..K of length Dt (Dt_s = Dt * 1e-6 s, float32):
 *   leak  P = r_l Dt_s, ON events;
 *   shot  P = (r_s Dt_s)(1 - I), I = clamp((L_j - shot_L0) * shot_inv_range)
 *         into [0, 1] (NaN -> 0), L_j the pixel's current log sample;
 *         random polarity;
 *   hot   P = r_h Dt_s on a fixed set of about hot_fraction of the pixels;
 *         random polarity.
 * Every draw comes from Philox4x32-10 (Salmon et al., SC 2011) with key
 * `seed` (low word first) and counter (x | y << 11, j, pair_index, kind):
 * kind 0 holds the three decisions of a pixel-substep (words 0, 1, 2 as
 * uniforms (w >> 8) 2^-24, an event when the uniform is < P), kinds 1-3 the
 * time t0 + min(floor((j - 1 + u) Dt), t1 - t0) and polarity (bit 0 of
 * word 1) of a leak, shot or hot event, kind 4 with j = pair = 0 the hot
 * set (word 0's uniform < hot_fraction).  Noise events do not move L_ref,
 * ignore the refractory period and leave t_last alone.  Give each env its
 * own seed and advance pair_index once per keyframe pair. */
typedef struct {
  float leak_rate_hz;     /* r_l >= 0, per pixel */
  float shot_rate_hz;     /* r_s >= 0, per pixel at normalised intensity 0 */
  float hot_rate_hz;      /* r_h >= 0, per hot pixel */
  float hot_fraction;     /* in [0, 1] */
  float shot_L0;          /* log intensity of normalised intensity 0 */
  float shot_inv_range;   /* normalised intensity per unit of log intensity (finite) */
  uint64_t seed;
  uint32_t pair_index;
  uint32_t reserved;
} evis_noise;

/* Per-pixel state carried from pair to pair (caller-owned device arrays). */
typedef struct {
  float *L_ref;     /* [H*W] reference log level of each pixel (Eq. 4) */
  int32_t *t_last;  /* [H*W] time of the last emitted event; may be NULL when refractory_us == 0 */
} evis_state;

typedef struct {
  evis_pair pair;
  evis_sensor sensor;
  evis_state state;
  int32_t env_id;             /* 0..EVIS_MAX_ENVS-1, written into each event */
  int32_t crop_margin;        /* over-render margin m >= 0 (0 = none), see evis_step_batch */
  const evis_noise *noise;    /* HOST pointer, or NULL: no noise events */
} evis_env;

typedef struct evis_ctx evis_ctx;

/* Lifetime.  evis_create binds the context to HIP device `device` and
 * allocates nothing else until a call needs scratch.  Returns EVIS_OK or a
 * negative status (ctx is then NULL). */
int evis_create(evis_ctx **ctx, int device);
void evis_destroy(evis_ctx *ctx);
/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char *evis_last_error(const evis_ctx *ctx);
int evis_abi_version(void);

/* Log intensity -- Eq. 3 Rec.709 luminance and the log intensity below it:
 * L = ln(Y + eps).  x is [n] luminance (channels == 1) or [n][3] linear RGB
 * (channels == 3); L_out is [n].  float32 arithmetic with the library's own
 * logarithm.  eps > 0. */
int evis_log_luminance(evis_ctx *ctx, const float *x, int32_t channels, int64_t n, float eps,
                       float *L_out, void *stream);

/* Defocus (Sec. "Sensor Calibration and Non-idealities": before event
 * generation the linear intensity is convolved with a separable Gaussian):
 * x and out are [H][W] (channels == 1) or [H][W][3] linear intensity,
 * out must not overlap x.  Taps k = -r..r, r = ceil(3 sigma), weights
 * exp(-k^2 / (2 sigma^2)) normalised to sum 1 (computed in double, used in
 * float32), edge pixels repeated; along x, then along y, each sum taken
 * in tap order in float32.  0 < sigma <= EVIS_MAX_DEFOCUS_SIGMA;
 * 1 <= H, W <= EVIS_MAX_DEFOCUS_DIM.  Apply it to the radiance before
 * evis_log_luminance. */
#define EVIS_MAX_DEFOCUS_SIGMA 10.0f
#define EVIS_MAX_DEFOCUS_DIM 16384
int evis_defocus(evis_ctx *ctx, const float *x, int32_t H, int32_t W, int32_t channels, float sigma,
                 float *out, void *stream);

/* The same blur of n images (imgs a HOST array; each image's own H, W;
 * the same channels and sigma), as few launches as possible (up to 64
 * images share one), so that many small frames fill the GPU. */
typedef struct {
  const float *x;
  float *out;
  int32_t H, W;
} evis_image;
int evis_defocus_batch(evis_ctx *ctx, const evis_image *imgs, int32_t n, int32_t channels,
                       float sigma, void *stream);

/* Colour events (Sec. "HDR Event Formation Model": each of R, G, B in
 * place of the luminance): x is [n][3] linear RGB, L_out is [3][n]
 * (channel-major), L_c = ln(x_c + eps) with the library's own logarithm.
 * Each channel plane is then the log frame of an env of its own (same
 * motion vectors and depth; give each channel its own env_id, state and
 * thresholds), so evis_step_batch emits the three colour streams in one
 * launch.  eps > 0. */
int evis_log_channels(evis_ctx *ctx, const float *x, int64_t n, float eps, float *L_out,
                      void *stream);

/* Initialise a pixel state from the first log frame: L_ref = L_first and,
 * when t_last is non-NULL, t_last = EVIS_T_LAST_INIT. */
int evis_state_init(evis_ctx *ctx, const float *L_first, int32_t H, int32_t W,
                    const evis_state *state, void *stream);

/* Substep count of one pair: the smallest K >= 1 with K^2 >= the
 * largest finite |m|^2 over m_A and m_B (float64), at most K_max; so no
 * motion vector moves a pixel by more than one pixel per substep.
 * K_out is a device int32. */
int evis_substep_count(evis_ctx *ctx, const evis_pair *pair, int32_t K_max, int32_t *K_out,
                       void *stream);

/* Sub-frames -- intermediate log frames j in [j_begin, j_end) of K (0 <= j_begin <
 * j_end <= K + 1, 1 <= K <= EVIS_MAX_K).  j = 0 and j = K return L_A and
 * L_B verbatim.  For 0 < j < K, f = j/K: keyframe A is splatted forward to
 * q = p - f m_A(p) over the bilinear footprint (corners with positive
 * weight), a 64-bit (depth bits << 32 | source index) z-buffer keeps the
 * nearest source (Eq. 6; depth from Eq. 7 with p_B = p - m_A(p), Z_B
 * sampled with edge clamping); keyframe B is warped per the mode word's
 * EVIS_WARP_* (default: gathered bilinearly at s = q - (1 - f) m_B(q));
 * the two are blended per its EVIS_BLEND_*, each side alone where the
 * other is missing, and lerp(L_A(q), L_B(q), alpha) where both are
 * missing.  L_out is [(j_end - j_begin)][H*W]; hole_mask (nullable) is the
 * same shape in bytes: bit 0 = A missing (no A source landed), bit 1 = B
 * missing (gather: s outside the image; splat: no B source landed). */
int evis_interpolate(evis_ctx *ctx, const evis_pair *pair, int32_t K, int32_t j_begin,
                     int32_t j_end, int32_t blend_mode, float *L_out, uint8_t *hole_mask,
                     void *stream);

/* Events from caller-supplied log frames L_seq[0..K] ([K+1][H*W];
 * L_seq[0] is the previous sample, events come from j = 1..K) between
 * t0_us and t1_us.  Per pixel and substep j: d = L_j - L_ref, polarity
 * sgn d, threshold c = theta_on/C_on or theta_off/C_off, n = floor(|d|/c)
 * exactly (Eq. 4), each crossing timed by linear interpolation of L between
 * L_{j-1} and L_j and floored to whole microseconds, dropped when the
 * refractory period has not elapsed since the last emitted event; then
 * L_ref moves by n*c (suppressed crossings included).  `state` is updated
 * in place.  The sensor's K, K_max and blend_mode are ignored here. */
int evis_generate_events(evis_ctx *ctx, const float *L_seq, int32_t H, int32_t W, int32_t K,
                         int64_t t0_us, int64_t t1_us, const evis_sensor *sensor,
                         const evis_state *state, int32_t env_id, evis_event *out,
                         int64_t capacity, int64_t *n_total, int32_t flags, void *stream);
/* The same with sensor noise (evis_noise, a HOST pointer; NULL = none),
 * drawn exactly as in evis_step_batch with this call's Dt and the pixel's
 * own coordinates. */
int evis_generate_events_noise(evis_ctx *ctx, const float *L_seq, int32_t H, int32_t W, int32_t K,
                               int64_t t0_us, int64_t t1_us, const evis_sensor *sensor,
                               const evis_state *state, int32_t env_id, const evis_noise *noise,
                               evis_event *out, int64_t capacity, int64_t *n_total,
                               int32_t flags, void *stream);

/* One env of a batch of the event model on caller frames: its samples
 * L_seq[0..K] ([K+1][H*W], device), times, sensor (C_on, C_off, theta_*,
 * refractory_us; K, K_max and blend_mode ignored), state and env id. */
typedef struct {
  const float *L_seq;
  int32_t H, W, K;
  int32_t env_id;
  int64_t t0_us, t1_us;
  evis_sensor sensor;
  evis_state state;
} evis_frames;

/* evis_generate_events for n_envs envs (1..EVIS_MAX_ENVS; envs is a HOST
 * array) in one launch: the same events, states and limits as one call per
 * env, all appended to one stream (Eq. 4, Eq. 8 and the refractory period
 * as above; no sensor noise).  Host-detected errors in any env enqueue
 * nothing. */
int evis_generate_events_batch(evis_ctx *ctx, const evis_frames *envs, int32_t n_envs,
                               evis_event *out, int64_t capacity, int64_t *n_total, int32_t flags,
                               void *stream);

/* Fused step -- one keyframe pair for each of n_envs environments
 * (1..EVIS_MAX_ENVS; envs is a HOST array of descriptors) in one
 * persistent launch: substep count, sub-frames and events of every env,
 * all events appended to one stream.  All envs of a call use the same
 * EVIS_WARP_* (else EVIS_ERR_UNSUPPORTED); blends may differ.  An env's
 * crop_margin m (0 <= 2m < min(H, W)) marks an over-rendered margin of m
 * pixels on every side (Sec. "Bidirectional Motion Vector Warping", last
 * paragraph): the warp uses the whole frame, only the inner
 * (H - 2m) x (W - 2m) pixels reach the event model and its noise, their
 * events carry the cropped frame's coordinates, and L_ref / t_last of the
 * margin are left untouched.  env.noise (nullable) adds sensor noise.  K_used (device [n_envs], nullable)
 * receives each env's K.  States are updated in place.  The launch
 * sequence is captured once into a HIP graph per (n_envs, out, cursor,
 * K_used, tuning) and replayed. */
int evis_step_batch(evis_ctx *ctx, const evis_env *envs, int32_t n_envs, evis_event *out,
                    int64_t capacity, int64_t *n_total, int32_t *K_used, int32_t flags,
                    void *stream);

/* evis_step_batch for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, but every scratch buffer of the call (descriptor
 * block, per-env substep counts, work queues, splat records, block bounds)
 * sits in one static device array of EVIS_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends.  The call
 * allocates nothing: no hipMalloc, hipFree or pinned host memory (the
 * descriptor block goes up through the context's staging ring, allocated by
 * evis_create), and it launches directly (no graph) with the context's
 * tuning.  Limit: the scratch a batch needs is about 17 bytes per pixel
 * (34 for the two-splat warps) plus 1 KB per env; a batch that needs more
 * than the array returns EVIS_ERR_UNSUPPORTED and enqueues nothing (64 MiB
 * hold about 3.8 M pixels, e.g. four 1280x720 envs).  Every call on one GPU
 * shares that GPU's array, from any context: calls that overlap on one GPU
 * (two streams, two threads, two contexts) race and must be serialised by
 * the caller.  Arguments, errors and results as evis_step_batch. */
#define EVIS_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
int evis_step_batch_noalloc(evis_ctx *ctx, const evis_env *envs, int32_t n_envs, evis_event *out,
                            int64_t capacity, int64_t *n_total, int32_t *K_used, int32_t flags,
                            void *stream);

/* Tuning of the fused launch: target tile shape and persistent grid size.
 * tile_w x tile_h in {16x16, 32x16, 32x32, 64x16, 64x32}; grid_mult >= 1
 * workgroups per compute unit (0 = occupancy limit); list_cap in 1..1024
 * caps the per-tile candidate list (the two-splat warps, whose list holds
 * both directions, take twice as many; smaller values force the
 * window-scan fallback; 0 = the maximum); use_graph 0/1. */
typedef struct {
  int32_t tile_w, tile_h;
  int32_t grid_mult;
  int32_t list_cap;
  int32_t use_graph;
  int32_t static_tiles;   /* 1 = skip warping of provably static tiles */
} evis_tuning;

int evis_get_tuning(const evis_ctx *ctx, evis_tuning *out);
int evis_set_tuning(evis_ctx *ctx, const evis_tuning *tuning);

/* Search the launch schedule on this batch and keep the fastest in ctx
 * (states and *n_total are restored afterwards from a private copy; each
 * trial times reps launches after one untimed launch).  The search runs
 * one axis at a time, each from the best point so far:
 *   1. tile shape, i.e. pixels per thread: 16x16 (1), 32x16 (2), 32x32 (4),
 *      64x16 (4); one or two pixels per thread are compiled for 4 waves per
 *      SIMD, four for 2 (64x32, eight per thread at 1 wave, is settable but
 *      not searched);
 *   2. grid_mult: the occupancy limit, then one and two workgroups per CU
 *      fewer;
 *   3. list_cap: 1024, 512, 256 candidate source blocks per tile.
 * best (host, nullable) receives the winner, best_ms (host, nullable) its
 * mean launch time in ms. */
int evis_autotune(evis_ctx *ctx, const evis_env *envs, int32_t n_envs, evis_event *out,
                  int64_t capacity, int64_t *n_total, int32_t reps, evis_tuning *best,
                  float *best_ms, void *stream);

/* One trial of the schedule search: the tuning and its mean launch time in
 * ms (negative if the trial failed). */
typedef struct {
  evis_tuning tuning;
  float ms;
  int32_t reserved;
} evis_tune_trial;

/* evis_autotune with a cache and the trials reported.  cache_path (host
 * string, nullable: no cache) names a text file of one JSON object per line,
 *   {"key": "...", "tile_w": W, "tile_h": H, "grid_mult": G, "list_cap": L, "ms": T}
 * keyed by the GPU architecture, this library build, the warp mode, the
 * noise flag, the sorted multiset of env sizes and the pixel-weighted mean
 * substep count of the batch rounded up to a power of two (measured by one
 * launch).  A key found there is applied without a search (*from_cache = 1,
 * no trials); otherwise the search runs and its winner is appended.
 * trials (host, nullable, max_trials entries) receive the trials in search
 * order, *n_trials (nullable) their number; from_cache nullable.  The
 * library opens the file only inside this call. */
int evis_autotune_ex(evis_ctx *ctx, const evis_env *envs, int32_t n_envs, evis_event *out,
                     int64_t capacity, int64_t *n_total, int32_t reps, const char *cache_path,
                     evis_tuning *best, float *best_ms, evis_tune_trial *trials,
                     int32_t max_trials, int32_t *n_trials, int32_t *from_cache, void *stream);

/* Smooth event-count surrogate and its gradient (a differentiable stand-in
 * for the crossing count of Eq. 4 that lets a contrast threshold and flow
 * corrections be fitted by gradient descent).  Per pixel
 *   S = sum_{j=1..K} sigmoid((|L_j - R_{j-1}| - C) / tau)
 * with L_j the sub-frames of evis_interpolate (same warp, same blend) and
 * R_0 = L_ref, R_j = R_{j-1} + p_j n_j C the hard reference level of Eq. 4
 * with threshold C both ways (integer counts n_j, polarity p_j).  Where the
 * counts do not change R does not move with L, and dR_j/dC = sum of p n up
 * to j; the gradient of C includes that term.  The backward pass returns dLoss/dL_A,
 * dLoss/dL_B, dLoss/dm_A (zero: the splat takes the winner's value, which
 * does not move with m_A), dLoss/dm_B (through the gather position) and
 * dLoss/dC per env, for a given dLoss/dS.  float32; gradients of L_A and L_B
 * are accumulated with atomics, so their last bits depend on ordering. */
typedef struct {
  evis_pair pair;       /* t0_us / t1_us are ignored */
  const float *L_ref;   /* [H*W] */
  float *S;             /* [H*W] forward output */
  const float *gS;      /* [H*W] backward input */
  float *gL_A, *gL_B;   /* [H*W] backward outputs (overwritten) */
  float *gm_A, *gm_B;   /* [H*W*2] backward outputs (overwritten) */
} evis_soft_env;

/* flags of evis_soft_count_backward: with EVIS_SOFT_HOLD_REF the reference
 * trajectory is treated as a constant (stop-gradient), so dS/dC is only the
 * direct -sigma'/tau term; without it dC also flows through R. */
enum { EVIS_SOFT_HOLD_REF = 1 };

/* K in 1..EVIS_MAX_K (same for all envs), tau > 0, blend_mode EVIS_BLEND_*
 * (the gather warp only; a splat warp is EVIS_ERR_UNSUPPORTED),
 * C a DEVICE float array [n_envs] (> 0), gC a DEVICE float array [n_envs],
 * flags 0 or EVIS_SOFT_HOLD_REF. */
int evis_soft_count_forward(evis_ctx *ctx, const evis_soft_env *envs, int32_t n_envs, int32_t K,
                            float tau, int32_t blend_mode, const float *C, void *stream);
int evis_soft_count_backward(evis_ctx *ctx, const evis_soft_env *envs, int32_t n_envs, int32_t K,
                             float tau, int32_t blend_mode, const float *C, float *gC,
                             int32_t flags, void *stream);

/* Event voxel grid (the per-polarity, 128-bin input of the paper's speed
 * estimator, Sec. "Sim-to-Real Rotational Speed Estimation" and its
 * appendix): events[0 .. min(*n_events, capacity)) (n_events a DEVICE
 * int64, e.g. the cursor of evis_step_batch) of env env_id with
 * t0_us <= t < t1_us sit at tau = (t - t0)(bins - 1)/(t1 - t0) on the axis
 * of bin centres and are spread over bins floor(tau) and floor(tau) + 1 by
 * linear interpolation in time; each (polarity, bin) plane is then divided
 * by its maximum (all zero when empty).
 * Number format (the library's, within a derived bound of the real-valued
 * grid): tau from the float32 scale fl32(fl32(bins - 1) / fl32(t1 - t0)),
 * the fraction q floored to 16 bits, 1 - q and q summed as uint32 fixed
 * point (exact and independent of event order), one float32 division per
 * voxel.  Limit: a voxel holds at most 65535 full-weight events per call
 * (beyond that its uint32 sum wraps and the grid is not defined).
 * out is [2][bins][H][W] float32, polarity 0 (OFF) first; it is also the
 * accumulator.  2 <= bins <= EVIS_MAX_VOXEL_BINS. */
#define EVIS_MAX_VOXEL_BINS 1024
int evis_voxel_grid(evis_ctx *ctx, const evis_event *events, const int64_t *n_events,
                    int64_t capacity, int32_t env_id, int32_t H, int32_t W, int64_t t0_us,
                    int64_t t1_us, int32_t bins, float *out, void *stream);

/* Kernel timing.  While profiling is enabled, each call records HIP events
 * on its stream around its main kernel (the fused tile kernel of
 * evis_step_batch, the tile kernel of evis_interpolate, the event kernel
 * of evis_generate_events); evis_step_batch then launches directly
 * instead of replaying its graph.  evis_profile_read waits for the
 * recorded events of one kind, returns their summed duration and count,
 * and forgets them. */
enum { EVIS_KERNEL_STEP = 0, EVIS_KERNEL_INTERP = 1, EVIS_KERNEL_EVENTS = 2 };
int evis_profile_enable(evis_ctx *ctx, int32_t enable);
int evis_profile_read(evis_ctx *ctx, int32_t kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* EVIS_H */
