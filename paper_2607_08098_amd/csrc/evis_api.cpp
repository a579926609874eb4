// C ABI of libevis: argument validation, per-context scratch, descriptor
// upload, HIP graph capture/replay of the fused launch, tuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "evis.h"
#include "evis_internal.h"

using namespace evis;

// Scratch of evis_step_batch_noalloc: device memory the library holds from
// load to process end (each GPU its own copy), so that entry point allocates
// nothing.  In host code this name is a host-side stand-in, never a device
// address: the address comes from hipGetSymbolAddress, once per device, at
// evis_create (noalloc_scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[EVIS_NOALLOC_SCRATCH_BYTES];

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

constexpr int kStageSlots = 4;

// Fixed-capacity vector: a call's descriptor plan lives on the stack, so no
// call allocates host memory for it (the capacity is the ABI's env limit).
template <typename T, int N>
struct FixedVec {
  T v[N];
  int n = 0;
  int size() const { return n; }
  bool empty() const { return n == 0; }
  void clear() { n = 0; }
  void push_back(const T& x) { v[n++] = x; }   // callers keep n <= N
  void assign(int m, const T& x) {
    n = m;
    for (int i = 0; i < m; ++i) v[i] = x;
  }
  T& operator[](int i) { return v[i]; }
  const T& operator[](int i) const { return v[i]; }
  T& back() { return v[n - 1]; }
  T* data() { return v; }
  const T* data() const { return v; }
  const T* begin() const { return v; }
  const T* end() const { return v + n; }
};

// Largest descriptor block of one call: EnvDesc per env plus the prefix table.
constexpr size_t kMetaMax = EVIS_MAX_ENVS * sizeof(EnvDesc) + (EVIS_MAX_ENVS + 1) * sizeof(int32_t);
using Blob = FixedVec<unsigned char, (int)kMetaMax>;

}  // namespace

struct evis_ctx {
  int device = 0;
  int n_cu = 256;
  std::string err;
  hipStream_t capture_stream = nullptr;
  // device scratch
  DevBuf meta;        // EnvDesc[n] followed by int32 src_prefix[n + 1]
  DevBuf dyn;         // EnvDyn[n]
  DevBuf sched;       // xbegin[8][n + 1], env_order[n], n_items[8], queue counters (256 B apart)
  DevBuf src;         // float4[16 per 4x4 source block]: per-source splat records
  DevBuf tb;          // float4[per 4x4 source block]: motion bounds
  DevBuf srcB;        // two-splat warps: B's splat records, same layout as src
  DevBuf tbB;         // two-splat warps: bounds of -m_B per block
  DevBuf sbb;         // motion bounds per superblock of source blocks
  DevBuf msq;         // one u64 for evis_substep_count
  DevBuf soft;        // item prefix + SoftPtrs of the surrogate calls
  DevBuf voxmax;      // per-plane maxima of evis_voxel_grid
  DevBuf evb;         // evis_generate_events_batch: EventArgs[n], then two int32 prefixes
  DevBuf evs;         // the sharded event stream of the wave-form event model
  bool evs_table_clean = false;   // its chunk table is all unpublished
  std::vector<unsigned char> soft_shadow;
  // host staging of the descriptor block (pinned ring)
  void* stage[kStageSlots] = {};
  size_t stage_bytes = 0;
  hipEvent_t stage_ev[kStageSlots] = {};
  int stage_next = 0;
  std::vector<unsigned char> shadow;   // what d_meta currently holds
  // the static scratch of evis_step_batch_noalloc on this context's device
  unsigned char* noalloc_scratch = nullptr;
  // graphs
  std::map<std::string, GraphEntry> graphs;
  evis_tuning tuning{32, 32, 0, kListCapMax, 1, 1};
  // kernel timing
  bool prof = false;
  struct Rec { int kind; hipEvent_t e0, e1; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> ev_pool;
};

namespace {

hipEvent_t pool_event(evis_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Start / stop a timed region around one kernel on stream s (profiling only).
struct ProfScope {
  evis_ctx* ctx;
  int kind;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(evis_ctx* c, int k, hipStream_t st) : ctx(c), kind(k), s(st) {
    if (!ctx->prof) return;
    e0 = pool_event(ctx);
    e1 = pool_event(ctx);
    if (e0) hipEventRecord(e0, s);
  }
  ~ProfScope() {
    if (!ctx->prof || !e0 || !e1) return;
    hipEventRecord(e1, s);
    ctx->recs.push_back({kind, e0, e1});
  }
};

int fail(evis_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(evis_ctx* c, hipError_t e, const char* where) {
  return fail(c, EVIS_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define EVIS_HIP(call, where)                      \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
  } while (0)

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int ensure(evis_ctx* ctx, DevBuf& b, size_t bytes, bool* grew = nullptr) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return EVIS_OK;
  if (b.p) {
    hipDeviceSynchronize();
    hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max(bytes, (size_t)4096);
  want = (want + 255) & ~(size_t)255;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(ctx, EVIS_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  b.bytes = want;
  if (grew) *grew = true;
  return EVIS_OK;
}

void drop_graphs(evis_ctx* ctx) {
  for (auto& kv : ctx->graphs) {
    if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) hipGraphDestroy(kv.second.graph);
  }
  ctx->graphs.clear();
}

// The sharded stream state of a wave-form event-model call writing to an
// output of `capacity` events (grown as needed, never shrunk).
int stream_state(evis_ctx* ctx, long long capacity, StreamState* st) {
  const size_t bytes = stream_state_layout(capacity, nullptr, nullptr);
  bool grew = false;
  const int rc = ensure(ctx, ctx->evs, bytes, &grew);
  if (rc) return rc;
  if (grew) ctx->evs_table_clean = false;
  stream_state_layout(capacity, ctx->evs.p, st);
  return EVIS_OK;
}

// Set-up, event-model launch (the caller's `launch`), fixup and clean-up of
// the sharded stream on stream s.  The table is cleared whole only when its
// state is unknown (new buffer, or a sequence that did not finish).
template <typename Launch>
int with_stream(evis_ctx* ctx, const StreamState& st, unsigned long long* cursor, int reset,
                evis_event* out, long long capacity, hipStream_t s, Launch launch) {
  const bool clear = !ctx->evs_table_clean;
  ctx->evs_table_clean = false;
  EVIS_HIP(launch_stream_init(st, cursor, reset, capacity, clear, s), "k_stream_init");
  EVIS_HIP(launch(), "k_events");
  EVIS_HIP(launch_stream_fixup(st, out, capacity, cursor, s), "k_stream_fixup");
  EVIS_HIP(launch_stream_clean(st, s), "k_stream_clean");
  ctx->evs_table_clean = true;
  return EVIS_OK;
}

int ensure_stage(evis_ctx* ctx, size_t bytes) {
  if (ctx->stage_bytes >= bytes) return EVIS_OK;
  for (int i = 0; i < kStageSlots; ++i) {
    if (ctx->stage_ev[i]) hipEventSynchronize(ctx->stage_ev[i]);
    if (ctx->stage[i]) hipHostFree(ctx->stage[i]);
    ctx->stage[i] = nullptr;
  }
  size_t want = std::max(bytes, (size_t)65536);
  for (int i = 0; i < kStageSlots; ++i) {
    hipError_t e = hipHostMalloc(&ctx->stage[i], want, hipHostMallocDefault);
    if (e != hipSuccess) return fail(ctx, EVIS_ERR_NOMEM, "hipHostMalloc of descriptor staging");
    if (!ctx->stage_ev[i]) {
      e = hipEventCreateWithFlags(&ctx->stage_ev[i], hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate");
    }
  }
  ctx->stage_bytes = want;
  return EVIS_OK;
}

// Copy a block of host data to a device buffer unless it already holds it
// (pinned staging ring; the copy is ordered on stream s).
// Copy bytes through the next slot of the pinned staging ring to dst on
// stream s (the slot's previous copy is waited for first).  The ring is
// allocated at evis_create for any descriptor block; only larger blocks
// (the surrogate's) make it grow.
int stage_copy(evis_ctx* ctx, void* dst, const void* data, size_t bytes, hipStream_t s) {
  int rc = ensure_stage(ctx, bytes);
  if (rc) return rc;
  const int slot = ctx->stage_next;
  ctx->stage_next = (slot + 1) % kStageSlots;
  EVIS_HIP(hipEventSynchronize(ctx->stage_ev[slot]), "hipEventSynchronize");
  std::memcpy(ctx->stage[slot], data, bytes);
  EVIS_HIP(hipMemcpyAsync(dst, ctx->stage[slot], bytes, hipMemcpyHostToDevice, s),
           "hipMemcpyAsync(descriptors)");
  EVIS_HIP(hipEventRecord(ctx->stage_ev[slot], s), "hipEventRecord");
  return EVIS_OK;
}

// Copy a block of host data to a device buffer unless it already holds it.
int upload_to(evis_ctx* ctx, DevBuf& dst, std::vector<unsigned char>& shadow,
              const unsigned char* data, size_t bytes, hipStream_t s) {
  bool grew = false;
  int rc = ensure(ctx, dst, bytes, &grew);
  if (rc) return rc;
  if (grew) {
    drop_graphs(ctx);
    shadow.clear();
  }
  if (shadow.size() == bytes && std::memcmp(shadow.data(), data, bytes) == 0) return EVIS_OK;
  rc = stage_copy(ctx, dst.p, data, bytes, s);
  if (rc) return rc;
  shadow.assign(data, data + bytes);
  return EVIS_OK;
}

int check_pair(evis_ctx* ctx, const evis_pair& p, const char* who) {
  if (p.H < 1 || p.W < 1) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": H and W must be >= 1");
  if (p.H > EVIS_MAX_DIM || p.W > EVIS_MAX_DIM)
    return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": H and W must be <= 2047");
  const void* ptrs[6] = {p.L_A, p.L_B, p.m_A, p.m_B, p.Z_A, p.Z_B};
  for (int i = 0; i < 6; ++i)
    if (!ptrs[i]) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": null frame pointer");
  if (!aligned(p.L_A, 4) || !aligned(p.L_B, 4) || !aligned(p.Z_A, 4) || !aligned(p.Z_B, 4) ||
      !aligned(p.m_A, 8) || !aligned(p.m_B, 8))
    return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": misaligned frame pointer");
  return EVIS_OK;
}

int check_times(evis_ctx* ctx, int64_t t0, int64_t t1, const char* who) {
  if (t0 < 0 || t1 <= t0 || t1 > 2147483647LL || t1 - t0 > EVIS_MAX_SPAN_US)
    return fail(ctx, EVIS_ERR_INVALID,
                std::string(who) + ": need 0 <= t0 < t1 <= 2^31-1 and t1 - t0 <= 2^24 us");
  return EVIS_OK;
}

// blend_mode carries an EVIS_BLEND_* value or'ed with an EVIS_WARP_* value
constexpr int kBlendMask = 0x0F, kWarpMask = 0x30;
bool mode_word_ok(int m) {
  const int b = m & kBlendMask, w = m & kWarpMask;
  return (m & ~(kBlendMask | kWarpMask)) == 0 && (b == EVIS_BLEND_TIME || b == EVIS_BLEND_B_PRIMARY) &&
         (w == EVIS_WARP_GATHER || w == EVIS_WARP_SPLAT || w == EVIS_WARP_JOINT);
}

int check_sensor(evis_ctx* ctx, const evis_sensor& s, const char* who, bool need_k) {
  const bool on_ok = s.theta_on ? aligned(s.theta_on, 4) : (s.C_on > 0.0f && std::isfinite(s.C_on));
  const bool off_ok = s.theta_off ? aligned(s.theta_off, 4) : (s.C_off > 0.0f && std::isfinite(s.C_off));
  if (!on_ok || !off_ok)
    return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": thresholds must be > 0 and finite");
  if (s.refractory_us < 0) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": refractory_us < 0");
  if (need_k) {
    if (s.K > EVIS_MAX_K) return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": K > 128");
    if (s.K <= 0 && (s.K_max < 1 || s.K_max > EVIS_MAX_K))
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": K_max must be in 1..128");
    if (!mode_word_ok(s.blend_mode))
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": unknown blend_mode");
  }
  return EVIS_OK;
}

int check_events_out(evis_ctx* ctx, const evis_event* out, int64_t capacity, const int64_t* n_total,
                     const char* who) {
  if (!n_total || !aligned(n_total, 8)) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": n_total");
  if (capacity < 0) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": capacity < 0");
  if (capacity > 0 && (!out || !aligned(out, 8)))
    return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": event buffer");
  return EVIS_OK;
}

int check_noise(evis_ctx* ctx, const evis_noise* nz, const char* who) {
  if (!nz) return EVIS_OK;
  auto rate_ok = [](float r) { return r >= 0.0f && std::isfinite(r); };
  if (!rate_ok(nz->leak_rate_hz) || !rate_ok(nz->shot_rate_hz) || !rate_ok(nz->hot_rate_hz))
    return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": noise rates must be >= 0 and finite");
  if (!(nz->hot_fraction >= 0.0f && nz->hot_fraction <= 1.0f))
    return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": noise hot_fraction must be in [0, 1]");
  if (!std::isfinite(nz->shot_L0) || !std::isfinite(nz->shot_inv_range))
    return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": noise shot_L0 / shot_inv_range");
  return EVIS_OK;
}

EnvDesc make_desc(const evis_pair& p, const evis_sensor& s, const evis_state& st, int env_id,
                  const evis_noise* nz = nullptr) {
  EnvDesc d{};
  d.LA = p.L_A;
  d.LB = p.L_B;
  d.mA = reinterpret_cast<const float2*>(p.m_A);
  d.mB = reinterpret_cast<const float2*>(p.m_B);
  d.ZA = p.Z_A;
  d.ZB = p.Z_B;
  d.Lref = st.L_ref;
  d.tlast = st.t_last;
  d.th_on = s.theta_on;
  d.th_off = s.theta_off;
  d.H = p.H;
  d.W = p.W;
  d.ntx_src = (p.W + kSrcBlk - 1) / kSrcBlk;
  d.nty_src = (p.H + kSrcBlk - 1) / kSrcBlk;
  d.ntx_sb = (d.ntx_src + kSbBlk - 1) / kSbBlk;
  d.nty_sb = (d.nty_src + kSbBlk - 1) / kSbBlk;
  d.K_fixed = s.K > 0 ? s.K : 0;
  d.K_max = s.K_max;
  d.blend = s.blend_mode & kBlendMask;
  d.warp = s.blend_mode & kWarpMask;
  d.C_on = s.C_on;
  d.C_off = s.C_off;
  d.refr = s.refractory_us;
  d.env_bits = (uint32_t)env_id << 23;
  d.t0 = p.t0_us;
  d.span = (int32_t)(p.t1_us - p.t0_us);
  if (nz && (nz->leak_rate_hz > 0.0f || nz->shot_rate_hz > 0.0f ||
             (nz->hot_rate_hz > 0.0f && nz->hot_fraction > 0.0f))) {
    d.noise_on = 1;
    d.leak_hz = nz->leak_rate_hz;
    d.shot_hz = nz->shot_rate_hz;
    d.hot_hz = nz->hot_rate_hz;
    d.hot_frac = nz->hot_fraction;
    d.shot_L0 = nz->shot_L0;
    d.shot_inv = nz->shot_inv_range;
    d.seed_lo = (uint32_t)(nz->seed & 0xFFFFFFFFull);
    d.seed_hi = (uint32_t)(nz->seed >> 32);
    d.pair_index = nz->pair_index;
  }
  return d;
}

// xbegin, env_order and n_items, then the queue counters from a 256-byte
// boundary, one per 256 bytes
size_t sched_head_ints(int n) { return ((size_t)kXcd * (n + 1) + n + kXcd + kQueueStride - 1) / kQueueStride * kQueueStride; }
size_t sched_ints(int n) { return sched_head_ints(n) + (size_t)kXcd * kQueueStride; }

struct Plan {
  FixedVec<EnvDesc, EVIS_MAX_ENVS> desc;
  FixedVec<int32_t, EVIS_MAX_ENVS + 1> src_prefix;   // n + 1: groups of four source blocks before each env
  long long px_total = 0;
  int src_total = 0;                 // groups of four source blocks (prep work units)
  int sb_total = 0;                  // superblocks of every env
  int sb_max = 0;                    // superblocks of the largest env
  int items = 0;
};

// Where a launch's scratch lives: the context's buffers, or the static
// array of evis_step_batch_noalloc.
struct ScratchView {
  void* meta;        // descriptor block: EnvDesc[n], then int32 src_prefix[n + 1]
  EnvDyn* dyn;       // [n]
  int32_t* sched;    // sched_ints(n)
};

ScratchView ctx_view(evis_ctx* ctx) {
  return ScratchView{ctx->meta.p, static_cast<EnvDyn*>(ctx->dyn.p), static_cast<int32_t*>(ctx->sched.p)};
}

// Point every env's splat records and block bounds into src / tb (and B's
// into srcB / tbB for the two-splat warps), four blocks per group.
void plan_bind(Plan& pl, float4* src, float4* tb, float4* srcB, float4* tbB, float4* sbb) {
  const bool two = pl.desc.size() > 0 && pl.desc[0].warp != EVIS_WARP_GATHER;   // one warp per plan
  long long sb0 = 0;
  for (int e = 0; e < pl.desc.size(); ++e) {
    const long long blk0 = 4LL * pl.src_prefix[e];
    pl.desc[e].src = src + blk0 * kBlkPx;
    pl.desc[e].tb = tb + blk0;
    pl.desc[e].sbb = sbb + sb0;
    pl.desc[e].srcB = two ? srcB + blk0 * kBlkPx : nullptr;
    pl.desc[e].tbB = two ? tbB + blk0 : nullptr;
    pl.desc[e].src_tile_base = pl.src_prefix[e];
    sb0 += (long long)pl.desc[e].ntx_sb * pl.desc[e].nty_sb;
  }
}

// Prefix of source-block groups, pixel and work-item totals.
void plan_layout(Plan& pl, int tw, int th) {
  const int n = pl.desc.size();
  long long px = 0;
  int src = 0, items = 0, sb = 0, sb_max = 0;
  pl.src_prefix.assign(n + 1, 0);
  for (int e = 0; e < n; ++e) {
    pl.src_prefix[e] = src;
    px += (long long)pl.desc[e].H * pl.desc[e].W;
    src += (pl.desc[e].ntx_src * pl.desc[e].nty_src + 3) / 4;
    items += ((pl.desc[e].W + tw - 1) / tw) * ((pl.desc[e].H + th - 1) / th);
    const int nsb = pl.desc[e].ntx_sb * pl.desc[e].nty_sb;
    sb += nsb;
    sb_max = std::max(sb_max, nsb);
  }
  pl.src_prefix[n] = src;
  pl.px_total = px;
  pl.src_total = src;
  pl.sb_total = sb;
  pl.sb_max = sb_max;
  pl.items = items;
}

// Lay out per-env scratch (splat records, tile bounds) in the context's
// buffers (grown as needed) and the descriptor block.
int plan_envs(evis_ctx* ctx, Plan& pl, int tw, int th) {
  const int n = pl.desc.size();
  plan_layout(pl, tw, th);
  const int src = pl.src_total;
  bool grew = false;
  // per block: one bounds record and 16 splat records (four blocks per group)
  int rc = ensure(ctx, ctx->src, (size_t)src * 4 * kBlkPx * sizeof(float4), &grew);
  if (rc) return rc;
  rc = ensure(ctx, ctx->tb, (size_t)src * 4 * sizeof(float4), &grew);
  if (rc) return rc;
  rc = ensure(ctx, ctx->sbb, (size_t)pl.sb_total * sizeof(float4), &grew);
  if (rc) return rc;
  const bool two = n > 0 && pl.desc[0].warp != EVIS_WARP_GATHER;   // one warp per plan
  if (two) {
    rc = ensure(ctx, ctx->srcB, (size_t)src * 4 * kBlkPx * sizeof(float4), &grew);
    if (rc) return rc;
    rc = ensure(ctx, ctx->tbB, (size_t)src * 4 * sizeof(float4), &grew);
    if (rc) return rc;
  }
  rc = ensure(ctx, ctx->dyn, (size_t)n * sizeof(EnvDyn), &grew);
  if (rc) return rc;
  rc = ensure(ctx, ctx->sched, sched_ints(n) * sizeof(int32_t), &grew);
  if (rc) return rc;
  if (grew) {
    drop_graphs(ctx);
    ctx->shadow.clear();
  }
  plan_bind(pl, static_cast<float4*>(ctx->src.p), static_cast<float4*>(ctx->tb.p),
            two ? static_cast<float4*>(ctx->srcB.p) : nullptr,
            two ? static_cast<float4*>(ctx->tbB.p) : nullptr, static_cast<float4*>(ctx->sbb.p));
  return EVIS_OK;
}

// The descriptor block of a plan.
void meta_blob(const Plan& pl, Blob& blob) {
  const size_t n = pl.desc.size();
  blob.n = (int)(n * sizeof(EnvDesc) + (n + 1) * sizeof(int32_t));
  std::memcpy(blob.data(), pl.desc.data(), n * sizeof(EnvDesc));
  std::memcpy(blob.data() + n * sizeof(EnvDesc), pl.src_prefix.data(), (n + 1) * sizeof(int32_t));
}

int upload_meta(evis_ctx* ctx, const Plan& pl, hipStream_t s) {
  Blob blob;
  meta_blob(pl, blob);
  return upload_to(ctx, ctx->meta, ctx->shadow, blob.data(), (size_t)blob.size(), s);
}

struct Sched {
  int32_t* xbegin;
  int32_t* env_order;
  int32_t* n_items;
  unsigned int* queue;
};

Sched sched_ptrs(int32_t* base, int n) {
  Sched s;
  s.xbegin = base;                               // kXcd * (n + 1)
  s.env_order = base + kXcd * (n + 1);           // n
  s.n_items = s.env_order + n;                   // kXcd
  s.queue = reinterpret_cast<unsigned int*>(base + sched_head_ints(n));   // kXcd * kQueueStride
  return s;
}

bool plan_has_noise(const Plan& pl) {
  for (const EnvDesc& d : pl.desc)
    if (d.noise_on) return true;
  return false;
}

// Enqueue reset, prep, queue and the tile kernel for the uploaded plan.
int enqueue_batch(evis_ctx* ctx, const ScratchView& sv, const Plan& pl, int mode, int tw, int th,
                  TileArgs ta, int32_t* K_used, unsigned long long* reset_cursor, hipStream_t s) {
  const int n = pl.desc.size();
  const EnvDesc* d_desc = static_cast<const EnvDesc*>(sv.meta);
  const int32_t* d_prefix = reinterpret_cast<const int32_t*>(
      static_cast<const unsigned char*>(sv.meta) + n * sizeof(EnvDesc));
  EnvDyn* d_dyn = sv.dyn;
  Sched sc = sched_ptrs(sv.sched, n);
  EVIS_HIP(launch_reset(d_dyn, n, sc.queue, reset_cursor, s), "k_reset");
  EVIS_HIP(launch_prep(d_desc, d_dyn, d_prefix, n, pl.src_total, s), "k_prep");
  EVIS_HIP(launch_superbounds(d_desc, n, pl.sb_max, s), "k_superbounds");
  if (!pl.desc.empty() && pl.desc[0].warp != EVIS_WARP_GATHER)   // one warp per plan
    EVIS_HIP(launch_prep_b(d_desc, d_prefix, n, pl.src_total, s), "k_prep_b");
  EVIS_HIP(launch_queue(d_desc, d_dyn, n, tw, th, sc.xbegin, sc.env_order, sc.n_items, K_used, s),
           "k_queue");
  ta.envs = d_desc;
  ta.dyn = d_dyn;
  ta.xbegin = sc.xbegin;
  ta.env_order = sc.env_order;
  ta.n_envs = n;
  ta.queue = sc.queue;
  ta.n_items = sc.n_items;
  const int warp = pl.desc.empty() ? EVIS_WARP_GATHER : pl.desc[0].warp;   // one warp per plan
  const bool noise = plan_has_noise(pl);
  int occ = tile_occupancy(tw, th, mode, warp, noise);
  int per_cu = ctx->tuning.grid_mult > 0 ? std::min(ctx->tuning.grid_mult, occ) : occ;
  int grid = std::max(1, std::min(pl.items, per_cu * ctx->n_cu));
  {
    ProfScope ps(ctx, mode == MODE_STEP ? EVIS_KERNEL_STEP : EVIS_KERNEL_INTERP, s);
    EVIS_HIP(launch_tile(tw, th, mode, warp, noise, ta, grid, s), "k_tile");
  }
  return EVIS_OK;
}

// Device address of `scratch` on `device`, taken once per device with that
// device current (the caller sets it); null if the runtime refuses.
unsigned char* noalloc_scratch_ptr(int device) {
  static std::mutex mu;
  static unsigned char* ptr[64] = {};
  static bool tried[64] = {};
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!tried[device]) {
    tried[device] = true;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) ptr[device] = static_cast<unsigned char*>(p);
  }
  return ptr[device];
}

// Carve a launch's scratch out of the static array: descriptor block,
// EnvDyn, schedule tables, splat records and block bounds (and B's for the
// two-splat warps), each from a 256-byte boundary.  Fails (nothing
// enqueued) when the batch needs more than the array holds.
int plan_static(evis_ctx* ctx, Plan& pl, int tw, int th, ScratchView& sv) {
  plan_layout(pl, tw, th);
  const int n = pl.desc.size();
  const bool two = n > 0 && pl.desc[0].warp != EVIS_WARP_GATHER;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t o_meta = take(n * sizeof(EnvDesc) + (n + 1) * sizeof(int32_t));
  const size_t o_dyn = take(n * sizeof(EnvDyn));
  const size_t o_sched = take(sched_ints(n) * sizeof(int32_t));
  const size_t rec = (size_t)pl.src_total * 4 * kBlkPx * sizeof(float4);
  const size_t bnd = (size_t)pl.src_total * 4 * sizeof(float4);
  const size_t o_src = take(rec), o_tb = take(bnd);
  const size_t o_srcB = two ? take(rec) : 0, o_tbB = two ? take(bnd) : 0;
  const size_t o_sbb = take((size_t)pl.sb_total * sizeof(float4));
  if (off > (size_t)EVIS_NOALLOC_SCRATCH_BYTES) {
    char b[200];
    std::snprintf(b, sizeof(b),
                  "evis_step_batch_noalloc: this batch needs %zu bytes of scratch, more than the "
                  "%zu the entry point holds",
                  off, (size_t)EVIS_NOALLOC_SCRATCH_BYTES);
    return fail(ctx, EVIS_ERR_UNSUPPORTED, b);
  }
  unsigned char* base = ctx->noalloc_scratch;
  sv = ScratchView{base + o_meta, reinterpret_cast<EnvDyn*>(base + o_dyn),
                   reinterpret_cast<int32_t*>(base + o_sched)};
  plan_bind(pl, reinterpret_cast<float4*>(base + o_src), reinterpret_cast<float4*>(base + o_tb),
            two ? reinterpret_cast<float4*>(base + o_srcB) : nullptr,
            two ? reinterpret_cast<float4*>(base + o_tbB) : nullptr,
            reinterpret_cast<float4*>(base + o_sbb));
  return EVIS_OK;
}

// Tuning cache: one JSON object per line, {"key": ..., "tile_w": ..., ...};
// the last line with a key wins.
#ifndef EVIS_BUILD_ID
#define EVIS_BUILD_ID "unversioned"
#endif

std::string tuning_key(evis_ctx* ctx, const Plan& pl, const evis_env* envs, int n_envs,
                       double mean_k) {
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == '"' || c == '\\') c = '_';
  std::map<std::pair<int, int>, int> sizes;
  for (int e = 0; e < n_envs; ++e) ++sizes[{envs[e].pair.H, envs[e].pair.W}];
  std::string shapes;
  for (const auto& kv : sizes) {
    char b[48];
    std::snprintf(b, sizeof(b), "%s%dx%d*%d", shapes.empty() ? "" : ",", kv.first.second,
                  kv.first.first, kv.second);
    shapes += b;
  }
  int kb = 1;
  while (kb < mean_k && kb < EVIS_MAX_K) kb *= 2;
  char b[160];
  std::snprintf(b, sizeof(b), "%s|%s|warp%d|noise%d|K<=%d|", arch.c_str(), EVIS_BUILD_ID,
                pl.desc.empty() ? 0 : pl.desc[0].warp, plan_has_noise(pl) ? 1 : 0, kb);
  return std::string(b) + shapes;
}

bool json_int(const char* line, const char* name, int* v) {
  const char* p = std::strstr(line, name);
  return p && std::sscanf(p + std::strlen(name), " : %d", v) == 1;
}

bool cache_lookup(const char* path, const std::string& key, evis_tuning& t, float& ms) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  const std::string want = "\"key\": \"" + key + "\"";
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    if (!std::strstr(line, want.c_str())) continue;
    evis_tuning c = t;
    double m = 0.0;
    const char* pm = std::strstr(line, "\"ms\"");
    if (json_int(line, "\"tile_w\"", &c.tile_w) && json_int(line, "\"tile_h\"", &c.tile_h) &&
        json_int(line, "\"grid_mult\"", &c.grid_mult) && json_int(line, "\"list_cap\"", &c.list_cap) &&
        pm && std::sscanf(pm + 4, " : %lf", &m) == 1 && tile_shape_supported(c.tile_w, c.tile_h) &&
        c.grid_mult >= 0 && c.list_cap >= 1 && c.list_cap <= kListCapMax) {
      t = c;
      ms = (float)m;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const evis_tuning& t, float ms) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"tile_w\": %d, \"tile_h\": %d, \"grid_mult\": %d, "
                  "\"list_cap\": %d, \"ms\": %.4f}\n",
               key.c_str(), t.tile_w, t.tile_h, t.grid_mult, t.list_cap, (double)ms);
  std::fclose(f);
}

}  // namespace

extern "C" {

int evis_abi_version(void) { return EVIS_ABI_VERSION; }

int evis_create(evis_ctx** out, int device) {
  if (!out) return EVIS_ERR_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return EVIS_ERR_INVALID;
  if (hipSetDevice(device) != hipSuccess) return EVIS_ERR_HIP;
  evis_ctx* ctx = new evis_ctx();
  ctx->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->n_cu = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return EVIS_ERR_HIP;
  }
  // set-up for evis_step_batch_noalloc: the static scratch's address on this
  // device and a staging ring large enough for any descriptor block
  ctx->noalloc_scratch = noalloc_scratch_ptr(device);
  if (ensure_stage(ctx, kMetaMax) != EVIS_OK) {
    evis_destroy(ctx);
    return EVIS_ERR_NOMEM;
  }
  *out = ctx;
  return EVIS_OK;
}

void evis_destroy(evis_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  drop_graphs(ctx);
  for (auto& r : ctx->recs) {
    hipEventDestroy(r.e0);
    hipEventDestroy(r.e1);
  }
  for (hipEvent_t e : ctx->ev_pool) hipEventDestroy(e);
  DevBuf* bufs[] = {&ctx->meta, &ctx->dyn, &ctx->sched, &ctx->src,    &ctx->tb,
                    &ctx->srcB, &ctx->tbB, &ctx->msq,   &ctx->soft,   &ctx->voxmax, &ctx->evb, &ctx->evs, &ctx->sbb};
  for (DevBuf* b : bufs)
    if (b->p) hipFree(b->p);
  for (int i = 0; i < kStageSlots; ++i) {
    if (ctx->stage[i]) hipHostFree(ctx->stage[i]);
    if (ctx->stage_ev[i]) hipEventDestroy(ctx->stage_ev[i]);
  }
  if (ctx->capture_stream) hipStreamDestroy(ctx->capture_stream);
  delete ctx;
}

const char* evis_last_error(const evis_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int evis_log_luminance(evis_ctx* ctx, const float* x, int32_t channels, int64_t n, float eps,
                       float* L_out, void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (!x || !L_out || !aligned(x, 4) || !aligned(L_out, 4))
    return fail(ctx, EVIS_ERR_INVALID, "evis_log_luminance: null or misaligned pointer");
  if (channels != 1 && channels != 3)
    return fail(ctx, EVIS_ERR_INVALID, "evis_log_luminance: channels must be 1 or 3");
  if (n < 0) return fail(ctx, EVIS_ERR_INVALID, "evis_log_luminance: n < 0");
  if (!(eps > 0.0f) || !std::isfinite(eps))
    return fail(ctx, EVIS_ERR_INVALID, "evis_log_luminance: eps must be > 0");
  if (n == 0) return EVIS_OK;
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  EVIS_HIP(launch_log_luminance(x, channels, n, eps, L_out, (hipStream_t)stream), "k_log_luminance");
  return EVIS_OK;
}

int evis_log_channels(evis_ctx* ctx, const float* x, int64_t n, float eps, float* L_out,
                      void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (!x || !L_out || !aligned(x, 4) || !aligned(L_out, 4))
    return fail(ctx, EVIS_ERR_INVALID, "evis_log_channels: null or misaligned pointer");
  if (n < 0) return fail(ctx, EVIS_ERR_INVALID, "evis_log_channels: n < 0");
  if (!(eps > 0.0f) || !std::isfinite(eps))
    return fail(ctx, EVIS_ERR_INVALID, "evis_log_channels: eps must be > 0");
  if (n == 0) return EVIS_OK;
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  EVIS_HIP(launch_log_channels(x, n, eps, L_out, (hipStream_t)stream), "k_log_channels");
  return EVIS_OK;
}

int evis_voxel_grid(evis_ctx* ctx, const evis_event* events, const int64_t* n_events,
                    int64_t capacity, int32_t env_id, int32_t H, int32_t W, int64_t t0_us,
                    int64_t t1_us, int32_t bins, float* out, void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (!n_events || !aligned(n_events, 8)) return fail(ctx, EVIS_ERR_INVALID, "evis_voxel_grid: n_events");
  if (capacity < 0 || (capacity > 0 && (!events || !aligned(events, 8))))
    return fail(ctx, EVIS_ERR_INVALID, "evis_voxel_grid: events / capacity");
  if (!out || !aligned(out, 4)) return fail(ctx, EVIS_ERR_INVALID, "evis_voxel_grid: out");
  if (H < 1 || W < 1) return fail(ctx, EVIS_ERR_INVALID, "evis_voxel_grid: H, W");
  if (H > EVIS_MAX_DIM || W > EVIS_MAX_DIM)
    return fail(ctx, EVIS_ERR_UNSUPPORTED, "evis_voxel_grid: H, W > 2047");
  if (bins < 2 || bins > EVIS_MAX_VOXEL_BINS)
    return fail(ctx, EVIS_ERR_INVALID, "evis_voxel_grid: bins must be in 2..1024");
  if (env_id < 0 || env_id >= EVIS_MAX_ENVS) return fail(ctx, EVIS_ERR_INVALID, "evis_voxel_grid: env_id");
  if (t1_us <= t0_us || t0_us < INT32_MIN || t1_us > (int64_t)INT32_MAX + 1)
    return fail(ctx, EVIS_ERR_INVALID, "evis_voxel_grid: need t0 < t1 within int32 time");
  VoxelArgs a{};
  a.events = events;
  a.n_events = reinterpret_cast<const long long*>(n_events);
  a.capacity = capacity;
  a.acc = reinterpret_cast<uint32_t*>(out);
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  int rc = ensure(ctx, ctx->voxmax, (size_t)2 * bins * sizeof(uint32_t));
  if (rc) return rc;
  a.maxbuf = static_cast<uint32_t*>(ctx->voxmax.p);
  a.t0 = t0_us;
  a.t1 = t1_us;
  a.scale = (float)(bins - 1) / (float)(t1_us - t0_us);
  a.env_id = env_id;
  a.H = H;
  a.W = W;
  a.bins = bins;
  EVIS_HIP(launch_voxel(a, (hipStream_t)stream), "k_voxel");
  return EVIS_OK;
}

int evis_defocus_batch(evis_ctx* ctx, const evis_image* imgs, int32_t n, int32_t channels,
                       float sigma, void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  const char* who = "evis_defocus";
  if (!imgs || n < 1) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": no images");
  if (channels != 1 && channels != 3)
    return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": channels must be 1 or 3");
  if (!(sigma > 0.0f && sigma <= EVIS_MAX_DEFOCUS_SIGMA))
    return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": sigma must be in (0, 10]");
  for (int i = 0; i < n; ++i) {
    const evis_image& im = imgs[i];
    if (!im.x || !im.out || !aligned(im.x, 4) || !aligned(im.out, 4))
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": null or misaligned pointer");
    if (im.H < 1 || im.W < 1) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": H, W");
    if (im.H > EVIS_MAX_DEFOCUS_DIM || im.W > EVIS_MAX_DEFOCUS_DIM)
      return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": H, W > 16384");
    const size_t bytes = (size_t)im.H * im.W * channels * sizeof(float);
    const char* xb = reinterpret_cast<const char*>(im.x);
    const char* ob = reinterpret_cast<const char*>(im.out);
    if (xb < ob + bytes && ob < xb + bytes)
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": out overlaps x");
  }
  DefocusArgs a{};
  a.C = channels;
  a.r = (int)std::ceil(3.0 * (double)sigma);
  double w[2 * kDefocusMaxR + 1], sum = 0.0;
  for (int k = -a.r; k <= a.r; ++k) {
    w[k + a.r] = std::exp(-(double)k * k / (2.0 * (double)sigma * (double)sigma));
    sum += w[k + a.r];
  }
  for (int k = 0; k <= 2 * a.r; ++k) a.w[k] = (float)(w[k] / sum);
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  for (int i0 = 0; i0 < n; i0 += kDefocusBatch) {   // up to kDefocusBatch images per launch
    a.n = std::min(kDefocusBatch, n - i0);
    int tiles = 0;
    for (int i = 0; i < a.n; ++i) {
      const evis_image& im = imgs[i0 + i];
      a.img[i] = DefocusImage{im.x, im.out, im.H, im.W, 0, 0};
      a.tile_prefix[i] = tiles;
      tiles += defocus_tiles(im.H, im.W, &a.img[i].tiles_x);
    }
    a.tile_prefix[a.n] = tiles;
    EVIS_HIP(launch_defocus(a, (hipStream_t)stream), "k_defocus");
  }
  return EVIS_OK;
}

int evis_defocus(evis_ctx* ctx, const float* x, int32_t H, int32_t W, int32_t channels, float sigma,
                 float* out, void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  const evis_image im{x, out, H, W};
  return evis_defocus_batch(ctx, &im, 1, channels, sigma, stream);
}

int evis_state_init(evis_ctx* ctx, const float* L_first, int32_t H, int32_t W,
                    const evis_state* state, void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (!state || !L_first || !state->L_ref || !aligned(L_first, 4) || !aligned(state->L_ref, 4) ||
      (state->t_last && !aligned(state->t_last, 4)))
    return fail(ctx, EVIS_ERR_INVALID, "evis_state_init: null or misaligned pointer");
  if (H < 1 || W < 1 || H > EVIS_MAX_DIM || W > EVIS_MAX_DIM)
    return fail(ctx, EVIS_ERR_INVALID, "evis_state_init: bad H, W");
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  EVIS_HIP(launch_state_init(L_first, (long long)H * W, state->L_ref, state->t_last, (hipStream_t)stream),
           "k_state_init");
  return EVIS_OK;
}

int evis_substep_count(evis_ctx* ctx, const evis_pair* pair, int32_t K_max, int32_t* K_out,
                       void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (!pair) return fail(ctx, EVIS_ERR_INVALID, "evis_substep_count: null pair");
  int rc = check_pair(ctx, *pair, "evis_substep_count");
  if (rc) return rc;
  if (K_max < 1 || K_max > EVIS_MAX_K) return fail(ctx, EVIS_ERR_INVALID, "evis_substep_count: K_max");
  if (!K_out || !aligned(K_out, 4)) return fail(ctx, EVIS_ERR_INVALID, "evis_substep_count: K_out");
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  rc = ensure(ctx, ctx->msq, sizeof(unsigned long long));
  if (rc) return rc;
  EVIS_HIP(launch_substep_count(reinterpret_cast<const float2*>(pair->m_A),
                                reinterpret_cast<const float2*>(pair->m_B),
                                (long long)pair->H * pair->W, K_max,
                                static_cast<unsigned long long*>(ctx->msq.p), K_out,
                                (hipStream_t)stream),
           "k_msq");
  return EVIS_OK;
}

int evis_interpolate(evis_ctx* ctx, const evis_pair* pair, int32_t K, int32_t j_begin,
                     int32_t j_end, int32_t blend_mode, float* L_out, uint8_t* hole_mask,
                     void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (!pair) return fail(ctx, EVIS_ERR_INVALID, "evis_interpolate: null pair");
  int rc = check_pair(ctx, *pair, "evis_interpolate");
  if (rc) return rc;
  if (K < 1) return fail(ctx, EVIS_ERR_INVALID, "evis_interpolate: K must be >= 1");
  if (K > EVIS_MAX_K) return fail(ctx, EVIS_ERR_UNSUPPORTED, "evis_interpolate: K > 128");
  if (j_begin < 0 || j_end <= j_begin || j_end > K + 1)
    return fail(ctx, EVIS_ERR_INVALID, "evis_interpolate: need 0 <= j_begin < j_end <= K + 1");
  if (!mode_word_ok(blend_mode))
    return fail(ctx, EVIS_ERR_INVALID, "evis_interpolate: unknown blend_mode");
  if (!L_out || !aligned(L_out, 4)) return fail(ctx, EVIS_ERR_INVALID, "evis_interpolate: L_out");
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  evis_sensor s{};
  s.C_on = s.C_off = 1.0f;
  s.K = K;
  s.K_max = K;
  s.blend_mode = blend_mode;
  evis_state st{};
  Plan pl;
  evis_pair p = *pair;
  p.t0_us = 0;
  p.t1_us = 1;
  pl.desc.push_back(make_desc(p, s, st, 0));
  const int tw = 32, th = 32;
  rc = plan_envs(ctx, pl, tw, th);
  if (rc) return rc;
  rc = upload_meta(ctx, pl, (hipStream_t)stream);
  if (rc) return rc;
  TileArgs ta{};
  ta.list_cap = std::min(std::max(ctx->tuning.list_cap, 1), kListCapMax);
  ta.static_tiles = 0;
  ta.L_out = L_out;
  ta.hole = hole_mask;
  ta.j_begin = j_begin;
  ta.j_end = j_end;
  return enqueue_batch(ctx, ctx_view(ctx), pl, MODE_INTERP, tw, th, ta, nullptr, nullptr,
                       (hipStream_t)stream);
}

int evis_generate_events(evis_ctx* ctx, const float* L_seq, int32_t H, int32_t W, int32_t K,
                         int64_t t0_us, int64_t t1_us, const evis_sensor* sensor,
                         const evis_state* state, int32_t env_id, evis_event* out,
                         int64_t capacity, int64_t* n_total, int32_t flags, void* stream) {
  return evis_generate_events_noise(ctx, L_seq, H, W, K, t0_us, t1_us, sensor, state, env_id,
                                    nullptr, out, capacity, n_total, flags, stream);
}

int evis_generate_events_noise(evis_ctx* ctx, const float* L_seq, int32_t H, int32_t W, int32_t K,
                               int64_t t0_us, int64_t t1_us, const evis_sensor* sensor,
                               const evis_state* state, int32_t env_id, const evis_noise* noise,
                               evis_event* out, int64_t capacity, int64_t* n_total,
                               int32_t flags, void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (!L_seq || !aligned(L_seq, 4)) return fail(ctx, EVIS_ERR_INVALID, "evis_generate_events: L_seq");
  if (H < 1 || W < 1) return fail(ctx, EVIS_ERR_INVALID, "evis_generate_events: H, W");
  if (H > EVIS_MAX_DIM || W > EVIS_MAX_DIM)
    return fail(ctx, EVIS_ERR_UNSUPPORTED, "evis_generate_events: H, W > 2047");
  if (K < 1) return fail(ctx, EVIS_ERR_INVALID, "evis_generate_events: K must be >= 1");
  if (K > EVIS_MAX_K) return fail(ctx, EVIS_ERR_UNSUPPORTED, "evis_generate_events: K > 128");
  int rc = check_times(ctx, t0_us, t1_us, "evis_generate_events");
  if (rc) return rc;
  if (!sensor || !state) return fail(ctx, EVIS_ERR_INVALID, "evis_generate_events: sensor/state");
  rc = check_sensor(ctx, *sensor, "evis_generate_events", false);
  if (rc) return rc;
  if (!state->L_ref || !aligned(state->L_ref, 4))
    return fail(ctx, EVIS_ERR_INVALID, "evis_generate_events: state.L_ref");
  if (sensor->refractory_us > 0 && !state->t_last)
    return fail(ctx, EVIS_ERR_INVALID, "evis_generate_events: refractory period needs state.t_last");
  if (state->t_last && !aligned(state->t_last, 4))
    return fail(ctx, EVIS_ERR_INVALID, "evis_generate_events: state.t_last");
  if (env_id < 0 || env_id >= EVIS_MAX_ENVS)
    return fail(ctx, EVIS_ERR_INVALID, "evis_generate_events: env_id");
  rc = check_events_out(ctx, out, capacity, n_total, "evis_generate_events");
  if (rc) return rc;
  rc = check_noise(ctx, noise, "evis_generate_events");
  if (rc) return rc;
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const int span = (int)(t1_us - t0_us);
  const float Dt = (float)span / (float)K;
  // the same per-substep probabilities as the fused step's (host float32
  // arithmetic in the same order)
  NoiseCfg nc{};
  const bool noisy = noise && (noise->leak_rate_hz > 0.0f || noise->shot_rate_hz > 0.0f ||
                               (noise->hot_rate_hz > 0.0f && noise->hot_fraction > 0.0f));
  if (noisy) {
    const float dts = Dt * 1e-6f;
    nc = NoiseCfg{noise->leak_rate_hz * dts, noise->shot_rate_hz * dts, noise->hot_rate_hz * dts,
                  noise->shot_L0, noise->shot_inv_range, noise->hot_fraction,
                  (uint32_t)(noise->seed & 0xFFFFFFFFull), (uint32_t)(noise->seed >> 32),
                  noise->pair_index};
  }
  const bool wave = events_wave_form(sensor->refractory_us, noisy);
  StreamState st{};
  if (wave) {
    rc = stream_state(ctx, capacity, &st);
    if (rc) return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* cursor = reinterpret_cast<unsigned long long*>(n_total);
  const int reset = (flags & EVIS_FLAG_RESET_CURSOR) ? 1 : 0;
  ProfScope ps(ctx, EVIS_KERNEL_EVENTS, s);
  auto launch = [&]() {
    return launch_events(L_seq, H, W, K, t0_us, span, Dt, sensor->C_on, sensor->C_off,
                         sensor->theta_on, sensor->theta_off, sensor->refractory_us,
                         (uint32_t)env_id << 23, state->L_ref, state->t_last, out, capacity,
                         cursor, reset, noisy ? &nc : nullptr, st, s);
  };
  if (wave) return with_stream(ctx, st, cursor, reset, out, capacity, s, launch);
  EVIS_HIP(launch(), "k_events");
  return EVIS_OK;
}

int evis_generate_events_batch(evis_ctx* ctx, const evis_frames* envs, int32_t n_envs,
                               evis_event* out, int64_t capacity, int64_t* n_total, int32_t flags,
                               void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  const char* who = "evis_generate_events_batch";
  if (!envs) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": null envs");
  if (n_envs < 1) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": n_envs must be >= 1");
  if (n_envs > EVIS_MAX_ENVS) return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": n_envs > 512");
  int rc = check_events_out(ctx, out, capacity, n_total, who);
  if (rc) return rc;
  // Envs without a refractory period go to the wave form, the others to
  // the workgroup form: two launches, each over its own descriptors.
  std::vector<EventArgs> descs;
  std::vector<EventArgs> descs_refr;
  descs.reserve(n_envs);
  for (int e = 0; e < n_envs; ++e) {
    const evis_frames& v = envs[e];
    if (!v.L_seq || !aligned(v.L_seq, 4)) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": L_seq");
    if (v.H < 1 || v.W < 1) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": H, W");
    if (v.H > EVIS_MAX_DIM || v.W > EVIS_MAX_DIM)
      return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": H, W > 2047");
    if (v.K < 1) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": K must be >= 1");
    if (v.K > EVIS_MAX_K) return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": K > 128");
    rc = check_times(ctx, v.t0_us, v.t1_us, who);
    if (rc) return rc;
    rc = check_sensor(ctx, v.sensor, who, false);
    if (rc) return rc;
    if (!v.state.L_ref || !aligned(v.state.L_ref, 4))
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": state.L_ref");
    if (v.sensor.refractory_us > 0 && !v.state.t_last)
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": refractory period needs state.t_last");
    if (v.state.t_last && !aligned(v.state.t_last, 4))
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": state.t_last");
    if (v.env_id < 0 || v.env_id >= EVIS_MAX_ENVS)
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": env_id");
    const int span = (int)(v.t1_us - v.t0_us);
    const EventArgs a{v.L_seq, v.H, v.W, v.K, v.t0_us, span, (float)span / (float)v.K,
                      v.sensor.C_on, v.sensor.C_off, v.sensor.theta_on, v.sensor.theta_off,
                      v.sensor.refractory_us, (uint32_t)v.env_id << 23, v.state.L_ref,
                      v.state.t_last, out, capacity, reinterpret_cast<unsigned long long*>(n_total),
                      NoiseCfg{}};
    (v.sensor.refractory_us > 0 ? descs_refr : descs).push_back(a);
  }
  const int n_wave = (int)descs.size(), n_refr = (int)descs_refr.size();
  descs.insert(descs.end(), descs_refr.begin(), descs_refr.end());
  // prefix of each group: [n_wave + 1] then [n_refr + 1]
  std::vector<int32_t> prefix;
  prefix.reserve(n_envs + 2);
  long long blocks_wave = 0, blocks_refr = 0;
  for (int g = 0; g < 2; ++g) {
    long long blocks = 0;
    const int b0 = g == 0 ? 0 : n_wave, b1 = g == 0 ? n_wave : n_envs;
    for (int e = b0; e < b1; ++e) {
      prefix.push_back((int32_t)blocks);
      blocks += events_batch_blocks((long long)descs[e].H * descs[e].W);
      if (blocks > 0x7FFFFFFFLL) return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": batch too large");
    }
    prefix.push_back((int32_t)blocks);
    (g == 0 ? blocks_wave : blocks_refr) = blocks;
  }
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const size_t off_prefix = ((size_t)n_envs * sizeof(EventArgs) + 255) & ~(size_t)255;
  std::vector<unsigned char> blob(off_prefix + prefix.size() * sizeof(int32_t));
  std::memcpy(blob.data(), descs.data(), (size_t)n_envs * sizeof(EventArgs));
  std::memcpy(blob.data() + off_prefix, prefix.data(), prefix.size() * sizeof(int32_t));
  rc = ensure(ctx, ctx->evb, blob.size());
  if (rc) return rc;
  rc = stage_copy(ctx, ctx->evb.p, blob.data(), blob.size(), s);
  if (rc) return rc;
  const EventArgs* d_descs = static_cast<const EventArgs*>(ctx->evb.p);
  const int32_t* d_prefix =
      reinterpret_cast<const int32_t*>(static_cast<unsigned char*>(ctx->evb.p) + off_prefix);
  StreamState st{};
  if (n_wave > 0) {
    rc = stream_state(ctx, capacity, &st);
    if (rc) return rc;
  }
  unsigned long long* cursor = reinterpret_cast<unsigned long long*>(n_total);
  const int reset = (flags & EVIS_FLAG_RESET_CURSOR) ? 1 : 0;
  ProfScope ps(ctx, EVIS_KERNEL_EVENTS, s);
  // the wave form through the sharded stream (which leaves the cursor at
  // its end), then the workgroup form at the cursor
  if (n_wave > 0) {
    rc = with_stream(ctx, st, cursor, reset, out, capacity, s, [&]() {
      return launch_events_batch(d_descs, d_prefix, n_wave, (int)blocks_wave, true, st, s);
    });
    if (rc) return rc;
  } else if (reset) {
    EVIS_HIP(launch_zero_u64(cursor, s), "k_zero_u64");
  }
  EVIS_HIP(launch_events_batch(d_descs + n_wave, d_prefix + n_wave + 1, n_refr, (int)blocks_refr,
                               false, st, s),
           "k_events_batch");
  return EVIS_OK;
}

static int validate_envs(evis_ctx* ctx, const evis_env* envs, int32_t n_envs, Plan& pl,
                         const char* who) {
  if (!envs) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": null envs");
  if (n_envs < 1) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": n_envs must be >= 1");
  if (n_envs > EVIS_MAX_ENVS) return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": n_envs > 512");
  pl.desc.clear();
  for (int e = 0; e < n_envs; ++e) {
    const evis_env& v = envs[e];
    int rc = check_pair(ctx, v.pair, who);
    if (rc) return rc;
    rc = check_times(ctx, v.pair.t0_us, v.pair.t1_us, who);
    if (rc) return rc;
    rc = check_sensor(ctx, v.sensor, who, true);
    if (rc) return rc;
    if (!v.state.L_ref || !aligned(v.state.L_ref, 4))
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": state.L_ref");
    if (v.sensor.refractory_us > 0 && !v.state.t_last)
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": refractory period needs state.t_last");
    if (v.state.t_last && !aligned(v.state.t_last, 4))
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": state.t_last");
    if (v.env_id < 0 || v.env_id >= EVIS_MAX_ENVS)
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": env_id");
    rc = check_noise(ctx, v.noise, who);
    if (rc) return rc;
    if (v.crop_margin < 0 || 2LL * v.crop_margin >= std::min(v.pair.H, v.pair.W))
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": crop_margin must satisfy 0 <= 2m < min(H, W)");
    pl.desc.push_back(make_desc(v.pair, v.sensor, v.state, v.env_id, v.noise));
    pl.desc.back().margin = v.crop_margin;
    if (pl.desc.back().warp != pl.desc[0].warp)
      return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": envs of one call need the same EVIS_WARP_*");
  }
  return EVIS_OK;
}

static int run_step(evis_ctx* ctx, Plan& pl, evis_event* out, int64_t capacity, int64_t* n_total,
                    int32_t* K_used, int32_t flags, hipStream_t s) {
  const evis_tuning tu = ctx->tuning;
  int rc = plan_envs(ctx, pl, tu.tile_w, tu.tile_h);
  if (rc) return rc;
  rc = upload_meta(ctx, pl, s);
  if (rc) return rc;
  TileArgs ta{};
  ta.list_cap = std::min(std::max(tu.list_cap, 1), kListCapMax);
  ta.static_tiles = tu.static_tiles ? 1 : 0;
  ta.out = out;
  ta.capacity = capacity;
  ta.cursor = reinterpret_cast<unsigned long long*>(n_total);
  unsigned long long* reset = (flags & EVIS_FLAG_RESET_CURSOR) ? ta.cursor : nullptr;
  if (!tu.use_graph || ctx->prof)
    return enqueue_batch(ctx, ctx_view(ctx), pl, MODE_STEP, tu.tile_w, tu.tile_h, ta, K_used, reset, s);

  char key[256];
  std::snprintf(key, sizeof(key), "%d|%d|%d|%p|%lld|%p|%p|%d|%d|%d|%d|%d|%d|%d|%d", (int)pl.desc.size(),
                pl.src_total, pl.items, (void*)out, (long long)capacity, (void*)n_total,
                (void*)K_used, flags & EVIS_FLAG_RESET_CURSOR, tu.tile_w, tu.tile_h, tu.grid_mult,
                ta.list_cap, ta.static_tiles, (int)ctx->meta.bytes,
                pl.desc[0].warp | (plan_has_noise(pl) ? 0x100 : 0));
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    if (ctx->graphs.size() >= 512) drop_graphs(ctx);
    GraphEntry g;
    hipStream_t cs = ctx->capture_stream;
    EVIS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    rc = enqueue_batch(ctx, ctx_view(ctx), pl, MODE_STEP, tu.tile_w, tu.tile_h, ta, K_used, reset, cs);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc) {
      if (graph) hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      hipGraphDestroy(graph);
      return hip_fail(ctx, e, "hipGraphInstantiate");
    }
    g.graph = graph;
    it = ctx->graphs.emplace(key, g).first;
  }
  EVIS_HIP(hipGraphLaunch(it->second.exec, s), "hipGraphLaunch");
  return EVIS_OK;
}

int evis_step_batch(evis_ctx* ctx, const evis_env* envs, int32_t n_envs, evis_event* out,
                    int64_t capacity, int64_t* n_total, int32_t* K_used, int32_t flags,
                    void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  Plan pl;
  int rc = validate_envs(ctx, envs, n_envs, pl, "evis_step_batch");
  if (rc) return rc;
  rc = check_events_out(ctx, out, capacity, n_total, "evis_step_batch");
  if (rc) return rc;
  if (K_used && !aligned(K_used, 4)) return fail(ctx, EVIS_ERR_INVALID, "evis_step_batch: K_used");
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  return run_step(ctx, pl, out, capacity, n_total, K_used, flags, (hipStream_t)stream);
}

int evis_step_batch_noalloc(evis_ctx* ctx, const evis_env* envs, int32_t n_envs, evis_event* out,
                            int64_t capacity, int64_t* n_total, int32_t* K_used, int32_t flags,
                            void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (!ctx->noalloc_scratch)
    return fail(ctx, EVIS_ERR_HIP, "evis_step_batch_noalloc: the static scratch has no device address");
  Plan pl;
  int rc = validate_envs(ctx, envs, n_envs, pl, "evis_step_batch_noalloc");
  if (rc) return rc;
  rc = check_events_out(ctx, out, capacity, n_total, "evis_step_batch_noalloc");
  if (rc) return rc;
  if (K_used && !aligned(K_used, 4))
    return fail(ctx, EVIS_ERR_INVALID, "evis_step_batch_noalloc: K_used");
  const evis_tuning tu = ctx->tuning;
  ScratchView sv{};
  rc = plan_static(ctx, pl, tu.tile_w, tu.tile_h, sv);
  if (rc) return rc;
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  // the descriptor block always goes up: other contexts on this device
  // share the array
  Blob blob;
  meta_blob(pl, blob);
  rc = stage_copy(ctx, sv.meta, blob.data(), (size_t)blob.size(), s);
  if (rc) return rc;
  TileArgs ta{};
  ta.list_cap = std::min(std::max(tu.list_cap, 1), kListCapMax);
  ta.static_tiles = tu.static_tiles ? 1 : 0;
  ta.out = out;
  ta.capacity = capacity;
  ta.cursor = reinterpret_cast<unsigned long long*>(n_total);
  unsigned long long* reset = (flags & EVIS_FLAG_RESET_CURSOR) ? ta.cursor : nullptr;
  return enqueue_batch(ctx, sv, pl, MODE_STEP, tu.tile_w, tu.tile_h, ta, K_used, reset, s);
}

int evis_profile_enable(evis_ctx* ctx, int32_t enable) {
  if (!ctx) return EVIS_ERR_INVALID;
  ctx->prof = enable != 0;
  return EVIS_OK;
}

int evis_profile_read(evis_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (kernel < EVIS_KERNEL_STEP || kernel > EVIS_KERNEL_EVENTS)
    return fail(ctx, EVIS_ERR_INVALID, "evis_profile_read: unknown kernel");
  double sum = 0.0;
  int64_t cnt = 0;
  std::vector<evis_ctx::Rec> keep;
  for (auto& r : ctx->recs) {
    if (r.kind != kernel) {
      keep.push_back(r);
      continue;
    }
    EVIS_HIP(hipEventSynchronize(r.e1), "hipEventSynchronize");
    float ms = 0.0f;
    EVIS_HIP(hipEventElapsedTime(&ms, r.e0, r.e1), "hipEventElapsedTime");
    sum += ms;
    ++cnt;
    ctx->ev_pool.push_back(r.e0);
    ctx->ev_pool.push_back(r.e1);
  }
  ctx->recs.swap(keep);
  if (total_ms) *total_ms = sum;
  if (launches) *launches = cnt;
  return EVIS_OK;
}

static int soft_call(evis_ctx* ctx, const evis_soft_env* envs, int32_t n_envs, int32_t K, float tau,
                     int32_t blend_mode, const float* C, float* gC, bool backward,
                     int32_t flags, hipStream_t s) {
  const char* who = backward ? "evis_soft_count_backward" : "evis_soft_count_forward";
  if (!envs) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": null envs");
  if (n_envs < 1) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": n_envs must be >= 1");
  if (n_envs > EVIS_MAX_ENVS) return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": n_envs > 512");
  if (K < 1) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": K must be >= 1");
  if (K > EVIS_MAX_K) return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": K > 128");
  if (!(tau > 0.0f) || !std::isfinite(tau)) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": tau");
  if (!mode_word_ok(blend_mode))
    return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": unknown blend_mode");
  if ((blend_mode & kWarpMask) != EVIS_WARP_GATHER)
    return fail(ctx, EVIS_ERR_UNSUPPORTED, std::string(who) + ": the surrogate supports the gather warp only");
  if (!C || !aligned(C, 4)) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": C");
  if (backward && (!gC || !aligned(gC, 4))) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": gC");
  if (flags & ~EVIS_SOFT_HOLD_REF) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": unknown flags");
  Plan pl;
  std::vector<SoftPtrs> ptrs(n_envs);
  evis_sensor sen{};
  sen.C_on = sen.C_off = 1.0f;
  sen.K = K;
  sen.K_max = K;
  sen.blend_mode = blend_mode;
  for (int e = 0; e < n_envs; ++e) {
    const evis_soft_env& v = envs[e];
    int rc = check_pair(ctx, v.pair, who);
    if (rc) return rc;
    const void* need[] = {v.L_ref, backward ? v.gS : v.S};
    for (const void* q : need)
      if (!q || !aligned(q, 4)) return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": L_ref / S / gS");
    if (backward && (!v.gL_A || !v.gL_B || !v.gm_A || !v.gm_B || !aligned(v.gL_A, 4) ||
                     !aligned(v.gL_B, 4) || !aligned(v.gm_A, 8) || !aligned(v.gm_B, 8)))
      return fail(ctx, EVIS_ERR_INVALID, std::string(who) + ": gradient outputs");
    evis_pair p = v.pair;
    p.t0_us = 0;
    p.t1_us = 1;
    evis_state st{};
    pl.desc.push_back(make_desc(p, sen, st, 0));
    SoftPtrs& P = ptrs[e];
    P.Lref = v.L_ref;
    P.S = v.S;
    P.gS = v.gS;
    P.gLA = v.gL_A;
    P.gLB = v.gL_B;
    P.gmA = reinterpret_cast<float2*>(v.gm_A);
    P.gmB = reinterpret_cast<float2*>(v.gm_B);
  }
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  int rc = plan_envs(ctx, pl, kSoftTW, kSoftTH);
  if (rc) return rc;
  rc = upload_meta(ctx, pl, s);
  if (rc) return rc;
  std::vector<int32_t> item_prefix(n_envs + 1, 0);
  for (int e = 0; e < n_envs; ++e)
    item_prefix[e + 1] = item_prefix[e] + ((pl.desc[e].W + kSoftTW - 1) / kSoftTW) *
                                              ((pl.desc[e].H + kSoftTH - 1) / kSoftTH);
  const size_t off_ptrs = ((n_envs + 1) * sizeof(int32_t) + 15) & ~(size_t)15;
  std::vector<unsigned char> blob(off_ptrs + n_envs * sizeof(SoftPtrs));
  std::memcpy(blob.data(), item_prefix.data(), (n_envs + 1) * sizeof(int32_t));
  std::memcpy(blob.data() + off_ptrs, ptrs.data(), n_envs * sizeof(SoftPtrs));
  rc = upload_to(ctx, ctx->soft, ctx->soft_shadow, blob.data(), blob.size(), s);
  if (rc) return rc;
  const EnvDesc* d_desc = static_cast<const EnvDesc*>(ctx->meta.p);
  const int32_t* d_prefix = reinterpret_cast<const int32_t*>(
      static_cast<const unsigned char*>(ctx->meta.p) + n_envs * sizeof(EnvDesc));
  EnvDyn* d_dyn = static_cast<EnvDyn*>(ctx->dyn.p);
  Sched sc = sched_ptrs(static_cast<int32_t*>(ctx->sched.p), n_envs);
  const SoftPtrs* d_ptrs = reinterpret_cast<const SoftPtrs*>(static_cast<unsigned char*>(ctx->soft.p) + off_ptrs);
  EVIS_HIP(launch_reset(d_dyn, n_envs, sc.queue, nullptr, s), "k_reset");
  EVIS_HIP(launch_prep(d_desc, d_dyn, d_prefix, n_envs, pl.src_total, s), "k_prep");
  EVIS_HIP(launch_superbounds(d_desc, n_envs, pl.sb_max, s), "k_superbounds");
  if (backward) EVIS_HIP(launch_soft_zero(d_ptrs, d_desc, n_envs, gC, s), "k_soft_zero");
  SoftArgs a{};
  a.envs = d_desc;
  a.dyn = d_dyn;
  a.item_prefix = static_cast<const int32_t*>(ctx->soft.p);
  a.ptrs = d_ptrs;
  a.n_envs = n_envs;
  a.K = K;
  a.inv_tau = 1.0f / tau;
  a.list_cap = std::min(std::max(ctx->tuning.list_cap, 1), kListCapMax);
  a.C = C;
  a.gC = gC;
  a.hold_ref = (flags & EVIS_SOFT_HOLD_REF) ? 1 : 0;
  EVIS_HIP(launch_soft(backward, a, item_prefix[n_envs], s), "k_soft");
  return EVIS_OK;
}

int evis_soft_count_forward(evis_ctx* ctx, const evis_soft_env* envs, int32_t n_envs, int32_t K,
                            float tau, int32_t blend_mode, const float* C, void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  return soft_call(ctx, envs, n_envs, K, tau, blend_mode, C, nullptr, false, 0, (hipStream_t)stream);
}

int evis_soft_count_backward(evis_ctx* ctx, const evis_soft_env* envs, int32_t n_envs, int32_t K,
                             float tau, int32_t blend_mode, const float* C, float* gC,
                             int32_t flags, void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  return soft_call(ctx, envs, n_envs, K, tau, blend_mode, C, gC, true, flags, (hipStream_t)stream);
}

int evis_get_tuning(const evis_ctx* ctx, evis_tuning* out) {
  if (!ctx || !out) return EVIS_ERR_INVALID;
  *out = ctx->tuning;
  return EVIS_OK;
}

int evis_set_tuning(evis_ctx* ctx, const evis_tuning* t) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (!t) return fail(ctx, EVIS_ERR_INVALID, "evis_set_tuning: null");
  if (!tile_shape_supported(t->tile_w, t->tile_h))
    return fail(ctx, EVIS_ERR_UNSUPPORTED, "evis_set_tuning: unsupported tile shape");
  if (t->grid_mult < 0 || t->list_cap < 0 || t->list_cap > kListCapMax)
    return fail(ctx, EVIS_ERR_INVALID, "evis_set_tuning: grid_mult / list_cap out of range");
  ctx->tuning = *t;
  if (ctx->tuning.list_cap == 0) ctx->tuning.list_cap = kListCapMax;
  return EVIS_OK;
}

int evis_autotune(evis_ctx* ctx, const evis_env* envs, int32_t n_envs, evis_event* out,
                  int64_t capacity, int64_t* n_total, int32_t reps, evis_tuning* best,
                  float* best_ms, void* stream) {
  return evis_autotune_ex(ctx, envs, n_envs, out, capacity, n_total, reps, nullptr, best, best_ms,
                          nullptr, 0, nullptr, nullptr, stream);
}

int evis_autotune_ex(evis_ctx* ctx, const evis_env* envs, int32_t n_envs, evis_event* out,
                     int64_t capacity, int64_t* n_total, int32_t reps, const char* cache_path,
                     evis_tuning* best, float* best_ms, evis_tune_trial* trials,
                     int32_t max_trials, int32_t* n_trials, int32_t* from_cache, void* stream) {
  if (!ctx) return EVIS_ERR_INVALID;
  if (n_trials) *n_trials = 0;
  if (from_cache) *from_cache = 0;
  Plan pl;
  int rc = validate_envs(ctx, envs, n_envs, pl, "evis_autotune");
  if (rc) return rc;
  rc = check_events_out(ctx, out, capacity, n_total, "evis_autotune");
  if (rc) return rc;
  if (reps < 1) return fail(ctx, EVIS_ERR_INVALID, "evis_autotune: reps must be >= 1");
  if (max_trials < 0 || (max_trials > 0 && !trials))
    return fail(ctx, EVIS_ERR_INVALID, "evis_autotune: trials / max_trials");
  EVIS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  // Private copy of every state (and of the cursor) so that trial launches
  // leave them untouched, and room for the substep counts of one launch.
  size_t bytes = 8 + 4 * (size_t)n_envs;
  for (int e = 0; e < n_envs; ++e) {
    const size_t px = (size_t)envs[e].pair.H * envs[e].pair.W;
    bytes += px * 4 * (envs[e].state.t_last ? 2 : 1);
  }
  void* saved = nullptr;
  EVIS_HIP(hipMalloc(&saved, bytes), "hipMalloc(autotune state copy)");
  int32_t* d_K = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(saved) + bytes - 4 * (size_t)n_envs);
  auto copy_states = [&](bool save) -> hipError_t {
    unsigned char* p = static_cast<unsigned char*>(saved);
    hipError_t e = save ? hipMemcpyAsync(p, n_total, 8, hipMemcpyDeviceToDevice, s)
                        : hipMemcpyAsync(n_total, p, 8, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    p += 8;
    for (int k = 0; k < n_envs; ++k) {
      const size_t px = (size_t)envs[k].pair.H * envs[k].pair.W;
      e = save ? hipMemcpyAsync(p, envs[k].state.L_ref, px * 4, hipMemcpyDeviceToDevice, s)
               : hipMemcpyAsync(envs[k].state.L_ref, p, px * 4, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
      p += px * 4;
      if (envs[k].state.t_last) {
        e = save ? hipMemcpyAsync(p, envs[k].state.t_last, px * 4, hipMemcpyDeviceToDevice, s)
                 : hipMemcpyAsync(envs[k].state.t_last, p, px * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        p += px * 4;
      }
    }
    return hipSuccess;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  const evis_tuning orig = ctx->tuning;
  evis_tuning winner = orig;
  float winner_ms = 1e30f;
  int n_done = 0;
  bool cached = false;
  std::string key;
  // Mean launch time of one tuning (the first launch of a shape also
  // captures its graph and is not timed); negative on failure.
  auto trial = [&](const evis_tuning& t) -> float {
    ctx->tuning = t;
    float total = 0.0f;
    for (int r = 0; r <= reps && rc == EVIS_OK; ++r) {
      hipError_t he = copy_states(false);
      if (he != hipSuccess) {
        rc = hip_fail(ctx, he, "evis_autotune state copy");
        break;
      }
      hipEventRecord(e0, s);
      Plan p2 = pl;
      rc = run_step(ctx, p2, out, capacity, n_total, nullptr, 0, s);
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float ms = 0.0f;
      hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) total += ms;
    }
    const float avg = rc == EVIS_OK ? total / (float)reps : -1.0f;
    if (trials && n_done < max_trials) trials[n_done] = evis_tune_trial{t, avg, 0};
    ++n_done;
    if (rc == EVIS_OK && avg < winner_ms) {
      winner_ms = avg;
      winner = t;
    }
    return avg;
  };
  hipError_t he = copy_states(true);
  if (he != hipSuccess) rc = hip_fail(ctx, he, "evis_autotune state copy");
  // the batch's substep counts, from one launch with the current tuning
  double mean_k = 1.0;
  if (rc == EVIS_OK) {
    Plan p2 = pl;
    rc = run_step(ctx, p2, out, capacity, n_total, d_K, 0, s);
    std::vector<int32_t> K(n_envs, 1);
    if (rc == EVIS_OK) {
      he = hipMemcpyAsync(K.data(), d_K, 4 * (size_t)n_envs, hipMemcpyDeviceToHost, s);
      if (he == hipSuccess) he = hipStreamSynchronize(s);
      if (he != hipSuccess) rc = hip_fail(ctx, he, "evis_autotune K readback");
    }
    double wk = 0.0, w = 0.0;
    for (int e = 0; e < n_envs; ++e) {
      const double px = (double)envs[e].pair.H * envs[e].pair.W;
      wk += px * K[e];
      w += px;
    }
    mean_k = w > 0.0 ? wk / w : 1.0;
  }
  if (rc == EVIS_OK && cache_path) {
    key = tuning_key(ctx, pl, envs, n_envs, mean_k);
    evis_tuning t = orig;
    float ms = 0.0f;
    if (cache_lookup(cache_path, key, t, ms)) {
      cached = true;
      winner = t;
      winner_ms = ms;
    }
  }
  if (rc == EVIS_OK && !cached) {
    // 1. tile shape (pixels per thread) at the occupancy limit and the full list
    const int shapes[4][2] = {{16, 16}, {32, 16}, {32, 32}, {64, 16}};
    for (int i = 0; i < 4 && rc == EVIS_OK; ++i) {
      evis_tuning t = orig;
      t.tile_w = shapes[i][0];
      t.tile_h = shapes[i][1];
      t.grid_mult = 0;
      t.list_cap = kListCapMax;
      trial(t);
    }
    // 2. workgroups per CU below the occupancy limit
    if (rc == EVIS_OK) {
      const int occ = tile_occupancy(winner.tile_w, winner.tile_h, MODE_STEP, pl.desc[0].warp,
                                     plan_has_noise(pl));
      const evis_tuning base = winner;
      for (int g = occ - 1; g >= std::max(1, occ - 2) && rc == EVIS_OK; --g) {
        evis_tuning t = base;
        t.grid_mult = g;
        trial(t);
      }
    }
    // 3. candidate-list capacity
    if (rc == EVIS_OK) {
      const evis_tuning base = winner;
      for (int cap : {kListCapMax / 2, kListCapMax / 4}) {
        if (rc != EVIS_OK) break;
        evis_tuning t = base;
        t.list_cap = cap;
        trial(t);
      }
    }
    if (rc == EVIS_OK && cache_path) cache_store(cache_path, key, winner, winner_ms);
  }
  he = copy_states(false);
  hipStreamSynchronize(s);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(saved);
  ctx->tuning = (rc == EVIS_OK && he == hipSuccess) ? winner : orig;
  if (rc) return rc;
  if (he != hipSuccess) return hip_fail(ctx, he, "evis_autotune state copy");
  if (best) *best = winner;
  if (best_ms) *best_ms = winner_ms;
  if (n_trials) *n_trials = n_done;
  if (from_cache) *from_cache = cached ? 1 : 0;
  return EVIS_OK;
}

}  // extern "C"
