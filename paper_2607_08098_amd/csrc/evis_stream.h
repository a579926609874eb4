// Sharded reservation of event-stream slots (gfx950).
//
// A same-address 64-bit atomic add runs at about 83 M/s on this GPU (one
// at a time, far from the CUs), so a kernel that reserves slots for a few
// hundred events at a time on the caller's cursor queues on that one
// address.  Here reservations are spread over kStreams counters instead:
// stream s hands out its slots i = 0, 1, 2, ... in blocks of kStreamChunk, and
// block k of a stream is placed in the output at a chunk drawn from one
// chunk counter (one atomic per kStreamChunk events).  The reservation that
// enters block k of a stream draws and publishes the chunk of block
// k + kAheadChunks, so a chunk is nearly always published long before
// anyone needs it; a reservation that finds its chunk not yet published
// waits for the wave about to publish it (that wave waits on nothing
// before it publishes).
//
// When the emitting kernel is done, only the last blocks of each stream
// are not full (at most kMaxHoleChunks of them).  The fixup kernel moves
// the events stored above the stream's end into those holes, so that
// out[base, min(base + T, capacity)) holds events (T: the events of the
// call), and sets the cursor to base + T.  Chunk slots at or past
// `capacity` go to a spill buffer large enough for every hole, so that
// prefix is filled whenever the caller's buffer holds it.
#pragma once

#include "evis_common.h"

namespace evis {

constexpr int kStreams = 32;
constexpr int kStreamChunkLog = 12;
constexpr int kStreamChunk = 1 << kStreamChunkLog;        // slots per block / chunk
constexpr int kAheadChunks = 3;               // blocks published ahead of use
constexpr int kMaxHoleChunks = kStreams * (kAheadChunks + 1);
constexpr long long kSpillEvents = (long long)kMaxHoleChunks * kStreamChunk;
constexpr int kChunkUnpublished = -1;
constexpr int kChunkDropped = -2;             // no place: past the output and the spill
constexpr int kStreamLine = 32;               // u64 counters 256 bytes apart

// Per-call values, written by the init kernel (one 256-byte line).
struct StreamHdr {
  long long base;          // cursor at the start of the call
  unsigned int nchunks;    // chunks drawn so far
  int gmax;                // chunks with a place (output or spill)
};

// Device state of the event stream of one call (all device memory).
struct StreamState {
  StreamHdr* hdr;
  unsigned long long* fill;   // [kStreams * kStreamLine]: slots reserved by stream s, at s * kStreamLine
  int* chunk_of;              // [kStreams][kmax]: chunk of block k of stream s, or unpublished / dropped
  int* owner;                 // [gmax_alloc]: s | k << 8 of chunk g
  evis_event* spill;          // [kSpillEvents]
  int kmax;                   // blocks per stream in chunk_of
};

// Chunk-table accesses are device-coherent but relaxed: a consumer uses
// only the chunk number itself (the owner table is read by the next
// kernel), and acquire / release would invalidate / write back the L2 of
// the whole die at every access.
__device__ __forceinline__ int load_chunk_entry(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_chunk_entry(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Draw the chunk of block k of stream s and publish it.
__device__ __forceinline__ void stream_publish(const StreamState& st, int gmax, int s, long long k) {
  if (k >= st.kmax) return;
  const int g = (int)__hip_atomic_fetch_add(&st.hdr->nchunks, 1u, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
  int* p = st.chunk_of + (long long)s * st.kmax + k;
  if (g < gmax) {
    st.owner[g] = s | ((int)k << 8);
    store_chunk_entry(p, g);
  } else {
    store_chunk_entry(p, kChunkDropped);
  }
}

// Reserve n >= 1 consecutive slots of stream s and publish the chunks the
// reservation makes due.  One lane calls it; returns the first slot.
__device__ __forceinline__ unsigned long long stream_reserve_lane(const StreamState& st, int gmax,
                                                                  int s, unsigned long long n) {
  const unsigned long long i0 = __hip_atomic_fetch_add(st.fill + s * kStreamLine, n,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // blocks entered: those whose first slot lies in [i0, i0 + n)
  const long long k_first = (long long)((i0 + kStreamChunk - 1) >> kStreamChunkLog);
  const long long k_end = (long long)((i0 + n + kStreamChunk - 1) >> kStreamChunkLog);
  for (long long k = k_first; k < k_end; ++k) stream_publish(st, gmax, s, k + kAheadChunks);
  return i0;
}

// The chunk of block k of stream s, once published.  The wait is bounded:
// after about 2^22 tries it gives up and the block's events are dropped
// (still counted), which a correct run never does.
__device__ __forceinline__ int stream_chunk(const StreamState& st, int s, long long k) {
  if (k >= st.kmax) return kChunkDropped;
  const int* p = st.chunk_of + (long long)s * st.kmax + k;
  int g = load_chunk_entry(p);
  for (int tries = 0; g == kChunkUnpublished && tries < (1 << 22); ++tries) {
    __builtin_amdgcn_s_sleep(2);
    g = load_chunk_entry(p);
  }
  return g == kChunkUnpublished ? kChunkDropped : g;
}

// Address of stream slot i in chunk g (null: dropped).
__device__ __forceinline__ evis_event* stream_slot_ptr(const StreamState& st, long long base, int g,
                                                       unsigned long long i, evis_event* out,
                                                       long long capacity) {
  if (g < 0) return nullptr;
  const long long pos = base + ((long long)g << kStreamChunkLog) + (long long)(i & (kStreamChunk - 1));
  if (pos < capacity) return out + pos;
  const long long sp = pos - capacity;
  return (capacity > base && sp < kSpillEvents) ? st.spill + sp : nullptr;
}

// Layout of a call's stream state in one device buffer, for an output of
// `capacity` events: the header line, the stream counters, chunk_of,
// owner, then the spill buffer.  Returns the bytes needed; with p, fills st.
inline size_t stream_state_layout(long long capacity, void* p, StreamState* st) {
  const long long cap = capacity > 0 ? capacity : 0;
  const long long gmax = (cap + kSpillEvents + kStreamChunk - 1) >> kStreamChunkLog;
  const long long kmax = gmax + kAheadChunks + 1;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_fill = 256;
  const size_t o_chunk = o_fill + up((size_t)kStreams * kStreamLine * sizeof(unsigned long long));
  const size_t o_owner = o_chunk + up((size_t)kStreams * (size_t)kmax * sizeof(int));
  const size_t o_spill = o_owner + up((size_t)gmax * sizeof(int));
  const size_t total = o_spill + (size_t)kSpillEvents * sizeof(evis_event);
  if (p && st) {
    unsigned char* b = static_cast<unsigned char*>(p);
    st->hdr = reinterpret_cast<StreamHdr*>(b);
    st->fill = reinterpret_cast<unsigned long long*>(b + o_fill);
    st->chunk_of = reinterpret_cast<int*>(b + o_chunk);
    st->owner = reinterpret_cast<int*>(b + o_owner);
    st->spill = reinterpret_cast<evis_event*>(b + o_spill);
    st->kmax = (int)kmax;
  }
  return total;
}

}  // namespace evis
