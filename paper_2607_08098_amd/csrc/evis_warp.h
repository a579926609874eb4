// Warp building blocks shared by the fused tile kernel and the surrogate
// kernels (gfx950): the candidate 4x4 source blocks of a target tile, the
// depth-tested splat of those sources into an LDS z-buffer (Eq. 5 q_A,
// bilinear footprint, Eq. 6, Eq. 7) and the bilinear gather of B at
// s = q - (1 - f) m_B(q).
//
// The two-splat warps also splat B backward to q_B = p + (1 - f) m_B(p).
// B's splat record holds -m_B, so that q_B = p - g (-m_B) with g = 1 - f is
// the same arithmetic as A's q_A = p - f m_A (the negation is exact, so
// the position is bit for bit p + g m_B), while the depth is still
// interpolated at f from A's side (Z_A at p + m_B) to B's (Z_B at p).
#pragma once

#include "evis_internal.h"

namespace evis {

// Splat direction: A forward, B backward, or A forward with its keys
// tagged (one z-buffer shared by both splats; a tagged key loses a depth
// tie to B's).
enum SplatDir { DIR_A = 0, DIR_B = 1, DIR_A_TAGGED = 2 };
constexpr uint32_t kATag = 0x80000000u;   // tag bit in the low word of a key

// ---------------------------------------------------------------------------
// candidate source blocks
// ---------------------------------------------------------------------------

// Conservative interval of substeps during which some source of the 4x4
// block [Sx0,Sx1]x[Sy0,Sy1] with motion bounds b can put a footprint corner
// into the target tile [Tx0,Tx1]x[Ty0,Ty1].  A corner lies in [Tx0,Tx1]
// only if q_x = p_x - f m_x is in [Tx0 - 1, Tx1 + 1); over the tile q_x lies
// in [Sx0 - f max m_x, Sx1 - f min m_x].
// bnd / a by the hardware reciprocal (relative error a few ulp)
__device__ __forceinline__ float fast_div(float bnd, float a) {
  return bnd * __builtin_amdgcn_rcpf(a);
}
__device__ __forceinline__ void lin_le(float a, float bnd, float& flo, float& fhi) {
  if (a > 0.0f) fhi = fminf(fhi, fast_div(bnd, a));        // a f <= bnd
  else if (a < 0.0f) flo = fmaxf(flo, fast_div(bnd, a));
  else if (bnd < 0.0f) flo = 2.0f;
}
__device__ __forceinline__ void lin_ge(float a, float bnd, float& flo, float& fhi) {
  if (a > 0.0f) flo = fmaxf(flo, fast_div(bnd, a));        // a f >= bnd
  else if (a < 0.0f) fhi = fminf(fhi, fast_div(bnd, a));
  else if (bnd > 0.0f) flo = 2.0f;
}

// The footprint test is conservative by 1/64 px (far above the rounding of
// q = p - f m for |q| < 4096 and |m| < 2^20) and the substep bounds by
// 1/256 of a substep (far above K = 128 times the few-ulp error of the
// reciprocal division for fractions in [0, 1]), so no source that can land
// in the tile at substep j is ever left out.
// With back = true the bounds are those of a backward splat, whose position
// fraction is g = 1 - f: the interval [flo, fhi] of g maps to substeps
// [K (1 - fhi), K (1 - flo)].
__device__ __forceinline__ bool substep_range(float4 b, int Sx0, int Sx1, int Sy0, int Sy1,
                                              int Tx0, int Tx1, int Ty0, int Ty1, int K,
                                              int& jlo, int& jhi, bool back = false) {
  if (!(b.x <= b.y) || !(b.z <= b.w)) return false;   // no finite source
  float flo = 0.0f, fhi = 1.0f;
  const float slack = 1.0f / 64.0f;
  lin_le(b.x, (float)(Sx1 - Tx0 + 1) + slack, flo, fhi);
  lin_ge(b.y, (float)(Sx0 - Tx1 - 1) - slack, flo, fhi);
  lin_le(b.z, (float)(Sy1 - Ty0 + 1) + slack, flo, fhi);
  lin_ge(b.w, (float)(Sy0 - Ty1 - 1) - slack, flo, fhi);
  if (!(flo <= fhi)) return false;
  const float Kf = (float)K;
  const float jl = back ? (1.0f - fhi) : flo, jh = back ? (1.0f - flo) : fhi;
  const int lo = max(1, (int)ceilf(jl * Kf - (1.0f / 256.0f)));
  const int hi = min(K - 1, (int)floorf(jh * Kf + (1.0f / 256.0f)));
  if (lo > hi) return false;
  jlo = lo;
  jhi = hi;
  return true;
}

// The LDS z-buffer of a TW x TH target tile has an apron of one cell on
// every side, so that every footprint corner of a source that lands in
// [Tx0 - 1, Tx1 + 1) x [Ty0 - 1, Ty1 + 1) has a cell; apron cells (and
// those of pixels outside the image) are written but never read.  Rows are
// ZS(TW) = TW + 4 keys long (TW a multiple of 16): consecutive rows start
// 32 bytes further along the banks, so the four rows of a 4x4 block's
// footprint fall in different banks.
template <int TW>
__device__ __forceinline__ constexpr int zrow() { return TW + 4; }
template <int TW, int TH>
__device__ __forceinline__ constexpr int zcells() { return zrow<TW>() * (TH + 2); }
// Cell of target pixel (lx, ly) of the tile (lx in [-1, TW], ly in [-1, TH]).
template <int TW>
__device__ __forceinline__ int zcell(int lx, int ly) { return (ly + 1) * zrow<TW>() + (lx + 1); }

// Candidate-list entry of a 4x4 source block: bx << 23 | by << 14 | j_lo << 7
// | j_hi (bx, by < 512; 1 <= j_lo <= j_hi <= 127), so 0 is never an entry
// and marks an empty slot.
__device__ __forceinline__ uint32_t cand_entry(int bx, int by, int jlo, int jhi) {
  return ((uint32_t)bx << 23) | ((uint32_t)by << 14) | ((uint32_t)jlo << 7) | (uint32_t)jhi;
}
__device__ __forceinline__ int cand_bx(uint32_t e) { return (int)(e >> 23); }
__device__ __forceinline__ int cand_by(uint32_t e) { return (int)((e >> 14) & 0x1FFu); }
__device__ __forceinline__ int cand_jlo(uint32_t e) { return (int)((e >> 7) & 0x7Fu); }
__device__ __forceinline__ int cand_jhi(uint32_t e) { return (int)(e & 0x7Fu); }

// Splat kChunk slots of four source blocks each (lane group g = lane / 16
// takes candidate entry blk[c] of slot c, one source per lane; 0 is empty)
// into the LDS z-buffers of target tile [Tx0,Tx1]x[Ty0,Ty1]: at fraction
// fs[t] into zs[t] for t < nf (nf <= NF consecutive substeps share the
// loads).  The loads of all slots are issued before any of them is used.
constexpr int kChunk = 3;

template <int TW, int NF, int DIR = DIR_A>
__device__ __forceinline__ void splat_chunk(const EnvDesc& d, const uint32_t (&blk)[kChunk],
                                            const float (&fs)[NF], int nf, int Tx0, int Tx1,
                                            int Ty0, int Ty1, unsigned long long* const (&zs)[NF]) {
  const int r = threadIdx.x & (kBlkPx - 1);   // lane within the block: (r & 3, r >> 2)
  const float4* recs = (DIR == DIR_B) ? d.srcB : d.src;
  float4 rec[kChunk];   // A: (m_A.x, m_A.y, Z_A, Zend - Z_A); B: (-m_B.x, -m_B.y, Zstart, Z_B - Zstart)
  int src[kChunk];      // source index, -1 outside the image or for an empty slot
  int sx[kChunk], sy[kChunk];
  // All loads first, unconditionally (a lane without a source reads a
  // record of its block, or of block 0), so that they are in flight
  // together.
#pragma unroll
  for (int c = 0; c < kChunk; ++c) {
    const uint32_t e = blk[c];
    const int bx = cand_bx(e), by = cand_by(e);
    sx[c] = bx * kSrcBlk + (r & 3);
    sy[c] = by * kSrcBlk + (r >> 2);
    const bool ok = e != 0u && sx[c] < d.W && sy[c] < d.H;
    // 24-bit products (full-rate v_mul_u32_u24): rows, columns and block
    // counts are below 2^12
    src[c] = ok ? (int)__umul24((unsigned)sy[c], (unsigned)d.W) + sx[c] : -1;
    // every candidate entry names a block of the env (an empty slot block
    // 0), so the record is read unconditionally: one 32-bit byte offset
    rec[c] = ldg_bytes(recs, ((__umul24((unsigned)by, (unsigned)d.ntx_src) + (unsigned)bx) *
                              (unsigned)(kBlkPx * sizeof(float4))) + (unsigned)r * (unsigned)sizeof(float4));
  }
  // image pixel (x, y) has z-buffer cell y ZS + x - corg (the apron's first
  // cell is pixel (Tx0 - 1, Ty0 - 1))
  const int corg = (Ty0 - 1) * zrow<TW>() + (Tx0 - 1);
#pragma unroll
  for (int c = 0; c < kChunk; ++c) {
    if (src[c] < 0) continue;
    const float px = (float)sx[c], py = (float)sy[c];
#pragma unroll
    for (int t = 0; t < NF; ++t) {
      if (t >= nf) break;   // uniform
      const float f = fs[t];
      const float fp = (DIR == DIR_B) ? 1.0f - f : f;   // position fraction
      const float qx = px - fp * rec[c].x;
      const float qy = py - fp * rec[c].y;
      const float zt = rec[c].z + f * rec[c].w;
      if (!(zt > 0.0f)) continue;
      if (!(qx >= (float)(Tx0 - 1) && qx < (float)(Tx1 + 1) && qy >= (float)(Ty0 - 1) &&
            qy < (float)(Ty1 + 1)))
        continue;
      const float fx0 = floorf(qx), fy0 = floorf(qy);
      const bool bx = qx > fx0, by = qy > fy0;   // corners of strictly positive weight
      const uint32_t low = (DIR == DIR_A_TAGGED) ? ((uint32_t)src[c] | kATag) : (uint32_t)src[c];
      const unsigned long long key = ((unsigned long long)__float_as_uint(zt) << 32) | low;
      // All four corners of the cell from one address.  A corner of zero
      // weight (an integer coordinate, rare) must not be written: it gets
      // the empty key, which changes nothing; the gather warp's splat
      // writes the one key four times when all four weights are positive.
      // y0 ZS + x0 is formed in float, exactly (|x0|, |y0| <= 2^12, so it
      // is an integer below 2^24).
      constexpr int ZS = zrow<TW>();
      unsigned long long* zb = zs[t] + ((int)fmaf(fy0, (float)ZS, fx0) - corg);
      atomicMin(zb, key);
      if (DIR == DIR_A && bx && by) {   // (the two-splat warps measured no faster with it)
        atomicMin(zb + 1, key);
        atomicMin(zb + ZS, key);
        atomicMin(zb + ZS + 1, key);
      } else {
        atomicMin(zb + 1, bx ? key : kEmptyKey);
        atomicMin(zb + ZS, by ? key : kEmptyKey);
        atomicMin(zb + ZS + 1, (bx && by) ? key : kEmptyKey);
      }
    }
  }
}

// B gather at fraction g = 1 - f for one target pixel (x, y): the sample
// position s = (x, y) - g m_B, its validity and the four taps of its cell.
struct BTaps {
  float a, b, c, d, wx, wy;
  bool v;
};

__device__ __forceinline__ BTaps b_taps(const EnvDesc& d, int x, int y, float2 mB, float g,
                                        bool pixel_ok) {
  BTaps t;
  const float sx = (float)x - g * mB.x;
  const float sy = (float)y - g * mB.y;
  t.v = pixel_ok && sx >= 0.0f && sx <= (float)(d.W - 1) && sy >= 0.0f && sy <= (float)(d.H - 1);
  const float sxc = t.v ? sx : 0.0f, syc = t.v ? sy : 0.0f;
  const float fx0 = floorf(sxc), fy0 = floorf(syc);
  t.wx = sxc - fx0;
  t.wy = syc - fy0;
  const int x0 = (int)fx0, y0 = (int)fy0;
  const int x1 = min(x0 + 1, d.W - 1), y1 = min(y0 + 1, d.H - 1);
  t.a = t.b = t.c = t.d = 0.0f;
  if (t.v) {
    const int r0 = (int)__umul24((unsigned)y0, (unsigned)d.W);   // y, W < 2^12: 24-bit products
    const int r1 = (int)__umul24((unsigned)y1, (unsigned)d.W);
    t.a = ldg(d.LB, r0 + x0);
    t.b = ldg(d.LB, r0 + x1);
    t.c = ldg(d.LB, r1 + x0);
    t.d = ldg(d.LB, r1 + x1);
  }
  return t;
}

__device__ __forceinline__ float b_value(const BTaps& t) {
  return lerp32(lerp32(t.a, t.b, t.wx), lerp32(t.c, t.d, t.wx), t.wy);
}

// Window of 4x4 source blocks that can reach a target tile: block columns
// [wx0, wx0 + nwx), nwin blocks in all.
struct Window {
  int wx0, wy0, nwx, nwin;
};

// Whether block (bx, by) can reach target tile [Tx0,Tx1]x[Ty0,Ty1], and during
// which substeps.  A block whose positions over the whole gap (f in [0, 1])
// stay clear of the tile by more than a pixel is rejected first, without
// the divisions of substep_range (which rejects it too).
template <bool BACK = false>
__device__ __forceinline__ bool block_range(const EnvDesc& d, int bx, int by, int Tx0, int Tx1,
                                            int Ty0, int Ty1, int K, int& jlo, int& jhi) {
  const float4 b = ldg(BACK ? d.tbB : d.tb, by * d.ntx_src + bx);
  const int Sx0 = bx * kSrcBlk, Sx1 = min(bx * kSrcBlk + kSrcBlk - 1, d.W - 1);
  const int Sy0 = by * kSrcBlk, Sy1 = min(by * kSrcBlk + kSrcBlk - 1, d.H - 1);
  // q = p - f m over f in [0, 1] lies in [S0 - max(m_max, 0), S1 - min(m_min, 0)]
  if ((float)Sx0 - fmaxf(b.y, 0.0f) >= (float)(Tx1 + 2) ||
      (float)Sx1 - fminf(b.x, 0.0f) <= (float)(Tx0 - 2) ||
      (float)Sy0 - fmaxf(b.w, 0.0f) >= (float)(Ty1 + 2) ||
      (float)Sy1 - fminf(b.z, 0.0f) <= (float)(Ty0 - 2))
    return false;
  return substep_range(b, Sx0, Sx1, Sy0, Sy1, Tx0, Tx1, Ty0, Ty1, K, jlo, jhi, BACK);
}

// Whether some source of superblock (sx, sy) can come within a pixel of
// target tile [Tx0,Tx1]x[Ty0,Ty1] over the gap: the test block_range makes
// first, on the superblock's extent and motion bounds.  Both only widen
// from a block to its superblock, so a block that passes it lies in a
// superblock that passes it.
__device__ __forceinline__ bool superblock_reaches(const EnvDesc& d, int sx, int sy, int Tx0,
                                                   int Tx1, int Ty0, int Ty1) {
  const float4 b = ldg(d.sbb, sy * d.ntx_sb + sx);
  if (!(b.x <= b.y) || !(b.z <= b.w)) return false;   // no finite source
  constexpr int SP = kSbBlk * kSrcBlk;                 // pixels per superblock side
  const int Sx0 = sx * SP, Sx1 = min(Sx0 + SP - 1, d.W - 1);
  const int Sy0 = sy * SP, Sy1 = min(Sy0 + SP - 1, d.H - 1);
  return !((float)Sx0 - fmaxf(b.y, 0.0f) >= (float)(Tx1 + 2) ||
           (float)Sx1 - fminf(b.x, 0.0f) <= (float)(Tx0 - 2) ||
           (float)Sy0 - fmaxf(b.w, 0.0f) >= (float)(Ty1 + 2) ||
           (float)Sy1 - fminf(b.z, 0.0f) <= (float)(Ty0 - 2));
}

// The window of source blocks that can reach target tile [Tx0,Tx1]x[Ty0,Ty1]
// (the env's largest motion around it); its last block column and row in
// wx1, wy1.
__device__ __forceinline__ void candidate_window(const EnvDesc& d, const EnvDyn& dy, int Tx0,
                                                 int Tx1, int Ty0, int Ty1, Window& w, int& wx1,
                                                 int& wy1) {
  const double M = __longlong_as_double((long long)dy.msq_bits);
  const int Rw = (M > 1.0e12) ? (1 << 20) : ((int)ceil(sqrt(M)) + 3);
  w.wx0 = max(0, Tx0 - Rw) / kSrcBlk;
  w.wy0 = max(0, Ty0 - Rw) / kSrcBlk;
  wx1 = min(d.ntx_src - 1, min(Tx1 + Rw, d.W - 1) / kSrcBlk);
  wy1 = min(d.nty_src - 1, min(Ty1 + Rw, d.H - 1) / kSrcBlk);
  w.nwx = wx1 - w.wx0 + 1;
  w.nwin = w.nwx * (wy1 - w.wy0 + 1);
}

// Candidate source blocks of target tile [Tx0,Tx1]x[Ty0,Ty1] and the substeps
// during which each can reach it, appended to the LDS list (at most cap
// entries, see cand_entry).  *count must be zero on entry; returns the
// number of candidates (uniform; more than cap means the list overflowed).
// The window of blocks follows from the env's largest motion; when it
// takes more than one pass, with the superblock bounds (sb_list: LDS
// [kBlock], *sb_count zero on entry) only the blocks of the window's
// superblocks that can reach the tile are tested, which on a scene whose
// motion varies is a fraction of the window.  The candidates are the same either way (their order in the
// list is not).  Holds a barrier (two with superblocks).
__device__ __forceinline__ int build_candidates(const EnvDesc& d, const EnvDyn& dy, int K,
                                                int Tx0, int Tx1, int Ty0, int Ty1,
                                                uint32_t* list, int* count, int cap, Window& w,
                                                int* sb_list = nullptr, int* sb_count = nullptr) {
  const int tid = threadIdx.x;
  int wx1, wy1;
  candidate_window(d, dy, Tx0, Tx1, Ty0, Ty1, w, wx1, wy1);
  auto test_block = [&](int bx, int by) {
    int jlo, jhi;
    if (block_range(d, bx, by, Tx0, Tx1, Ty0, Ty1, K, jlo, jhi)) {
      const int slot = atomicAdd(count, 1);
      if (slot < cap) list[slot] = cand_entry(bx, by, jlo, jhi);
    }
  };
  const int sx0 = w.wx0 / kSbBlk, sx1 = wx1 / kSbBlk, sy0 = w.wy0 / kSbBlk, sy1 = wy1 / kSbBlk;
  const int nsx = sx1 - sx0 + 1, nsb = nsx * (sy1 - sy0 + 1);
  // (a window the workgroup scans in one pass is left to the plain scan:
  // the superblock pass would only add a barrier)
  if (sb_list != nullptr && d.sbb != nullptr && w.nwin > kBlock && nsb <= kBlock) {   // uniform
    if (tid < nsb) {
      const int sx = sx0 + tid % nsx, sy = sy0 + tid / nsx;
      if (superblock_reaches(d, sx, sy, Tx0, Tx1, Ty0, Ty1)) sb_list[atomicAdd(sb_count, 1)] = sx | (sy << 16);
    }
    __syncthreads();
    constexpr int NB = kSbBlk * kSbBlk;
    const int n_items = __builtin_amdgcn_readfirstlane(*sb_count) * NB;
    for (int i = tid; i < n_items; i += kBlock) {
      const int e = sb_list[i / NB], bi = i % NB;
      const int bx = (e & 0xFFFF) * kSbBlk + bi % kSbBlk, by = (e >> 16) * kSbBlk + bi / kSbBlk;
      if (bx >= w.wx0 && bx <= wx1 && by >= w.wy0 && by <= wy1) test_block(bx, by);
    }
  } else {
    for (int i = tid; i < w.nwin; i += kBlock) test_block(w.wx0 + i % w.nwx, w.wy0 + i / w.nwx);
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*count);
}

// Both directions' candidates (two-splat warps) in one list of cap entries:
// A's from the front, B's from the back (B's entry e at cap - 1 - e).  One
// 64-bit LDS counter holds A's count in its low and B's in its high word;
// an entry is stored only if the two counts before its own increment leave
// it room, which also keeps the two ends from meeting (of two entries
// that would share a slot, the one counted second finds the list full).
// *count must be zero on entry; nA and nB are uniform, and nA + nB > cap
// means the list overflowed.  Holds a barrier.
__device__ __forceinline__ void build_candidates_two(const EnvDesc& d, const EnvDyn& dy, int K,
                                                     int Tx0, int Tx1, int Ty0, int Ty1,
                                                     uint32_t* list, unsigned long long* count,
                                                     int cap, Window& w, int& nA, int& nB) {
  const int tid = threadIdx.x;
  const int W = d.W, H = d.H;
  const double M = __longlong_as_double((long long)dy.msq_bits);
  const int Rw = (M > 1.0e12) ? (1 << 20) : ((int)ceil(sqrt(M)) + 3);
  w.wx0 = max(0, Tx0 - Rw) / kSrcBlk;
  w.wy0 = max(0, Ty0 - Rw) / kSrcBlk;
  const int wx1 = min(d.ntx_src - 1, min(Tx1 + Rw, W - 1) / kSrcBlk);
  const int wy1 = min(d.nty_src - 1, min(Ty1 + Rw, H - 1) / kSrcBlk);
  w.nwx = wx1 - w.wx0 + 1;
  w.nwin = w.nwx * (wy1 - w.wy0 + 1);
  for (int i = tid; i < w.nwin; i += kBlock) {
    const int bx = w.wx0 + i % w.nwx, by = w.wy0 + i / w.nwx;
    int jlo, jhi;
    if (block_range<false>(d, bx, by, Tx0, Tx1, Ty0, Ty1, K, jlo, jhi)) {
      const unsigned long long old = atomicAdd(count, 1ull);
      const int a = (int)(old & 0xFFFFFFFFull), b = (int)(old >> 32);
      if (a + b < cap) list[a] = cand_entry(bx, by, jlo, jhi);
    }
    if (block_range<true>(d, bx, by, Tx0, Tx1, Ty0, Ty1, K, jlo, jhi)) {
      const unsigned long long old = atomicAdd(count, 1ull << 32);
      const int a = (int)(old & 0xFFFFFFFFull), b = (int)(old >> 32);
      if (a + b < cap) list[cap - 1 - b] = cand_entry(bx, by, jlo, jhi);
    }
  }
  __syncthreads();
  const unsigned long long c = *count;
  nA = __builtin_amdgcn_readfirstlane((int)(c & 0xFFFFFFFFull));
  nB = __builtin_amdgcn_readfirstlane((int)(c >> 32));
}

// Splat every source that can reach the target tile at substeps j .. j+nf-1
// (fractions fs, z-buffers zs): the candidate-list entries active at any of
// them, or, if the list overflowed, the active blocks of the whole window.
// Each wave takes every fourth entry, packs its active entries into its
// 64-entry LDS slice `wl` and splats them four blocks (one per lane group)
// per slot.  Entry e sits at list[lbase + lstep * e] (lstep = -1 for the
// backward splat's entries at the back of a shared list).
template <int TW, int NF, int DIR = DIR_A, int SCAN = 1>
__device__ __forceinline__ void splat_candidates(const EnvDesc& d, const uint32_t* list, int nlist,
                                                 bool overflow, const Window& w, int K, int j,
                                                 int nf, const float (&fs)[NF], int Tx0, int Tx1,
                                                 int Ty0, int Ty1, uint32_t* wl,
                                                 unsigned long long* const (&zs)[NF],
                                                 int lbase = 0, int lstep = 1) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int g = lane >> 4;
  const int jz = j + nf - 1;
  if (!overflow) {
    for (int base = 0; base < nlist; base += kBlock) {
      const int e2 = base + lane * kWavesPerBlock + wave;
      uint32_t ent = 0u;
      bool act = false;
      if (e2 < nlist) {
        ent = lds_ld(list, lbase + lstep * e2);
        act = (jz >= cand_jlo(ent)) && (j <= cand_jhi(ent));
      }
      const unsigned long long mask = __ballot(act);
      const int nact = __popcll(mask);
      if (act) lds_st(wl, __popcll(mask & ((1ull << lane) - 1ull)), ent);
      for (int s0 = 0; s0 < nact; s0 += 4 * kChunk) {
        uint32_t blk[kChunk];
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
          const int i = s0 + c * 4 + g;
          blk[c] = (i < nact) ? lds_ld(wl, i) : 0u;
        }
        splat_chunk<TW, NF, DIR>(d, blk, fs, nf, Tx0, Tx1, Ty0, Ty1, zs);
      }
    }
  } else {
    // Window scan (the candidate list did not fit): each pass of a wave
    // tests and splats 4 SCAN blocks of the window (SCAN <= kChunk slots of
    // the chunk; more slots take more registers, which the kernels at
    // their register limit pay for in spills).
    static_assert(SCAN >= 1 && SCAN <= kChunk, "window scan slots");
    for (int i0 = wave * 4 * SCAN; i0 < w.nwin; i0 += 4 * SCAN * kWavesPerBlock) {
      uint32_t blk[kChunk];
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        const int i = i0 + c * 4 + g;
        blk[c] = 0u;
        if (c < SCAN && i < w.nwin) {
          const int bx = w.wx0 + i % w.nwx, by = w.wy0 + i / w.nwx;
          int jlo, jhi;
          if (block_range<DIR == DIR_B>(d, bx, by, Tx0, Tx1, Ty0, Ty1, K, jlo, jhi) && jz >= jlo &&
              j <= jhi)
            blk[c] = cand_entry(bx, by, jlo, jhi);
        }
      }
      splat_chunk<TW, NF, DIR>(d, blk, fs, nf, Tx0, Tx1, Ty0, Ty1, zs);
    }
  }
}

}  // namespace evis
