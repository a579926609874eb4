// Event voxel grid (the per-polarity, 128-bin representation of the
// paper's speed-estimation experiment): events of one env in [t0, t1) are
// spread over two neighbouring time bins by linear interpolation, in 16-bit
// fixed point so that the sums are integers (uint32 atomics, exact and
// independent of order), then each (polarity, bin) plane is divided by its
// maximum.  HBM-bound: a fill, one pass over the event stream (which also
// finds the plane maxima) and a read-write pass over the grid.
#include "evis_internal.h"

namespace evis {

constexpr uint32_t kVoxelOne = 1u << 16;

__global__ __launch_bounds__(kBlock) void k_voxel_fill(uint32_t* __restrict__ acc, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) acc[i] = 0u;
}

// The accumulation also finds each plane's maximum: a voxel's sums only
// grow, so the largest sum an add returns is the plane's final maximum.
// Each workgroup keeps its planes' maxima in LDS and raises the global
// ones once at its end.
__global__ __launch_bounds__(kBlock) void k_voxel_acc(const VoxelArgs a) {
  extern __shared__ uint32_t s_pmax[];   // [2 * bins]
  for (int i = threadIdx.x; i < 2 * a.bins; i += kBlock) s_pmax[i] = 0u;
  __syncthreads();
  const long long n = min((long long)*a.n_events, a.capacity);
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long plane = (long long)a.H * a.W;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const evis_event e = a.events[i];
    const uint32_t w = e.xyp;
    if ((int)(w >> 23) != a.env_id) continue;
    const long long t = e.t_us;
    if (t < a.t0 || t >= a.t1) continue;
    const int x = (int)(w & 0x7FFu), y = (int)((w >> 11) & 0x7FFu), p = (int)((w >> 22) & 1u);
    if (x >= a.W || y >= a.H) continue;
    const float tau = (float)(t - a.t0) * a.scale;
    int b = (int)floorf(tau);
    uint32_t q1 = 0u;
    if (b >= a.bins - 1) {
      b = a.bins - 1;
    } else {
      q1 = (uint32_t)floorf((tau - (float)b) * 65536.0f);
    }
    const int pl = p * a.bins + b;
    uint32_t* base = a.acc + ((long long)pl * plane + (long long)y * a.W + x);
    const uint32_t w0 = kVoxelOne - q1;
    atomicMax(&s_pmax[pl], atomicAdd(base, w0) + w0);
    if (q1) atomicMax(&s_pmax[pl + 1], atomicAdd(base + plane, q1) + q1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * a.bins; i += kBlock)
    if (s_pmax[i]) atomicMax(a.maxbuf + i, s_pmax[i]);
}

// Each voxel divided by its plane's maximum, in place (uint32 sums in,
// float32 out); workgroup (chunk, plane) reads a chunk of a plane, 16
// bytes per lane when the grid starts on 16 bytes and a plane is a whole
// number of 16-byte groups (the chunks are, see launch_voxel).
__global__ __launch_bounds__(kBlock) void k_voxel_div(uint32_t* __restrict__ acc, long long plane,
                                                      long long chunk, const uint32_t* maxbuf) {
  uint32_t* pl = acc + (long long)blockIdx.y * plane;
  float* out = reinterpret_cast<float*>(pl);
  const uint32_t mx = maxbuf[blockIdx.y];
  const float fm = (float)mx;
  const long long i0 = (long long)blockIdx.x * chunk, i1 = min(plane, i0 + chunk);
  if ((plane & 3) == 0 && (reinterpret_cast<uintptr_t>(acc) & 15) == 0) {   // uniform
    uint4* p4 = reinterpret_cast<uint4*>(pl);
    float4* o4 = reinterpret_cast<float4*>(pl);
#pragma unroll 4
    for (long long i = (i0 >> 2) + threadIdx.x; i < (i1 >> 2); i += kBlock) {
      const uint4 v = p4[i];
      o4[i] = mx ? make_float4((float)v.x / fm, (float)v.y / fm, (float)v.z / fm, (float)v.w / fm)
                 : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  } else {
    for (long long i = i0 + threadIdx.x; i < i1; i += kBlock) {
      const uint32_t v = pl[i];
      out[i] = mx ? (float)v / fm : 0.0f;
    }
  }
}

hipError_t launch_voxel(const VoxelArgs& a, hipStream_t s) {
  const long long plane = (long long)a.H * a.W;
  const long long total = 2LL * a.bins * plane;
  const int fill_blocks = (int)std::min<long long>((total + kBlock - 1) / kBlock, 256LL * 8);
  hipLaunchKernelGGL(k_voxel_fill, dim3(fill_blocks), dim3(kBlock), 0, s, a.acc, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_voxel_fill, dim3(1), dim3(kBlock), 0, s, a.maxbuf, 2LL * a.bins);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int acc_blocks = (int)std::max<long long>(1, std::min<long long>((a.capacity + kBlock - 1) / kBlock, 256LL * 8));
  hipLaunchKernelGGL(k_voxel_acc, dim3(acc_blocks), dim3(kBlock), 2 * a.bins * sizeof(uint32_t), s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // enough workgroups to fill the chip: chunks of at least 16 K voxels, a
  // multiple of 4 (whole 16-byte groups)
  const long long chunk = (std::max<long long>(16384, (plane + 7) / 8) + 3) & ~3LL;
  const int nchunks = (int)((plane + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_voxel_div, dim3(nchunks, 2 * a.bins), dim3(kBlock), 0, s, a.acc, plane, chunk,
                     a.maxbuf);
  return hipGetLastError();
}

}  // namespace evis
