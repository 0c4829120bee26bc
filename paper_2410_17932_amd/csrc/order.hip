// Spatial (Morton, Z-order) permutation of a point set.  A storage-layout
// step for a static scene, run once at load time: points adjacent in memory
// are then adjacent in space, so their projections land on nearby pixels
// and per-point lookups of screen-space buffers (the depth cull's depth and
// transmittance reads) share cache lines.  The per-frame path gives the same
// result for any point order, up to the order of exactly equal depths.
//
//   k_bbox_init, k_bbox   axis-aligned bounds (order-preserving integer
//                         encoding of floats, so min/max are integer atomics)
//   k_morton              10 bits per axis, interleaved x, y, z -> 30-bit key
//   radix sort            stable, 30 bits: ties keep index order
#include <mutex>

#include "vrs_common.h"

namespace vrs {
namespace {

__device__ inline uint32_t f2ord(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ord2f(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void k_bbox_init(uint32_t* bb) {
  if (threadIdx.x < 3) {
    bb[threadIdx.x] = 0xffffffffu;   // min
    bb[3 + threadIdx.x] = 0u;        // max
  }
}

__global__ __launch_bounds__(256) void k_bbox(const float* __restrict__ pos, int64_t n,
                                              uint32_t* bb) {
  uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float v = pos[a * n + i];
      if (!isfinite(v)) continue;
      const uint32_t o = f2ord(v);
      lo[a] = o < lo[a] ? o : lo[a];
      hi[a] = o > hi[a] ? o : hi[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
      const uint32_t l = __shfl_xor(lo[a], s, 64), h = __shfl_xor(hi[a], s, 64);
      lo[a] = l < lo[a] ? l : lo[a];
      hi[a] = h > hi[a] ? h : hi[a];
    }
  }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      atomicMin(&bb[a], lo[a]);
      atomicMax(&bb[3 + a], hi[a]);
    }
}

// spread the low 10 bits of v to every third bit
__device__ inline uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ pos, int64_t n,
                                                const uint32_t* __restrict__ bb,
                                                uint32_t* __restrict__ key,
                                                uint32_t* __restrict__ val) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = ord2f(bb[a]), hi = ord2f(bb[3 + a]);
    const float v = pos[a * n + i];
    float t = 0.0f;
    if (hi > lo && isfinite(v)) t = ((v - lo) / (hi - lo)) * 1024.0f;
    t = t < 0.0f ? 0.0f : (t > 1023.0f ? 1023.0f : t);
    q[a] = isfinite(v) ? (uint32_t)t : 1023u;
  }
  key[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  val[i] = (uint32_t)i;
}

__global__ void k_copy_u32(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                           int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

struct OrderWs {
  size_t bb, k0, k1, v1, sort_tmp, total;
};

bool order_layout(int64_t n, OrderWs* L) {
  if (n < 1 || n >= (int64_t(1) << 31)) return false;
  Carver c;
  L->bb = c.take(6 * 4);
  L->k0 = c.take((size_t)n * 4);
  L->k1 = c.take((size_t)n * 4);
  L->v1 = c.take((size_t)n * 4);
  L->sort_tmp = c.take(sort_tmp_bytes(n, 30, 8));
  L->total = c.off;
  return true;
}

// Allocation-free variant: its scratch is a file-scope device array sized
// for kNoAllocMaxPoints points (the layout above at that size: bounds, Morton
// keys, the sort's second key and value buffers and its partition counts).
constexpr int64_t kNoAllocMaxPoints = int64_t(1) << 20;
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kNoAllocBytes =
    align256(align256(align256(align256(24) + kNoAllocMaxPoints * 4) + kNoAllocMaxPoints * 4) +
             kNoAllocMaxPoints * 4) +
    (256 + 256 * (size_t)((kNoAllocMaxPoints + 2047) / 2048)) * 4;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on each device, taken once per device (with
// that device current) on the first call there.  In host code the array's
// name is only a stand-in symbol; kernels and copies get this address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

vrs_status spatial_order_run(const float* pos, int64_t n, uint32_t* perm, void* ws,
                             const OrderWs& L, hipStream_t st) {
  uint32_t* bb = at<uint32_t>(ws, L.bb);
  hipLaunchKernelGGL(k_bbox_init, dim3(1), dim3(64), 0, st, bb);
  VRS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bbox, dim3((unsigned)std::min<int64_t>(1024, div_up(n, 256))), dim3(256), 0,
                     st, pos, n, bb);
  VRS_LAUNCH_CHECK();
  // indices start in perm, so an even number of passes leaves the result there
  hipLaunchKernelGGL(k_morton, dim3(div_up(n, 256)), dim3(256), 0, st, pos, n, bb,
                     at<uint32_t>(ws, L.k0), perm);
  VRS_LAUNCH_CHECK();
  bool in1 = false;
  VRS_HIP_CHECK(radix_sort_u32(at<uint32_t>(ws, L.k0), perm, at<uint32_t>(ws, L.k1),
                               at<uint32_t>(ws, L.v1), nullptr, n, 30, 8,
                               at<void>(ws, L.sort_tmp), nullptr, st, &in1));
  if (in1) {
    hipLaunchKernelGGL(k_copy_u32, dim3((unsigned)std::min<int64_t>(4096, div_up(n, 256))),
                       dim3(256), 0, st, at<uint32_t>(ws, L.v1), perm, n);
    VRS_LAUNCH_CHECK();
  }
  return VRS_OK;
}

}  // namespace
}  // namespace vrs

using namespace vrs;

extern "C" size_t vrs_spatial_order_workspace_size(int64_t n) {
  OrderWs L;
  return order_layout(n, &L) ? L.total : 0;
}

extern "C" vrs_status vrs_spatial_order(const float* pos, int64_t n, uint32_t* perm, void* ws,
                                        size_t ws_bytes, void* stream) {
  OrderWs L;
  if (!pos || !perm || !ws || !order_layout(n, &L) || ws_bytes < L.total) return VRS_EINVAL;
  return spatial_order_run(pos, n, perm, ws, L, static_cast<hipStream_t>(stream));
}

extern "C" vrs_status vrs_spatial_order_noalloc(const float* pos, int64_t n, uint32_t* perm,
                                                void* stream) {
  OrderWs L;
  if (!pos || !perm || n > kNoAllocMaxPoints || !order_layout(n, &L) || L.total > kNoAllocBytes)
    return VRS_EINVAL;
  void* ws = nullptr;
  VRS_HIP_CHECK(scratch_address(&ws));
  return spatial_order_run(pos, n, perm, ws, L, static_cast<hipStream_t>(stream));
}
