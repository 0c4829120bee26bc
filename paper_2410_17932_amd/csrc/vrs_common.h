// Shared host/device definitions of the vrsplat HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "vrsplat.h"

#define VRS_HIP_CHECK(expr)                         \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return VRS_EHIP;          \
  } while (0)

#define VRS_LAUNCH_CHECK() VRS_HIP_CHECK(hipGetLastError())

namespace vrs {

constexpr int kWave = 64;

// View as the kernels see it (kernel-argument copy of vrs_view plus the
// camera centre, computed on the host in double precision).
struct KView {
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float znear;
  float cam[3];
  int W, H;
};

struct KViews {
  KView v[VRS_MAX_VIEWS];
  int n;
};

struct KCrop {
  int view, x0, y0, size;
  float gx, gy;
  int pix_base;   // first layer pixel of this crop in the packed pyramid
  int out_base;   // first element of this crop in packed [crop][3][S][S]
};

struct KCrops {
  KCrop c[VRS_MAX_CROPS];
  int n;
};

// Status words written from device code.
__device__ inline void set_status(int32_t* st, int32_t code) {
  if (st) atomicCAS(st, 0, code);
}

// Workspace carving on the host: 256-byte aligned sub-buffers.
struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = (off + 255) & ~size_t(255);
    off = o + bytes;
    return o;
  }
};

template <typename T>
inline T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

bool make_views(const vrs_view* views, int n, KViews* out);

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------ primitives
// Device-wide exclusive scan of uint32 counts (single pass, decoupled
// look-back, Merrill & Garland 2016).  in[i] (or in[idx[i]] when idx is not
// null) for i < n, n = min(*n_dev, n_max) (n_dev may be null).  Writes
// out[i] and *total (may be null) = sum.  tmp: scan_tmp_bytes(n_max).
// cleared: an earlier kernel on the stream zeroed those bytes of tmp since
// their last use, so the scan runs as one launch.
size_t scan_tmp_bytes(int64_t n_max);
hipError_t exclusive_scan_u32(const uint32_t* in, const uint32_t* idx, uint32_t* out,
                              uint32_t* total, const uint32_t* n_dev, int64_t n_max, void* tmp,
                              int32_t* status, hipStream_t st, bool cleared = false);

// Stable LSD radix sort of (uint32 key, value) pairs over the low key_bits
// bits, 8 bits per pass, reduce-then-scan per pass (digit counts per
// partition, their scan per digit, then a ranking scatter; Merrill &
// Grimshaw's structure with wave-ballot multisplit ranking).  Ping-pongs
// between (k0, v0) and (k1, v1); returns through *result_in_1 whether the
// sorted data ended in the second buffer.  n = min(*n_dev, n_max).
size_t sort_tmp_bytes(int64_t n_max, int key_bits);
// gather_src/gather_dst (both or neither): the last pass also writes
// gather_dst[i] = gather_src[value i] in sorted order (a per-value word
// carried into the sorted order without a pass of its own).
hipError_t radix_sort_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                          const uint32_t* n_dev, int64_t n_max, int key_bits, void* tmp,
                          int32_t* status, hipStream_t st, bool* result_in_1,
                          const uint32_t* gather_src = nullptr, uint32_t* gather_dst = nullptr);
hipError_t radix_sort_u64(uint32_t* k0, uint64_t* v0, uint32_t* k1, uint64_t* v1,
                          const uint32_t* n_dev, int64_t n_max, int key_bits, void* tmp,
                          int32_t* status, hipStream_t st, bool* result_in_1);
// After a sort, the key count of each digit value of its last pass
// (uint32 [256], device): for a one-pass sort, the run length of every key.
const uint32_t* radix_sort_digit_totals(const void* tmp);

// Stage timing hook (vrs_trace_set).
void trace_begin(int stage, hipStream_t st);
void trace_end(int stage, hipStream_t st);

// Fill n words with a value (graph-safe replacement for memset).
hipError_t fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t st);

}  // namespace vrs
