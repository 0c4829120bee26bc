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
  int mx0, my0;   // largest origin inside the view: W - size, H - size
};

// Crop table as kernels see it: views, sizes and packing fixed on the host;
// origins and gazes from the host values, or, when `place` is set, from a
// device table read at run time (vrs_crop_place: x0, y0, gaze_x, gaze_y),
// so a captured frame takes a new fixation without being captured again.
// Origins from the device table are clamped into the view.
struct KCrops {
  KCrop c[VRS_MAX_CROPS];
  int n;
  const int4* place;
};

__device__ inline int clamp_origin(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }
__device__ inline int crop_x0(const KCrops& kc, int k) {
  return kc.place ? clamp_origin(kc.place[k].x, kc.c[k].mx0) : kc.c[k].x0;
}
__device__ inline int crop_y0(const KCrops& kc, int k) {
  return kc.place ? clamp_origin(kc.place[k].y, kc.c[k].my0) : kc.c[k].y0;
}
__device__ inline float crop_gx(const KCrops& kc, int k) {
  return kc.place ? __int_as_float(kc.place[k].z) : kc.c[k].gx;
}
__device__ inline float crop_gy(const KCrops& kc, int k) {
  return kc.place ? __int_as_float(kc.place[k].w) : kc.c[k].gy;
}

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
// Compute units of the current device (queried once per device).
int device_cus();
hipError_t exclusive_scan_u32(const uint32_t* in, const uint32_t* idx, uint32_t* out,
                              uint32_t* total, const uint32_t* n_dev, int64_t n_max, void* tmp,
                              int32_t* status, hipStream_t st, bool cleared = false);

// Stable LSD radix sort of (uint32 key, value) pairs over the low key_bits
// bits, radix_bits (4, 6, 8 or 11) bits per pass, reduce-then-scan per pass
// (digit counts per partition, their scan per digit, then a ranking scatter;
// Merrill & Grimshaw's structure with wave-ballot multisplit ranking).
// Ping-pongs between (k0, v0) and (k1, v1); returns through *result_in_1
// whether the sorted data ended in the second buffer.  n = min(*n_dev,
// n_max).
bool radix_bits_ok(int radix_bits);
size_t sort_tmp_bytes(int64_t n_max, int key_bits, int radix_bits);
// gather_src/gather_dst (both or neither): the last pass also writes
// gather_dst[i] = gather_src[value i] in sorted order (a per-value word
// carried into the sorted order without a pass of its own).  iota: the
// values are the items' input positions, not read from v0 (v0 is still the
// buffer of the even passes' output).
hipError_t radix_sort_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                          const uint32_t* n_dev, int64_t n_max, int key_bits, int radix_bits,
                          void* tmp, int32_t* status, hipStream_t st, bool* result_in_1,
                          const uint32_t* gather_src = nullptr, uint32_t* gather_dst = nullptr,
                          bool iota = false);
hipError_t radix_sort_u64(uint32_t* k0, uint64_t* v0, uint32_t* k1, uint64_t* v1,
                          const uint32_t* n_dev, int64_t n_max, int key_bits, int radix_bits,
                          void* tmp, int32_t* status, hipStream_t st, bool* result_in_1);
// After a sort, the key count of each digit value of its last pass
// (uint32 [2^radix_bits], device): for a one-pass sort, the run length of
// every key.
const uint32_t* radix_sort_digit_totals(const void* tmp);

// Stage timing: the caller's HIP events recorded around a stage's kernels
// (a plan's trace table, vrs_plan_trace); null: no timing.
constexpr int kTraceStages = 16;
struct Trace {
  hipEvent_t start[kTraceStages], stop[kTraceStages];
};
inline void trace_begin(const Trace* tr, int stage, hipStream_t st) {
  if (tr && tr->start[stage]) (void)hipEventRecord(tr->start[stage], st);
}
inline void trace_end(const Trace* tr, int stage, hipStream_t st) {
  if (tr && tr->stop[stage]) (void)hipEventRecord(tr->stop[stage], st);
}

// Stage entry points as the frame runtime calls them (the extern "C"
// entries call these with no trace table and, for the periphery, with the
// adjoint's and work-count outputs on).
constexpr int kRenderStats = 1;
vrs_status render_impl(const float* mean, const float* cov, const float* opacity,
                       const float* sh, int sh_degree, int64_t n, const vrs_view* views,
                       int n_views, const vrs_raster_opts* opts, float* rgb, float* depth,
                       float* t_final, int32_t* n_contrib, void* ws, size_t ws_bytes,
                       int64_t max_pairs, int32_t* dev_status, void* stream, int flags,
                       const Trace* tr);
vrs_status splat_impl(const float* pos, const float* radius, const uint16_t* feat,
                      const float* opacity, int64_t np, int channels, int levels,
                      const vrs_view* views, int n_views, const vrs_crop* crops, int n_crops,
                      const vrs_crop_place* place, const float* depth, const float* t_final,
                      float cov_min, float slack, const uint32_t* point_ids, float* pyramid,
                      void* ws, size_t ws_bytes, int64_t max_frags, int32_t* dev_status,
                      void* stream, const Trace* tr, const float* gaze = nullptr);
vrs_status decode_impl_entry(const float* pyramid, int levels, const float* rgb_periphery,
                             const vrs_view* views, int n_views, const vrs_crop* crops,
                             int n_crops, const vrs_crop_place* place, const float* weights,
                             const vrs_decoder_desc* dd, float* fovea_rgb, void* ws,
                             size_t ws_bytes, void* stream, const Trace* tr);
vrs_status composite_impl(const float* rgb_periphery, int n_views, int width, int height,
                          const float* fovea_rgb, const vrs_crop* crops, int n_crops,
                          const vrs_crop_place* place, int mode, float ring, float m, float gamma,
                          float* out, void* stream, const Trace* tr);

// Fill n words with a value (graph-safe replacement for memset).
hipError_t fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t st);

}  // namespace vrs
