// Device-wide primitives written for gfx950 wave64: fill, single-pass
// exclusive scan with decoupled look-back, and an onesweep LSD radix sort
// with wave-level multisplit ranking in LDS.
//
// Forward progress: scan partitions and sort partitions take their index
// from an atomic counter in launch order, so every predecessor a block waits
// on has already started.  Every wait is bounded (kSpinLimit polls); on
// expiry the kernel records VRS_ETIMEOUT in the status word and proceeds, so
// every wave always exits.
#include "vrs_common.h"

namespace vrs {
namespace {

constexpr int kSpinLimit = 1 << 22;

__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of m at lanes below this lane
__device__ inline uint32_t count_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t ld_agent64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  return x;
}

__global__ void k_fill(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ------------------------------------------------------------------ scan
constexpr int kScanBlock = 256, kScanItems = 8, kScanTile = kScanBlock * kScanItems;
constexpr uint64_t kFlagAgg = 1ull << 32, kFlagPre = 2ull << 32;

__global__ void k_scan_clear(uint32_t* counter, uint64_t* flags, const uint32_t* n_dev,
                             int64_t n_max) {
  int64_t n = n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)n_max) : n_max;
  int64_t parts = (n + kScanTile - 1) / kScanTile;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) *counter = 0;
  for (; i < parts; i += (int64_t)gridDim.x * blockDim.x) flags[i] = 0;
}

__global__ __launch_bounds__(kScanBlock) void k_scan(const uint32_t* __restrict__ in,
                                                      const uint32_t* __restrict__ idx,
                                                      uint32_t* __restrict__ out,
                                                      uint32_t* total, const uint32_t* n_dev,
                                                      int64_t n_max, uint32_t* counter,
                                                      uint64_t* flags, int32_t* status,
                                                      int flags_mode) {
  __shared__ uint32_t s_part, s_prefix;
  __shared__ uint32_t s_wsum[kScanBlock / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_part = atomicAdd(counter, 1u);
  __syncthreads();
  const int64_t part = s_part;
  const int64_t n = n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)n_max) : n_max;
  const int64_t base = part * kScanTile;
  if (base >= n) return;
  uint32_t v[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + (int64_t)tid * kScanItems + j;
    uint32_t x = 0;
    if (i < n) x = idx ? in[idx[i]] : in[i];
    if (flags_mode) x = x != 0u;
    v[j] = sum;
    sum += x;
  }
  uint32_t incl = wave_incl_scan(sum);
  if (lane == 63) s_wsum[wave] = incl;
  __syncthreads();
  uint32_t woff = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < kScanBlock / 64; ++w) {
    if (w < wave) woff += s_wsum[w];
    btot += s_wsum[w];
  }
  if (tid == 0) {
    uint32_t excl = 0;
    if (part == 0) {
      st_agent64(&flags[0], kFlagPre | btot);
    } else {
      st_agent64(&flags[part], kFlagAgg | btot);
      int64_t p = part - 1;
      int spins = 0;
      while (p >= 0) {
        uint64_t w = ld_agent64(&flags[p]);
        if ((w >> 32) == 0) {
          if (++spins > kSpinLimit) { set_status(status, VRS_ETIMEOUT); break; }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += (uint32_t)w;
        if ((w & kFlagPre) != 0) break;
        --p;
      }
      st_agent64(&flags[part], kFlagPre | (uint64_t)(excl + btot));
    }
    s_prefix = excl;
    if (total && base + kScanTile >= n) *total = excl + btot;
  }
  __syncthreads();
  const uint32_t off = s_prefix + woff + (incl - sum);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + (int64_t)tid * kScanItems + j;
    if (i < n) out[i] = off + v[j];
  }
}

// ------------------------------------------------------------------ sort
constexpr int kSortBlock = 256, kSortWaves = kSortBlock / 64, kSortItems = 15;
constexpr int kWaveChunk = 64 * kSortItems, kSortTile = kSortBlock * kSortItems;  // 3840
constexpr uint32_t kLbAgg = 1u << 30, kLbPre = 2u << 30, kLbVal = (1u << 30) - 1;

__global__ void k_sort_clear(uint32_t* hist, int passes, uint32_t* lookback, int64_t parts_max,
                             const uint32_t* n_dev, int64_t n_max) {
  int64_t n = n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)n_max) : n_max;
  int64_t parts = (n + kSortTile - 1) / kSortTile;
  int64_t per = parts * 256;
  int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < passes * 256 + passes; i += stride) hist[i] = 0;  // hist + counters
  for (int p = 0; p < passes; ++p)
    for (int64_t i = i0; i < per; i += stride) lookback[p * parts_max * 256 + i] = 0;
}

__global__ __launch_bounds__(256) void k_sort_hist(const uint32_t* __restrict__ keys,
                                                    const uint32_t* n_dev, int64_t n_max,
                                                    int passes, uint32_t* hist) {
  __shared__ uint32_t s_h[4][256];
  const int tid = threadIdx.x;
  for (int p = 0; p < 4; ++p) s_h[p][tid] = 0;
  __syncthreads();
  const int64_t n = n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)n_max) : n_max;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + tid; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t k = keys[i];
    for (int p = 0; p < passes; ++p) atomicAdd(&s_h[p][(k >> (8 * p)) & 255u], 1u);
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p)
    if (s_h[p][tid]) atomicAdd(&hist[p * 256 + tid], s_h[p][tid]);
}

template <typename V>
__global__ __launch_bounds__(kSortBlock) void k_onesweep(
    const uint32_t* __restrict__ kin, const V* __restrict__ vin, uint32_t* __restrict__ kout,
    V* __restrict__ vout, const uint32_t* n_dev, int64_t n_max, int pass,
    const uint32_t* __restrict__ hist, uint32_t* counters, uint32_t* lookback, int32_t* status) {
  __shared__ uint32_t s_part;
  __shared__ uint32_t s_wh[kSortWaves][256];
  __shared__ uint32_t s_lstart[256], s_gstart[256], s_scan[kSortWaves];
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ V s_vals[kSortTile];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int shift = 8 * pass;
  if (tid == 0) s_part = atomicAdd(&counters[pass], 1u);
#pragma unroll
  for (int w = 0; w < kSortWaves; ++w) s_wh[w][tid] = 0;
  __syncthreads();
  const int64_t part = s_part;
  const int64_t n = n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)n_max) : n_max;
  const int64_t base = part * kSortTile;
  if (base >= n) return;

  // load: wave w owns [base + w*960, +960); item j of lane l at j*64 + l
  uint32_t key[kSortItems];
  V val[kSortItems];
  uint32_t rank[kSortItems];
  const int64_t wbase = base + (int64_t)wave * kWaveChunk;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    int64_t i = wbase + j * 64 + lane;
    bool ok = i < n;
    key[j] = ok ? kin[i] : 0xffffffffu;
    val[j] = ok ? vin[i] : V(0);
  }
  // stable rank within the wave: match lanes with equal digit by ballots
  volatile uint32_t* wh = s_wh[wave];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const bool ok = wbase + j * 64 + lane < n;
    const uint32_t d = (key[j] >> shift) & 255u;
    uint64_t m = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t below = count_below(m);
    const uint32_t prev = wh[d];
    rank[j] = prev + below;
    __builtin_amdgcn_wave_barrier();
    if (ok && below == 0) wh[d] = prev + (uint32_t)__popcll(m);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit: exclusive prefix over waves, block count
  const uint32_t d = tid;
  uint32_t cnt = 0;
#pragma unroll
  for (int w = 0; w < kSortWaves; ++w) {
    uint32_t c = s_wh[w][d];
    s_wh[w][d] = cnt;
    cnt += c;
  }
  // publish this partition's aggregate for digit d
  uint32_t* lb = lookback + (int64_t)pass * ((n_max + kSortTile - 1) / kSortTile) * 256;
  if (part == 0) st_agent(&lb[d], kLbPre | cnt);
  else st_agent(&lb[part * 256 + d], kLbAgg | cnt);
  // block-wide exclusive scan of counts over digits -> local start
  uint32_t incl = wave_incl_scan(cnt);
  if (lane == 63) s_scan[wave] = incl;
  // global digit offsets from the histogram of this pass
  uint32_t h = hist[pass * 256 + d];
  uint32_t hincl = wave_incl_scan(h);
  __syncthreads();
  uint32_t woff = 0;
  for (int w = 0; w < wave; ++w) woff += s_scan[w];
  s_lstart[d] = woff + incl - cnt;
  __syncthreads();
  if (lane == 63) s_scan[wave] = hincl;
  __syncthreads();
  uint32_t hoff = 0;
  for (int w = 0; w < wave; ++w) hoff += s_scan[w];
  const uint32_t gdig = hoff + hincl - h;
  // decoupled look-back for digit d
  uint32_t excl = 0;
  if (part > 0) {
    int64_t p = part - 1;
    int spins = 0;
    while (p >= 0) {
      uint32_t w = ld_agent(&lb[p * 256 + d]);
      if ((w & (kLbAgg | kLbPre)) == 0) {
        if (++spins > kSpinLimit) { set_status(status, VRS_ETIMEOUT); break; }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += w & kLbVal;
      if (w & kLbPre) break;
      --p;
    }
    st_agent(&lb[part * 256 + d], kLbPre | (excl + cnt));
  }
  s_gstart[d] = gdig + excl;
  __syncthreads();
  // scatter into LDS in block-sorted order
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    if (wbase + j * 64 + lane < n) {
      const uint32_t dj = (key[j] >> shift) & 255u;
      const uint32_t lpos = s_lstart[dj] + s_wh[wave][dj] + rank[j];
      s_keys[lpos] = key[j];
      s_vals[lpos] = val[j];
    }
  }
  __syncthreads();
  const int cnt_tile = (int)min((int64_t)kSortTile, n - base);
  for (int i = tid; i < cnt_tile; i += kSortBlock) {
    const uint32_t k = s_keys[i];
    const uint32_t dk = (k >> shift) & 255u;
    const uint32_t g = s_gstart[dk] + (uint32_t)i - s_lstart[dk];
    kout[g] = k;
    vout[g] = s_vals[i];
  }
}

template <typename V>
hipError_t radix_sort_impl(uint32_t* k0, V* v0, uint32_t* k1, V* v1, const uint32_t* n_dev,
                           int64_t n_max, int key_bits, void* tmp, int32_t* status,
                           hipStream_t st, bool* result_in_1) {
  const int passes = key_bits <= 0 ? 0 : (key_bits + 7) / 8;
  *result_in_1 = (passes & 1) != 0;
  if (passes == 0 || n_max == 0) return hipSuccess;
  const int64_t parts = (n_max + kSortTile - 1) / kSortTile;
  uint32_t* hist = static_cast<uint32_t*>(tmp);
  uint32_t* counters = hist + passes * 256;
  uint32_t* lookback = hist + ((passes * 256 + passes + 63) / 64) * 64;
  int clear_blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (parts * 256 + 255) / 256));
  hipLaunchKernelGGL(k_sort_clear, dim3(clear_blocks), dim3(256), 0, st, hist, passes, lookback,
                     parts, n_dev, n_max);
  int hist_blocks = (int)std::min<int64_t>(2048, std::max<int64_t>(1, (n_max + 4095) / 4096));
  hipLaunchKernelGGL(k_sort_hist, dim3(hist_blocks), dim3(256), 0, st, k0, n_dev, n_max, passes,
                     hist);
  uint32_t* kb[2] = {k0, k1};
  V* vb[2] = {v0, v1};
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(k_onesweep<V>, dim3((unsigned)parts), dim3(kSortBlock), 0, st, kb[p & 1],
                       vb[p & 1], kb[(p + 1) & 1], vb[(p + 1) & 1], n_dev, n_max, p, hist,
                       counters, lookback, status);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, st, p, value, n);
  return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t n_max) {
  int64_t parts = (n_max + kScanTile - 1) / kScanTile;
  return 256 + (size_t)std::max<int64_t>(parts, 1) * 8;
}

static hipError_t scan_impl(const uint32_t* in, const uint32_t* idx, uint32_t* out,
                            uint32_t* total, const uint32_t* n_dev, int64_t n_max, void* tmp,
                            int32_t* status, hipStream_t st, int flags_mode) {
  if (n_max <= 0) {
    if (total) return fill_u32(total, 0, 1, st);
    return hipSuccess;
  }
  uint32_t* counter = static_cast<uint32_t*>(tmp);
  uint64_t* flags = reinterpret_cast<uint64_t*>(static_cast<char*>(tmp) + 256);
  int64_t parts = (n_max + kScanTile - 1) / kScanTile;
  int cb = (int)std::min<int64_t>(1024, (parts + 255) / 256 + 1);
  hipLaunchKernelGGL(k_scan_clear, dim3(cb), dim3(256), 0, st, counter, flags, n_dev, n_max);
  if (total) {
    // n may turn out to be 0 on the device: start from a defined total
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, total, 0u, (int64_t)1);
  }
  hipLaunchKernelGGL(k_scan, dim3((unsigned)parts), dim3(kScanBlock), 0, st, in, idx, out, total,
                     n_dev, n_max, counter, flags, status, flags_mode);
  return hipGetLastError();
}

hipError_t exclusive_scan_u32(const uint32_t* in, const uint32_t* idx, uint32_t* out,
                              uint32_t* total, const uint32_t* n_dev, int64_t n_max, void* tmp,
                              int32_t* status, hipStream_t st) {
  return scan_impl(in, idx, out, total, n_dev, n_max, tmp, status, st, 0);
}

hipError_t exclusive_scan_flags_u32(const uint32_t* in, uint32_t* out, uint32_t* total,
                                    int64_t n, void* tmp, int32_t* status, hipStream_t st) {
  return scan_impl(in, nullptr, out, total, nullptr, n, tmp, status, st, 1);
}

size_t sort_tmp_bytes(int64_t n_max, int key_bits) {
  const int passes = std::max(1, (key_bits + 7) / 8);
  const int64_t parts = std::max<int64_t>(1, (n_max + kSortTile - 1) / kSortTile);
  size_t head = ((passes * 256 + passes + 63) / 64) * 64 * 4;
  return head + (size_t)passes * parts * 256 * 4;
}

hipError_t radix_sort_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                          const uint32_t* n_dev, int64_t n_max, int key_bits, void* tmp,
                          int32_t* status, hipStream_t st, bool* result_in_1) {
  return radix_sort_impl<uint32_t>(k0, v0, k1, v1, n_dev, n_max, key_bits, tmp, status, st,
                                   result_in_1);
}

hipError_t radix_sort_u64(uint32_t* k0, uint64_t* v0, uint32_t* k1, uint64_t* v1,
                          const uint32_t* n_dev, int64_t n_max, int key_bits, void* tmp,
                          int32_t* status, hipStream_t st, bool* result_in_1) {
  return radix_sort_impl<uint64_t>(k0, v0, k1, v1, n_dev, n_max, key_bits, tmp, status, st,
                                   result_in_1);
}

}  // namespace vrs
