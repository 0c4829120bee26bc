// Device-wide primitives written for gfx950 wave64: fill, single-pass
// exclusive scan with a wave-parallel decoupled look-back, and a
// reduce-then-scan LSD radix sort with wave-level multisplit ranking in LDS.
//
// Forward progress: scan partitions take their index from an atomic counter
// in launch order, so every predecessor a workgroup waits on has already
// started; every wait is bounded and records VRS_ETIMEOUT on expiry, so every
// wave always exits.  The sort never waits on another workgroup.
#include "lookback.h"

namespace vrs {
namespace {


__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of m at lanes below this lane
__device__ inline uint32_t count_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
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
// Partition shapes: direct reads of 2M items or more take 16K-item
// partitions (1024 threads x 16 items: fewer partitions, so fewer ticket
// atomics and look-back rounds); gathered reads (in[idx[i]]) and smaller
// scans take 4K-item partitions (512 x 8), where more workgroups keep more
// reads in flight.  Temporaries are sized for the smaller one.
constexpr int kScanTileMin = 4096;

// Clears the partition counter, the look-back flags the scan will use and
// the total (n may turn out to be 0 on the device: the total is then 0).
__global__ void k_scan_clear(uint32_t* counter, uint64_t* flags, uint32_t* total,
                             const uint32_t* n_dev, int64_t n_max) {
  int64_t n = n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)n_max) : n_max;
  int64_t parts = (n + kScanTileMin - 1) / kScanTileMin;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) {
    *counter = 0;
    if (total) *total = 0;
  }
  for (; i < parts; i += (int64_t)gridDim.x * blockDim.x) flags[i] = 0;
}

// Thread t of a partition owns kScanItems consecutive items of it; when the
// input is read directly (no index) and 16-byte aligned, they come in as
// 16-byte loads.
template <int kScanBlock, int kScanItems>
__global__ __launch_bounds__(kScanBlock) void k_scan(const uint32_t* __restrict__ in,
                                                      const uint32_t* __restrict__ idx,
                                                      uint32_t* __restrict__ out,
                                                      uint32_t* total, const uint32_t* n_dev,
                                                      int64_t n_max, uint32_t* counter,
                                                      uint64_t* flags, int32_t* status) {
  __shared__ uint32_t s_part, s_prefix;
  constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanItems;
  static_assert(kScanTile >= kScanTileMin && kScanItems % 4 == 0, "partition shape");
  __shared__ uint32_t s_wsum[kScanBlock / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // the grid is sized for n_max; blocks beyond the partitions n needs leave
  // before taking a partition id, so exactly those take ids 0..parts-1
  const int64_t n = n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)n_max) : n_max;
  if ((int64_t)blockIdx.x * kScanTile >= n) {
    if (n == 0 && blockIdx.x == 0 && tid == 0 && total) *total = 0;
    return;
  }
  if (tid == 0) s_part = atomicAdd(counter, 1u);
  __syncthreads();
  const int64_t part = s_part;
  const int64_t base = part * kScanTile;
  const int64_t i0 = base + (int64_t)tid * kScanItems;
  uint32_t x[kScanItems];
  if (!idx && i0 + kScanItems <= n && (reinterpret_cast<uintptr_t>(in) & 15) == 0) {
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
      const uint4 a = *reinterpret_cast<const uint4*>(in + i0 + 4 * q);
      x[4 * q] = a.x; x[4 * q + 1] = a.y; x[4 * q + 2] = a.z; x[4 * q + 3] = a.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int64_t i = i0 + j;
      x[j] = i < n ? (idx ? in[idx[i]] : in[i]) : 0u;
    }
  }
  uint32_t v[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = sum;
    sum += x[j];
  }
  const uint32_t incl = wave_incl_scan(sum);
  if (lane == 63) s_wsum[wave] = incl;
  __syncthreads();
  uint32_t woff = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < kScanBlock / 64; ++w) {
    if (w < wave) woff += s_wsum[w];
    btot += s_wsum[w];
  }
  if (wave == 0) {
    const uint32_t excl = wave_lookback(flags, part, btot, status);
    if (lane == 0) {
      s_prefix = excl;
      if (total && base + kScanTile >= n) *total = excl + btot;
    }
  }
  __syncthreads();
  const uint32_t off = s_prefix + woff + (incl - sum);
  if (i0 + kScanItems <= n && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q)
      *reinterpret_cast<uint4*>(out + i0 + 4 * q) =
          make_uint4(off + v[4 * q], off + v[4 * q + 1], off + v[4 * q + 2], off + v[4 * q + 3]);
  } else {
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
      if (i0 + j < n) out[i0 + j] = off + v[j];
  }
}

// ------------------------------------------------------------------ sort
// LSD radix sort, R bits per pass (R = 4, 6, 8 or 11: the digit width is
// tuned per workload; fewer wider passes move the data fewer times, narrower
// digits keep the per-partition histograms small), reduce-then-scan: per
// pass an upsweep counts each partition's digits, one workgroup per digit
// scans those counts over partitions, and the downsweep ranks its partition
// in LDS and writes every item straight to its final position.  No
// inter-workgroup waiting anywhere; deterministic.
constexpr int kSortBlock = 256, kSortWaves = kSortBlock / 64, kSortItems = 8;
constexpr int kWaveChunk = 64 * kSortItems, kSortTile = kSortBlock * kSortItems;  // 2048
constexpr int64_t kSortGrid = 1024;

__device__ inline int64_t sort_n(const uint32_t* n_dev, int64_t n_max) {
  return n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)n_max) : n_max;
}

// Upsweep: digit counts of a partition, stored digit-major (counts[d * parts
// + p]).  Keys often come in runs (pairs of one Gaussian, pixels of one
// point): where all active lanes hold the same digit the wave adds once.
// Workgroups take partitions in grid-stride order: the grid is sized for at
// most kSortGrid workgroups whatever the capacity, the count is read on the
// device.
template <int R>
__global__ __launch_bounds__(kSortBlock) void k_sort_count(const uint32_t* __restrict__ keys,
                                                            const uint32_t* n_dev, int64_t n_max,
                                                            int shift, int64_t parts,
                                                            uint32_t* __restrict__ counts) {
  constexpr int NB = 1 << R;
  constexpr uint32_t MASK = NB - 1;
  __shared__ uint32_t s_h[NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = sort_n(n_dev, n_max);
  for (int64_t part = blockIdx.x; part * kSortTile < n; part += gridDim.x) {
    const int64_t base = part * kSortTile;
    for (int d = tid; d < NB; d += kSortBlock) s_h[d] = 0;
    __syncthreads();
    const int64_t wbase = base + (int64_t)wave * kWaveChunk;
    uint32_t kv[kSortItems];   // every load in flight before the first atomic
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int64_t i = wbase + j * 64 + lane;
      kv[j] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int64_t i = wbase + j * 64 + lane;
      if (i < n) {
        const uint32_t d = (kv[j] >> shift) & MASK;
        const uint64_t act = __ballot(true);
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        if (__ballot(d != d0) == 0) {
          if (count_below(act) == 0) atomicAdd(&s_h[d0], (uint32_t)__popcll(act));
        } else {
          atomicAdd(&s_h[d], 1u);
        }
      }
    }
    __syncthreads();
    for (int d = tid; d < NB; d += kSortBlock) counts[(int64_t)d * parts + part] = s_h[d];
    __syncthreads();   // s_h is cleared for the next partition
  }
}

// One workgroup per digit: exclusive scan of the digit's counts over the
// partitions n needs (in place), the digit total to totals[d].
__global__ __launch_bounds__(256) void k_sort_scan(uint32_t* counts, const uint32_t* n_dev,
                                                   int64_t n_max, int64_t parts,
                                                   uint32_t* __restrict__ totals) {
  __shared__ uint32_t s_w[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = sort_n(n_dev, n_max);
  const int64_t used = (n + kSortTile - 1) / kSortTile;
  uint32_t* c = counts + (int64_t)blockIdx.x * parts;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < used; b0 += 256 * 4) {
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = b0 + tid * 4 + j;
      const uint32_t x = i < used ? c[i] : 0u;
      v[j] = sum;
      sum += x;
    }
    const uint32_t incl = wave_incl_scan(sum);
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t woff = 0, btot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if (w < wave) woff += s_w[w];
      btot += s_w[w];
    }
    const uint32_t off = carry + woff + incl - sum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = b0 + tid * 4 + j;
      if (i < used) c[i] = off + v[j];
    }
    carry += btot;
    __syncthreads();   // s_w is rewritten by the next chunk
  }
  if (tid == 0) totals[blockIdx.x] = carry;
}

// Exclusive scan over the NB digits of a workgroup: thread t owns digits
// [t DPT, t DPT + DPT) (DPT = NB / 256, or one digit for t < NB when NB is
// smaller); x[j] is digit t DPT + j's value, replaced by its exclusive prefix.
template <int NB>
__device__ inline void block_digit_scan(uint32_t* x, uint32_t* s_scan) {
  constexpr int DPT = NB >= kSortBlock ? NB / kSortBlock : 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const uint32_t v = x[j];
    x[j] = sum;
    sum += v;
  }
  const uint32_t incl = wave_incl_scan(sum);
  if (lane == 63) s_scan[wave] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (int w = 0; w < wave; ++w) woff += s_scan[w];
  __syncthreads();   // s_scan is reused by the caller's next scan
#pragma unroll
  for (int j = 0; j < DPT; ++j) x[j] += woff + incl - sum;
}

// Downsweep of a partition (grid-stride order, as the upsweep): stable rank of every item among the
// partition's items of the same digit (wave ballots, then waves in order),
// items regrouped by digit in LDS, then written to
//   base(digit) + count of the digit in earlier partitions + local rank,
// with base(digit) the exclusive scan of the digit totals.
template <typename V, int R>
__global__ __launch_bounds__(kSortBlock) void k_sort_scatter(
    const uint32_t* __restrict__ kin, const V* __restrict__ vin, uint32_t* __restrict__ kout,
    V* __restrict__ vout, const uint32_t* n_dev, int64_t n_max, int shift, int64_t parts,
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ totals,
    const uint32_t* __restrict__ gsrc, uint32_t* __restrict__ gdst) {
  constexpr int NB = 1 << R;
  constexpr uint32_t MASK = NB - 1;
  constexpr int DPT = NB >= kSortBlock ? NB / kSortBlock : 1;
  __shared__ uint32_t s_wh[kSortWaves][NB];
  __shared__ uint32_t s_lstart[NB], s_gstart[NB], s_scan[kSortWaves];
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ V s_vals[kSortTile];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = sort_n(n_dev, n_max);
  for (int64_t part = blockIdx.x; part * kSortTile < n; part += gridDim.x) {
    const int64_t base = part * kSortTile;
    for (int d = tid; d < NB; d += kSortBlock)
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) s_wh[w][d] = 0;
    __syncthreads();
    // load: wave w owns [base + w*512, +512); item j of lane l at j*64 + l
    uint32_t key[kSortItems];
    V val[kSortItems];
    uint32_t rank[kSortItems];
    const int64_t wbase = base + (int64_t)wave * kWaveChunk;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int64_t i = wbase + j * 64 + lane;
      const bool ok = i < n;
      key[j] = ok ? kin[i] : 0xffffffffu;
      // no input values: each item's value is its input position
      val[j] = ok ? (vin ? vin[i] : (V)i) : V(0);
    }
    // stable rank within the wave: match lanes with equal digit by ballots
    volatile uint32_t* wh = s_wh[wave];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const bool ok = wbase + j * 64 + lane < n;
      const uint32_t d = (key[j] >> shift) & MASK;
      uint64_t m = __ballot(ok);
#pragma unroll
      for (int b = 0; b < R; ++b) {
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
    // per digit: exclusive prefix over waves and the partition's count; the
    // local start of each digit (scan of those counts) and its global base
    // (scan of the digit totals plus the earlier partitions' count)
    uint32_t cnt[DPT], glob[DPT];
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = tid * DPT + j;
      uint32_t c = 0;
      if (d < NB) {
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
          const uint32_t x = s_wh[w][d];
          s_wh[w][d] = c;
          c += x;
        }
      }
      cnt[j] = c;
      glob[j] = d < NB ? totals[d] : 0u;
    }
    block_digit_scan<NB>(cnt, s_scan);
    block_digit_scan<NB>(glob, s_scan);
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = tid * DPT + j;
      if (d < NB) {
        s_lstart[d] = cnt[j];
        s_gstart[d] = glob[j] + counts[(int64_t)d * parts + part];
      }
    }
    __syncthreads();
    // regroup by digit in LDS, then coalesced runs to the output
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      if (wbase + j * 64 + lane < n) {
        const uint32_t dj = (key[j] >> shift) & MASK;
        const uint32_t lpos = s_lstart[dj] + s_wh[wave][dj] + rank[j];
        s_keys[lpos] = key[j];
        s_vals[lpos] = val[j];
      }
    }
    __syncthreads();
    const int cnt_tile = (int)min((int64_t)kSortTile, n - base);
    for (int i = tid; i < cnt_tile; i += kSortBlock) {
      const uint32_t k = s_keys[i];
      const uint32_t dk = (k >> shift) & MASK;
      const uint32_t g = s_gstart[dk] + (uint32_t)i - s_lstart[dk];
      kout[g] = k;
      vout[g] = s_vals[i];
      if (gdst) gdst[g] = gsrc[(uint64_t)s_vals[i]];   // last pass: gather in sorted order
    }
    __syncthreads();   // LDS is rewritten by the next partition
  }
}

template <typename V, int R>
hipError_t radix_sort_r(uint32_t* k0, V* v0, uint32_t* k1, V* v1, const uint32_t* n_dev,
                        int64_t n_max, int key_bits, void* tmp, hipStream_t st,
                        bool* result_in_1, const uint32_t* gather_src, uint32_t* gather_dst,
                        bool iota) {
  constexpr int NB = 1 << R;
  const int passes = key_bits <= 0 ? 0 : (key_bits + R - 1) / R;
  *result_in_1 = (passes & 1) != 0;
  if (passes == 0 || n_max == 0) return hipSuccess;
  const int64_t parts = (n_max + kSortTile - 1) / kSortTile;
  const unsigned grid = (unsigned)std::min<int64_t>(parts, kSortGrid);
  uint32_t* totals = static_cast<uint32_t*>(tmp);
  uint32_t* counts = totals + NB;
  uint32_t* kb[2] = {k0, k1};
  V* vb[2] = {v0, v1};
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(k_sort_count<R>, dim3(grid), dim3(kSortBlock), 0, st, kb[p & 1],
                       n_dev, n_max, R * p, parts, counts);
    hipLaunchKernelGGL(k_sort_scan, dim3(NB), dim3(256), 0, st, counts, n_dev, n_max, parts,
                       totals);
    const bool last = p == passes - 1;
    hipLaunchKernelGGL((k_sort_scatter<V, R>), dim3(grid), dim3(kSortBlock), 0, st,
                       kb[p & 1], (p == 0 && iota) ? nullptr : vb[p & 1], kb[(p + 1) & 1],
                       vb[(p + 1) & 1], n_dev, n_max,
                       R * p, parts, counts, totals, last ? gather_src : nullptr,
                       last ? gather_dst : nullptr);
  }
  return hipGetLastError();
}

template <typename V>
hipError_t radix_sort_impl(uint32_t* k0, V* v0, uint32_t* k1, V* v1, const uint32_t* n_dev,
                           int64_t n_max, int key_bits, int radix_bits, void* tmp,
                           int32_t* status, hipStream_t st, bool* result_in_1,
                           const uint32_t* gather_src, uint32_t* gather_dst, bool iota) {
  (void)status;   // nothing in the sort waits on another workgroup
  switch (radix_bits) {
    case 4:
      return radix_sort_r<V, 4>(k0, v0, k1, v1, n_dev, n_max, key_bits, tmp, st, result_in_1,
                                gather_src, gather_dst, iota);
    case 6:
      return radix_sort_r<V, 6>(k0, v0, k1, v1, n_dev, n_max, key_bits, tmp, st, result_in_1,
                                gather_src, gather_dst, iota);
    case 11:
      return radix_sort_r<V, 11>(k0, v0, k1, v1, n_dev, n_max, key_bits, tmp, st, result_in_1,
                                 gather_src, gather_dst, iota);
    default:
      return radix_sort_r<V, 8>(k0, v0, k1, v1, n_dev, n_max, key_bits, tmp, st, result_in_1,
                                gather_src, gather_dst, iota);
  }
}

}  // namespace

hipError_t fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, st, p, value, n);
  return hipGetLastError();
}

int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int v = 0;
    cached[dev] = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) ==
                          hipSuccess && v > 0
                      ? v
                      : 256;
  }
  return cached[dev];
}

size_t scan_tmp_bytes(int64_t n_max) {
  int64_t parts = (n_max + kScanTileMin - 1) / kScanTileMin;
  return 256 + (size_t)std::max<int64_t>(parts, 1) * 8;
}

static hipError_t scan_impl(const uint32_t* in, const uint32_t* idx, uint32_t* out,
                            uint32_t* total, const uint32_t* n_dev, int64_t n_max, void* tmp,
                            int32_t* status, hipStream_t st, bool cleared) {
  if (n_max <= 0) {
    if (total) return fill_u32(total, 0, 1, st);
    return hipSuccess;
  }
  uint32_t* counter = static_cast<uint32_t*>(tmp);
  uint64_t* flags = reinterpret_cast<uint64_t*>(static_cast<char*>(tmp) + 256);
  // 4K-item partitions for gathers and below 2M items (more workgroups in
  // flight: a 1M-item scan has only 62 partitions of 16K), 16K above
  const bool small = idx || n_max < (int64_t(2) << 20);
  const int64_t tile = small ? 512 * 8 : 1024 * 16;
  const int64_t parts = (n_max + tile - 1) / tile;
  if (!cleared) {
    const int cb = (int)std::min<int64_t>(1024, (parts + 255) / 256 + 1);
    hipLaunchKernelGGL(k_scan_clear, dim3(cb), dim3(256), 0, st, counter, flags, total, n_dev,
                       n_max);
  }
  if (small)
    hipLaunchKernelGGL((k_scan<512, 8>), dim3((unsigned)parts), dim3(512), 0, st, in, idx, out,
                       total, n_dev, n_max, counter, flags, status);
  else
    hipLaunchKernelGGL((k_scan<1024, 16>), dim3((unsigned)parts), dim3(1024), 0, st, in, idx, out,
                       total, n_dev, n_max, counter, flags, status);
  return hipGetLastError();
}

hipError_t exclusive_scan_u32(const uint32_t* in, const uint32_t* idx, uint32_t* out,
                              uint32_t* total, const uint32_t* n_dev, int64_t n_max, void* tmp,
                              int32_t* status, hipStream_t st, bool cleared) {
  return scan_impl(in, idx, out, total, n_dev, n_max, tmp, status, st, cleared);
}

const uint32_t* radix_sort_digit_totals(const void* tmp) {
  return static_cast<const uint32_t*>(tmp);   // totals lead the temporary
}

bool radix_bits_ok(int radix_bits) {
  return radix_bits == 4 || radix_bits == 6 || radix_bits == 8 || radix_bits == 11;
}

size_t sort_tmp_bytes(int64_t n_max, int key_bits, int radix_bits) {
  (void)key_bits;   // one counts matrix, reused by every pass
  const int64_t parts = std::max<int64_t>(1, (n_max + kSortTile - 1) / kSortTile);
  const int64_t nb = int64_t(1) << (radix_bits_ok(radix_bits) ? radix_bits : 8);
  return (size_t)(nb + nb * parts) * 4;
}

hipError_t radix_sort_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                          const uint32_t* n_dev, int64_t n_max, int key_bits, int radix_bits,
                          void* tmp, int32_t* status, hipStream_t st, bool* result_in_1,
                          const uint32_t* gather_src, uint32_t* gather_dst, bool iota) {
  return radix_sort_impl<uint32_t>(k0, v0, k1, v1, n_dev, n_max, key_bits, radix_bits, tmp,
                                   status, st, result_in_1, gather_src, gather_dst, iota);
}

hipError_t radix_sort_u64(uint32_t* k0, uint64_t* v0, uint32_t* k1, uint64_t* v1,
                          const uint32_t* n_dev, int64_t n_max, int key_bits, int radix_bits,
                          void* tmp, int32_t* status, hipStream_t st, bool* result_in_1) {
  return radix_sort_impl<uint64_t>(k0, v0, k1, v1, n_dev, n_max, key_bits, radix_bits, tmp,
                                   status, st, result_in_1, nullptr, nullptr, false);
}

}  // namespace vrs
