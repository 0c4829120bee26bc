// Decoupled look-back (Merrill & Garland, "Single-pass Parallel Prefix Scan
// with Decoupled Look-back", 2016) run by one whole wave.
//
// Each partition owns a 64-bit status word: flag in the high half (0 = not
// yet published, kLbFlagAgg = block aggregate, kLbFlagPre = inclusive
// prefix), value in the low half, so flag and value are read together.  A
// round reads the 64 predecessors of a window in one load per lane, waits
// until every word of the window is published, and stops at the nearest
// predecessor that holds an inclusive prefix; otherwise it adds the 64
// aggregates and moves the window down.  Partition ids must come from an
// atomic counter in launch order so that every predecessor has started;
// every wait is bounded and records VRS_ETIMEOUT on expiry, after which
// unpublished words count as zero so the wave always finishes.
#pragma once
#include "vrs_common.h"

namespace vrs {

constexpr uint64_t kLbFlagAgg = 1ull << 32, kLbFlagPre = 2ull << 32;
constexpr int kLbSpinLimit = 1 << 22;

__device__ inline uint64_t lb_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void lb_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Publishes `agg` as partition `part`'s aggregate, finds the exclusive
// prefix, publishes the inclusive prefix.  Called by all 64 lanes of one
// wave with the same arguments; returns the exclusive prefix in every lane.
__device__ inline uint32_t wave_lookback(uint64_t* flags, int64_t part, uint32_t agg,
                                         int32_t* status) {
  const int lane = threadIdx.x & 63;
  if (part == 0) {
    if (lane == 0) lb_store(&flags[0], kLbFlagPre | agg);
    return 0;
  }
  if (lane == 0) lb_store(&flags[part], kLbFlagAgg | agg);
  uint32_t excl = 0;
  int64_t top = part;   // window [top - 64, top)
  int spins = 0;
  while (true) {
    const int64_t p = top - 64 + lane;
    uint64_t w = p >= 0 ? lb_load(&flags[p]) : kLbFlagPre;
    while (__ballot((w >> 32) == 0) != 0) {
      if (++spins > kLbSpinLimit) {
        if (lane == 0) set_status(status, VRS_ETIMEOUT);
        if ((w >> 32) == 0) w = kLbFlagPre;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      if ((w >> 32) == 0) w = lb_load(&flags[p]);
    }
    const uint64_t pre = __ballot((w & kLbFlagPre) != 0);
    if (pre != 0) {
      const int hi = 63 - __builtin_clzll(pre);
      excl += wave_sum_u32(lane >= hi ? (uint32_t)w : 0u);
      break;
    }
    excl += wave_sum_u32((uint32_t)w);
    top -= 64;
  }
  if (lane == 0) lb_store(&flags[part], kLbFlagPre | (uint64_t)(excl + agg));
  return excl;
}

}  // namespace vrs
