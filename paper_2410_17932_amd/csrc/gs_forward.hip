// Peripheral 3D Gaussian splatting, forward (Sec. 3.2 of VR-Splatting: the
// full image P and the approximate depth of Eq. 1).
//
// Pipeline per call, all views in the same launches:
//   k_gs_preprocess   one thread per Gaussian, attributes read once for all
//                     views; EWA projection, SH colour, 48-byte record,
//                     depth key and super-tile count per (view, Gaussian);
//                     per-block totals of tile pairs
//   radix sort        (depth bits) of all (view, Gaussian) entries
//   scan              super-tile counts in depth order -> offsets (device)
//   k_gs_emit_super   output-parallel: one (super-tile, Gaussian) pair per
//                     8 x 8-tile super-tile a rectangle reaches, carrying
//                     the rectangle's part inside it; stores coalesce
//   radix sort        (super-tile id) of those pairs, stable: keeps depth
//                     order, and there are few of them (a Gaussian reaches
//                     far fewer super-tiles than tiles)
//   k_gs_runs         each super-tile's run [begin, end) in the sorted pairs
//   k_gs_units        runs cut into work units of 256 pairs (a scan), and
//                     the exact tile pair total
//   k_gs_bin_count    one wave per unit: per tile (tile = lane of an 8 x 8
//                     super-tile) the unit's pairs reaching it, from row
//                     and column ballots
//   k_gs_bin_prefix   per super-tile: prefix of those counts over its units,
//                     the tile totals and their length buckets; the last
//                     workgroup scans the super-tile totals (lists are laid
//                     out super-tile by super-tile) and the bucket counts
//   k_gs_schedule     one wave per super-tile: tile list offsets,
//                     [begin, end) per tile and the blend order, longest
//                     list first (counting sort by length bucket)
//   k_gs_bin_scatter  one wave per unit: every Gaussian index goes to its
//                     final place in each tile list it belongs to, its rank
//                     within a round from one ballot per tile
//   k_gs_blend        (gs_blend.hip) one workgroup per tile in that order,
//                     one wave per sub-tile; records staged in LDS in
//                     batches, front-to-back blend with per-wave and
//                     block-wide early exit
#include <type_traits>

#include "gs_layout.h"

namespace vrs {

// ------------------------------------------------------------ preprocess
// The SH degree is a template parameter, so the coefficient reads have no
// branches between them and are all in flight together.
template <int DEG>
__global__ __launch_bounds__(256) void k_gs_preprocess(
    const float* __restrict__ mean, const float* __restrict__ cov,
    const float* __restrict__ opacity, const float* __restrict__ sh, int64_t n,
    KViews views, GsOpt o, float4* __restrict__ rec, uint2* __restrict__ rect,
    uint32_t* __restrict__ dkey,
    uint32_t* __restrict__ nsup, uint64_t* __restrict__ psum,
    uint32_t* __restrict__ scan_clear, int64_t clear_words) {
  __shared__ uint64_t s_p[4];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  // the depth-order scan's temporary, zeroed here so that scan is one launch
  for (int64_t w = i; w < clear_words; w += (int64_t)gridDim.x * blockDim.x) scan_clear[w] = 0u;
  uint64_t pairs = 0;   // tiles reached, over the views
  if (i < n) {
    const float mx = mean[i], my = mean[n + i], mz = mean[2 * n + i];
    float S6[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) S6[k] = cov[k * n + i];
    const float op = opacity[i];
    constexpr int K = (DEG + 1) * (DEG + 1);
    float coef[16][3];
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k < K)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) coef[k][ch] = sh[(k * 3 + ch) * n + i];
    for (int v = 0; v < views.n; ++v) {
      const KView& cv = views.v[v];
      const int64_t e = v * n + i;
      Geom g;
      const bool ok = gs_geom32(cv, mx, my, mz, S6, o.lowpass, o.extent, g);
      if (!ok) {
        dkey[e] = 0xffffffffu;
        nsup[e] = 0;
        rec[3 * e + 0] = make_float4(0, 0, 0, 0);
        rec[3 * e + 1] = make_float4(0, 0, 0, 0);
        rec[3 * e + 2] = make_float4(0, 0, __uint_as_float(0xffffffffu), 0);
        rect[e] = make_uint2(0xffffffffu, 0u);
        continue;
      }
      const float inv = 1.0f / g.det;
      const float A = g.c * inv, B = -g.b * inv, C = g.a * inv;
      // view-dependent colour
      float dx = mx - cv.cam[0], dy = my - cv.cam[1], dz = mz - cv.cam[2];
      const float rn = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
      dx *= rn; dy *= rn; dz *= rn;
      float Y[16];
      sh_eval(DEG, dx, dy, dz, Y);
      float col[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.5f;
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k < K) acc += Y[k] * coef[k][ch];
        col[ch] = acc > 0.0f ? acc : 0.0f;
      }
      const int tile = o.tile;
      const int tx0 = g.x0 / tile, tx1 = g.x1 / tile, ty0 = g.y0 / tile, ty1 = g.y1 / tile;
      dkey[e] = __float_as_uint(g.t[2]);
      pairs += (uint64_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
      nsup[e] = (uint32_t)(((tx1 / kSuper) - (tx0 / kSuper) + 1) *
                           ((ty1 / kSuper) - (ty0 / kSuper) + 1));
      rec[3 * e + 0] = make_float4(g.px, g.py, A, B);
      rec[3 * e + 1] = make_float4(C, op, col[0], col[1]);
      rec[3 * e + 2] = make_float4(col[2], g.t[2], __uint_as_float(pack_xy(g.x0, g.y0)),
                                   __uint_as_float(pack_xy(g.x1, g.y1)));
      rect[e] = make_uint2(pack_xy(g.x0, g.y0), pack_xy(g.x1, g.y1));
    }
  }
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) pairs += __shfl_xor(pairs, s, 64);
  if ((threadIdx.x & 63) == 0) s_p[threadIdx.x >> 6] = pairs;
  __syncthreads();
  if (threadIdx.x == 0) psum[blockIdx.x] = s_p[0] + s_p[1] + s_p[2] + s_p[3];
}

// ------------------------------------------------------------------ emit
// Output-parallel emission of (super-tile, Gaussian) pairs.  A block owns
// 256 consecutive depth-ordered entries; their pair offsets and rectangles
// are staged in LDS, and each thread writes pairs p = first + tid, first +
// tid + 256, ... of the block's range, finding the owning entry (last i with
// off[i] <= p) by binary search in LDS.  Stores of consecutive p are
// consecutive, so they coalesce.  key = view * supers_per_view + super-tile;
// value = Gaussian index | (tile rectangle inside the super-tile, 3 bits per
// bound: x0, x1, y0, y1) << 32.
constexpr int kEmitBlock = 256;
__global__ __launch_bounds__(kEmitBlock) void k_gs_emit_super(
    const uint32_t* __restrict__ offs, const uint32_t* __restrict__ sorted_e,
    const uint2* __restrict__ rect, const uint32_t* __restrict__ total_p, int64_t vn,
    int64_t n, int64_t max_pairs, int tile, int64_t sxn, int64_t spv,
    uint32_t* __restrict__ skey, uint64_t* __restrict__ sval, int64_t st_total,
    uint2* __restrict__ srange, int32_t* status) {
  __shared__ uint32_t s_off[kEmitBlock + 1];
  __shared__ uint32_t s_base[kEmitBlock];   // key of the entry's first super-tile
  __shared__ uint32_t s_w[kEmitBlock];      // super-tiles per rectangle row
  __shared__ uint32_t s_id[kEmitBlock];
  __shared__ uint32_t s_lo[kEmitBlock], s_hi[kEmitBlock];   // tile rectangle (x | y << 16)
  const int tid = threadIdx.x;
  const int64_t total = *total_p;
  const int64_t cap = std::min<int64_t>(total, max_pairs);
  if (blockIdx.x == 0 && tid == 0 && total > max_pairs) set_status(status, VRS_ECAPACITY);
  // the run ranges are filled in after the sort; absent super-tiles keep (0, 0)
  for (int64_t i = blockIdx.x * (int64_t)kEmitBlock + tid; i < st_total;
       i += (int64_t)gridDim.x * kEmitBlock)
    srange[i] = make_uint2(0u, 0u);
  const int64_t j0 = (int64_t)blockIdx.x * kEmitBlock;
  const int64_t j = j0 + tid;
  if (j < vn) {
    s_off[tid] = offs[j];
    const uint32_t e = sorted_e[j];
    const int64_t v = e / n, gi = e - v * n;
    // the entry's rectangle from its own 8-byte array: a gather from the
    // 48-byte records would fetch a record line for 8 bytes
    const uint2 r = rect[e];
    const uint32_t lo_xy = r.x, hi_xy = r.y;
    const int tx0 = (int)(lo_xy & 0xffffu) / tile, ty0 = (int)(lo_xy >> 16) / tile;
    const int tx1 = (int)(hi_xy & 0xffffu) / tile, ty1 = (int)(hi_xy >> 16) / tile;
    s_base[tid] = (uint32_t)(v * spv + (int64_t)(ty0 / kSuper) * sxn + tx0 / kSuper);
    s_w[tid] = (uint32_t)(tx1 / kSuper - tx0 / kSuper + 1);
    s_id[tid] = (uint32_t)gi;
    s_lo[tid] = (uint32_t)tx0 | ((uint32_t)ty0 << 16);
    s_hi[tid] = (uint32_t)tx1 | ((uint32_t)ty1 << 16);
  } else {
    s_off[tid] = (uint32_t)total;
  }
  if (tid == 0) s_off[kEmitBlock] = j0 + kEmitBlock < vn ? offs[j0 + kEmitBlock] : (uint32_t)total;
  __syncthreads();
  const int64_t first = s_off[0];
  const int64_t last = std::min<int64_t>((int64_t)s_off[kEmitBlock], cap);
  int lo = 0;
  for (int64_t p = first + tid; p < last; p += kEmitBlock) {
    // s_off[lo] <= p holds on entry (p only grows); find the last such index
    int hi = kEmitBlock - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((int64_t)s_off[mid] <= p) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t k = (uint32_t)(p - (int64_t)s_off[lo]);
    const uint32_t w = s_w[lo];
    const uint32_t row = k / w, col = k - row * w;
    const int tx0 = (int)(s_lo[lo] & 0xffffu), ty0 = (int)(s_lo[lo] >> 16);
    const int tx1 = (int)(s_hi[lo] & 0xffffu), ty1 = (int)(s_hi[lo] >> 16);
    const int sx = tx0 / kSuper + (int)col, sy = ty0 / kSuper + (int)row;
    const int lx0 = max(tx0 - sx * kSuper, 0), lx1 = min(tx1 - sx * kSuper, kSuper - 1);
    const int ly0 = max(ty0 - sy * kSuper, 0), ly1 = min(ty1 - sy * kSuper, kSuper - 1);
    const uint32_t r12 = (uint32_t)(lx0 | (lx1 << 3) | (ly0 << 6) | (ly1 << 9));
    skey[p] = s_base[lo] + row * (uint32_t)sxn + col;
    sval[p] = ((uint64_t)r12 << 32) | s_id[lo];
  }
}

// ----------------------------------------------------------------- blend
// First index in [0, cnt) whose key is >= target (cnt if none).  The 32
// lanes of one half-wave search together: each round probes 32 evenly spaced
// keys and keeps the gap in which the comparison flips, so a list of 2^25
// pairs takes five dependent loads.
__device__ inline uint32_t halfwave_lower_bound(const uint32_t* __restrict__ keys, uint32_t cnt,
                                                uint32_t target) {
  const int lane = threadIdx.x & 63, j = lane & 31;
  const bool upper = lane >= 32;
  uint32_t lo = 0, hi = cnt;
  while (lo < hi) {
    const uint32_t step = (hi - lo + 31) / 32;
    const uint32_t p = lo + (uint32_t)j * step;
    const bool less = p < hi && keys[p] < target;
    const uint64_t b = __ballot(less);
    const uint32_t c = (uint32_t)__popc(upper ? (uint32_t)(b >> 32) : (uint32_t)b);
    if (c == 0) {
      hi = lo;
    } else {
      const uint32_t nhi = lo + c * step;
      lo = lo + (c - 1) * step + 1;
      hi = nhi < hi ? nhi : hi;
    }
  }
  return lo;
}

// ------------------------------------------------------------- binning
// After the stable sort by super-tile, each super-tile's pairs form a run in
// depth order.  Runs are cut into work units of kBinUnit pairs, one wave
// each, taken 64 pairs (one per lane) per round.  Lane l stands for tile
// (l / 8, l % 8) of the super-tile.  The pairs reaching a tile row or column
// are one ballot each, so the pairs reaching a tile are the AND of two of
// them: their count per tile, and, when scattering, each pair's rank among
// them (pairs in lower lanes come first, which is depth order).

// R[r] (X[c]): lanes whose rectangle reaches tile row r (column c); rp, cp:
// the same per lane
__device__ inline void bin_masks(uint32_t r12, bool ok, uint64_t* R, uint64_t* X) {
  const int lx0 = (int)(r12 & 7u), lx1 = (int)((r12 >> 3) & 7u);
  const int ly0 = (int)((r12 >> 6) & 7u), ly1 = (int)((r12 >> 9) & 7u);
#pragma unroll
  for (int k = 0; k < kSuper; ++k) {
    R[k] = __builtin_amdgcn_ballot_w64(ok && ly0 <= k && k <= ly1);
    X[k] = __builtin_amdgcn_ballot_w64(ok && lx0 <= k && k <= lx1);
  }
}

// pairs of the round that reach lane l's tile
__device__ inline uint32_t bin_lane_count(const uint64_t* R, const uint64_t* X, int lane) {
  const int r = lane >> 3, c = lane & 7;
  uint64_t a = R[0], b = X[0];
#pragma unroll
  for (int k = 1; k < kSuper; ++k) {
    a = r == k ? R[k] : a;
    b = c == k ? X[k] : b;
  }
  return (uint32_t)__popcll(a & b);
}

// global index of lane l's tile in super-tile s; false where it lies
// outside the view
__device__ inline bool bin_tile(int64_t s, int lane, int64_t sxn, int64_t spv, int64_t tiles_x,
                                int64_t tiles_y, int64_t* t) {
  const int64_t v = s / spv, sl = s - v * spv;
  const int64_t sy = sl / sxn, sx = sl - sy * sxn;
  const int64_t ty = sy * kSuper + (lane >> 3), tx = sx * kSuper + (lane & 7);
  *t = (v * tiles_y + ty) * tiles_x + tx;
  return ty < tiles_y && tx < tiles_x;
}

// Run boundaries: [begin, end) of every super-tile present in the sorted
// keys (absent ones keep the zeroed range).
__global__ __launch_bounds__(256) void k_gs_runs(const uint32_t* __restrict__ skeys,
                                                 const uint32_t* __restrict__ stotal_p,
                                                 int64_t max_pairs, uint2* __restrict__ srange) {
  const int64_t cnt = std::min<int64_t>(*stotal_p, max_pairs);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = skeys[i];
    if (i == 0 || skeys[i - 1] != k) srange[k].x = (uint32_t)i;
    if (i == cnt - 1 || skeys[i + 1] != k) srange[k].y = (uint32_t)(i + 1);
  }
}

// One workgroup: units per run, their exclusive scan (first unit of each
// super-tile, ubase[st_total] = number of units), and the exact number of
// tile pairs from the preprocess blocks' partial sums (whatever the
// capacity).  With run lengths given (a one-pass sort's digit counts) the
// runs are their exclusive scan, written here; else k_gs_runs found them.
constexpr int kUnitsBlock = 1024;
__global__ __launch_bounds__(kUnitsBlock) void k_gs_units(uint2* __restrict__ srange,
                                                          const uint32_t* __restrict__ run_len,
                                                          int64_t st_total,
                                                          const uint64_t* __restrict__ psum,
                                                          int64_t nps, uint32_t* __restrict__ ubase,
                                                          uint32_t* __restrict__ nunits,
                                                          uint32_t* __restrict__ pair_count) {
  __shared__ uint32_t s_w[kUnitsBlock / 64];
  __shared__ uint64_t s_p[kUnitsBlock / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint64_t p = 0;
  for (int64_t k = tid; k < nps; k += kUnitsBlock) p += psum[k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
  if (lane == 0) s_p[wave] = p;
  // block-wide exclusive scan of x over the chunk's super-tiles; returns the
  // chunk total
  auto block_scan = [&](uint32_t x, uint32_t& excl) {
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t woff = 0, btot = 0;
#pragma unroll
    for (int w = 0; w < kUnitsBlock / 64; ++w) {
      woff += w < wave ? s_w[w] : 0u;
      btot += s_w[w];
    }
    excl = woff + incl - x;
    __syncthreads();   // s_w is rewritten by the next scan
    return btot;
  };
  uint32_t carry = 0, rcarry = 0;
  for (int64_t s0 = 0; s0 < st_total; s0 += kUnitsBlock) {
    const int64_t s = s0 + tid;
    uint32_t len = 0;
    if (s < st_total) {
      if (run_len) {
        len = run_len[s];
      } else {
        const uint2 r = srange[s];
        len = r.y > r.x ? r.y - r.x : 0u;
      }
    }
    if (run_len) {
      uint32_t b;
      const uint32_t tot = block_scan(len, b);
      if (s < st_total) srange[s] = make_uint2(rcarry + b, rcarry + b + len);
      rcarry += tot;
    }
    const uint32_t u = (len + kBinUnit - 1) / kBinUnit;
    uint32_t ue;
    const uint32_t utot = block_scan(u, ue);
    if (s < st_total) ubase[s] = carry + ue;
    carry += utot;
  }
  if (tid == 0) {
    ubase[st_total] = carry;
    *nunits = carry;
    uint64_t q = 0;
    for (int w = 0; w < kUnitsBlock / 64; ++w) q += s_p[w];
    *pair_count = (uint32_t)std::min<uint64_t>(q, 0xffffffffull);
  }
}

// Unit u of the scan -> its super-tile (last s with ubase[s] <= u) and pair
// range [lo, hi).
__device__ inline int64_t bin_unit(const uint32_t* __restrict__ ubase, int64_t st_total,
                                   const uint2* __restrict__ srange, uint32_t u, uint32_t* lo,
                                   uint32_t* hi) {
  const int64_t s = (int64_t)halfwave_lower_bound(ubase, (uint32_t)st_total, u + 1) - 1;
  const uint2 r = srange[s];
  *lo = r.x + (u - ubase[s]) * kBinUnit;
  *hi = std::min<uint32_t>(r.y, *lo + kBinUnit);
  return s;
}

// Per unit and tile: pairs of the unit reaching the tile.  Waves take units
// in grid-stride order; the grid is sized for the capacity, the count is
// read on the device.
__global__ __launch_bounds__(256) void k_gs_bin_count(const uint64_t* __restrict__ svals,
                                                      const uint2* __restrict__ srange,
                                                      const uint32_t* __restrict__ ubase,
                                                      const uint32_t* __restrict__ nunits_p,
                                                      int64_t st_total,
                                                      uint32_t* __restrict__ ucnt) {
  const int lane = threadIdx.x & 63;
  const uint32_t nunits = *nunits_p;
  for (uint32_t u = blockIdx.x * 4u + (threadIdx.x >> 6); u < nunits; u += gridDim.x * 4u) {
    uint32_t lo, hi;
    bin_unit(ubase, st_total, srange, u, &lo, &hi);
    uint32_t r12[kBinUnit / 64];   // every load of the unit in flight first
#pragma unroll
    for (int k = 0; k < kBinUnit / 64; ++k) {
      const uint32_t j = lo + 64 * k + lane;
      r12[k] = j < hi ? (uint32_t)(svals[j] >> 32) : 0u;
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < kBinUnit / 64; ++k) {
      if (lo + 64 * k >= hi) break;   // uniform over the wave
      uint64_t R[kSuper], X[kSuper];
      bin_masks(r12[k], lo + 64 * k + lane < hi, R, X);
      cnt += bin_lane_count(R, X, lane);
    }
    ucnt[(int64_t)u * 64 + lane] = cnt;
  }
}

// One workgroup per super-tile: exclusive prefix of its units' counts per
// tile (in place) and the tile totals.  Wave w takes a contiguous share of
// the units, loads kPrefixBatch of them at a time.
// Device-coherent word access for the last-workgroup hand-over below.
__device__ inline uint32_t coh_load32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void coh_store32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Length bucket of a tile list: descending in 16 log2(1 + length), so that
// the blend runs long lists first (work per tile is very uneven, and
// starting the long lists first keeps them off the end of the blend).
__device__ inline uint32_t sched_bucket(uint32_t len) {
  const float lb = 16.0f * log2f(1.0f + (float)len);
  return 255u - (uint32_t)fminf(lb, 255.0f);
}
// The active lanes holding the same 8-bit value b (eight ballots): one
// atomic per distinct bucket of a wave.
__device__ inline uint64_t match_u8(uint32_t b) {
  uint64_t m = __ballot(true);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const bool bit = (b >> i) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

constexpr int kPrefixWaves = 16, kPrefixBatch = 8;
__global__ __launch_bounds__(64 * kPrefixWaves) void k_gs_bin_prefix(
    const uint32_t* __restrict__ ubase, int64_t sxn, int64_t spv, int64_t tiles_x,
    int64_t tiles_y, uint32_t* __restrict__ ucnt, uint32_t* __restrict__ tcnt,
    const uint32_t* __restrict__ total_p, int64_t max_pairs, int64_t st_total,
    uint32_t* __restrict__ stot, uint32_t* __restrict__ sbase, uint32_t* __restrict__ sched) {
  __shared__ uint32_t s_c[kPrefixWaves][64];
  __shared__ uint32_t s_w[kPrefixWaves];
  __shared__ bool s_last;
  const int64_t s = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t u0 = ubase[s], nu = ubase[s + 1] - u0;
  const uint32_t a = u0 + (uint32_t)((uint64_t)nu * wave / kPrefixWaves);
  const uint32_t b = u0 + (uint32_t)((uint64_t)nu * (wave + 1) / kPrefixWaves);
  uint32_t sum = 0;
  for (uint32_t u = a; u < b; u += kPrefixBatch) {
    uint32_t c[kPrefixBatch];
#pragma unroll
    for (int k = 0; k < kPrefixBatch; ++k)
      c[k] = u + k < b ? ucnt[(int64_t)(u + k) * 64 + lane] : 0u;
#pragma unroll
    for (int k = 0; k < kPrefixBatch; ++k) sum += c[k];
  }
  s_c[wave][lane] = sum;
  __syncthreads();
  uint32_t run = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kPrefixWaves; ++w) {
    run += w < wave ? s_c[w][lane] : 0u;
    tot += s_c[w][lane];
  }
  for (uint32_t u = a; u < b; u += kPrefixBatch) {
    uint32_t c[kPrefixBatch];
#pragma unroll
    for (int k = 0; k < kPrefixBatch; ++k)
      c[k] = u + k < b ? ucnt[(int64_t)(u + k) * 64 + lane] : 0u;
#pragma unroll
    for (int k = 0; k < kPrefixBatch; ++k) {
      if (u + k < b) ucnt[(int64_t)(u + k) * 64 + lane] = run;
      run += c[k];
    }
  }
  int64_t t;
  if (wave == 0) {
    // the tile totals, the super-tile's total and the tiles' length buckets
    // (past the capacity every list is empty)
    const bool valid = bin_tile(s, lane, sxn, spv, tiles_x, tiles_y, &t);
    const uint32_t c = valid && (int64_t)*total_p <= max_pairs ? tot : 0u;
    if (valid) tcnt[t] = tot;
    uint32_t st = c;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) st += __shfl_xor(st, o, 64);
    if (lane == 0) coh_store32(&stot[s], st);
    if (valid) {
      const uint32_t bk = sched_bucket(c);
      const uint64_t m = match_u8(bk);
      if (lane == __builtin_ctzll(m)) atomicAdd(&sched[kSchedHist + bk], (uint32_t)__popcll(m));
    }
  }
  // the last workgroup to finish: list bases of the super-tiles (their tile
  // lists are laid out super-tile by super-tile) and the bucket cursors.
  // The hand-over words are device-coherent (agent-scope store, device
  // atomics); wave 0, which wrote them, waits until they have completed
  // before it counts the workgroup done.
  if (wave == 0) {
    __builtin_amdgcn_s_waitcnt(0);   // every counter drained: vector memory included
    if (lane == 0) s_last = atomicAdd(&sched[kSchedDone], 1u) == (uint32_t)(st_total - 1);
  }
  __syncthreads();
  if (!s_last) return;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < st_total; b0 += 64 * kPrefixWaves) {
    const int64_t i = b0 + tid;
    const uint32_t x = i < st_total ? coh_load32(&stot[i]) : 0u;
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t woff = 0, btot = 0;
#pragma unroll
    for (int w = 0; w < kPrefixWaves; ++w) {
      woff += w < wave ? s_w[w] : 0u;
      btot += s_w[w];
    }
    if (i < st_total) sbase[i] = carry + woff + incl - x;
    carry += btot;
    __syncthreads();   // s_w is rewritten by the next chunk
  }
  if (wave == 0) {   // exclusive scan of the 256 buckets, four per lane
    uint32_t h[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      h[q] = sum;
      sum += coh_load32(&sched[kSchedHist + lane * 4 + q]);
    }
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) sched[kSchedCursor + lane * 4 + q] = incl - sum + h[q];
  }
}

// One wave per super-tile, one lane per tile: the tile's list offset (its
// super-tile's base plus the counts of the super-tile's earlier tiles), its
// [begin, end) range and its place in the blend order (the next place of
// its length bucket; the order within a bucket is free: tiles are
// independent).  Past the capacity every list is left empty.
__global__ __launch_bounds__(64) void k_gs_schedule(
    const uint32_t* __restrict__ tcnt, const uint32_t* __restrict__ sbase,
    const uint32_t* __restrict__ total_p, int64_t max_pairs, int64_t sxn, int64_t spv,
    int64_t tiles_x, int64_t tiles_y, uint32_t* __restrict__ sched, uint32_t* __restrict__ toff,
    uint2* __restrict__ ranges, uint32_t* __restrict__ order, int32_t* status) {
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  const bool over = (int64_t)*total_p > max_pairs;
  if (s == 0 && lane == 0 && over) set_status(status, VRS_ECAPACITY);
  int64_t t;
  const bool valid = bin_tile(s, lane, sxn, spv, tiles_x, tiles_y, &t);
  const uint32_t c = valid && !over ? tcnt[t] : 0u;
  uint32_t incl = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (!valid) return;
  const uint32_t b = sbase[s] + incl - c;
  toff[t] = b;
  ranges[t] = make_uint2(b, b + c);
  const uint32_t bk = sched_bucket(c);
  const uint64_t m = match_u8(bk);
  const int leader = __builtin_ctzll(m);
  uint32_t at = 0;
  if (lane == leader) at = atomicAdd(&sched[kSchedCursor + bk], (uint32_t)__popcll(m));
  at = __shfl(at, leader, 64);
  order[at + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = (uint32_t)t;
}

// Per unit: tile l's cursor starts at the tile's list offset plus the counts
// of the run's earlier units; per round and tile the reaching pairs'
// Gaussian indices go to cursor + rank.  Nothing is written past the
// capacity (the lists are then left empty).
__global__ __launch_bounds__(256) void k_gs_bin_scatter(
    const uint64_t* __restrict__ svals, const uint2* __restrict__ srange,
    const uint32_t* __restrict__ ubase, const uint32_t* __restrict__ nunits_p, int64_t st_total,
    const uint32_t* __restrict__ ucnt, const uint32_t* __restrict__ toff,
    const uint32_t* __restrict__ total_p, int64_t max_pairs, int64_t sxn, int64_t spv,
    int64_t tiles_x, int64_t tiles_y, uint32_t* __restrict__ ids) {
  // the unit's pairs, staged per wave: a lane reads back only what it wrote
  __shared__ uint64_t s_unit[4][kBinUnit];
  const int lane = threadIdx.x & 63;
  if ((int64_t)*total_p > max_pairs) return;
  const uint32_t nunits = *nunits_p;
  uint64_t* su = s_unit[threadIdx.x >> 6];
  for (uint32_t u = blockIdx.x * 4u + (threadIdx.x >> 6); u < nunits; u += gridDim.x * 4u) {
    uint32_t lo, hi;
    const int64_t s = bin_unit(ubase, st_total, srange, u, &lo, &hi);
    int64_t t;
    uint32_t cursor = 0;
    if (bin_tile(s, lane, sxn, spv, tiles_x, tiles_y, &t))
      cursor = toff[t] + ucnt[(int64_t)u * 64 + lane];
    // Every load of the unit in flight at once, then parked in LDS.  A load
    // issued inside the round loop would have to complete before the next
    // round, and the loads and stores of one wave share a single in-order
    // completion counter: that wait would drain the round's 64 stores too.
    {
      uint64_t r[kBinUnit / 64];
#pragma unroll
      for (int k = 0; k < kBinUnit / 64; ++k) {
        const uint32_t j = lo + 64 * k + lane;
        r[k] = j < hi ? svals[j] : 0ull;
      }
#pragma unroll
      for (int k = 0; k < kBinUnit / 64; ++k) su[64 * k + lane] = r[k];
    }
    for (uint32_t i = lo, k = 0; i < hi; i += 64, ++k) {
      const uint64_t cur = su[64 * k + lane];
      const uint32_t gi = (uint32_t)cur;
      uint64_t R[kSuper], X[kSuper];
      bin_masks((uint32_t)(cur >> 32), i + lane < hi, R, X);
#pragma unroll
      for (int l = 0; l < 64; ++l) {
        // the lanes reaching tile l are those of M (a wave-uniform mask, the
        // store's execution mask): the rank is a bit count
        const uint64_t M = R[l >> 3] & X[l & 7];
        const uint32_t at_l = (uint32_t)__builtin_amdgcn_readlane((int)cursor, l);
        if (__builtin_amdgcn_inverse_ballot_w64(M))
          ids[at_l + __builtin_amdgcn_mbcnt_hi((uint32_t)(M >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)M, 0u))] = gi;
      }
      cursor += bin_lane_count(R, X, lane);
    }
  }
}

}  // namespace vrs

using namespace vrs;

static bool read_opts(const vrs_raster_opts* ro, GsOpt* o) {
  if (!ro) return false;
  o->tile = ro->tile;
  o->aclamp = ro->alpha_clamp;
  o->amin = ro->alpha_min;
  o->tmin = ro->t_min;
  o->lowpass = ro->lowpass;
  o->extent = ro->extent;
  for (int k = 0; k < 3; ++k) o->bg[k] = ro->bg[k];
  o->order = ro->order;
  return (o->tile == 8 || o->tile == 16 || o->tile == 32) && radix_bits_ok(opts_radix(ro)) &&
         (o->order == VRS_ORDER_PRIMITIVE || o->order == VRS_ORDER_PIXEL) && o->extent > 0 &&
         o->lowpass >= 0 && o->amin >= 0;
}

// Per-pixel order runs one pixel per lane with its window in registers:
// tiles of 8 and 16 pixels (a 32-pixel tile's 1024-lane workgroup would leave
// too few registers per lane).
static bool order_supported(const GsOpt& o) {
  return o.order != VRS_ORDER_PIXEL || o.tile <= 16;
}

static bool same_dims(const vrs_view* views, int nv) {
  for (int i = 1; i < nv; ++i)
    if (views[i].width != views[0].width || views[i].height != views[0].height) return false;
  return true;
}

extern "C" size_t vrs_render_workspace_size(int64_t n, int n_views, const vrs_view* views,
                                            const vrs_raster_opts* opts, int64_t max_pairs) {
  RenderWs L;
  if (!opts || !render_layout(n, n_views, views, opts->tile, opts_radix(opts), max_pairs, &L,
                             opts->order))
    return 0;
  return L.total;
}

extern "C" vrs_status vrs_render_workspace_layout(int64_t n, int n_views, const vrs_view* views,
                                                  const vrs_raster_opts* opts,
                                                  int64_t max_pairs, vrs_render_layout* out) {
  RenderWs L;
  if (!opts || !out ||
      !render_layout(n, n_views, views, opts->tile, opts_radix(opts), max_pairs, &L,
                     opts->order))
    return VRS_EINVAL;
  out->pair_count = L.pair_count;
  out->sorted_ids = L.ids;
  out->tile_ranges = L.ranges;
  out->tiles_x = L.tiles_x;
  out->tiles_y = L.tiles_y;
  out->tiles_total = L.tiles_total;
  out->pixel_evals = L.evals;
  out->super_pair_count = L.super_count;
  out->exact_pass_count = L.fix_count;
  out->tile_words = L.tkey;
  return VRS_OK;
}

namespace vrs {
// flags: kRenderStats keeps the per-pixel last positions (for the adjoint)
// and evaluation counts in the workspace.
vrs_status render_impl(const float* mean, const float* cov, const float* opacity,
                       const float* sh, int sh_degree, int64_t n, const vrs_view* views,
                       int n_views, const vrs_raster_opts* opts, float* rgb, float* depth,
                       float* t_final, int32_t* n_contrib, void* ws, size_t ws_bytes,
                       int64_t max_pairs, int32_t* dev_status, void* stream, int flags,
                       const Trace* tr) {
  GsOpt o;
  KViews kv;
  RenderWs L;
  if (!read_opts(opts, &o) || !make_views(views, n_views, &kv) || !same_dims(views, n_views))
    return VRS_EINVAL;
  if (!order_supported(o)) return VRS_EUNSUPPORTED;
  if (n < 0 || n > (int64_t(1) << 28) || (n > 0 && (!mean || !cov || !opacity || !sh)))
    return VRS_EINVAL;
  if (sh_degree < 0 || sh_degree > 3) return VRS_EINVAL;
  if (!rgb || !depth || !t_final || !n_contrib || !ws) return VRS_EINVAL;
  if (max_pairs < 0 || max_pairs >= (int64_t(1) << 30)) return VRS_EINVAL;
  if (!render_layout(n, n_views, views, o.tile, opts_radix(opts), max_pairs, &L, o.order) ||
      ws_bytes < L.total)
    return VRS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t vn = L.vn;
  uint32_t* pair_count = at<uint32_t>(ws, L.pair_count);
  uint32_t* super_count = at<uint32_t>(ws, L.super_count);
  const int64_t nps = div_up(n, 256);
  bool s1 = false;
  if (vn > 0) {
    trace_begin(tr, VRS_TRACE_GS_PREPROCESS, st);
    auto pre = sh_degree == 0   ? k_gs_preprocess<0>
               : sh_degree == 1 ? k_gs_preprocess<1>
               : sh_degree == 2 ? k_gs_preprocess<2>
                                : k_gs_preprocess<3>;
    hipLaunchKernelGGL(pre, dim3((unsigned)nps), dim3(256), 0, st, mean, cov, opacity, sh, n, kv,
                       o, at<float4>(ws, L.rec), at<uint2>(ws, L.rect), at<uint32_t>(ws, L.dkey0),
                       at<uint32_t>(ws, L.nsup),
                       at<uint64_t>(ws, L.psum), at<uint32_t>(ws, L.scan_tmp),
                       (int64_t)((L.sched - L.scan_tmp) / 4 + kSchedDone + 1));
    VRS_LAUNCH_CHECK();
    if (o.order == VRS_ORDER_PIXEL) {
      launch_gs_pixdepth(L, ws, mean, cov, n, kv, st);
      VRS_LAUNCH_CHECK();
    }
    trace_end(tr, VRS_TRACE_GS_PREPROCESS, st);
    trace_begin(tr, VRS_TRACE_GS_DEPTH_SORT, st);
    bool d1 = false;
    // the last pass also lays the super-tile counts out in depth order
    VRS_HIP_CHECK(radix_sort_u32(at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0),
                                 at<uint32_t>(ws, L.dkey1), at<uint32_t>(ws, L.dval1), nullptr, vn,
                                 32, L.radix, at<void>(ws, L.sort_tmp), dev_status, st, &d1,
                                 at<uint32_t>(ws, L.nsup), at<uint32_t>(ws, L.nsorted), true));
    const uint32_t* sorted_e = at<uint32_t>(ws, d1 ? L.dval1 : L.dval0);
    VRS_HIP_CHECK(exclusive_scan_u32(at<uint32_t>(ws, L.nsorted), nullptr,
                                     at<uint32_t>(ws, L.soffs), super_count, nullptr, vn,
                                     at<void>(ws, L.scan_tmp), dev_status, st, true));
    trace_end(tr, VRS_TRACE_GS_DEPTH_SORT, st);
    trace_begin(tr, VRS_TRACE_GS_EMIT, st);
    hipLaunchKernelGGL(k_gs_emit_super, dim3(div_up(vn, kEmitBlock)), dim3(kEmitBlock), 0, st,
                       at<uint32_t>(ws, L.soffs), sorted_e, at<uint2>(ws, L.rect), super_count,
                       vn, n, max_pairs, o.tile, L.sxn, L.spv, at<uint32_t>(ws, L.skey0),
                       at<uint64_t>(ws, L.sval0), L.st_total, at<uint2>(ws, L.srange),
                       dev_status);
    VRS_LAUNCH_CHECK();
    trace_end(tr, VRS_TRACE_GS_EMIT, st);
    trace_begin(tr, VRS_TRACE_GS_SORT, st);
    VRS_HIP_CHECK(radix_sort_u64(at<uint32_t>(ws, L.skey0), at<uint64_t>(ws, L.sval0),
                                 at<uint32_t>(ws, L.skey1), at<uint64_t>(ws, L.sval1), super_count,
                                 max_pairs, L.st_bits, L.radix, at<void>(ws, L.sort_tmp),
                                 dev_status, st, &s1));
  } else {
    trace_begin(tr, VRS_TRACE_GS_SORT, st);
    VRS_HIP_CHECK(fill_u32(super_count, 0, 1, st));
    VRS_HIP_CHECK(fill_u32(at<uint32_t>(ws, L.srange), 0, 2 * L.st_total, st));
    VRS_HIP_CHECK(fill_u32(at<uint32_t>(ws, L.sched), 0, kSchedDone + 1, st));
  }
  // binning: runs, units, per unit and tile counts, tile offsets, ranges and
  // the longest-first schedule, scatter.  Timed with the sorts, so the blend
  // stage is the blend alone.
  const uint32_t* skeys = at<uint32_t>(ws, s1 ? L.skey1 : L.skey0);
  const uint64_t* svals = at<uint64_t>(ws, s1 ? L.sval1 : L.sval0);
  const int64_t mp = std::max<int64_t>(max_pairs, 1);
  const unsigned unit_blocks =
      (unsigned)std::min<int64_t>(2048, div_up(bin_units_max(mp, L.st_total), 4));
  // one sort pass: its digit counts are the run lengths; else find the runs
  const bool one_pass = vn > 0 && L.st_bits <= L.radix;
  if (!one_pass) {
    hipLaunchKernelGGL(k_gs_runs, dim3((unsigned)std::min<int64_t>(4096, div_up(mp, 256))),
                       dim3(256), 0, st, skeys, super_count, max_pairs, at<uint2>(ws, L.srange));
    VRS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_gs_units, dim3(1), dim3(kUnitsBlock), 0, st, at<uint2>(ws, L.srange),
                     one_pass ? radix_sort_digit_totals(at<void>(ws, L.sort_tmp)) : nullptr,
                     L.st_total, at<uint64_t>(ws, L.psum), vn > 0 ? nps : 0,
                     at<uint32_t>(ws, L.ubase), at<uint32_t>(ws, L.nunits), pair_count);
  VRS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gs_bin_count, dim3(unit_blocks), dim3(256), 0, st, svals,
                     at<uint2>(ws, L.srange), at<uint32_t>(ws, L.ubase),
                     at<uint32_t>(ws, L.nunits), L.st_total, at<uint32_t>(ws, L.ucnt));
  VRS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gs_bin_prefix, dim3((unsigned)L.st_total), dim3(64 * kPrefixWaves), 0, st,
                     at<uint32_t>(ws, L.ubase), L.sxn, L.spv, L.tiles_x, L.tiles_y,
                     at<uint32_t>(ws, L.ucnt), at<uint32_t>(ws, L.tcnt), pair_count, max_pairs,
                     L.st_total, at<uint32_t>(ws, L.stot), at<uint32_t>(ws, L.sbase),
                     at<uint32_t>(ws, L.sched));
  VRS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gs_schedule, dim3((unsigned)L.st_total), dim3(64), 0, st,
                     at<uint32_t>(ws, L.tcnt), at<uint32_t>(ws, L.sbase), pair_count, max_pairs,
                     L.sxn, L.spv, L.tiles_x, L.tiles_y, at<uint32_t>(ws, L.sched),
                     at<uint32_t>(ws, L.toff), at<uint2>(ws, L.ranges), at<uint32_t>(ws, L.order),
                     dev_status);
  VRS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gs_bin_scatter, dim3(unit_blocks), dim3(256), 0, st, svals,
                     at<uint2>(ws, L.srange), at<uint32_t>(ws, L.ubase),
                     at<uint32_t>(ws, L.nunits), L.st_total, at<uint32_t>(ws, L.ucnt),
                     at<uint32_t>(ws, L.toff), pair_count, max_pairs, L.sxn, L.spv, L.tiles_x,
                     L.tiles_y, at<uint32_t>(ws, L.ids));
  VRS_LAUNCH_CHECK();
  const uint32_t* order = at<uint32_t>(ws, L.order);
  if (o.order == VRS_ORDER_PIXEL) {
    launch_gs_tile_zsort(L, ws, n, kv, o.tile, st);
    VRS_LAUNCH_CHECK();
  }
  trace_end(tr, VRS_TRACE_GS_SORT, st);
  trace_begin(tr, VRS_TRACE_GS_BLEND, st);
  if (o.order == VRS_ORDER_PIXEL)
    launch_gs_blend_px(L, ws, n, order, kv, o, rgb, depth, t_final, n_contrib, st);
  else
    launch_gs_blend((flags & kRenderStats) != 0, L, ws, n, order, kv, o, rgb, depth, t_final,
                    n_contrib, st);
  VRS_LAUNCH_CHECK();
  trace_end(tr, VRS_TRACE_GS_BLEND, st);
  return VRS_OK;
}
}  // namespace vrs

extern "C" vrs_status vrs_render_gaussians(const float* mean, const float* cov,
                                           const float* opacity, const float* sh, int sh_degree,
                                           int64_t n, const vrs_view* views, int n_views,
                                           const vrs_raster_opts* opts, float* rgb, float* depth,
                                           float* t_final, int32_t* n_contrib, void* ws,
                                           size_t ws_bytes, int64_t max_pairs,
                                           int32_t* dev_status, void* stream) {
  return render_impl(mean, cov, opacity, sh, sh_degree, n, views, n_views, opts, rgb, depth,
                     t_final, n_contrib, ws, ws_bytes, max_pairs, dev_status, stream,
                     kRenderStats, nullptr);
}
