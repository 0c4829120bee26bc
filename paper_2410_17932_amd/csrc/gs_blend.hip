// Periphery blend (Sec. 3.2): front-to-back alpha blending of each tile's
// depth-ordered Gaussian list with Eq. 1 depth, the hot loop of the
// periphery.  The tile lists, their ranges and the longest-first schedule
// come from the binning in gs_forward.hip.
#include <type_traits>

#include "gs_layout.h"

namespace vrs {

// One workgroup per (view, tile).  The tile is cut into SUB x SUB sub-tiles,
// one wave each; a lane holds PPT pixels of its sub-tile (a column, rows
// 64/SUB apart).  Records of the tile list are staged in LDS in batches of
// BLOCK (one per thread, conic pre-scaled for exp2); while staging, each wave
// ballots which of the batch's records reach each sub-tile, so a wave walks
// only the records that touch its sub-tile, in list order, with scalar bit
// scans.  The per-pixel step is branch-free: every lane evaluates, and
// selects decide.  A wave stops evaluating once all its pixels have
// stopped; the block leaves the list when every wave has.  Workgroup i
// takes the i-th tile of the longest-first schedule.

// A 64-bit value known to be equal in every lane, moved to scalar registers
// (the builtin returns a signed 32-bit int: each half goes through uint32_t
// so that the low half is not sign-extended into the high one).
__device__ inline uint64_t wave_uniform_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// A lane flag as the wave's mask (bit l = lane l) and back: the mask lives
// in scalar registers and every combination of flags is a scalar operation.
__device__ inline uint64_t wave_mask(bool b) { return __builtin_amdgcn_ballot_w64(b); }
__device__ inline bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }
// c + 1 in the lanes of mask m, c elsewhere: one vector add with m as its
// carry-in (the compiler would select and add)
__device__ inline int count_lanes(int c, uint64_t m) {
  uint64_t carry_out;
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %2" : "+v"(c), "=s"(carry_out) : "s"(m));
  (void)carry_out;
  return c;
}

// Lower bound of G(d) = ga dx^2 + gb dx dy + gc dy^2 (positive definite)
// over the box dx in [X0, X1], dy in [Y0, Y1]: 0 if the box holds the
// origin, else the least of the four edge minima (the minimiser of a convex
// quadratic over a box lies on its boundary; on an edge it is the clamped
// stationary point).  ia, ic = 1 / (2 ga), 1 / (2 gc): a stationary point off
// by a relative rounding error changes the edge minimum by its square, far
// inside the caller's margin.
__device__ inline float box_min_quadratic(float ga, float gb, float gc, float ia, float ic,
                                          float X0, float X1, float Y0, float Y1) {
  if (X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f) return 0.0f;
  float m = 3.0e38f;
  float Xe[2] = {X0, X1}, Ye[2] = {Y0, Y1};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float X = Xe[i];
    const float dy = fminf(fmaxf(-gb * X * ic, Y0), Y1);
    m = fminf(m, ga * X * X + gb * X * dy + gc * dy * dy);
    const float Y = Ye[i];
    const float dx = fminf(fmaxf(-gb * Y * ia, X0), X1);
    m = fminf(m, ga * dx * dx + gb * dx * Y + gc * Y * Y);
  }
  return m;
}

template <int TILE, int SUB>
struct BlendCfg {
  static constexpr int NQ = TILE / SUB;          // sub-tiles per side
  static constexpr int NW = NQ * NQ;             // waves per block
  static constexpr int BLOCK = 64 * NW;
  static constexpr int PPT = SUB * SUB / 64;     // pixels per lane
  static constexpr int ROWS = 64 / SUB;          // rows between a lane's pixels
};

// Register budget for five waves per SIMD (96 VGPRs; no spills): the
// staging and the per-pixel state compete for registers, and occupancy hides
// the LDS and gather latency better than the extra registers would help.
// STATS: also write each pixel's last contributing list position (the
// adjoint's replay start) and its evaluation count (the work count); an
// inference frame leaves both out, and with them the counting of records
// out of reach of the ellipse.
template <int TILE, int SUB, bool STATS>
__global__ __launch_bounds__((BlendCfg<TILE, SUB>::BLOCK))
__attribute__((amdgpu_waves_per_eu(5, 8))) void k_gs_blend(
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ ids,
    const float4* __restrict__ rec, int64_t n, KViews views, GsOpt o, int64_t tiles_x,
    int64_t tiles_per_view, const uint2* __restrict__ ranges, float* __restrict__ out_rgb,
    float* __restrict__ out_depth,
    float* __restrict__ out_t, int32_t* __restrict__ out_n, uint32_t* __restrict__ out_last,
    uint32_t* __restrict__ out_evals) {
  using Cfg = BlendCfg<TILE, SUB>;
  constexpr int BLOCK = Cfg::BLOCK, PPT = Cfg::PPT, NW = Cfg::NW, NQ = Cfg::NQ;
  __shared__ float4 s_a[BLOCK], s_b[BLOCK], s_c[BLOCK];
  __shared__ uint64_t s_mask[NW][NW];   // [sub-tile][group of 64 records]: rectangle reaches it
  __shared__ uint64_t s_full[NW][NW];   // ... and the contributing ellipse may too
  __shared__ uint64_t s_cover[NW][NW];  // ... and the rectangle holds its in-image pixels
  const int64_t tglob = order[blockIdx.x];
  const int v = (int)(tglob / tiles_per_view);
  const int64_t tl = tglob - (int64_t)v * tiles_per_view;
  const int ty = (int)(tl / tiles_x), tx = (int)(tl - (int64_t)ty * tiles_x);
  const KView& cv = views.v[v];
  const int W = cv.W, H = cv.H;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // sub-tile of this wave and the lane's pixels
  const int sx0 = tx * TILE + (wave % NQ) * SUB, sy0 = ty * TILE + (wave / NQ) * SUB;
  const int px = sx0 + lane % SUB;
  // lm[q]: the wave's lanes whose pixel q is in the image and has not
  // stopped (one bit per lane, in scalar registers: liveness costs no vector
  // instructions); stopcov[q]: the count of sub-tile-holding records when
  // the pixel stopped (statistics only)
  int py[PPT];
  uint64_t lm[PPT];
  float T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT];
  int cnt[PPT];
  uint32_t last[PPT], evals[PPT], stopcov[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    py[q] = sy0 + lane / SUB + q * Cfg::ROWS;
    lm[q] = wave_mask(px < W && py[q] < H);
    T[q] = 1.0f;
    C0[q] = C1[q] = C2[q] = D[q] = 0.0f;
    cnt[q] = 0;
    last[q] = 0;
    evals[q] = 0;
    stopcov[q] = 0;
  }
  const uint2 rg = ranges[tglob];
  const uint32_t begin = rg.x, end = rg.y;
  const float aclamp = o.aclamp, amin = o.amin, tmin = o.tmin;
  const float inv_amin = 1.0f / amin;   // infinite for alpha_min = 0: never out of reach
  const float xc = (float)px + 0.5f;
  float yc[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) yc[q] = (float)py[q] + 0.5f;
  auto any_live = [&]() {
    uint64_t a = 0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) a |= lm[q];
    return a != 0;   // wave-uniform
  };
  bool alive = any_live();
  // records whose rectangle holds the sub-tile, so far: every live pixel
  // evaluated each of them, so they are counted per wave, not per pixel
  uint32_t ncov = 0;
  for (uint32_t b0 = begin; b0 < end; b0 += BLOCK) {
    if (__syncthreads_count(alive) == 0) break;
    const uint32_t jr = b0 + tid;
    bool has = jr < end;
    int x0 = 1, x1 = 0, y0 = 1, y1 = 0;
    // contributing region: alpha >= alpha_min <=> G(d) = -q(d) <= log2(op /
    // alpha_min); thr carries a margin far above the rounding of q so that a
    // sub-tile is declared out of reach only where every pixel's own test
    // would fail
    float cx = 0.0f, cy = 0.0f, ga = 1.0f, gb = 0.0f, gc = 1.0f, ia = 0.5f, ic = 0.5f, thr = -1.0f;
    if (has) {
      const uint32_t id = ids[jr];
      const int64_t e = (int64_t)v * n + (id < (uint64_t)n ? id : 0);
      float4 a, b, c;
      gs_stage(rec, e, a, b, c);
      s_a[tid] = a;
      s_b[tid] = b;
      s_c[tid] = c;
      const uint32_t lo = __float_as_uint(b.z), hi = __float_as_uint(b.w);
      x0 = (int)(lo & 0xffffu); y0 = (int)(lo >> 16);
      x1 = (int)(hi & 0xffffu); y1 = (int)(hi >> 16);
      cx = a.x; cy = a.y;
      ga = -a.z; gb = -a.w; gc = -b.x;
      ia = 0.5f * __builtin_amdgcn_rcpf(ga);
      ic = 0.5f * __builtin_amdgcn_rcpf(gc);
      // (hardware log2 and reciprocal: their error is far inside the margin)
      thr = b.y >= amin ? __builtin_amdgcn_logf(b.y * inv_amin) * 1.001f + 1.0e-3f : -1.0f;
      if (!(ga > 0.0f && gc > 0.0f)) thr = 3.0e38f;   // never declared out of reach
    }
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int qx0 = tx * TILE + (w % NQ) * SUB, qy0 = ty * TILE + (w / NQ) * SUB;
      const int xlo = max(x0, qx0), xhi = min(x1, qx0 + SUB - 1);
      const int ylo = max(y0, qy0), yhi = min(y1, qy0 + SUB - 1);
      const bool hit = has && xlo <= xhi && ylo <= yhi;
      const bool cover = hit && x0 <= qx0 && x1 >= min(qx0 + SUB - 1, W - 1) && y0 <= qy0 &&
                         y1 >= min(qy0 + SUB - 1, H - 1);
      bool full = false;
      if (hit) {
        // d = centre - pixel centre over the pixel centres of the overlap
        const float g = box_min_quadratic(ga, gb, gc, ia, ic, cx - ((float)xhi + 0.5f),
                                          cx - ((float)xlo + 0.5f), cy - ((float)yhi + 0.5f),
                                          cy - ((float)ylo + 0.5f));
        full = !(g > thr);
      }
      const uint64_t m = __ballot(hit), mf = __ballot(full), mc = __ballot(cover);
      if (lane == 0) {
        s_mask[w][wave] = m;
        s_full[w][wave] = mf;
        s_cover[w][wave] = mc;
      }
    }
    __syncthreads();
    if (!alive) continue;
    for (int g = 0; g < NW && alive; ++g) {
      uint64_t m = wave_uniform_u64(s_mask[wave][g]);
      const uint64_t mfull = wave_uniform_u64(s_full[wave][g]);
      const uint64_t mcov = wave_uniform_u64(s_cover[wave][g]);
      while (m) {
        // Records out of reach of the ellipse before the next one that may
        // contribute: no pixel can pass alpha_min, so only the evaluation
        // count of in-rectangle live pixels moves.  Those whose rectangle
        // holds the whole sub-tile are only counted; the others are tested
        // per pixel, in a loop of their own: the blend state flows through
        // this loop alone.
        const uint64_t mf = m & mfull;
        const uint64_t cheap = mf ? (m & ((mf & (~mf + 1ull)) - 1ull)) : m;
        m &= ~cheap;
        if constexpr (STATS) {
          ncov += (uint32_t)__popcll(cheap & mcov);
          uint64_t cpart = cheap & ~mcov;
          while (cpart) {
            const int kc = g * 64 + __builtin_ctzll(cpart);
            cpart &= cpart - 1;
            const float4 bc = s_b[kc];
            const uint32_t clo = __float_as_uint(bc.z), chi = __float_as_uint(bc.w);
            const int cx0 = (int)(clo & 0xffffu), cy0 = (int)(clo >> 16);
            const bool cin = (uint32_t)(px - cx0) <= (uint32_t)((int)(chi & 0xffffu) - cx0);
            const uint32_t cspan = (uint32_t)((int)(chi >> 16) - cy0);
#pragma unroll
            for (int q = 0; q < PPT; ++q)
              evals[q] += (lane_in(lm[q]) & cin & ((uint32_t)(py[q] - cy0) <= cspan)) ? 1u : 0u;
          }
        }
        if (!m) break;
        const int bit = __builtin_ctzll(m);
        const int k = g * 64 + bit;
        m &= m - 1;
        const float4 a = s_a[k], b = s_b[k], c = s_c[k];
        const uint32_t pos = b0 + (uint32_t)k + 1u - begin;
        const float dx = a.x - xc;
        // the exponent's per-column part (same operations as gs_exponent)
        const float P = (a.z * dx) * dx, R = a.w * dx;
        // One record over the lane's pixels.  inr[q]: the pixel is live and
        // inside the record's rectangle (where the rectangle holds the
        // sub-tile, liveness alone).  The two cases differ in these masks
        // only, so the blend state has a single update path.
        const bool cov = (mcov >> bit) & 1ull;   // uniform
        uint64_t inr[PPT];
        if (cov) {
          if constexpr (STATS) ++ncov;
#pragma unroll
          for (int q = 0; q < PPT; ++q) inr[q] = lm[q];
        } else {
          const uint32_t lo = __float_as_uint(b.z), hi = __float_as_uint(b.w);
          const int rx0 = (int)(lo & 0xffffu), ry0 = (int)(lo >> 16);
          const uint64_t inx =
              wave_mask((uint32_t)(px - rx0) <= (uint32_t)((int)(hi & 0xffffu) - rx0));
          const uint32_t ry_span = (uint32_t)((int)(hi >> 16) - ry0);
#pragma unroll
          for (int q = 0; q < PPT; ++q)
            inr[q] = lm[q] & inx & wave_mask((uint32_t)(py[q] - ry0) <= ry_span);
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
#pragma clang fp contract(off)   // T - w0 rounded once, the same in test and update
          const float dy = a.y - yc[q];
          const float qq = fmaf(dy, fmaf(b.x, dy, R), P);
          const float e = __builtin_amdgcn_exp2f(qq);
          const float al = fminf(b.y * e, aclamp);
          // w0 = alpha T is the contribution's weight and T - w0 the new
          // transmittance: every state update below is then in place
          const float w0 = al * T[q];
          const float Tn = T[q] - w0;
          // the decisions as wave masks: each comparison is one vector
          // instruction, their combinations scalar ones
          const uint64_t ok0 = inr[q] & wave_mask(al >= amin);
          const uint64_t stop = ok0 & wave_mask(Tn < tmin);
          const uint64_t okm = ok0 & ~stop;
          lm[q] &= ~stop;
          const bool ok = lane_in(okm);
          if constexpr (STATS) {
            stopcov[q] = lane_in(stop) ? ncov : stopcov[q];
            last[q] = ok ? pos : last[q];
            if (!cov) evals[q] += lane_in(inr[q]) ? 1u : 0u;
          }
          const float wgt = ok ? w0 : 0.0f;
          C0[q] = fmaf(c.x, wgt, C0[q]);
          C1[q] = fmaf(c.y, wgt, C1[q]);
          C2[q] = fmaf(c.z, wgt, C2[q]);
          D[q] = fmaf(c.w, wgt, D[q]);
          T[q] -= wgt;
          cnt[q] = count_lanes(cnt[q], okm);
        }
        if (!any_live()) {
          alive = false;
          break;
        }
      }
    }
  }
  // sub-tile-holding records: up to its stop, or all of them
#pragma unroll
  for (int q = 0; q < PPT; ++q)
    if constexpr (STATS) evals[q] += lane_in(lm[q]) ? ncov : stopcov[q];
  const int64_t plane = (int64_t)W * H;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    if (px >= W || py[q] >= H) continue;
    const int64_t off = (int64_t)py[q] * W + px;
    const int64_t pix = (int64_t)v * plane + off;
    float* rgb = out_rgb + (int64_t)v * 3 * plane + off;
    rgb[0] = C0[q] + T[q] * o.bg[0];
    rgb[plane] = C1[q] + T[q] * o.bg[1];
    rgb[2 * plane] = C2[q] + T[q] * o.bg[2];
    out_depth[pix] = D[q];
    out_t[pix] = T[q];
    out_n[pix] = cnt[q];
    if constexpr (STATS) {
      out_last[pix] = last[q];
      out_evals[pix] = evals[q];
    }
  }
}

// Sub-tile edge per tile size: 16x16 sub-tiles (4 pixels per lane) for
// 32-pixel tiles, 8x8 (one pixel per lane) below.
template <int TILE, bool STATS>
void launch_blend_t(const RenderWs& L, void* ws, int64_t n, const uint32_t* order,
                         const KViews& kv, const GsOpt& o, float* rgb, float* depth, float* tf,
                         int32_t* nc, hipStream_t st) {
  constexpr int SUB = TILE == 32 ? 16 : 8;
  const uint32_t* ids = at<uint32_t>(ws, L.ids);
  hipLaunchKernelGGL((k_gs_blend<TILE, SUB, STATS>), dim3((unsigned)L.tiles_total),
                     dim3(BlendCfg<TILE, SUB>::BLOCK), 0, st, order, ids, at<float4>(ws, L.rec), n,
                     kv, o, L.tiles_x, L.tiles_x * L.tiles_y, at<uint2>(ws, L.ranges), rgb, depth,
                     tf, nc, at<uint32_t>(ws, L.last), at<uint32_t>(ws, L.evals));
}

void launch_gs_blend(bool stats, const RenderWs& L, void* ws, int64_t n, const uint32_t* order,
                     const KViews& kv, const GsOpt& o, float* rgb, float* depth, float* tf,
                     int32_t* nc, hipStream_t st) {
  switch (o.tile * 2 + (stats ? 1 : 0)) {
    case 16: launch_blend_t<8, false>(L, ws, n, order, kv, o, rgb, depth, tf, nc, st); break;
    case 17: launch_blend_t<8, true>(L, ws, n, order, kv, o, rgb, depth, tf, nc, st); break;
    case 32: launch_blend_t<16, false>(L, ws, n, order, kv, o, rgb, depth, tf, nc, st); break;
    case 33: launch_blend_t<16, true>(L, ws, n, order, kv, o, rgb, depth, tf, nc, st); break;
    case 65: launch_blend_t<32, true>(L, ws, n, order, kv, o, rgb, depth, tf, nc, st); break;
    default: launch_blend_t<32, false>(L, ws, n, order, kv, o, rgb, depth, tf, nc, st); break;
  }
}


}  // namespace vrs
