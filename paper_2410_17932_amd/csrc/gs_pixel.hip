// Periphery in per-pixel order (Sec. 3.2: Gaussian contributions sorted per
// pixel instead of per primitive, the sorting of Radl and Steiner et al. that
// removes popping).  The depth of Gaussian g at pixel p is the camera depth
// z* of the maximum of g's 3D density along the ray through p's centre:
// with the camera-space mean mu, camera-space precision M and the ray
// direction d = (u, v, 1), z* = (d^T M mu) / (d^T M d).  Each pixel blends its
// Gaussians in (z*, index) order, and Eq. 1 accumulates z*.
//
// The exact per-pixel order without per-pixel lists:
//   k_gs_pixdepth   per (view, Gaussian): the key's coefficients in single
//                   precision (the order decision, in a documented operation
//                   order) and z_lo, a lower bound of the key over every
//                   pixel of the Gaussian's rectangle; z_lo replaces the
//                   depth-sort key, so each tile list comes out in z_lo order
//   k_gs_blend_px   one lane per pixel keeps a sorted window of its pending
//                   contributions (key, index, alpha); before record j is
//                   considered, every pending entry with key below z_lo(j)
//                   precedes all later records (their keys are at least
//                   their z_lo, which is at least z_lo(j)) and is blended.  A
//                   pixel whose window fills up with no entry so released
//                   has its order unresolved: it is queued
//   k_gs_blend_px_fix  one wave per queued pixel redoes it exactly: each
//                   round selects the least (key, index) above the last one
//                   over the pixel's whole tile list
// The adjoint is not provided for this order.
#include "gs_layout.h"

namespace vrs {

constexpr int kPxWindow = 16;   // pending contributions per pixel

// order-preserving unsigned image of a float, and back
__device__ inline uint32_t f2ord(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ord2f(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ inline float dot3f(float a0, float a1, float a2, float b0, float b1, float b2) {
#pragma clang fp contract(off)
  float s = a0 * b0;
  s = s + a1 * b1;
  return s + a2 * b2;
}

// Key coefficients (m00, 2 m01, 2 m02, m11, 2 m12, m22, b0, b1, b2), b = M mu,
// in single precision: Sigma^-1 by cofactors over ((s00 c00 + s01 c01) +
// s02 c02), Q = R Sigma^-1, M_ij = Q_i . R_j, b_i = M_i . mu.  A non-positive
// or non-finite determinant gives the mean depth at every pixel.
__device__ inline void pix_coef32(const KView& cv, const float t[3], const float* s, float* k) {
#pragma clang fp contract(off)
  const float c00 = s[3] * s[5] - s[4] * s[4], c01 = s[2] * s[4] - s[1] * s[5];
  const float c02 = s[1] * s[4] - s[2] * s[3], c11 = s[0] * s[5] - s[2] * s[2];
  const float c12 = s[1] * s[2] - s[0] * s[4], c22 = s[0] * s[3] - s[1] * s[1];
  float det = s[0] * c00;
  det = det + s[1] * c01;
  det = det + s[2] * c02;
  if (!(det > 0.0f) || !isfinite(det)) {
    for (int q = 0; q < 9; ++q) k[q] = 0.0f;
    k[5] = 1.0f;
    k[8] = t[2];
    return;
  }
  const float id = 1.0f / det;
  const float P[3][3] = {{c00 * id, c01 * id, c02 * id},
                         {c01 * id, c11 * id, c12 * id},
                         {c02 * id, c12 * id, c22 * id}};
  float Q[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int q = 0; q < 3; ++q)
      Q[a][q] = dot3f(cv.R[3 * a], cv.R[3 * a + 1], cv.R[3 * a + 2], P[0][q], P[1][q], P[2][q]);
  float M[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b)
      M[a][b] = dot3f(Q[a][0], Q[a][1], Q[a][2], cv.R[3 * b], cv.R[3 * b + 1], cv.R[3 * b + 2]);
  k[0] = M[0][0];
  k[1] = 2.0f * M[0][1];
  k[2] = 2.0f * M[0][2];
  k[3] = M[1][1];
  k[4] = 2.0f * M[1][2];
  k[5] = M[2][2];
  k[6] = dot3f(M[0][0], M[0][1], M[0][2], t[0], t[1], t[2]);
  k[7] = dot3f(M[0][1], M[1][1], M[1][2], t[0], t[1], t[2]);
  k[8] = dot3f(M[0][2], M[1][2], M[2][2], t[0], t[1], t[2]);
}

// Ray coordinates of a pixel-centre coordinate: ((x + 0.5) - c) / f.
__device__ inline float pix_ray(int x, float c, float f) {
#pragma clang fp contract(off)
  return (((float)x + 0.5f) - c) / f;
}

// Numerator and denominator of the key at ray coordinates (u, v), with the
// coefficients staged as q0 = (m00, 2m01, 2m02, m11), q1 = (2m12, m22, b0,
// b1), q2 = (b2, z_lo, -, -).
__device__ inline void pix_numden(const float4& q0, const float4& q1, const float4& q2, float u,
                                  float v, float& num, float& den) {
#pragma clang fp contract(off)
  num = q1.z * u;
  num = num + q1.w * v;
  num = num + q2.x;
  float a = q0.x * u;
  a = a + q0.y * v;
  a = a + q0.z;
  float b = q0.w * v;
  b = b + q1.x;
  den = a * u;
  den = den + b * v;
  den = den + q1.y;
}

__device__ inline uint32_t pix_key_bits(const float4& q0, const float4& q1, const float4& q2,
                                        float u, float v) {
  float num, den;
  pix_numden(q0, q1, q2, u, v, num, den);
  return f2ord(num / den);
}

// Coefficients and the sort key z_lo of every (view, Gaussian) entry the
// preprocess kept (its depth key is replaced; culled entries keep theirs).
// z_lo: the numerator is linear in (u, v) and the denominator a convex
// quadratic, so over the box of the rectangle's pixel centres the key is at
// least (least corner numerator) / (largest corner denominator) when that
// numerator is positive (else no bound: -inf); it is lowered by 2^-12 of
// itself, far above the rounding of either side.  Thread 0 also clears the
// count of pixels queued for the exact pass.
__global__ __launch_bounds__(256) void k_gs_pixdepth(const float* __restrict__ mean,
                                                     const float* __restrict__ cov, int64_t n,
                                                     KViews views,
                                                     const float4* __restrict__ rec,
                                                     uint32_t* __restrict__ dkey,
                                                     float4* __restrict__ pcoef,
                                                     uint32_t* __restrict__ fix_count) {
  const int64_t vn = n * views.n;
  if (blockIdx.x == 0 && threadIdx.x == 0) *fix_count = 0u;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < vn;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (dkey[e] == 0xffffffffu) {   // culled by the preprocess
      pcoef[3 * e] = pcoef[3 * e + 1] = pcoef[3 * e + 2] = make_float4(0, 0, 0, 0);
      continue;
    }
    const int v = (int)(e / n);
    const int64_t i = e - (int64_t)v * n;
    const KView& cv = views.v[v];
    float t[3];
    {
#pragma clang fp contract(off)
      const float mx = mean[i], my = mean[n + i], mz = mean[2 * n + i];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        float p = cv.R[3 * a + 0] * mx;
        float q = cv.R[3 * a + 1] * my;
        float s = p + q;
        float r = cv.R[3 * a + 2] * mz;
        s = s + r;
        t[a] = s + cv.t[a];
      }
    }
    float s6[6], k[9];
#pragma unroll
    for (int q = 0; q < 6; ++q) s6[q] = cov[q * n + i];
    pix_coef32(cv, t, s6, k);
    const float4 q0 = make_float4(k[0], k[1], k[2], k[3]);
    const float4 q1 = make_float4(k[4], k[5], k[6], k[7]);
    const float4 r2 = rec[3 * e + 2];
    const uint32_t lo = __float_as_uint(r2.z), hi = __float_as_uint(r2.w);
    const float u0 = pix_ray((int)(lo & 0xffffu), cv.cx, cv.fx);
    const float u1 = pix_ray((int)(hi & 0xffffu), cv.cx, cv.fx);
    const float v0 = pix_ray((int)(lo >> 16), cv.cy, cv.fy);
    const float v1 = pix_ray((int)(hi >> 16), cv.cy, cv.fy);
    float nmin = 3.0e38f, dmax = -3.0e38f;
    const float us[2] = {u0, u1}, vs[2] = {v0, v1};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        float num, den;
        pix_numden(q0, q1, make_float4(k[8], 0, 0, 0), us[a], vs[b], num, den);
        nmin = fminf(nmin, num);
        dmax = fmaxf(dmax, den);
      }
    float zlo = -INFINITY;
    if (nmin > 0.0f && dmax > 0.0f && isfinite(nmin) && isfinite(dmax)) {
      zlo = nmin / dmax;
      zlo = zlo - zlo * 0x1p-12f;
    }
    pcoef[3 * e] = q0;
    pcoef[3 * e + 1] = q1;
    pcoef[3 * e + 2] = make_float4(k[8], zlo, 0.0f, 0.0f);
    dkey[e] = f2ord(zlo);
  }
}

// A lane's pending contributions, ascending in (key bits << 32 | index),
// with their alphas; free slots hold ~0.  Fixed-size and fully unrolled so
// that it stays in registers.
template <int K>
struct PxWindow {
  // vector types are register values (element access needs no memory)
  typedef unsigned long long KeyV __attribute__((ext_vector_type(K)));
  typedef float AlphaV __attribute__((ext_vector_type(K)));
  KeyV k;
  AlphaV a;
  int n;
  __device__ __attribute__((always_inline)) void clear() {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      k[q] = ~0ull;
      a[q] = 0.0f;
    }
    n = 0;
  }
  // drop the first entry where `go`
  __device__ __attribute__((always_inline)) void shift(bool go) {
#pragma unroll
    for (int q = 0; q < K - 1; ++q) {
      k[q] = go ? k[q + 1] : k[q];
      a[q] = go ? a[q + 1] : a[q];
    }
    k[K - 1] = go ? ~0ull : k[K - 1];
    n -= go ? 1 : 0;
  }
  // insert into a window with a free slot: one compare-exchange pass
  __device__ __attribute__((always_inline)) void insert(uint64_t key, float al) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const bool lt = key < k[q];
      const uint64_t tk = lt ? k[q] : key;
      const float ta = lt ? a[q] : al;
      k[q] = lt ? key : k[q];
      a[q] = lt ? al : a[q];
      key = tk;
      al = ta;
    }
    ++n;
  }
};

template <int TILE>
struct PxCfg {
  static constexpr int NQ = TILE / 8;     // 8x8 sub-tiles per side, one wave each
  static constexpr int NW = NQ * NQ;
  static constexpr int BLOCK = 64 * NW;
};

// One workgroup per tile in the longest-first schedule, one wave per 8x8
// sub-tile, one pixel per lane.  Records are staged in batches with a ballot
// per sub-tile of those whose rectangle reaches it.  A lane's window holds
// (key bits << 32 | index) ascending with the contribution's alpha; free
// slots hold ~0.
template <int TILE>
__global__ __launch_bounds__(PxCfg<TILE>::BLOCK) void k_gs_blend_px(
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ ids,
    const float4* __restrict__ rec, const float4* __restrict__ pcoef, int64_t n, KViews views,
    GsOpt o, int64_t tiles_x, int64_t tiles_per_view, const uint2* __restrict__ ranges,
    float* __restrict__ out_rgb, float* __restrict__ out_depth, float* __restrict__ out_t,
    int32_t* __restrict__ out_n, uint32_t* __restrict__ fix_list,
    uint32_t* __restrict__ fix_count) {
  using Cfg = PxCfg<TILE>;
  constexpr int BLOCK = Cfg::BLOCK, NW = Cfg::NW, NQ = Cfg::NQ, K = kPxWindow;
  __shared__ float4 s_a[BLOCK], s_b[BLOCK], s_q0[BLOCK], s_q1[BLOCK], s_q2[BLOCK];
  __shared__ uint32_t s_id[BLOCK];
  __shared__ uint64_t s_mask[NW][NW];
  const int64_t tglob = order[blockIdx.x];
  const int v = (int)(tglob / tiles_per_view);
  const int64_t tl = tglob - (int64_t)v * tiles_per_view;
  const int ty = (int)(tl / tiles_x), tx = (int)(tl - (int64_t)ty * tiles_x);
  const KView& cv = views.v[v];
  const int W = cv.W, H = cv.H;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int px = tx * TILE + (wave % NQ) * 8 + (lane & 7);
  const int py = ty * TILE + (wave / NQ) * 8 + (lane >> 3);
  const float xc = (float)px + 0.5f, yc = (float)py + 0.5f;
  const float ur = pix_ray(px, cv.cx, cv.fx), vr = pix_ray(py, cv.cy, cv.fy);
  const float aclamp = o.aclamp, amin = o.amin, tmin = o.tmin;
  bool alive = px < W && py < H;
  bool inexact = false;
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D = 0.0f;
  int cnt = 0;
  PxWindow<K> win;
  win.clear();
  // blend the window's first entry (lanes where `go`), then shift it out
  auto pop = [&](bool go) __attribute__((always_inline)) {
    if (go) {
      const uint32_t gi = (uint32_t)win.k[0];
      const int64_t e = (int64_t)v * n + gi;
      const float4 r1 = rec[3 * e + 1], r2 = rec[3 * e + 2];
      const float w0 = win.a[0] * T;
      const float Tn = T - w0;
      if (Tn < tmin) {
        alive = false;   // stops before this contribution; the rest is moot
      } else {
        C0 = fmaf(r1.z, w0, C0);
        C1 = fmaf(r1.w, w0, C1);
        C2 = fmaf(r2.x, w0, C2);
        D = fmaf(ord2f((uint32_t)(win.k[0] >> 32)), w0, D);
        T = Tn;
        ++cnt;
      }
    }
    win.shift(go);
  };
  const uint2 rg = ranges[tglob];
  const uint32_t begin = rg.x, end = rg.y;
  for (uint32_t b0 = begin; b0 < end; b0 += BLOCK) {
    if (__syncthreads_count(alive) == 0) break;
    const uint32_t jr = b0 + tid;
    const bool has = jr < end;
    int x0 = 1, x1 = 0, y0 = 1, y1 = 0;
    if (has) {
      const uint32_t id = ids[jr];
      const int64_t e = (int64_t)v * n + (id < (uint64_t)n ? id : 0);
      float4 a, b, c;
      gs_stage(rec, e, a, b, c);
      s_a[tid] = a;
      s_b[tid] = b;
      s_q0[tid] = pcoef[3 * e];
      s_q1[tid] = pcoef[3 * e + 1];
      s_q2[tid] = pcoef[3 * e + 2];
      s_id[tid] = id;
      const uint32_t lo = __float_as_uint(b.z), hi = __float_as_uint(b.w);
      x0 = (int)(lo & 0xffffu); y0 = (int)(lo >> 16);
      x1 = (int)(hi & 0xffffu); y1 = (int)(hi >> 16);
    }
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int qx0 = tx * TILE + (w % NQ) * 8, qy0 = ty * TILE + (w / NQ) * 8;
      const bool hit = has && max(x0, qx0) <= min(x1, qx0 + 7) && max(y0, qy0) <= min(y1, qy0 + 7);
      const uint64_t m = __ballot(hit);
      if (lane == 0) s_mask[w][wave] = m;
    }
    __syncthreads();
    for (int g = 0; g < NW; ++g) {
      uint64_t m = s_mask[wave][g];
      while (m && __ballot(alive)) {
        const int k = g * 64 + __builtin_ctzll(m);
        m &= m - 1;
        const float4 q2 = s_q2[k];
        const uint32_t zlo = f2ord(q2.y);
        // pending entries below this record's bound precede every later one
        while (true) {
          const bool go = alive && win.n > 0 && (uint32_t)(win.k[0] >> 32) < zlo;
          if (!__ballot(go)) break;
          pop(go);
        }
        const float4 a = s_a[k], b = s_b[k];
        const uint32_t lo = __float_as_uint(b.z), hi = __float_as_uint(b.w);
        const bool inr = alive && px >= (int)(lo & 0xffffu) && px <= (int)(hi & 0xffffu) &&
                         py >= (int)(lo >> 16) && py <= (int)(hi >> 16);
        const float dx = a.x - xc, dy = a.y - yc;
        const float P = (a.z * dx) * dx, R = a.w * dx;
        const float qq = fmaf(dy, fmaf(b.x, dy, R), P);
        const float al = fminf(b.y * __builtin_amdgcn_exp2f(qq), aclamp);
        const bool ok = inr && al >= amin;
        if (ok) {
          const uint64_t key = ((uint64_t)pix_key_bits(s_q0[k], s_q1[k], q2, ur, vr) << 32) |
                               s_id[k];
          // a full window must release its least entry before it is known
          // to be the next: the pixel is redone exactly
          const bool full = win.n == K;
          if (full && !((uint32_t)(win.k[0] >> 32) < zlo)) inexact = true;
          if (full) pop(true);
          if (alive) win.insert(key, al);
        }
      }
    }
  }
  // the rest of the window, in order
  while (true) {
    const bool go = alive && win.n > 0;
    if (!__ballot(go)) break;
    pop(go);
  }
  if (px < W && py < H) {
    const int64_t plane = (int64_t)W * H;
    const int64_t off = (int64_t)py * W + px;
    float* rgb = out_rgb + (int64_t)v * 3 * plane + off;
    rgb[0] = C0 + T * o.bg[0];
    rgb[plane] = C1 + T * o.bg[1];
    rgb[2 * plane] = C2 + T * o.bg[2];
    out_depth[(int64_t)v * plane + off] = D;
    out_t[(int64_t)v * plane + off] = T;
    out_n[(int64_t)v * plane + off] = cnt;
    if (inexact) fix_list[atomicAdd(fix_count, 1u)] = (uint32_t)((int64_t)v * plane + off);
  }
}

// Exact per-pixel order for the queued pixels: one wave per pixel; every
// round the lanes scan the pixel's tile list for the least (key, index) above
// the last blended one, reduce it over the wave and blend it, until the pixel
// stops or no contribution is left.
__global__ __launch_bounds__(256) void k_gs_blend_px_fix(
    const uint32_t* __restrict__ fix_list, const uint32_t* __restrict__ fix_count,
    const uint32_t* __restrict__ ids, const float4* __restrict__ rec,
    const float4* __restrict__ pcoef, int64_t n, KViews views, GsOpt o, int tile,
    int64_t tiles_x, int64_t tiles_per_view, const uint2* __restrict__ ranges,
    float* __restrict__ out_rgb, float* __restrict__ out_depth, float* __restrict__ out_t,
    int32_t* __restrict__ out_n) {
  const int lane = threadIdx.x & 63;
  const uint32_t nfix = *fix_count;
  for (uint32_t f = blockIdx.x * 4u + (threadIdx.x >> 6); f < nfix; f += gridDim.x * 4u) {
    const int64_t pix = fix_list[f];
    const KView& cv0 = views.v[0];
    const int64_t plane = (int64_t)cv0.W * cv0.H;
    const int v = (int)(pix / plane);
    const int64_t off = pix - (int64_t)v * plane;
    const KView& cv = views.v[v];
    const int py = (int)(off / cv.W), px = (int)(off - (int64_t)py * cv.W);
    const float xc = (float)px + 0.5f, yc = (float)py + 0.5f;
    const float ur = pix_ray(px, cv.cx, cv.fx), vr = pix_ray(py, cv.cy, cv.fy);
    const uint2 rg = ranges[(int64_t)v * tiles_per_view + (int64_t)(py / tile) * tiles_x + px / tile];
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D = 0.0f;
    int cnt = 0;
    uint64_t last = 0;
    bool first = true;
    while (true) {
      uint64_t best = ~0ull;
      float best_al = 0.0f;
      for (uint32_t j = rg.x + lane; j < rg.y; j += 64) {
        const uint32_t id = ids[j];
        const int64_t e = (int64_t)v * n + id;
        float4 a, b, c;
        gs_stage(rec, e, a, b, c);
        const uint32_t lo = __float_as_uint(b.z), hi = __float_as_uint(b.w);
        if (!(px >= (int)(lo & 0xffffu) && px <= (int)(hi & 0xffffu) && py >= (int)(lo >> 16) &&
              py <= (int)(hi >> 16)))
          continue;
        const float dx = a.x - xc, dy = a.y - yc;
        const float P = (a.z * dx) * dx, R = a.w * dx;
        const float qq = fmaf(dy, fmaf(b.x, dy, R), P);
        const float al = fminf(b.y * __builtin_amdgcn_exp2f(qq), o.aclamp);
        if (!(al >= o.amin)) continue;
        const uint64_t key =
            ((uint64_t)pix_key_bits(pcoef[3 * e], pcoef[3 * e + 1], pcoef[3 * e + 2], ur, vr)
             << 32) | id;
        if ((first || key > last) && key < best) {
          best = key;
          best_al = al;
        }
      }
      uint64_t mn = best;
#pragma unroll
      for (int s = 32; s > 0; s >>= 1) {
        const uint64_t y = __shfl_xor(mn, s, 64);
        mn = y < mn ? y : mn;
      }
      if (mn == ~0ull) break;   // wave-uniform
      const uint64_t holders = __ballot(best == mn);
      const float al = __shfl(best_al, __builtin_ctzll(holders), 64);
      const int64_t e = (int64_t)v * n + (uint32_t)mn;
      const float4 r1 = rec[3 * e + 1], r2 = rec[3 * e + 2];
      const float w0 = al * T;
      const float Tn = T - w0;
      if (Tn < o.tmin) break;
      C0 = fmaf(r1.z, w0, C0);
      C1 = fmaf(r1.w, w0, C1);
      C2 = fmaf(r2.x, w0, C2);
      D = fmaf(ord2f((uint32_t)(mn >> 32)), w0, D);
      T = Tn;
      ++cnt;
      last = mn;
      first = false;
    }
    if (lane == 0) {
      float* rgb = out_rgb + (int64_t)v * 3 * plane + off;
      rgb[0] = C0 + T * o.bg[0];
      rgb[plane] = C1 + T * o.bg[1];
      rgb[2 * plane] = C2 + T * o.bg[2];
      out_depth[(int64_t)v * plane + off] = D;
      out_t[(int64_t)v * plane + off] = T;
      out_n[(int64_t)v * plane + off] = cnt;
    }
  }
}

void launch_gs_pixdepth(const RenderWs& L, void* ws, const float* mean, const float* cov,
                        int64_t n, const KViews& kv, hipStream_t st) {
  const int64_t vn = L.vn;
  hipLaunchKernelGGL(k_gs_pixdepth, dim3((unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, div_up(vn, 256)))),
                     dim3(256), 0, st, mean, cov, n, kv, at<float4>(ws, L.rec),
                     at<uint32_t>(ws, L.dkey0), at<float4>(ws, L.pcoef),
                     at<uint32_t>(ws, L.fix_count));
}

void launch_gs_blend_px(const RenderWs& L, void* ws, int64_t n, const uint32_t* order,
                        const KViews& kv, const GsOpt& o, float* rgb, float* depth, float* tf,
                        int32_t* nc, hipStream_t st) {
  const uint32_t* ids = at<uint32_t>(ws, L.ids);
  const float4* rec = at<float4>(ws, L.rec);
  const float4* pc = at<float4>(ws, L.pcoef);
  const uint2* ranges = at<uint2>(ws, L.ranges);
  uint32_t* fl = at<uint32_t>(ws, L.fix_list);
  uint32_t* fc = at<uint32_t>(ws, L.fix_count);
  const int64_t tpv = L.tiles_x * L.tiles_y;
  switch (o.tile) {
    case 8:
      hipLaunchKernelGGL(k_gs_blend_px<8>, dim3((unsigned)L.tiles_total), dim3(PxCfg<8>::BLOCK),
                         0, st, order, ids, rec, pc, n, kv, o, L.tiles_x, tpv, ranges, rgb, depth,
                         tf, nc, fl, fc);
      break;
    case 16:
      hipLaunchKernelGGL(k_gs_blend_px<16>, dim3((unsigned)L.tiles_total), dim3(PxCfg<16>::BLOCK),
                         0, st, order, ids, rec, pc, n, kv, o, L.tiles_x, tpv, ranges, rgb, depth,
                         tf, nc, fl, fc);
      break;
    default:
      hipLaunchKernelGGL(k_gs_blend_px<32>, dim3((unsigned)L.tiles_total), dim3(PxCfg<32>::BLOCK),
                         0, st, order, ids, rec, pc, n, kv, o, L.tiles_x, tpv, ranges, rgb, depth,
                         tf, nc, fl, fc);
      break;
  }
  hipLaunchKernelGGL(k_gs_blend_px_fix, dim3(1024), dim3(256), 0, st, fl, fc, ids, rec, pc, n, kv,
                     o, o.tile, L.tiles_x, tpv, ranges, rgb, depth, tf, nc);
}

}  // namespace vrs
