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
//                   order) and a lower bound of the key over the Gaussian's
//                   rectangle, which replaces the depth-sort key (only an
//                   initial order: the tile lists are sorted again)
//   k_gs_tile_zsort per tile: bound words for the list positions (see
//                   zs_word), the first kZsPrefix records sorted by z_t, a
//                   rigorous lower bound of the single-precision key over
//                   the tile's pixels
//   k_gs_blend_px   one lane per pixel keeps a sorted window of its pending
//                   contributions (key, index, alpha, colour).  Before record
//                   j is considered, a pending entry whose key is below
//                   every later record's least key over the 8x8 sub-tile
//                   precedes all of them and is blended.  At tile 8 that
//                   bound is j's bound word; with several sub-tiles, per
//                   staged batch, a suffix minimum of exact sub-tile minima
//                   (one wave minimum per record), closed by the bound word
//                   of the next batch's first position.  A pixel whose window fills
//                   up with no entry so released has its order unresolved:
//                   it is queued
//   k_gs_blend_px_fix  one wave per queued pixel redoes it exactly, in
//                   rounds of streaming selection of the least keys above
//                   the last blended one (scans cut off by the bound words)
// The adjoint is not provided for this order.
#include "gs_layout.h"

namespace vrs {

constexpr int kPxWindow = 20;   // pending contributions per pixel
constexpr int kPxRing = 1024;   // records whose colours stay in LDS

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
// b1), q2 = (b2, z_lo, -, -) with z_lo the bound below over the Gaussian's
// whole rectangle.
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

// A lower bound of the single-precision key over every pixel centre of the
// box [x0, x1] x [y0, y1] (-inf where none is proven).
//   The exact numerator N is linear in the ray coordinates (u, v) and the
//   exact denominator D a quadratic, convex when its 2x2 part is positive
//   definite (checked with a margin).  The evaluation order of the key
//   rounds N by at most An = 8 eps sum|terms| and D by at most Bd = 16 eps
//   sum|terms| (eps = 2^-24; three and six roundings deep), the sums taken
//   at the largest |u| and |v| of the box, so wherever N - An > 0 and
//   D - Bd > 0 the key is at least f = (N - An) / (D + Bd) (1 - eps).  For
//   c > 0, (N - An) - c (D + Bd) is concave, so its least value over the box
//   is at a corner: f is least at a corner, and the corners are pixel
//   centres.  Positivity: N's least value is at a corner; D is at least its
//   tangent plane at the (u0, v0) corner, least at one of the box's ends.  Corner values are computed with
//   2 An and 2 Bd to cover their own rounding, and the result is lowered by
//   2^-20 of itself, which covers the last few roundings.  Ray coordinates
//   round monotonically, so every pixel's (u, v) lies in the corners' box.
__device__ inline float pix_box_bound_uv(const float4& q0, const float4& q1, const float4& q2,
                                         float u0, float u1, float v0, float v1) {
#pragma clang fp contract(off)
  const float m00 = q0.x, m01 = 0.5f * q0.y, m11 = q0.w;
  const float pd = m00 * m11, od = m01 * m01;
  if (!(m00 > 0.0f) || !(m11 > 0.0f) || !(pd > od * (1.0f + 0x1p-20f)) || !isfinite(pd))
    return -INFINITY;
  const float U = fmaxf(fabsf(u0), fabsf(u1)), V = fmaxf(fabsf(v0), fabsf(v1));
  const float nabs = (fabsf(q1.z) * U + fabsf(q1.w) * V) + fabsf(q2.x);
  const float dabs = ((fabsf(q0.x) * U + fabsf(q0.y) * V) + fabsf(q0.z)) * U +
                     (fabsf(q0.w) * V + fabsf(q1.x)) * V + fabsf(q1.y);
  const float An = 0x1p-21f * nabs, Bd = 0x1p-20f * dabs;
  // tangent plane of D at (u0, v0) over the box
  const float du = (u1 - u0) * (1.0f + 0x1p-20f), dv = (v1 - v0) * (1.0f + 0x1p-20f);
  float n00, d00;
  pix_numden(q0, q1, q2, u0, v0, n00, d00);
  const float gu = ((2.0f * q0.x) * u0 + q0.y * v0) + q0.z;
  const float gv = (q0.y * u0 + (2.0f * q0.w) * v0) + q1.x;
  const float dlb = (d00 + fminf(gu * du, 0.0f)) + fminf(gv * dv, 0.0f);
  const float dlb_abs =
      (dabs + (((2.0f * fabsf(q0.x)) * U + fabsf(q0.y) * V) + fabsf(q0.z)) * fabsf(du)) +
      ((fabsf(q0.y) * U + (2.0f * fabsf(q0.w)) * V) + fabsf(q1.x)) * fabsf(dv);
  if (!(dlb - 0x1p-20f * dlb_abs > 2.0f * Bd) || !isfinite(dlb_abs)) return -INFINITY;
  const float us[2] = {u0, u1}, vs[2] = {v0, v1};
  float z = INFINITY;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      float num, den;
      pix_numden(q0, q1, q2, us[a], vs[b], num, den);
      const float nn = num - 2.0f * An;
      if (!(nn > 0.0f)) return -INFINITY;
      z = fminf(z, nn / (den + 2.0f * Bd));
    }
  if (!isfinite(z)) return -INFINITY;
  return z - z * 0x1p-20f;
}

__device__ inline float pix_box_bound(const float4& q0, const float4& q1, const float4& q2,
                                      const KView& cv, int x0, int x1, int y0, int y1) {
  return pix_box_bound_uv(q0, q1, q2, pix_ray(x0, cv.cx, cv.fx), pix_ray(x1, cv.cx, cv.fx),
                          pix_ray(y0, cv.cy, cv.fy), pix_ray(y1, cv.cy, cv.fy));
}

// Coefficients and the sort key of every (view, Gaussian) entry the
// preprocess kept (its depth key is replaced; culled entries keep theirs):
// z_lo, the bound above over the Gaussian's whole rectangle, so that every
// tile list comes out of the binning in z_lo order.  Thread 0 also clears
// the count of pixels queued for the exact pass.
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
    const float zlo = pix_box_bound(q0, q1, make_float4(k[8], 0.0f, 0.0f, 0.0f), cv,
                                    (int)(lo & 0xffffu), (int)(hi & 0xffffu), (int)(lo >> 16),
                                    (int)(hi >> 16));
    pcoef[3 * e] = q0;
    pcoef[3 * e + 1] = q1;
    pcoef[3 * e + 2] = make_float4(k[8], zlo, 0.0f, 0.0f);
    dkey[e] = f2ord(zlo);
  }
}

// ---------------------------------------------------------------- tile sort
// Bound words.  Every list position j gets w(j) = beta(j) << 32 | index with
// beta non-decreasing along the list and every key of every record at
// positions >= j, at every pixel of the tile in its rectangle, at least
// beta(j) (order-preserving bits throughout).  The first kZsPrefix records
// (or all) are sorted by z_t, the bound over the tile's pixel box, its bits
// rounded down to 20 (so that a 32-bit word carries it with a 12-bit slot
// in the prefix): beta = min(rounded z_t, z_lo of the first record after the
// prefix).  After the prefix the list keeps its z_lo order and beta = z_lo.
// Blending stops long before most lists end, so only the prefix is sorted; a
// pixel that reads past it still gets valid, if looser, bounds.
constexpr int kZsBlock = 256, kZsPrefix = 4096, kZsSlotBits = 12;
static_assert(kZsPrefix == 1 << kZsSlotBits, "one slot per prefix position");

__device__ inline uint64_t zs_word(const uint64_t* __restrict__ tkey,
                                   const uint32_t* __restrict__ ids,
                                   const float4* __restrict__ pcoef, int64_t vbase, uint32_t begin,
                                   uint32_t j) {
  if (j - begin < (uint32_t)kZsPrefix) return tkey[j];
  const uint32_t id = ids[j];
  return ((uint64_t)f2ord(pcoef[3 * (vbase + id) + 2].y) << 32) | id;
}

// One workgroup per tile: the prefix's words, sorted in LDS (bitonic over
// 32-bit (rounded z_t bits | slot) words).
__global__ __launch_bounds__(kZsBlock) void k_gs_tile_zsort(
    const uint32_t* __restrict__ ids, const float4* __restrict__ pcoef, int64_t n, KViews views,
    int tile, int64_t tiles_x, int64_t tiles_per_view, const uint2* __restrict__ ranges,
    uint64_t* __restrict__ out) {
  __shared__ uint32_t s[kZsPrefix];
  const int64_t tglob = blockIdx.x;
  const uint2 rg = ranges[tglob];
  const uint32_t begin = rg.x;
  const int len = (int)(rg.y - rg.x);
  if (len <= 0) return;
  const int v = (int)(tglob / tiles_per_view);
  const int64_t tl = tglob - (int64_t)v * tiles_per_view;
  const int ty = (int)(tl / tiles_x), tx = (int)(tl - (int64_t)ty * tiles_x);
  const KView& cv = views.v[v];
  const int X0 = tx * tile, Y0 = ty * tile;
  const int X1 = min(X0 + tile, cv.W) - 1, Y1 = min(Y0 + tile, cv.H) - 1;
  const float u0 = pix_ray(X0, cv.cx, cv.fx), u1 = pix_ray(X1, cv.cx, cv.fx);
  const float v0 = pix_ray(Y0, cv.cy, cv.fy), v1 = pix_ray(Y1, cv.cy, cv.fy);
  const int64_t vbase = (int64_t)v * n;
  const int m = min(len, kZsPrefix);
  uint32_t cap = 0xffffffffu;   // z_lo of the first record after the prefix
  if (len > m) cap = f2ord(pcoef[3 * (vbase + ids[begin + m]) + 2].y);
  int P = 64;
  while (P < m) P <<= 1;
  constexpr uint32_t kSlot = (1u << kZsSlotBits) - 1u;
  for (int i = threadIdx.x; i < P; i += kZsBlock) {
    uint32_t w = 0xffffffffu;
    if (i < m) {
      const int64_t e = vbase + ids[begin + i];
      const float z = pix_box_bound_uv(pcoef[3 * e], pcoef[3 * e + 1], pcoef[3 * e + 2], u0, u1,
                                       v0, v1);
      w = (f2ord(z) & ~kSlot) | (uint32_t)i;
    }
    s[i] = w;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < (P >> 1); i += kZsBlock) {
        const int a = ((i & ~(j - 1)) << 1) | (i & (j - 1)), b = a + j;
        const uint32_t x = s[a], y = s[b];
        if ((x > y) == ((a & k) == 0)) {
          s[a] = y;
          s[b] = x;
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < m; i += kZsBlock) {
    const uint32_t w = s[i];
    const uint32_t beta = min(w & ~kSlot, cap);
    out[begin + i] = ((uint64_t)beta << 32) | ids[begin + (w & kSlot)];
  }
}

// A lane's pending contributions, ascending in (key bits << 32 | index),
// with their alphas and list positions (the colour waits in the tile's LDS
// ring under the position); free slots hold ~0.  Fixed-size and fully
// unrolled so that it stays in registers.
template <int K>
struct PxWindow {
  // vector types are register values (element access needs no memory)
  typedef unsigned long long KeyV __attribute__((ext_vector_type(K)));
  typedef float AlphaV __attribute__((ext_vector_type(K)));
  typedef unsigned int PosV __attribute__((ext_vector_type(K)));
  KeyV k;
  AlphaV a;
  PosV p;
  int n;
  __device__ __attribute__((always_inline)) void clear() {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      k[q] = ~0ull;
      a[q] = 0.0f;
      p[q] = 0u;
    }
    n = 0;
  }
  // drop the first entry where `go`.  Written as masked bit moves: with
  // selects on one condition for every slot the compiler rebuilds the shift
  // as a variable-index gather, quadratic in the window size.
  __device__ __attribute__((always_inline)) void shift(bool go) {
    const uint64_t m64 = go ? ~0ull : 0ull;
    const uint32_t m32 = (uint32_t)m64;
#pragma unroll
    for (int q = 0; q < K - 1; ++q) {
      k[q] = k[q] ^ ((k[q] ^ k[q + 1]) & m64);
      const uint32_t u = __float_as_uint(a[q]);
      a[q] = __uint_as_float(u ^ ((u ^ __float_as_uint(a[q + 1])) & m32));
      p[q] = p[q] ^ ((p[q] ^ p[q + 1]) & m32);
    }
    k[K - 1] = k[K - 1] | m64;
    n -= go ? 1 : 0;
  }
  // insert into a window with a free slot.  The slots are ascending, so the
  // slots above the key are a suffix: slot q takes the key if it is the
  // first of them, its lower neighbour if it is a later one, and keeps its
  // entry otherwise (two selects per word; every index static).
  __device__ __attribute__((always_inline)) void insert(uint64_t key, float al, uint32_t pos) {
    bool above[K];
#pragma unroll
    for (int q = 0; q < K; ++q) above[q] = key < k[q];
#pragma unroll
    for (int q = K - 1; q >= 1; --q) {
      const bool take = above[q], from_left = above[q - 1];
      k[q] = take ? (from_left ? k[q - 1] : key) : k[q];
      a[q] = take ? (from_left ? a[q - 1] : al) : a[q];
      p[q] = take ? (from_left ? p[q - 1] : pos) : p[q];
    }
    k[0] = above[0] ? key : k[0];
    a[0] = above[0] ? al : a[0];
    p[0] = above[0] ? pos : p[0];
    ++n;
  }
  // least list position among the entries (~0 when empty)
  __device__ __attribute__((always_inline)) uint32_t oldest() const {
    uint32_t m = 0xffffffffu;
#pragma unroll
    for (int q = 0; q < K; ++q) m = q < n ? min(m, p[q]) : m;
    return m;
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
// (key bits << 32 | index) ascending with the contribution's alpha and list
// position (its colour is in the LDS ring); free slots hold ~0.
template <int TILE>
__global__ __launch_bounds__(PxCfg<TILE>::BLOCK) void k_gs_blend_px(
    const uint32_t* __restrict__ order, const uint64_t* __restrict__ tkey,
    const uint32_t* __restrict__ ids, const float4* __restrict__ rec, const float4* __restrict__ pcoef, int64_t n, KViews views,
    GsOpt o, int64_t tiles_x, int64_t tiles_per_view, const uint2* __restrict__ ranges,
    float* __restrict__ out_rgb, float* __restrict__ out_depth, float* __restrict__ out_t,
    int32_t* __restrict__ out_n, uint32_t* __restrict__ fix_list,
    uint32_t* __restrict__ fix_count) {
  using Cfg = PxCfg<TILE>;
  constexpr int BLOCK = Cfg::BLOCK, NW = Cfg::NW, NQ = Cfg::NQ, K = kPxWindow;
  static_assert(kPxRing % BLOCK == 0, "batches fill whole ring slots");
  __shared__ float4 s_a[BLOCK], s_b[BLOCK], s_q0[BLOCK], s_q1[BLOCK], s_q2[BLOCK];
  __shared__ float s_ring[3][kPxRing];      // colours by list position mod kPxRing
  __shared__ uint32_t s_id[BLOCK];
  __shared__ uint64_t s_mask[NW][NW];
  __shared__ uint32_t s_beta[BLOCK];         // per record: its position's bound word
  __shared__ uint32_t s_bound[NW][BLOCK];   // per sub-tile and record: release bound
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
      const float w0 = win.a[0] * T;
      const float Tn = T - w0;
      if (Tn < tmin) {
        alive = false;   // stops before this contribution; the rest is moot
      } else {
        const uint32_t slot = win.p[0] & (kPxRing - 1);
        C0 = fmaf(s_ring[0][slot], w0, C0);
        C1 = fmaf(s_ring[1][slot], w0, C1);
        C2 = fmaf(s_ring[2][slot], w0, C2);
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
    // this batch's colours overwrite the ring slots of positions b0 - kPxRing
    // onwards: a pixel still holding one of those cannot be finished here
    if (alive && win.n > 0 && win.oldest() + kPxRing < (b0 - begin) + BLOCK) {
      inexact = true;
      alive = false;
    }
    if (__syncthreads_count(alive) == 0) break;
    const uint32_t jr = b0 + tid;
    const bool has = jr < end;
    int x0 = 1, x1 = 0, y0 = 1, y1 = 0;
    if (has) {
      const uint64_t wd = zs_word(tkey, ids, pcoef, (int64_t)v * n, begin, jr);
      const uint32_t id = (uint32_t)wd;
      s_beta[tid] = (uint32_t)(wd >> 32);
      const int64_t e = (int64_t)v * n + (id < (uint64_t)n ? id : 0);
      float4 a, b, c;
      gs_stage(rec, e, a, b, c);
      s_a[tid] = a;
      s_b[tid] = b;
      const uint32_t slot = (jr - begin) & (kPxRing - 1);
      s_ring[0][slot] = c.x;
      s_ring[1][slot] = c.y;
      s_ring[2][slot] = c.z;
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
    if (!__ballot(alive)) continue;
    // Release bounds.  One sub-tile: the bound word of record k's position.
    // Several: walking this batch's records backwards, before record k every
    // later key at any pixel of the sub-tile is at least the least key of
    // records k.. of the batch over the sub-tile's pixels (a wave minimum of
    // exact keys), and at least the bound word of the next batch's first
    // position.
    if constexpr (NW > 1) {
      uint32_t bound =
          b0 + BLOCK < end
              ? (uint32_t)(zs_word(tkey, ids, pcoef, (int64_t)v * n, begin, b0 + BLOCK) >> 32)
              : 0xffffffffu;
      for (int g = NW - 1; g >= 0; --g) {
        uint64_t m = s_mask[wave][g];
        while (m) {
          const int bit = 63 - __builtin_clzll(m);
          m &= ~(1ull << bit);
          const int k = g * 64 + bit;
          const float4 b = s_b[k];
          const uint32_t lo = __float_as_uint(b.z), hi = __float_as_uint(b.w);
          const bool inr = px < W && py < H && px >= (int)(lo & 0xffffu) &&
                           px <= (int)(hi & 0xffffu) && py >= (int)(lo >> 16) &&
                           py <= (int)(hi >> 16);
          uint32_t kb = inr ? pix_key_bits(s_q0[k], s_q1[k], s_q2[k], ur, vr) : 0xffffffffu;
#pragma unroll
          for (int sh = 32; sh > 0; sh >>= 1) kb = min(kb, (uint32_t)__shfl_xor((int)kb, sh, 64));
          bound = min(bound, kb);
          if (lane == 0) s_bound[wave][k] = bound;
        }
      }
      // lane 0's bounds are read by the whole wave below
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (int g = 0; g < NW; ++g) {
      uint64_t m = s_mask[wave][g];
      while (m && __ballot(alive)) {
        const int k = g * 64 + __builtin_ctzll(m);
        m &= m - 1;
        const float4 q2 = s_q2[k];
        const uint32_t zlo = NW > 1 ? s_bound[wave][k] : s_beta[k];
        // pending entries below the bound precede every later contribution
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
          if (win.n == K) {
            if ((uint32_t)(win.k[0] >> 32) < zlo) {
              pop(true);
            } else {
              inexact = true;   // the rest of this pixel is moot
              alive = false;
            }
          }
          if (alive) win.insert(key, al, b0 - begin + (uint32_t)k);
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

// Exact per-pixel order for the queued pixels, one wave per pixel, in
// rounds.  A round streams the pixel's tile list 64 records at a time and
// keeps, in LDS, the kFixCap least (key, index) above the last blended one:
// candidates go into a buffer of twice that size; when it overflows it is
// sorted and cut back, and its kFixCap-th key becomes a threshold below
// which a candidate must lie.  The scan stops at the first position whose
// bound word exceeds the threshold (every later key is at least that word),
// so the kept entries are exactly the least ones of the whole list.  They
// are blended in order; a round that keeps fewer than kFixCap entries has
// exhausted the list.
constexpr int kFixCap = 256, kFixWaves = 4;

struct FixAcc {
  float T, C0, C1, C2, D;
  int cnt;
  bool stop;
};

// Blend one contribution (wave-uniform values); false once the pixel stops.
__device__ __attribute__((always_inline)) inline bool fix_blend(FixAcc& s, float al, float r0,
                                                                float r1, float r2, float z,
                                                                float tmin) {
  const float w0 = al * s.T;
  const float Tn = s.T - w0;
  if (Tn < tmin) {
    s.stop = true;
    return false;
  }
  s.C0 = fmaf(r0, w0, s.C0);
  s.C1 = fmaf(r1, w0, s.C1);
  s.C2 = fmaf(r2, w0, s.C2);
  s.D = fmaf(z, w0, s.D);
  s.T = Tn;
  ++s.cnt;
  return true;
}

__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Ascending bitonic sort of one wave's (key, alpha) pairs in LDS, P a power
// of two (pads hold ~0).
__device__ inline void wave_sort(uint64_t* ck, float* ca, int P, int lane) {
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < (P >> 1); i += 64) {
        const int a = ((i & ~(j - 1)) << 1) | (i & (j - 1)), b = a + j;
        const uint64_t x = ck[a], y = ck[b];
        if ((x > y) == ((a & k) == 0)) {
          ck[a] = y;
          ck[b] = x;
          const float t = ca[a];
          ca[a] = ca[b];
          ca[b] = t;
        }
      }
      wave_sync_lds();
    }
}

__global__ __launch_bounds__(64 * kFixWaves) void k_gs_blend_px_fix(
    const uint32_t* __restrict__ fix_list, const uint32_t* __restrict__ fix_count,
    const uint64_t* __restrict__ tkey, const uint32_t* __restrict__ ids,
    const float4* __restrict__ rec, const float4* __restrict__ pcoef, int64_t n, KViews views,
    GsOpt o, int tile, int64_t tiles_x, int64_t tiles_per_view, const uint2* __restrict__ ranges,
    float* __restrict__ out_rgb, float* __restrict__ out_depth, float* __restrict__ out_t,
    int32_t* __restrict__ out_n) {
  constexpr int CAP2 = 2 * kFixCap;
  __shared__ uint64_t s_ck[kFixWaves][CAP2];
  __shared__ float s_ca[kFixWaves][CAP2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t* ck = s_ck[wave];
  float* ca = s_ca[wave];
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t nfix = *fix_count;
  for (uint32_t f = blockIdx.x * kFixWaves + wave; f < nfix; f += gridDim.x * kFixWaves) {
    const int64_t pix = fix_list[f];
    const KView& cv0 = views.v[0];
    const int64_t plane = (int64_t)cv0.W * cv0.H;
    const int v = (int)(pix / plane);
    const int64_t off = pix - (int64_t)v * plane;
    const KView& cv = views.v[v];
    const int py = (int)(off / cv.W), px = (int)(off - (int64_t)py * cv.W);
    const float xc = (float)px + 0.5f, yc = (float)py + 0.5f;
    const float ur = pix_ray(px, cv.cx, cv.fx), vr = pix_ray(py, cv.cy, cv.fy);
    const uint2 rg =
        ranges[(int64_t)v * tiles_per_view + (int64_t)(py / tile) * tiles_x + px / tile];
    const int64_t vbase = (int64_t)v * n;
    FixAcc acc{1.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0, false};
    uint64_t last = 0;   // the last blended (key, index), valid unless `first`
    bool first = true;
    while (!acc.stop) {
      int nc = 0;
      uint64_t thr = ~0ull;   // candidates must lie below
      for (uint32_t c0 = rg.x; c0 < rg.y; c0 += 64) {
        if (thr != ~0ull &&
            (uint32_t)(zs_word(tkey, ids, pcoef, vbase, rg.x, c0) >> 32) > (uint32_t)(thr >> 32))
          break;   // every key from here on is above the threshold
        const uint32_t j = c0 + lane;
        uint64_t key = ~0ull;
        float al = 0.0f;
        bool ok = false;
        if (j < rg.y) {
          const uint32_t id = (uint32_t)zs_word(tkey, ids, pcoef, vbase, rg.x, j);
          const int64_t e = vbase + id;
          float4 a, b, c;
          gs_stage(rec, e, a, b, c);
          const uint32_t lo = __float_as_uint(b.z), hi = __float_as_uint(b.w);
          if (px >= (int)(lo & 0xffffu) && px <= (int)(hi & 0xffffu) && py >= (int)(lo >> 16) &&
              py <= (int)(hi >> 16)) {
            const float dx = a.x - xc, dy = a.y - yc;
            const float P = (a.z * dx) * dx, R = a.w * dx;
            const float qq = fmaf(dy, fmaf(b.x, dy, R), P);
            al = fminf(b.y * __builtin_amdgcn_exp2f(qq), o.aclamp);
            if (al >= o.amin) {
              key = ((uint64_t)pix_key_bits(pcoef[3 * e], pcoef[3 * e + 1], pcoef[3 * e + 2], ur,
                                            vr) << 32) | id;
              ok = (first || key > last) && key < thr;
            }
          }
        }
        const uint64_t m = __ballot(ok);
        if (ok) {
          const int q = nc + __builtin_popcountll(m & below);
          ck[q] = key;
          ca[q] = al;
        }
        nc += __builtin_popcountll(m);
        wave_sync_lds();
        if (nc > kFixCap + (CAP2 - kFixCap - 64)) {
          // buffer nearly full: keep the kFixCap least, tighten the threshold
          for (int i = nc + lane; i < CAP2; i += 64) ck[i] = ~0ull;
          wave_sync_lds();
          wave_sort(ck, ca, CAP2, lane);
          nc = kFixCap;
          thr = ck[kFixCap - 1];
        }
      }
      // the round's least entries, in order
      int P = 64;
      while (P < nc) P <<= 1;
      for (int i = nc + lane; i < P; i += 64) ck[i] = ~0ull;
      wave_sync_lds();
      wave_sort(ck, ca, P, lane);
      const int m = min(nc, kFixCap);
      for (int b0 = 0; b0 < m && !acc.stop; b0 += 64) {
        const int i = b0 + lane;
        const uint64_t k = i < m ? ck[i] : ~0ull;
        const float al = i < m ? ca[i] : 0.0f;
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
        if (i < m) {
          const int64_t e = vbase + (uint32_t)k;
          const float4 r1 = rec[3 * e + 1], r2 = rec[3 * e + 2];
          c0 = r1.z;
          c1 = r1.w;
          c2 = r2.x;
        }
        const int cnt = min(64, m - b0);
        for (int q = 0; q < cnt; ++q) {
          const uint64_t kq = __shfl(k, q, 64);
          if (!fix_blend(acc, __shfl(al, q, 64), __shfl(c0, q, 64), __shfl(c1, q, 64),
                         __shfl(c2, q, 64), ord2f((uint32_t)(kq >> 32)), o.tmin))
            break;
          last = kq;
          first = false;
        }
      }
      wave_sync_lds();
      if (nc < kFixCap) break;   // the list is exhausted
    }
    if (lane == 0) {
      float* rgb = out_rgb + (int64_t)v * 3 * plane + off;
      rgb[0] = acc.C0 + acc.T * o.bg[0];
      rgb[plane] = acc.C1 + acc.T * o.bg[1];
      rgb[2 * plane] = acc.C2 + acc.T * o.bg[2];
      out_depth[(int64_t)v * plane + off] = acc.D;
      out_t[(int64_t)v * plane + off] = acc.T;
      out_n[(int64_t)v * plane + off] = acc.cnt;
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

void launch_gs_tile_zsort(const RenderWs& L, void* ws, int64_t n, const KViews& kv, int tile,
                         hipStream_t st) {
  if (L.tiles_total == 0) return;
  hipLaunchKernelGGL(k_gs_tile_zsort, dim3((unsigned)L.tiles_total), dim3(kZsBlock), 0, st,
                     at<uint32_t>(ws, L.ids), at<float4>(ws, L.pcoef), n, kv, tile, L.tiles_x,
                     L.tiles_x * L.tiles_y, at<uint2>(ws, L.ranges), at<uint64_t>(ws, L.tkey));
}

void launch_gs_blend_px(const RenderWs& L, void* ws, int64_t n, const uint32_t* order,
                        const KViews& kv, const GsOpt& o, float* rgb, float* depth, float* tf,
                        int32_t* nc, hipStream_t st) {
  const uint64_t* tk = at<uint64_t>(ws, L.tkey);
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
                         0, st, order, tk, ids, rec, pc, n, kv, o, L.tiles_x, tpv, ranges, rgb,
                         depth, tf, nc, fl, fc);
      break;
    default:  // 16 (the entry point rejects larger tiles in this order)
      hipLaunchKernelGGL(k_gs_blend_px<16>, dim3((unsigned)L.tiles_total), dim3(PxCfg<16>::BLOCK),
                         0, st, order, tk, ids, rec, pc, n, kv, o, L.tiles_x, tpv, ranges, rgb,
                         depth, tf, nc, fl, fc);
      break;
  }
  hipLaunchKernelGGL(k_gs_blend_px_fix, dim3(1024), dim3(64 * kFixWaves), 0, st, fl, fc, tk, ids,
                     rec, pc, n, kv, o, o.tile, L.tiles_x, tpv, ranges, rgb, depth, tf, nc);
}

}  // namespace vrs
