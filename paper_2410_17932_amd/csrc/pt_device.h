// Device-side pieces of the foveal neural-point splat shared by the forward
// and backward kernels.
#pragma once
#include <hip/hip_fp16.h>

#include "vrs_common.h"

namespace vrs {

struct PtGeom {
  float t[3];
  float ux, uy, px, py, s;
  int l0;
  bool two;
};

// Projection and pyramid layer of one point in view cv (Sec. 3.3), single
// precision in the documented operation order.  Returns false if the point
// is culled by the near plane or projects to a non-finite position or size.
__device__ inline bool pt_geom32(const KView& cv, float x, float y, float z, float radius,
                                 int levels, PtGeom& g) {
#pragma clang fp contract(off)
  for (int i = 0; i < 3; ++i) {
    float a = cv.R[3 * i + 0] * x;
    float b = cv.R[3 * i + 1] * y;
    float s = a + b;
    float e = cv.R[3 * i + 2] * z;
    s = s + e;
    g.t[i] = s + cv.t[i];
  }
  if (!(g.t[2] > cv.znear)) return false;
  g.ux = g.t[0] / g.t[2];
  g.uy = g.t[1] / g.t[2];
  const float fxu = cv.fx * g.ux, fyu = cv.fy * g.uy;
  g.px = fxu + cv.cx;
  g.py = fyu + cv.cy;
  if (!(isfinite(g.px) && isfinite(g.py))) return false;
  const float f2 = 2.0f * cv.fx;
  const float num = f2 * radius;
  g.s = num / g.t[2];
  if (!isfinite(g.s)) return false;
  g.l0 = 0;
  g.two = false;
  if (g.s > 1.0f) {
    int e;
    const float m = frexpf(g.s, &e);
    g.l0 = e - 1;
    if (g.l0 >= levels - 1) g.l0 = levels - 1;
    else g.two = m > 0.5f;
  }
  return true;
}

// Depth-occlusion cull against the periphery's approximate depth (Eq. 1)
// at the pixel under the point: where the periphery's coverage 1 - T' is at
// least cov_min, a point farther than slack x (depth / coverage) is hidden.
// pt_cull_pixel gives the pixel (false outside the view: never hidden);
// pt_hidden decides from that pixel's T' and depth, so callers can issue
// both loads early.  Every other culling test is independent of this one.
__device__ inline bool pt_cull_pixel(const KView& cv, const PtGeom& g, int64_t& pi) {
  if (!(g.px >= 0.0f && g.px < (float)cv.W && g.py >= 0.0f && g.py < (float)cv.H)) return false;
  const int X = (int)floorf(g.px), Y = (int)floorf(g.py);
  pi = (int64_t)Y * cv.W + X;
  return true;
}
__device__ inline bool pt_hidden(float tz, float tf, float dep, float cov_min, float slack) {
#pragma clang fp contract(off)
  const float A = 1.0f - tf;
  if (!(A >= cov_min)) return false;
  const float q = dep / A;
  const float lim = slack * q;
  return tz > lim;
}

// Layer-l coordinates of the point in a crop with origin (x0, y0) and the
// integer corner of its bilinear footprint.  Returns false if no target of
// the footprint lies inside the S_l x S_l layer.
__device__ inline bool pt_layer32(const PtGeom& g, int x0, int y0, int l, int Sl, float& xl,
                                  float& yl, int& ix, int& iy) {
#pragma clang fp contract(off)
  const float sc = ldexpf(1.0f, -l);
  const float ax = g.px - (float)x0, ay = g.py - (float)y0;
  const float bx = ax * sc, by = ay * sc;
  xl = bx - 0.5f;
  yl = by - 0.5f;
  if (!(xl >= -1.0f && xl < (float)Sl && yl >= -1.0f && yl < (float)Sl)) return false;
  ix = (int)floorf(xl);
  iy = (int)floorf(yl);
  return true;
}

// ------------------------------------------------ compensated positions
// The integer decisions above are taken on the single-precision view pixel
// coordinate p = fx (t.x / t.z) + cx.  Far from the image origin (x ~ 2000)
// that coordinate carries up to ~1e-4 px of rounding, which the bilinear
// weights would inherit.  The continuous part of a fragment (its bilinear
// fractions) is therefore taken from the same single-precision inputs in
// float-float arithmetic (an unevaluated sum hi + lo; Dekker's two-product
// via fma and Knuth's two-sum), in the crop's own frame: the sub-frustum's
// principal point c - x0 (Sec. 3.3) is formed before the projected offset
// is added, so no large coordinate is ever rounded.
struct FF {
  float hi, lo;
};
__device__ inline FF ff_two_sum(float a, float b) {
#pragma clang fp contract(off)
  const float s = a + b;
  const float bb = s - a;
  const float e = (a - (s - bb)) + (b - bb);
  return FF{s, e};
}
__device__ inline FF ff_quick(float a, float b) {   // |a| >= |b| or a == 0
#pragma clang fp contract(off)
  const float s = a + b;
  return FF{s, b - (s - a)};
}
__device__ inline FF ff_two_prod(float a, float b) {
#pragma clang fp contract(off)
  const float p = a * b;
  return FF{p, fmaf(a, b, -p)};
}
__device__ inline FF ff_add(FF a, FF b) {
#pragma clang fp contract(off)
  const FF s = ff_two_sum(a.hi, b.hi);
  return ff_quick(s.hi, s.lo + (a.lo + b.lo));
}
__device__ inline FF ff_div(FF a, FF b) {
#pragma clang fp contract(off)
  const float q = a.hi / b.hi;
  float r = fmaf(-q, b.hi, a.hi);   // exact remainder of the rounded quotient
  r = r + a.lo;
  r = r - q * b.lo;
  return ff_quick(q, r / b.hi);
}

// Camera-plane position (t.x / t.z, t.y / t.z) of a point in float-float.
__device__ inline void pt_plane_ff(const KView& cv, float x, float y, float z, FF& ux, FF& uy) {
  FF t[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    FF s = ff_add(ff_two_prod(cv.R[3 * i + 0], x), ff_two_prod(cv.R[3 * i + 1], y));
    s = ff_add(s, ff_two_prod(cv.R[3 * i + 2], z));
    t[i] = ff_add(s, FF{cv.t[i], 0.0f});
  }
  ux = ff_div(t[0], t[2]);
  uy = ff_div(t[1], t[2]);
}

// Bilinear fraction along one axis in layer l of a crop with integer
// origin x0: xl - ix with xl = (f u + (c - x0)) 2^-l - 1/2 and ix the
// layer footprint's integer corner decided by pt_layer32.
__device__ inline float pt_frac_ff(float f, FF u, float c, int x0, int l, int ix) {
#pragma clang fp contract(off)
  FF a = ff_two_prod(f, u.hi);
  a = ff_quick(a.hi, a.lo + f * u.lo);
  a = ff_add(a, ff_two_sum(c, -(float)x0));
  const float sc = ldexpf(1.0f, -l);     // exact scaling
  FF d = ff_two_sum(a.hi * sc, -0.5f);
  d.lo = d.lo + a.lo * sc;
  return (d.hi - (float)ix) + d.lo;
}

__device__ inline int pt_targets(int ix, int iy, int Sl) {
  const int nx = (ix >= 0 ? 1 : 0) + (ix + 1 <= Sl - 1 ? 1 : 0);
  const int ny = (iy >= 0 ? 1 : 0) + (iy + 1 <= Sl - 1 ? 1 : 0);
  return nx * ny;
}

// Half precision bits -> float.
__device__ inline float h2f(uint16_t h) { return __half2float(__ushort_as_half(h)); }

}  // namespace vrs
