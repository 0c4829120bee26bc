// Device-side pieces of the 3D Gaussian splatting periphery shared by the
// forward and backward kernels: the single-precision EWA projection whose
// operation order fixes the integer decisions, and real spherical harmonics.
#pragma once
#include "vrs_common.h"

namespace vrs {

struct GsOpt {
  float aclamp, amin, tmin, lowpass, extent;
  float bg[3];
  int tile;
  int order;   // VRS_ORDER_PRIMITIVE or VRS_ORDER_PIXEL
};

struct Geom {
  float t[3];
  float ux, uy, jx, jy, j02, j12;  // projection intermediates
  float M[2][3];                   // J R
  float a, b, c, det;              // dilated 2D covariance
  float px, py;
  int x0, y0, x1, y1;              // pixel rectangle (inclusive)
};

__device__ inline float clamp_f(float v, float lo, float hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// EWA projection of one Gaussian into view cv, single precision, each
// operation rounded on its own in the documented order (3D Gaussian
// splatting as used for the periphery, Sec. 3.2).  Returns false if culled.
__device__ inline bool gs_geom32(const KView& cv, float mx, float my, float mz, const float* S6,
                                 float lowpass, float extent, Geom& g) {
#pragma clang fp contract(off)
  for (int i = 0; i < 3; ++i) {
    float a = cv.R[3 * i + 0] * mx;
    float b = cv.R[3 * i + 1] * my;
    float s = a + b;
    float e = cv.R[3 * i + 2] * mz;
    s = s + e;
    g.t[i] = s + cv.t[i];
  }
  if (!(g.t[2] > cv.znear)) return false;
  g.ux = g.t[0] / g.t[2];
  g.uy = g.t[1] / g.t[2];
  const float limx = 1.3f * ((0.5f * (float)cv.W) / cv.fx);
  const float limy = 1.3f * ((0.5f * (float)cv.H) / cv.fy);
  g.jx = cv.fx / g.t[2];
  g.jy = cv.fy / g.t[2];
  g.j02 = -(g.jx * clamp_f(g.ux, -limx, limx));
  g.j12 = -(g.jy * clamp_f(g.uy, -limy, limy));
  for (int k = 0; k < 3; ++k) {
    float p = g.jx * cv.R[k];
    float q = g.j02 * cv.R[6 + k];
    g.M[0][k] = p + q;
    p = g.jy * cv.R[3 + k];
    q = g.j12 * cv.R[6 + k];
    g.M[1][k] = p + q;
  }
  const float S[3][3] = {{S6[0], S6[1], S6[2]}, {S6[1], S6[3], S6[4]}, {S6[2], S6[4], S6[5]}};
  float U[2][3];
  for (int a = 0; a < 2; ++a)
    for (int k = 0; k < 3; ++k) {
      float p = g.M[a][0] * S[0][k];
      float q = g.M[a][1] * S[1][k];
      float s = p + q;
      float e = g.M[a][2] * S[2][k];
      U[a][k] = s + e;
    }
  float d0, d1, d2;
  {
    float p = U[0][0] * g.M[0][0], q = U[0][1] * g.M[0][1];
    float s = p + q;
    float e = U[0][2] * g.M[0][2];
    d0 = s + e;
    p = U[0][0] * g.M[1][0]; q = U[0][1] * g.M[1][1];
    s = p + q;
    e = U[0][2] * g.M[1][2];
    d1 = s + e;
    p = U[1][0] * g.M[1][0]; q = U[1][1] * g.M[1][1];
    s = p + q;
    e = U[1][2] * g.M[1][2];
    d2 = s + e;
  }
  g.a = d0 + lowpass;
  g.b = d1;
  g.c = d2 + lowpass;
  const float ac = g.a * g.c, bb = g.b * g.b;
  g.det = ac - bb;
  if (!(g.det > 0.0f)) return false;
  const float hd = 0.5f * (g.a - g.c);
  const float hd2 = hd * hd;
  const float disc = hd2 + bb;
  const float half = 0.5f * (g.a + g.c);
  const float lam = half + sqrtf(disc);
  const float sl = sqrtf(lam);
  const float r = ceilf(extent * sl);
  const float fxu = cv.fx * g.ux, fyu = cv.fy * g.uy;
  g.px = fxu + cv.cx;
  g.py = fyu + cv.cy;
  if (!(isfinite(g.px) && isfinite(g.py) && isfinite(r))) return false;
  float x0 = ceilf((g.px - r) - 0.5f), x1 = floorf((g.px + r) - 0.5f);
  float y0 = ceilf((g.py - r) - 0.5f), y1 = floorf((g.py + r) - 0.5f);
  x0 = x0 < 0.0f ? 0.0f : x0;
  y0 = y0 < 0.0f ? 0.0f : y0;
  x1 = x1 > (float)(cv.W - 1) ? (float)(cv.W - 1) : x1;
  y1 = y1 > (float)(cv.H - 1) ? (float)(cv.H - 1) : y1;
  if (x0 > x1 || y0 > y1) return false;
  g.x0 = (int)x0; g.y0 = (int)y0; g.x1 = (int)x1; g.y1 = (int)y1;
  return true;
}

// Real orthonormal spherical harmonics, degree <= 3, graphics sign
// convention (Sloan, "Stupid Spherical Harmonics Tricks").  Constants are
// 1/(2 sqrt(pi)), sqrt(3/(4 pi)), sqrt(15/pi)/2, sqrt(5/pi)/4,
// sqrt(15/pi)/4, sqrt(35/(2 pi))/4, sqrt(105/pi)/2, sqrt(21/(2 pi))/4,
// sqrt(7/pi)/4, sqrt(105/pi)/4.
struct ShC {
  static constexpr float c0 = 0.28209479177387814f;
  static constexpr float c1 = 0.48860251190291992f;
  static constexpr float c2a = 1.0925484305920792f;
  static constexpr float c2b = 0.31539156525252005f;
  static constexpr float c2c = 0.54627421529603959f;
  static constexpr float c3a = 0.59004358992664352f;
  static constexpr float c3b = 2.8906114426405538f;
  static constexpr float c3c = 0.45704579946446572f;
  static constexpr float c3d = 0.3731763325901154f;
  static constexpr float c3e = 1.4453057213202769f;
};

__device__ inline void sh_eval(int deg, float x, float y, float z, float* Y) {
  Y[0] = ShC::c0;
  if (deg < 1) return;
  Y[1] = -ShC::c1 * y;
  Y[2] = ShC::c1 * z;
  Y[3] = -ShC::c1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = ShC::c2a * x * y;
  Y[5] = -ShC::c2a * y * z;
  Y[6] = ShC::c2b * (2.0f * zz - xx - yy);
  Y[7] = -ShC::c2a * x * z;
  Y[8] = ShC::c2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -ShC::c3a * y * (3.0f * xx - yy);
  Y[10] = ShC::c3b * x * y * z;
  Y[11] = -ShC::c3c * y * (4.0f * zz - xx - yy);
  Y[12] = ShC::c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -ShC::c3c * x * (4.0f * zz - xx - yy);
  Y[14] = ShC::c3e * z * (xx - yy);
  Y[15] = -ShC::c3a * x * (xx - 3.0f * yy);
}

// Blend-time form of a projected Gaussian, staged in LDS once per tile
// batch: a = (px, py, A', B'), b = (C', opacity, rect_lo, rect_hi),
// c = (r, g, b, z), with the conic pre-scaled for a base-2 exponential:
// A' = -log2(e)/2 A, B' = -log2(e) B, C' = -log2(e)/2 C, so that
// alpha = min(alpha_clamp, opacity 2^(A' dx^2 + B' dx dy + C' dy^2)).
constexpr float kLog2e = 1.4426950408889634f;

__device__ inline void gs_stage(const float4* __restrict__ rec, int64_t e, float4& a, float4& b,
                                float4& c) {
  const float4 r0 = rec[3 * e + 0], r1 = rec[3 * e + 1], r2 = rec[3 * e + 2];
  a = make_float4(r0.x, r0.y, -0.5f * kLog2e * r0.z, -kLog2e * r0.w);
  b = make_float4(-0.5f * kLog2e * r1.x, r1.y, r2.z, r2.w);
  c = make_float4(r1.z, r1.w, r2.x, r2.y);
}

// Exponent q = P + dy (C' dy + R) with P = (A' dx) dx and R = B' dx: P and R
// are shared by every pixel of a column.
__device__ inline float gs_exponent(const float4& a, const float4& b, float dx, float dy) {
  const float P = (a.z * dx) * dx, R = a.w * dx;
  return fmaf(dy, fmaf(b.x, dy, R), P);
}

// Opacity at a pixel centre.  The conic is positive definite (the dilated
// covariance has a positive determinant), so the exponent is never positive
// but for rounding within a few units of the last place of zero, at the
// centre, where the opacity is the Gaussian's own either way: no guard on its
// sign is taken.  The forward blend evaluates the same operations inline and
// the backward calls this, so both take the same threshold decisions; e = 2^q
// is returned for the adjoint.
__device__ inline float gs_alpha(const float4& a, const float4& b, float xc, float yc,
                                 float aclamp, float& dx, float& dy, float& e) {
  dx = a.x - xc;
  dy = a.y - yc;
  const float q = gs_exponent(a, b, dx, dy);
  e = __builtin_amdgcn_exp2f(q);
  return fminf(b.y * e, aclamp);
}

// Packed rectangle: low 16 bits x, high 16 bits y.
__device__ inline uint32_t pack_xy(int x, int y) { return (uint32_t)x | ((uint32_t)y << 16); }

}  // namespace vrs
