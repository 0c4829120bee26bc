// Test infrastructure, not product code: a plain, slow FP64 CPU reference of
// the foveated hybrid renderer (VR-Splatting, Franke, Fink & Stamminger).
// Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
// may load it.  It shares no code with the HIP library.
//
// Everything continuous is computed in double precision.  Where floating
// point decides an integer (which Gaussians are culled, a splat's pixel
// rectangle and tile rectangle, the depth key that orders primitives, a neural
// point's pyramid layer and target pixels, the depth-occlusion cull) the
// decision is taken in IEEE single precision with the operation order written
// out below (no contraction, correctly rounded + - * / sqrt), which is the
// precision of the GPU kernels.  The two implementations are written
// independently from that order.
//
// Periphery: Sec. 3.2 (3D Gaussian splatting of the full image P, Eq. 1 depth).
// Fovea: Sec. 3.3 (sub-frustum neural point splat, depth cull) and Sec. 4
// "Inference" (all pyramid layers in one pass).  Decoder: Sec. 3.3 (small
// CNN, periphery crop injected, finest level halved).  Combination: Sec. 3.4
// (Eqs. 2-5).
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- cameras
// View record (17 floats): fx, fy, cx, cy, R[9] (world->camera, row-major),
// t[3], znear.  Dims: width, height.
struct CamF {
  float fx, fy, cx, cy, R[9], t[3], znear;
  int W, H;
};
struct CamD {
  double fx, fy, cx, cy, R[9], t[3], znear, o[3];
  int W, H;
};

CamF cam_f(const float* v, const int* d) {
  CamF c;
  c.fx = v[0]; c.fy = v[1]; c.cx = v[2]; c.cy = v[3];
  for (int i = 0; i < 9; ++i) c.R[i] = v[4 + i];
  for (int i = 0; i < 3; ++i) c.t[i] = v[13 + i];
  c.znear = v[16];
  c.W = d[0]; c.H = d[1];
  return c;
}

CamD cam_d(const float* v, const int* d) {
  CamD c;
  c.fx = v[0]; c.fy = v[1]; c.cx = v[2]; c.cy = v[3];
  for (int i = 0; i < 9; ++i) c.R[i] = v[4 + i];
  for (int i = 0; i < 3; ++i) c.t[i] = v[13 + i];
  c.znear = v[16];
  c.W = d[0]; c.H = d[1];
  // camera centre o = -R^T t
  for (int i = 0; i < 3; ++i)
    c.o[i] = -(c.R[0 * 3 + i] * c.t[0] + c.R[1 * 3 + i] * c.t[1] + c.R[2 * 3 + i] * c.t[2]);
  return c;
}

uint32_t fbits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }

// Single-precision camera transform: t_i = ((R_i0 x + R_i1 y) + R_i2 z) + T_i.
void xform32(const CamF& c, float x, float y, float z, float* t) {
  for (int i = 0; i < 3; ++i) {
    float a = c.R[3 * i + 0] * x;
    float b = c.R[3 * i + 1] * y;
    float s = a + b;
    float e = c.R[3 * i + 2] * z;
    s = s + e;
    t[i] = s + c.t[i];
  }
}

float clampf(float v, float lo, float hi) { return v < lo ? lo : (v > hi ? hi : v); }
double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

// --------------------------------------------------- spherical harmonics
// Real orthonormal spherical harmonics up to degree 3 in the usual graphics
// sign convention (P.-P. Sloan, "Stupid Spherical Harmonics Tricks", 2008),
// evaluated at the unit direction (x, y, z).  Y[(l)^2 + l + m].
void sh_basis(int deg, double x, double y, double z, double* Y) {
  const double c0 = 0.5 * std::sqrt(1.0 / M_PI);
  Y[0] = c0;
  if (deg < 1) return;
  const double c1 = std::sqrt(3.0 / (4.0 * M_PI));
  Y[1] = -c1 * y;
  Y[2] = c1 * z;
  Y[3] = -c1 * x;
  if (deg < 2) return;
  const double c2a = 0.5 * std::sqrt(15.0 / M_PI);
  const double c2b = 0.25 * std::sqrt(5.0 / M_PI);
  const double c2c = 0.25 * std::sqrt(15.0 / M_PI);
  Y[4] = c2a * x * y;
  Y[5] = -c2a * y * z;
  Y[6] = c2b * (2 * z * z - x * x - y * y);
  Y[7] = -c2a * x * z;
  Y[8] = c2c * (x * x - y * y);
  if (deg < 3) return;
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * M_PI));
  const double c3b = 0.5 * std::sqrt(105.0 / M_PI);
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * M_PI));
  const double c3d = 0.25 * std::sqrt(7.0 / M_PI);
  const double c3e = 0.25 * std::sqrt(105.0 / M_PI);
  Y[9] = -c3a * y * (3 * x * x - y * y);
  Y[10] = c3b * x * y * z;
  Y[11] = -c3c * y * (4 * z * z - x * x - y * y);
  Y[12] = c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
  Y[13] = -c3c * x * (4 * z * z - x * x - y * y);
  Y[14] = c3e * z * (x * x - y * y);
  Y[15] = -c3a * x * (x * x - 3 * y * y);
}

}  // namespace

extern "C" {

int orc_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_sh_basis(int deg, int64_t n, const double* dirs, double* out) {
  const int K = (deg + 1) * (deg + 1);
  for (int64_t i = 0; i < n; ++i) {
    double Y[16];
    sh_basis(deg, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], Y);
    for (int k = 0; k < K; ++k) out[i * K + k] = Y[k];
  }
}

// ------------------------------------------------------------------ bake
// Sec. 4 "Inference": covariances and opacities are baked into the
// primitives.  Sigma = R(q) diag(s^2) R(q)^T with s = exp(logscale) and R(q)
// the rotation of the unit quaternion (w, x, y, z); opacity = sigmoid(logit).
// cov out [6][n] = (xx, xy, xz, yy, yz, zz).
void orc_bake(int64_t n, const float* ls, const float* quat, const float* logit,
              double* cov, double* opac) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double w = quat[i], x = quat[n + i], y = quat[2 * n + i], z = quat[3 * n + i];
    double qn = std::sqrt(w * w + x * x + y * y + z * z);
    w /= qn; x /= qn; y /= qn; z /= qn;
    double R[3][3] = {
        {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
        {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
        {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    double s2[3];
    for (int k = 0; k < 3; ++k) s2[k] = std::exp(2.0 * (double)ls[k * n + i]);
    double S[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += R[a][k] * s2[k] * R[b][k];
        S[a][b] = acc;
      }
    cov[0 * n + i] = S[0][0]; cov[1 * n + i] = S[0][1]; cov[2 * n + i] = S[0][2];
    cov[3 * n + i] = S[1][1]; cov[4 * n + i] = S[1][2]; cov[5 * n + i] = S[2][2];
    opac[i] = 1.0 / (1.0 + std::exp(-(double)logit[i]));
  }
}

// ---------------------------------------------- Gaussian projection, FP32
// Decisions of the 3DGS projection (Sec. 3.2; EWA splatting as in the 3DGS
// method the paper builds on) in single precision, operation by operation:
//   t = R mean + T (xform32);            cull unless tz > znear
//   ux = tx/tz, uy = ty/tz;  limx = 1.3*((0.5*W)/fx), limy likewise
//   jx = fx/tz, jy = fy/tz;  j02 = -(jx*clamp(ux)), j12 = -(jy*clamp(uy))
//   M0k = jx*R0k + j02*R2k,  M1k = jy*R1k + j12*R2k          (M = J R)
//   U_ik = (M_i0 S_0k + M_i1 S_1k) + M_i2 S_2k                 (U = M Sigma)
//   a = ((U00 M00 + U01 M01) + U02 M02) + lowpass
//   b =  (U00 M10 + U01 M11) + U02 M12
//   c = ((U10 M10 + U11 M11) + U12 M12) + lowpass
//   det = a*c - b*b;  cull unless det > 0
//   hd = 0.5*(a - c); lam = 0.5*(a + c) + sqrt(hd*hd + b*b)
//   r = ceil(extent * sqrt(lam))
//   px = fx*ux + cx, py = fy*uy + cy;  cull unless finite
//   xmin = max(ceil((px - r) - 0.5), 0), xmax = min(floor((px + r) - 0.5), W-1)
//   (y likewise); cull if the rectangle is empty.
// Pixel (i, j) has its centre at (i + 0.5, j + 0.5).  A Gaussian contributes
// to a pixel only if the pixel lies in this integer rectangle; tiles are
// derived from it, so the image does not depend on the tile size.
// Output: rect [v][n][4] = xmin, ymin, xmax, ymax (all -1 when culled),
// zbits [v][n] = bit pattern of tz (0xffffffff when culled).
void orc_gauss_geom32(int64_t n, const float* mean, const float* cov, int nv,
                      const float* views, const int* dims, float lowpass, float extent,
                      int32_t* rect, uint32_t* zbits) {
  for (int v = 0; v < nv; ++v) {
    const CamF c = cam_f(views + 17 * v, dims + 2 * v);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      int32_t* rr = rect + ((int64_t)v * n + i) * 4;
      uint32_t* zb = zbits + (int64_t)v * n + i;
      rr[0] = rr[1] = rr[2] = rr[3] = -1;
      *zb = 0xffffffffu;
      float t[3];
      xform32(c, mean[i], mean[n + i], mean[2 * n + i], t);
      if (!(t[2] > c.znear)) continue;
      float ux = t[0] / t[2], uy = t[1] / t[2];
      float limx = 1.3f * ((0.5f * (float)c.W) / c.fx);
      float limy = 1.3f * ((0.5f * (float)c.H) / c.fy);
      float jx = c.fx / t[2], jy = c.fy / t[2];
      float j02 = -(jx * clampf(ux, -limx, limx));
      float j12 = -(jy * clampf(uy, -limy, limy));
      float M[2][3];
      for (int k = 0; k < 3; ++k) {
        float p = jx * c.R[0 * 3 + k];
        float q = j02 * c.R[2 * 3 + k];
        M[0][k] = p + q;
        p = jy * c.R[1 * 3 + k];
        q = j12 * c.R[2 * 3 + k];
        M[1][k] = p + q;
      }
      float s0 = cov[i], s1 = cov[n + i], s2 = cov[2 * n + i], s3 = cov[3 * n + i],
            s4 = cov[4 * n + i], s5 = cov[5 * n + i];
      float S[3][3] = {{s0, s1, s2}, {s1, s3, s4}, {s2, s4, s5}};
      float U[2][3];
      for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k) {
          float p = M[a][0] * S[0][k];
          float q = M[a][1] * S[1][k];
          float s = p + q;
          float e = M[a][2] * S[2][k];
          U[a][k] = s + e;
        }
      auto dot3 = [](const float* u, const float* m) {
        float p = u[0] * m[0];
        float q = u[1] * m[1];
        float s = p + q;
        float e = u[2] * m[2];
        return s + e;
      };
      float a = dot3(U[0], M[0]) + lowpass;
      float b = dot3(U[0], M[1]);
      float cc = dot3(U[1], M[1]) + lowpass;
      float ac = a * cc, bb = b * b;
      float det = ac - bb;
      if (!(det > 0.0f)) continue;
      float hd = 0.5f * (a - cc);
      float hd2 = hd * hd;
      float disc = hd2 + bb;
      float lam = 0.5f * (a + cc) + std::sqrt(disc);
      float r = std::ceil(extent * std::sqrt(lam));
      float px = c.fx * ux + c.cx;
      float py = c.fy * uy + c.cy;
      if (!(std::isfinite(px) && std::isfinite(py) && std::isfinite(r))) continue;
      float x0 = std::ceil((px - r) - 0.5f), x1 = std::floor((px + r) - 0.5f);
      float y0 = std::ceil((py - r) - 0.5f), y1 = std::floor((py + r) - 0.5f);
      x0 = x0 < 0.0f ? 0.0f : x0;
      y0 = y0 < 0.0f ? 0.0f : y0;
      x1 = x1 > (float)(c.W - 1) ? (float)(c.W - 1) : x1;
      y1 = y1 > (float)(c.H - 1) ? (float)(c.H - 1) : y1;
      if (x0 > x1 || y0 > y1) continue;
      rr[0] = (int32_t)x0; rr[1] = (int32_t)y0; rr[2] = (int32_t)x1; rr[3] = (int32_t)y1;
      *zb = fbits(t[2]);
    }
  }
}

// ---------------------------------------------- Gaussian projection, FP64
// The continuous quantities of the same projection in double precision:
// rec [v][n][10] = px, py, conic A, B, C (inverse of the dilated 2D
// covariance: (c, -b, a)/det), opacity, r, g, b, tz.
// Colour: dir = (mean - o)/|mean - o| with o the camera centre;
// rgb = max(0, 0.5 + sum_k Y_k(dir) sh_k).  Culled entries are left as zero.
void orc_gauss_project64(int64_t n, const float* mean, const float* cov, const float* opac,
                         const float* sh, int deg, int nv, const float* views,
                         const int* dims, double lowpass, double* rec) {
  const int K = (deg + 1) * (deg + 1);
  for (int v = 0; v < nv; ++v) {
    const CamD c = cam_d(views + 17 * v, dims + 2 * v);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double* o = rec + ((int64_t)v * n + i) * 10;
      for (int k = 0; k < 10; ++k) o[k] = 0;
      double m[3] = {mean[i], mean[n + i], mean[2 * n + i]};
      double t[3];
      for (int a = 0; a < 3; ++a)
        t[a] = c.R[3 * a] * m[0] + c.R[3 * a + 1] * m[1] + c.R[3 * a + 2] * m[2] + c.t[a];
      if (!(t[2] > 0)) continue;
      double ux = t[0] / t[2], uy = t[1] / t[2];
      double limx = 1.3 * (0.5 * c.W / c.fx), limy = 1.3 * (0.5 * c.H / c.fy);
      double J[2][3] = {{c.fx / t[2], 0, -c.fx / t[2] * clampd(ux, -limx, limx)},
                        {0, c.fy / t[2], -c.fy / t[2] * clampd(uy, -limy, limy)}};
      double M[2][3];
      for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k)
          M[a][k] = J[a][0] * c.R[k] + J[a][1] * c.R[3 + k] + J[a][2] * c.R[6 + k];
      double S[3][3] = {{cov[i], cov[n + i], cov[2 * n + i]},
                        {cov[n + i], cov[3 * n + i], cov[4 * n + i]},
                        {cov[2 * n + i], cov[4 * n + i], cov[5 * n + i]}};
      double C2[2][2];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          double acc = 0;
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) acc += M[a][k] * S[k][l] * M[b][l];
          C2[a][b] = acc;
        }
      double A = C2[0][0] + lowpass, B = C2[0][1], Cc = C2[1][1] + lowpass;
      double det = A * Cc - B * B;
      o[0] = c.fx * ux + c.cx;
      o[1] = c.fy * uy + c.cy;
      o[2] = Cc / det;
      o[3] = -B / det;
      o[4] = A / det;
      o[5] = opac[i];
      double d[3] = {m[0] - c.o[0], m[1] - c.o[1], m[2] - c.o[2]};
      double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double Y[16];
      sh_basis(deg, d[0] / dn, d[1] / dn, d[2] / dn, Y);
      for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.5;
        for (int k = 0; k < K; ++k) acc += Y[k] * (double)sh[((int64_t)k * 3 + ch) * n + i];
        o[6 + ch] = acc > 0 ? acc : 0;
      }
      o[9] = t[2];
    }
  }
}

// --------------------------------------------------- per-pixel depth
// Per-pixel order of the periphery (Sec. 3.2: contributions sorted per
// pixel instead of per primitive, after Radl and Steiner et al.): the depth
// of Gaussian g at pixel p is the camera depth z* of the maximum of g's 3D
// density along the ray through p's centre.  With the camera-space mean
// mu = R mean + T, camera-space precision M = (R Sigma R^T)^-1 and the ray
// direction d = ((p_x + 1/2 - cx)/fx, (p_y + 1/2 - cy)/fy, 1) (z = 1), the
// density along t d is largest at t* = (d^T M mu) / (d^T M d), and z* = t*.
// Coefficients per (view, Gaussian): (m00, 2 m01, 2 m02, m11, 2 m12, m22,
// b0, b1, b2) with b = M mu, so that
//   num = (b0 u + b1 v) + b2
//   den = ((m00 u + 2m01 v + 2m02) u + (m11 v + 2m12) v) + m22
//   z*  = num / den.
// Single precision, as the order decision (documented operation order, no
// contraction): Sigma^-1 by cofactors over the determinant
// ((s00 c00 + s01 c01) + s02 c02), Q = R Sigma^-1 (rows, each sum as
// ((a0 b0 + a1 b1) + a2 b2)), M_ij = Q_i . R_j, b_i = M_i . mu; per pixel
// u = ((x + 0.5) - cx) / fx, v likewise.  A Gaussian with a non-positive or
// non-finite determinant takes its mean depth at every pixel.
static float dot3f(float a0, float a1, float a2, float b0, float b1, float b2) {
  float s = a0 * b0;
  s = s + a1 * b1;
  return s + a2 * b2;
}

void orc_gauss_pixdepth32(int64_t n, const float* mean, const float* cov, int nv,
                          const float* views, const int* dims, float* coef) {
  for (int v = 0; v < nv; ++v) {
    const CamF c = cam_f(views + 17 * v, dims + 2 * v);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      float* o = coef + ((int64_t)v * n + i) * 9;
      float t[3];
      xform32(c, mean[i], mean[n + i], mean[2 * n + i], t);
      const float s00 = cov[i], s01 = cov[n + i], s02 = cov[2 * n + i];
      const float s11 = cov[3 * n + i], s12 = cov[4 * n + i], s22 = cov[5 * n + i];
      const float c00 = s11 * s22 - s12 * s12, c01 = s02 * s12 - s01 * s22;
      const float c02 = s01 * s12 - s02 * s11, c11 = s00 * s22 - s02 * s02;
      const float c12 = s01 * s02 - s00 * s12, c22 = s00 * s11 - s01 * s01;
      float det = s00 * c00;
      det = det + s01 * c01;
      det = det + s02 * c02;
      if (!(det > 0.0f) || !std::isfinite(det)) {
        for (int k = 0; k < 9; ++k) o[k] = 0.0f;
        o[5] = 1.0f;    // den = 1, num = b2 = mean depth
        o[8] = t[2];
        continue;
      }
      const float id = 1.0f / det;
      const float P[3][3] = {{c00 * id, c01 * id, c02 * id},
                             {c01 * id, c11 * id, c12 * id},
                             {c02 * id, c12 * id, c22 * id}};
      float Q[3][3];
      for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k)
          Q[a][k] = dot3f(c.R[3 * a], c.R[3 * a + 1], c.R[3 * a + 2], P[0][k], P[1][k], P[2][k]);
      float M[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b)
          M[a][b] = dot3f(Q[a][0], Q[a][1], Q[a][2], c.R[3 * b], c.R[3 * b + 1], c.R[3 * b + 2]);
      o[0] = M[0][0];
      o[1] = 2.0f * M[0][1];
      o[2] = 2.0f * M[0][2];
      o[3] = M[1][1];
      o[4] = 2.0f * M[1][2];
      o[5] = M[2][2];
      o[6] = dot3f(M[0][0], M[0][1], M[0][2], t[0], t[1], t[2]);
      o[7] = dot3f(M[0][1], M[1][1], M[1][2], t[0], t[1], t[2]);
      o[8] = dot3f(M[0][2], M[1][2], M[2][2], t[0], t[1], t[2]);
    }
  }
}

static float pixdepth_key32(const float* k, const CamF& c, int x, int y) {
  const float u = (((float)x + 0.5f) - c.cx) / c.fx;
  const float v = (((float)y + 0.5f) - c.cy) / c.fy;
  float num = k[6] * u;
  num = num + k[7] * v;
  num = num + k[8];
  float a = k[0] * u;
  a = a + k[1] * v;
  a = a + k[2];
  float b = k[3] * v;
  b = b + k[4];
  float den = a * u;
  den = den + b * v;
  den = den + k[5];
  return num / den;
}

// The same coefficients in double precision (the value accumulated into
// Eq. 1's depth in per-pixel order): the exact inverse and products.
void orc_gauss_pixdepth64(int64_t n, const float* mean, const float* cov, int nv,
                          const float* views, const int* dims, double* coef) {
  for (int v = 0; v < nv; ++v) {
    const CamD c = cam_d(views + 17 * v, dims + 2 * v);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double* o = coef + ((int64_t)v * n + i) * 9;
      double t[3];
      for (int a = 0; a < 3; ++a)
        t[a] = c.R[3 * a] * mean[i] + c.R[3 * a + 1] * mean[n + i] + c.R[3 * a + 2] * mean[2 * n + i] +
               c.t[a];
      const double s00 = cov[i], s01 = cov[n + i], s02 = cov[2 * n + i];
      const double s11 = cov[3 * n + i], s12 = cov[4 * n + i], s22 = cov[5 * n + i];
      const double c00 = s11 * s22 - s12 * s12, c01 = s02 * s12 - s01 * s22;
      const double c02 = s01 * s12 - s02 * s11, c11 = s00 * s22 - s02 * s02;
      const double c12 = s01 * s02 - s00 * s12, c22 = s00 * s11 - s01 * s01;
      const double det = s00 * c00 + s01 * c01 + s02 * c02;
      if (!(det > 0)) {
        for (int k = 0; k < 9; ++k) o[k] = 0;
        o[5] = 1;
        o[8] = t[2];
        continue;
      }
      const double P[3][3] = {{c00 / det, c01 / det, c02 / det},
                              {c01 / det, c11 / det, c12 / det},
                              {c02 / det, c12 / det, c22 / det}};
      double M[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double acc = 0;
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) acc += c.R[3 * a + k] * P[k][l] * c.R[3 * b + l];
          M[a][b] = acc;
        }
      o[0] = M[0][0]; o[1] = 2 * M[0][1]; o[2] = 2 * M[0][2];
      o[3] = M[1][1]; o[4] = 2 * M[1][2]; o[5] = M[2][2];
      for (int a = 0; a < 3; ++a) o[6 + a] = M[a][0] * t[0] + M[a][1] * t[1] + M[a][2] * t[2];
    }
  }
}

static double pixdepth64(const double* k, const CamD& c, int x, int y) {
  const double u = (x + 0.5 - c.cx) / c.fx, v = (y + 0.5 - c.cy) / c.fy;
  const double num = k[6] * u + k[7] * v + k[8];
  const double den = k[0] * u * u + k[1] * u * v + k[2] * u + k[3] * v * v + k[4] * v + k[5];
  return num / den;
}

// order-preserving unsigned image of a float (negative values first)
static uint32_t ford(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ------------------------------------------------------------ tile lists
// Per (view, tile): every non-culled Gaussian whose tile rectangle
// [xmin/T, xmax/T] x [ymin/T, ymax/T] contains the tile, ordered by
// (depth key bits, Gaussian index).  sel [nsel][2] = (view, tile index
// ty*tiles_x + tx).  offsets [nsel+1]; ids may be null (count only).
// Returns the total number of entries.
int64_t orc_tile_lists(int64_t n, int nv, const int* dims, int tile, const int32_t* rect,
                       const uint32_t* zbits, int64_t nsel, const int32_t* sel,
                       int64_t* offsets, int32_t* ids) {
  std::vector<std::vector<std::pair<uint32_t, int32_t>>> lists(nsel);
#pragma omp parallel for schedule(dynamic)
  for (int64_t s = 0; s < nsel; ++s) {
    int v = sel[2 * s];
    int tx_n = (dims[2 * v] + tile - 1) / tile;
    int tx = sel[2 * s + 1] % tx_n, ty = sel[2 * s + 1] / tx_n;
    for (int64_t i = 0; i < n; ++i) {
      const int32_t* r = rect + ((int64_t)v * n + i) * 4;
      if (r[0] < 0) continue;
      if (r[0] / tile <= tx && tx <= r[2] / tile && r[1] / tile <= ty && ty <= r[3] / tile)
        lists[s].push_back({zbits[(int64_t)v * n + i], (int32_t)i});
    }
    std::sort(lists[s].begin(), lists[s].end());
  }
  offsets[0] = 0;
  for (int64_t s = 0; s < nsel; ++s) offsets[s + 1] = offsets[s] + (int64_t)lists[s].size();
  if (ids)
    for (int64_t s = 0; s < nsel; ++s)
      for (size_t k = 0; k < lists[s].size(); ++k) ids[offsets[s] + k] = lists[s][k].second;
  return offsets[nsel];
}

// ------------------------------------------------------------- blending
// Front-to-back alpha blending per pixel (Sec. 3.2) with the approximate
// depth of Eq. 1.  For pixel p of view v, walk the Gaussians whose rectangle
// holds p in (depth key, index) order, with T = 1, C = D = 0:
//   d = (px, py) - (p + 0.5);  q = -0.5 (A dx^2 + C dy^2) - B dx dy
//   skip if q > 0;  alpha = min(alpha_clamp, opacity e^q); skip if
//   alpha < alpha_min;  T' = T (1 - alpha);  stop (without this Gaussian)
//   if T' < t_min;  else C += rgb alpha T, D += tz alpha T, T = T'.
// Outputs rgb = C + T bg, depth = D (Eq. 1 as printed), T_final = T,
// ncontrib = number of Gaussians blended, evals = number of Gaussians whose
// rectangle holds the pixel that it evaluated up to and including the one
// that stopped it.  margin = smallest relative
// distance of any threshold decision taken (alpha vs alpha_min, T' vs t_min)
// to its threshold: the pixels where single-precision arithmetic may take
// the other branch.
// opts = alpha_clamp, alpha_min, t_min, bg0, bg1, bg2.
// pix [npix][3] = (view, x, y); null renders every pixel of every view in
// [v][y][x] order (npix ignored).
// Per-pixel order (pix32/pix64 given: the coefficients of
// orc_gauss_pixdepth32/64 and views [v][17]): the Gaussians whose rectangle
// holds p are ordered by (order-preserving bits of their single-precision
// per-pixel depth key, index) instead, and Eq. 1 accumulates their
// double-precision per-pixel depth z* instead of tz; nothing else changes.
void orc_render(int64_t n, int nv, const int* dims, int tile, const int32_t* rect,
                const uint32_t* zbits, const double* rec, const double* opts, int64_t npix,
                const int32_t* pix, double* rgb, double* depth, double* tfinal,
                int32_t* ncontrib, double* margin, int32_t* evals, const float* pix32,
                const double* pix64, const float* views) {
  // enumerate requested pixels
  std::vector<int32_t> all;
  if (!pix) {
    npix = 0;
    for (int v = 0; v < nv; ++v) npix += (int64_t)dims[2 * v] * dims[2 * v + 1];
    all.resize(npix * 3);
    int64_t k = 0;
    for (int v = 0; v < nv; ++v)
      for (int y = 0; y < dims[2 * v + 1]; ++y)
        for (int x = 0; x < dims[2 * v]; ++x) {
          all[3 * k] = v; all[3 * k + 1] = x; all[3 * k + 2] = y; ++k;
        }
    pix = all.data();
  }
  // bin the Gaussians into the tiles that hold requested pixels
  std::vector<int64_t> tile_base(nv + 1, 0);
  for (int v = 0; v < nv; ++v) {
    int tx_n = (dims[2 * v] + tile - 1) / tile, ty_n = (dims[2 * v + 1] + tile - 1) / tile;
    tile_base[v + 1] = tile_base[v] + (int64_t)tx_n * ty_n;
  }
  std::vector<char> want(tile_base[nv], 0);
  for (int64_t k = 0; k < npix; ++k) {
    int v = pix[3 * k], x = pix[3 * k + 1], y = pix[3 * k + 2];
    int tx_n = (dims[2 * v] + tile - 1) / tile;
    want[tile_base[v] + (y / tile) * tx_n + x / tile] = 1;
  }
  std::vector<std::vector<std::pair<uint32_t, int32_t>>> lists(tile_base[nv]);
  for (int v = 0; v < nv; ++v) {
    int tx_n = (dims[2 * v] + tile - 1) / tile;
    for (int64_t i = 0; i < n; ++i) {
      const int32_t* r = rect + ((int64_t)v * n + i) * 4;
      if (r[0] < 0) continue;
      for (int ty = r[1] / tile; ty <= r[3] / tile; ++ty)
        for (int tx = r[0] / tile; tx <= r[2] / tile; ++tx) {
          int64_t t = tile_base[v] + (int64_t)ty * tx_n + tx;
          if (want[t]) lists[t].push_back({zbits[(int64_t)v * n + i], (int32_t)i});
        }
    }
  }
#pragma omp parallel for schedule(dynamic)
  for (int64_t t = 0; t < tile_base[nv]; ++t) std::sort(lists[t].begin(), lists[t].end());

  const double aclamp = opts[0], amin = opts[1], tmin = opts[2];
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < npix; ++k) {
    int v = pix[3 * k], x = pix[3 * k + 1], y = pix[3 * k + 2];
    int tx_n = (dims[2 * v] + tile - 1) / tile;
    const auto* L = &lists[tile_base[v] + (y / tile) * tx_n + x / tile];
    std::vector<std::pair<uint32_t, int32_t>> own;   // per-pixel order
    std::vector<double> zstar;
    if (pix32) {
      const CamF cf = cam_f(views + 17 * v, dims + 2 * v);
      for (const auto& e : *L) {
        const int32_t* r = rect + ((int64_t)v * n + e.second) * 4;
        if (x < r[0] || x > r[2] || y < r[1] || y > r[3]) continue;
        own.push_back({ford(pixdepth_key32(pix32 + ((int64_t)v * n + e.second) * 9, cf, x, y)),
                       e.second});
      }
      std::sort(own.begin(), own.end());
      const CamD cd = cam_d(views + 17 * v, dims + 2 * v);
      for (const auto& e : own)
        zstar.push_back(pixdepth64(pix64 + ((int64_t)v * n + e.second) * 9, cd, x, y));
      L = &own;
    }
    double T = 1, C[3] = {0, 0, 0}, D = 0, mg = INFINITY;
    int cnt = 0, ev = 0;
    for (size_t j = 0; j < L->size(); ++j) {
      const auto& e = (*L)[j];
      int64_t i = e.second;
      const int32_t* r = rect + ((int64_t)v * n + i) * 4;
      if (x < r[0] || x > r[2] || y < r[1] || y > r[3]) continue;
      ++ev;
      const double* g = rec + ((int64_t)v * n + i) * 10;
      const double di = pix32 ? zstar[j] : g[9];
      double dx = g[0] - (x + 0.5), dy = g[1] - (y + 0.5);
      double q = -0.5 * (g[2] * dx * dx + g[4] * dy * dy) - g[3] * dx * dy;
      if (q > 0) continue;
      double a = std::min(aclamp, g[5] * std::exp(q));
      mg = std::min(mg, std::fabs(a - amin) / amin);
      if (a < amin) continue;
      double Tn = T * (1 - a);
      mg = std::min(mg, std::fabs(Tn - tmin) / tmin);
      if (Tn < tmin) break;
      for (int ch = 0; ch < 3; ++ch) C[ch] += g[6 + ch] * a * T;
      D += di * a * T;
      T = Tn;
      ++cnt;
    }
    for (int ch = 0; ch < 3; ++ch) rgb[3 * k + ch] = C[ch] + T * opts[3 + ch];
    depth[k] = D;
    tfinal[k] = T;
    ncontrib[k] = cnt;
    margin[k] = mg;
    if (evals) evals[k] = ev;
  }
}

// ------------------------------------------------------- neural points
// Foveal neural-point splat (Sec. 3.3, Sec. 4 "Inference"): crop k = (view,
// x0, y0, S) is a sub-frustum with the view's focal lengths and principal
// point shifted by (-x0, -y0); its pyramid layer l is (S >> l)^2 pixels.
// Per point and view, in single precision:
//   t = R pos + T (xform32); cull unless tz > znear
//   px = fx*(tx/tz) + cx, py = fy*(ty/tz) + cy      (view pixel coordinates)
//   depth cull (when a depth buffer is given): if 0 <= px < W and
//   0 <= py < H, with X = floor(px), Y = floor(py), A = 1 - T_final(X, Y):
//   cull if A >= cov_min and tz > slack * (D(X, Y) / A)
//   s = ((2*fx)*radius)/tz (projected diameter, pixels); cull unless finite
//   layer: s <= 1 -> l0 = 0, single layer; else s = m 2^e (frexp),
//   l0 = e - 1, single layer if l0 >= L-1 (then l0 = L-1) or m == 0.5,
//   otherwise layers l0 and l0+1.
// Per crop of the view and per layer l used:
//   xl = ((px - x0) * 2^-l) - 0.5, yl likewise; none if not
//   (-1 <= xl < S_l and -1 <= yl < S_l); ix = floor(xl), iy = floor(yl);
//   targets (ix+dx, iy+dy), dx, dy in {0,1}, kept when inside the layer.
// Double precision: lambda = log2(s) gives layer weights (1 - f, f) with
// f = lambda - l0 (weight 1 for a single layer); bilinear weights from
// fx = xl - ix, fy = yl - iy; fragment weight w = layer weight x bilinear
// weight.  Per layer pixel the fragments are ordered by (depth key bits,
// point index) and blended front to back: alpha = w * opacity,
// F += feature alpha T, T *= 1 - alpha (no thresholds).
// crops [k][4] = view, x0, y0, S.  Pyramid packed [crop][layer][y][x][C].
struct Frag {
  int64_t key;  // layer pixel index in the packed pyramid
  uint32_t zb;
  int32_t id;
  double w;
  int32_t crop, layer, ix, iy, l0, two;  // the integer decisions behind w
};

static void point_fragments(int64_t np, const float* pos, const float* radius, int nv,
                            const float* views, const int* dims, int ncrops,
                            const int32_t* crops, int L, const float* depth,
                            const float* tfinal, float cov_min, float slack,
                            std::vector<Frag>& out, std::vector<int64_t>& pix_base) {
  pix_base.assign((size_t)ncrops * L + 1, 0);
  for (int k = 0; k < ncrops; ++k)
    for (int l = 0; l < L; ++l) {
      int64_t s = crops[4 * k + 3] >> l;
      pix_base[(size_t)k * L + l + 1] = pix_base[(size_t)k * L + l] + s * s;
    }
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  std::vector<std::vector<Frag>> part(nth);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
#pragma omp for schedule(static)
    for (int64_t i = 0; i < np; ++i) {
      for (int v = 0; v < nv; ++v) {
        bool any = false;
        for (int k = 0; k < ncrops; ++k) any |= crops[4 * k] == v;
        if (!any) continue;
        const CamF c = cam_f(views + 17 * v, dims + 2 * v);
        float t[3];
        xform32(c, pos[i], pos[np + i], pos[2 * np + i], t);
        if (!(t[2] > c.znear)) continue;
        float ux = t[0] / t[2], uy = t[1] / t[2];
        float px = c.fx * ux + c.cx, py = c.fy * uy + c.cy;
        if (!(std::isfinite(px) && std::isfinite(py))) continue;
        if (tfinal && px >= 0.0f && px < (float)c.W && py >= 0.0f && py < (float)c.H) {
          int X = (int)std::floor(px), Y = (int)std::floor(py);
          int64_t pi = (int64_t)v * c.W * c.H + (int64_t)Y * c.W + X;
          float A = 1.0f - tfinal[pi];
          if (A >= cov_min && t[2] > slack * (depth[pi] / A)) continue;
        }
        float s = ((2.0f * c.fx) * radius[i]) / t[2];
        if (!std::isfinite(s)) continue;
        int l0 = 0;
        bool two = false;
        if (s > 1.0f) {
          int e;
          float m = std::frexp(s, &e);
          l0 = e - 1;
          if (l0 >= L - 1) l0 = L - 1;
          else two = m > 0.5f;
        }
        // double-precision weights
        const CamD cd = cam_d(views + 17 * v, dims + 2 * v);
        double td[3];
        for (int a = 0; a < 3; ++a)
          td[a] = cd.R[3 * a] * (double)pos[i] + cd.R[3 * a + 1] * (double)pos[np + i] +
                  cd.R[3 * a + 2] * (double)pos[2 * np + i] + cd.t[a];
        double pxd = cd.fx * td[0] / td[2] + cd.cx, pyd = cd.fy * td[1] / td[2] + cd.cy;
        double sd = 2.0 * cd.fx * (double)radius[i] / td[2];
        double f = two ? std::log2(sd) - l0 : 0.0;
        uint32_t zb = fbits(t[2]);
        for (int k = 0; k < ncrops; ++k) {
          if (crops[4 * k] != v) continue;
          int x0 = crops[4 * k + 1], y0 = crops[4 * k + 2], S = crops[4 * k + 3];
          for (int li = 0; li < (two ? 2 : 1); ++li) {
            int l = l0 + li;
            double wl = two ? (li == 0 ? 1.0 - f : f) : 1.0;
            int Sl = S >> l;
            float sc = std::ldexp(1.0f, -l);
            float xl = (px - (float)x0) * sc - 0.5f;
            float yl = (py - (float)y0) * sc - 0.5f;
            if (!(xl >= -1.0f && xl < (float)Sl && yl >= -1.0f && yl < (float)Sl)) continue;
            int ix = (int)std::floor(xl), iy = (int)std::floor(yl);
            double xld = (pxd - x0) * std::ldexp(1.0, -l) - 0.5;
            double yld = (pyd - y0) * std::ldexp(1.0, -l) - 0.5;
            double bx = xld - ix, by = yld - iy;
            for (int dy = 0; dy < 2; ++dy)
              for (int dx = 0; dx < 2; ++dx) {
                int xx = ix + dx, yy = iy + dy;
                if (xx < 0 || xx >= Sl || yy < 0 || yy >= Sl) continue;
                double wb = (dx ? bx : 1.0 - bx) * (dy ? by : 1.0 - by);
                Frag fr;
                fr.key = pix_base[(size_t)k * L + l] + (int64_t)yy * Sl + xx;
                fr.zb = zb;
                fr.id = (int32_t)i;
                fr.w = wl * wb;
                fr.crop = k; fr.layer = l; fr.ix = ix; fr.iy = iy; fr.l0 = l0; fr.two = two;
                part[tid].push_back(fr);
              }
          }
        }
      }
    }
  }
  out.clear();
  for (auto& p : part) out.insert(out.end(), p.begin(), p.end());
  std::sort(out.begin(), out.end(), [](const Frag& a, const Frag& b) {
    if (a.key != b.key) return a.key < b.key;
    if (a.zb != b.zb) return a.zb < b.zb;
    return a.id < b.id;
  });
}

// Number of layer pixels of the packed pyramid.
int64_t orc_pyramid_pixels(int ncrops, const int32_t* crops, int L) {
  int64_t s = 0;
  for (int k = 0; k < ncrops; ++k)
    for (int l = 0; l < L; ++l) {
      int64_t e = crops[4 * k + 3] >> l;
      s += e * e;
    }
  return s;
}

// Fragment lists: offsets [pixels+1] per layer pixel; ids (may be null)
// hold the point indices in blend order.  Returns the fragment count.
int64_t orc_point_lists(int64_t np, const float* pos, const float* radius, int nv,
                        const float* views, const int* dims, int ncrops, const int32_t* crops,
                        int L, const float* depth, const float* tfinal, float cov_min,
                        float slack, int64_t* offsets, int32_t* ids) {
  std::vector<Frag> fr;
  std::vector<int64_t> base;
  point_fragments(np, pos, radius, nv, views, dims, ncrops, crops, L, depth, tfinal, cov_min,
                  slack, fr, base);
  int64_t P = base.back();
  std::fill(offsets, offsets + P + 1, 0);
  for (const auto& f : fr) offsets[f.key + 1]++;
  for (int64_t p = 0; p < P; ++p) offsets[p + 1] += offsets[p];
  if (ids)
    for (size_t k = 0; k < fr.size(); ++k) ids[k] = fr[k].id;
  return (int64_t)fr.size();
}

// Fragments in blend order with their integer decisions:
// out [nfrag][8] = key, point id, crop, layer, ix, iy, l0, two.
// Returns the count; out may be null (count only).
int64_t orc_point_frags(int64_t np, const float* pos, const float* radius, int nv,
                        const float* views, const int* dims, int ncrops, const int32_t* crops,
                        int L, const float* depth, const float* tfinal, float cov_min,
                        float slack, int64_t* out) {
  std::vector<Frag> fr;
  std::vector<int64_t> base;
  point_fragments(np, pos, radius, nv, views, dims, ncrops, crops, L, depth, tfinal, cov_min,
                  slack, fr, base);
  if (out)
    for (size_t k = 0; k < fr.size(); ++k) {
      int64_t* o = out + 8 * k;
      o[0] = fr[k].key; o[1] = fr[k].id; o[2] = fr[k].crop; o[3] = fr[k].layer;
      o[4] = fr[k].ix; o[5] = fr[k].iy; o[6] = fr[k].l0; o[7] = fr[k].two;
    }
  return (int64_t)fr.size();
}

// Pyramid features (double) packed [crop][layer][y][x][C].
// feat: [np][C] IEEE half bits; opacity may be null (all ones).
void orc_splat_points(int64_t np, const float* pos, const float* radius, const uint16_t* feat,
                      const float* opacity, int C, int nv, const float* views, const int* dims,
                      int ncrops, const int32_t* crops, int L, const float* depth,
                      const float* tfinal, float cov_min, float slack, double* pyramid) {
  std::vector<Frag> fr;
  std::vector<int64_t> base;
  point_fragments(np, pos, radius, nv, views, dims, ncrops, crops, L, depth, tfinal, cov_min,
                  slack, fr, base);
  int64_t P = base.back();
  std::fill(pyramid, pyramid + P * C, 0.0);
  // half -> double (exact)
  auto h2d = [](uint16_t h) {
    int s = h >> 15, e = (h >> 10) & 31, m = h & 1023;
    double v;
    if (e == 0) v = std::ldexp((double)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = std::ldexp((double)(m + 1024), e - 25);
    return s ? -v : v;
  };
  size_t a = 0;
  while (a < fr.size()) {
    size_t b = a;
    while (b < fr.size() && fr[b].key == fr[a].key) ++b;
    double T = 1;
    double* out = pyramid + fr[a].key * C;
    for (size_t k = a; k < b; ++k) {
      double o = opacity ? (double)opacity[fr[k].id] : 1.0;
      double al = fr[k].w * o;
      for (int ch = 0; ch < C; ++ch) out[ch] += h2d(feat[(int64_t)fr[k].id * C + ch]) * al * T;
      T *= 1 - al;
    }
    a = b;
  }
}

// --------------------------------------------------------------- decoder
// Small gated CNN that resolves the pyramid into the foveal image F
// (Sec. 3.3; the periphery crop is injected and the finest level is kept
// narrow).  Levels l = 0 (finest, S x S) .. n-1, each one gated 3x3
// convolution with zero padding:
//   G_l(x) = ELU(W_f * x + b_f) (.) sigmoid(W_g * x + b_g)
//   h_{n-1} = G_{n-1}(X_{n-1});  h_l = G_l([X_l, up2(h_{l+1}), Pcrop if l=0])
//   F = W_o h_0 + b_o  (1x1, 3 channels)
// up2 = bilinear x2 with half-pixel centres and edge clamp.  Weights packed as
// for level 0..n-1: W_l [2K][3][3][Cin], b_l [2K]; then W_o [3][K_0], b_o [3].
// pyramid: double, packed [crop][layer][y][x][C] with L layers.
// periph: double [nv][3][H][W].  out: double packed [crop][3][S][S].
static double elu(double x) { return x > 0 ? x : std::expm1(x); }
static double sigm(double x) { return 1.0 / (1.0 + std::exp(-x)); }

void orc_decode(int ncrops, const int32_t* crops, int L, int C, const double* pyramid,
                const double* periph, const int* dims, int nd, const int* widths,
                const double* weights, double* out) {
  int64_t pbase = 0, obase = 0;
  for (int k = 0; k < ncrops; ++k) {
    int v = crops[4 * k], x0 = crops[4 * k + 1], y0 = crops[4 * k + 2], S = crops[4 * k + 3];
    int W = dims[2 * v], H = dims[2 * v + 1];
    std::vector<int64_t> lay(L);
    int64_t acc = pbase;
    for (int l = 0; l < L; ++l) { lay[l] = acc; acc += (int64_t)(S >> l) * (S >> l) * C; }
    pbase = acc;
    // weight offsets
    std::vector<int64_t> woff(nd), boff(nd);
    std::vector<int> cin(nd);
    int64_t o = 0;
    for (int l = 0; l < nd; ++l) {
      cin[l] = C + (l + 1 < nd ? widths[l + 1] : 0) + (l == 0 ? 3 : 0);
      woff[l] = o; o += (int64_t)2 * widths[l] * 9 * cin[l];
      boff[l] = o; o += 2 * widths[l];
    }
    int64_t hw = o, hb = o + 3 * widths[0];
    std::vector<double> hprev;  // h_{l+1}, [S_{l+1}][S_{l+1}][K_{l+1}]
    for (int l = nd - 1; l >= 0; --l) {
      int Sl = S >> l, K = widths[l], Ci = cin[l];
      std::vector<double> x((size_t)Sl * Sl * Ci);
      for (int yy = 0; yy < Sl; ++yy)
        for (int xx = 0; xx < Sl; ++xx) {
          double* px = &x[((size_t)yy * Sl + xx) * Ci];
          int c = 0;
          for (int ch = 0; ch < C; ++ch) px[c++] = pyramid[lay[l] + ((int64_t)yy * Sl + xx) * C + ch];
          if (l + 1 < nd) {
            int Sp = Sl / 2, Kp = widths[l + 1];
            double sx = (xx + 0.5) / 2 - 0.5, sy = (yy + 0.5) / 2 - 0.5;
            int ax = (int)std::floor(sx), ay = (int)std::floor(sy);
            double fx = sx - ax, fy = sy - ay;
            int ax0 = std::min(std::max(ax, 0), Sp - 1), ax1 = std::min(std::max(ax + 1, 0), Sp - 1);
            int ay0 = std::min(std::max(ay, 0), Sp - 1), ay1 = std::min(std::max(ay + 1, 0), Sp - 1);
            for (int ch = 0; ch < Kp; ++ch) {
              double v00 = hprev[((size_t)ay0 * Sp + ax0) * Kp + ch];
              double v01 = hprev[((size_t)ay0 * Sp + ax1) * Kp + ch];
              double v10 = hprev[((size_t)ay1 * Sp + ax0) * Kp + ch];
              double v11 = hprev[((size_t)ay1 * Sp + ax1) * Kp + ch];
              px[c++] = (1 - fy) * ((1 - fx) * v00 + fx * v01) + fy * ((1 - fx) * v10 + fx * v11);
            }
          }
          if (l == 0)
            for (int ch = 0; ch < 3; ++ch)
              px[c++] = periph[(((int64_t)v * 3 + ch) * H + (y0 + yy)) * W + (x0 + xx)];
        }
      std::vector<double> h((size_t)Sl * Sl * K);
      const double* Wl = weights + woff[l];
      const double* bl = weights + boff[l];
#pragma omp parallel for schedule(static)
      for (int yy = 0; yy < Sl; ++yy)
        for (int xx = 0; xx < Sl; ++xx)
          for (int kk = 0; kk < K; ++kk) {
            double f = bl[kk], g = bl[K + kk];
            for (int ky = 0; ky < 3; ++ky)
              for (int kx = 0; kx < 3; ++kx) {
                int sy = yy + ky - 1, sx = xx + kx - 1;
                if (sy < 0 || sy >= Sl || sx < 0 || sx >= Sl) continue;
                const double* px = &x[((size_t)sy * Sl + sx) * Ci];
                const double* wf = Wl + (((int64_t)kk * 3 + ky) * 3 + kx) * Ci;
                const double* wg = Wl + (((int64_t)(K + kk) * 3 + ky) * 3 + kx) * Ci;
                for (int c = 0; c < Ci; ++c) { f += wf[c] * px[c]; g += wg[c] * px[c]; }
              }
            h[((size_t)yy * Sl + xx) * K + kk] = elu(f) * sigm(g);
          }
      hprev.swap(h);
    }
    int K0 = widths[0];
    for (int ch = 0; ch < 3; ++ch)
      for (int yy = 0; yy < S; ++yy)
        for (int xx = 0; xx < S; ++xx) {
          double a = weights[hb + ch];
          for (int kk = 0; kk < K0; ++kk)
            a += weights[hw + ch * K0 + kk] * hprev[((size_t)yy * S + xx) * K0 + kk];
          out[obase + ((int64_t)ch * S + yy) * S + xx] = a;
        }
    obase += (int64_t)3 * S * S;
  }
}

// ------------------------------------------------------------- composite
// Combination of the periphery P and the foveal crops F (Sec. 3.4).
// For every crop of a view, in index order, and every pixel (u, v) of the
// crop, with r the distance from the pixel centre to the gaze point e and
// d_f = S/2 the fovea radius:
//   mode 0 (linear ring): c = clamp((d_f - r)/ring, 0, 1)
//   mode 1 (Eqs. 2-5): r_n = clamp(r/d_f, 0, 1) (Eq. 2),
//     f_p = (r_n - m)/(1 - m) (Eq. 3), f_e = |Sobel(mean_rgb(F))|/4 with
//     replicated crop borders (Eq. 4), c = 1 - S2(clamp(f_p + gamma f_e,
//     0, 1)) with S2(x) = 6x^5 - 15x^4 + 10x^3 (Eq. 5)
//   out = (1 - c) out + c F.
// Outside every crop out = P.  P, out: [nv][3][H][W]; F packed
// [crop][3][S][S]; gaze [k][2].
static double smootherstep(double x) { return x * x * x * (x * (6 * x - 15) + 10); }

void orc_composite(int nv, const int* dims, const double* P, int ncrops, const int32_t* crops,
                   const float* gaze, const double* F, int mode, double ring, double m,
                   double gamma, double* out) {
  int64_t tot = 0;
  for (int v = 0; v < nv; ++v) tot += (int64_t)3 * dims[2 * v] * dims[2 * v + 1];
  std::memcpy(out, P, sizeof(double) * tot);
  int64_t fbase = 0;
  for (int k = 0; k < ncrops; ++k) {
    int v = crops[4 * k], x0 = crops[4 * k + 1], y0 = crops[4 * k + 2], S = crops[4 * k + 3];
    int W = dims[2 * v], H = dims[2 * v + 1];
    int64_t vb = 0;
    for (int u = 0; u < v; ++u) vb += (int64_t)3 * dims[2 * u] * dims[2 * u + 1];
    const double* Fk = F + fbase;
    double df = 0.5 * S;
    auto gray = [&](int x, int y) {
      x = std::min(std::max(x, 0), S - 1);
      y = std::min(std::max(y, 0), S - 1);
      return (Fk[(0 * S + y) * S + x] + Fk[((int64_t)1 * S + y) * S + x] +
              Fk[((int64_t)2 * S + y) * S + x]) / 3.0;
    };
    for (int y = 0; y < S; ++y)
      for (int x = 0; x < S; ++x) {
        double dx = (x0 + x + 0.5) - gaze[2 * k], dy = (y0 + y + 0.5) - gaze[2 * k + 1];
        double r = std::sqrt(dx * dx + dy * dy);
        double c;
        if (mode == 0) {
          c = clampd((df - r) / ring, 0, 1);
        } else {
          double rn = clampd(r / df, 0, 1);
          double fp = (rn - m) / (1 - m);
          double gx = (gray(x + 1, y - 1) + 2 * gray(x + 1, y) + gray(x + 1, y + 1)) -
                      (gray(x - 1, y - 1) + 2 * gray(x - 1, y) + gray(x - 1, y + 1));
          double gy = (gray(x - 1, y + 1) + 2 * gray(x, y + 1) + gray(x + 1, y + 1)) -
                      (gray(x - 1, y - 1) + 2 * gray(x, y - 1) + gray(x + 1, y - 1));
          double fe = std::sqrt(gx * gx + gy * gy) / 4.0;
          c = 1.0 - smootherstep(clampd(fp + gamma * fe, 0, 1));
        }
        for (int ch = 0; ch < 3; ++ch) {
          int64_t oi = vb + ((int64_t)ch * H + (y0 + y)) * W + (x0 + x);
          out[oi] = (1 - c) * out[oi] + c * Fk[((int64_t)ch * S + y) * S + x];
        }
      }
    fbase += (int64_t)3 * S * S;
  }
}

}  // extern "C"
