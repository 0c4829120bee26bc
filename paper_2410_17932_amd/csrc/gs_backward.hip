// Peripheral 3D Gaussian splatting, backward (end-to-end fitting, Sec. 3.5).
//
//   k_gs_blend_bwd        one workgroup per tile; every pixel replays its
//                         list back to front from its stored stop position
//                         and final transmittance (T before an entry is
//                         T after it divided by 1 - alpha), so no per-pixel
//                         lists are stored; per-entry screen-space gradients
//                         are summed over the wave with cross-lane
//                         reductions before one atomic add per wave
//   k_gs_project_bwd      one thread per Gaussian: chain rule through the
//                         conic inverse, the EWA Jacobian, the camera
//                         transform and the spherical harmonics, summed
//                         over views, accumulated into the caller's
//                         gradient planes
#include "gs_layout.h"

namespace vrs {

constexpr int kG2d = 10;  // px, py, A, B, C, opacity, r, g, b, z
constexpr float kLn2 = 0.69314718055994531f;

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int TILE>
struct BwdCfg {
  static constexpr int PIX = TILE * TILE;
  static constexpr int BLOCK = PIX < 256 ? PIX : 256;
  static constexpr int PPT = PIX / BLOCK;
};

template <int TILE>
__global__ __launch_bounds__(BwdCfg<TILE>::BLOCK) void k_gs_blend_bwd(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids,
    const float4* __restrict__ rec, int64_t n, KViews views, GsOpt o, int64_t tiles_x,
    int64_t tiles_per_view, const uint32_t* __restrict__ last_pos,
    const float* __restrict__ tfinal, const float* __restrict__ d_rgb,
    const float* __restrict__ d_depth, float* __restrict__ g2d) {
  using Cfg = BwdCfg<TILE>;
  constexpr int BLOCK = Cfg::BLOCK, PPT = Cfg::PPT;
  __shared__ float4 s_a[BLOCK], s_b[BLOCK], s_c[BLOCK];
  __shared__ uint32_t s_id[BLOCK];
  __shared__ uint32_t s_maxlast;
  const int64_t tglob = blockIdx.x;
  const int v = (int)(tglob / tiles_per_view);
  const int64_t tl = tglob - (int64_t)v * tiles_per_view;
  const int ty = (int)(tl / tiles_x), tx = (int)(tl - (int64_t)ty * tiles_x);
  const KView& cv = views.v[v];
  const int W = cv.W, H = cv.H;
  const int tid = threadIdx.x;
  const int64_t plane = (int64_t)W * H;
  int px[PPT], py[PPT];
  uint32_t last[PPT];
  float T[PPT], acc0[PPT], acc1[PPT], acc2[PPT], accd[PPT], g0[PPT], g1[PPT], g2[PPT], gd[PPT];
  if (tid == 0) s_maxlast = 0;
  __syncthreads();
  uint32_t mymax = 0;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int l = tid + q * BLOCK;
    px[q] = tx * TILE + (l % TILE);
    py[q] = ty * TILE + (l / TILE);
    last[q] = 0;
    T[q] = 1.0f;
    acc0[q] = o.bg[0]; acc1[q] = o.bg[1]; acc2[q] = o.bg[2]; accd[q] = 0.0f;
    g0[q] = g1[q] = g2[q] = gd[q] = 0.0f;
    if (px[q] < W && py[q] < H) {
      const int64_t pix = (int64_t)v * plane + (int64_t)py[q] * W + px[q];
      const int64_t rp = (int64_t)v * 3 * plane + (int64_t)py[q] * W + px[q];
      last[q] = last_pos[pix];
      T[q] = tfinal[pix];
      g0[q] = d_rgb[rp];
      g1[q] = d_rgb[rp + plane];
      g2[q] = d_rgb[rp + 2 * plane];
      gd[q] = d_depth ? d_depth[pix] : 0.0f;
      mymax = last[q] > mymax ? last[q] : mymax;
    }
  }
  atomicMax(&s_maxlast, mymax);
  __syncthreads();
  const uint2 rg = ranges[tglob];
  const uint32_t begin = rg.x;
  const uint32_t stop = begin + s_maxlast;
  const float aclamp = o.aclamp, amin = o.amin;
  for (int64_t b1 = stop; b1 > (int64_t)begin; b1 -= BLOCK) {
    const int64_t b0 = b1 - BLOCK > (int64_t)begin ? b1 - BLOCK : (int64_t)begin;
    const int cnt = (int)(b1 - b0);
    __syncthreads();
    if (tid < cnt) {
      const uint32_t id = ids[b0 + tid];
      const uint32_t idc = id < (uint64_t)n ? id : 0;
      const int64_t e = (int64_t)v * n + idc;
      float4 a, b, c;
      gs_stage(rec, e, a, b, c);
      s_a[tid] = a;
      s_b[tid] = b;
      s_c[tid] = c;
      s_id[tid] = idc;
    }
    __syncthreads();
    for (int k = cnt - 1; k >= 0; --k) {
      const uint32_t pos = (uint32_t)(b0 - begin) + k;  // position in the tile list
      const float4 a = s_a[k], bq = s_b[k], c = s_c[k];
      const uint32_t lo = __float_as_uint(bq.z), hi = __float_as_uint(bq.w);
      float dpx = 0, dpy = 0, dA = 0, dB = 0, dC = 0, dop = 0, dr = 0, dg = 0, db = 0, dz = 0;
      bool any = false;
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        if (pos >= last[q]) continue;
        const uint32_t x = (uint32_t)px[q], y = (uint32_t)py[q];
        if (x < (lo & 0xffffu) || x > (hi & 0xffffu) || y < (lo >> 16) || y > (hi >> 16)) continue;
        float dx, dy, eq;
        const float al = gs_alpha(a, bq, (float)px[q] + 0.5f, (float)py[q] + 0.5f, aclamp, dx, dy, eq);
        if (!(al >= amin)) continue;
        any = true;
        const float Tb = T[q] / (1.0f - al);
        const float w = al * Tb;
        dr += w * g0[q];
        dg += w * g1[q];
        db += w * g2[q];
        dz += w * gd[q];
        const float dal = Tb * (g0[q] * (c.x - acc0[q]) + g1[q] * (c.y - acc1[q]) +
                                g2[q] * (c.z - acc2[q]) + gd[q] * (c.w - accd[q]));
        acc0[q] = c.x * al + (1.0f - al) * acc0[q];
        acc1[q] = c.y * al + (1.0f - al) * acc1[q];
        acc2[q] = c.z * al + (1.0f - al) * acc2[q];
        accd[q] = c.w * al + (1.0f - al) * accd[q];
        T[q] = Tb;
        if (bq.y * eq < aclamp) {   // alpha not clamped: flows to opacity and the exponent
          dop += dal * eq;
          // exponent s = -(A dx^2 + C dy^2)/2 - B dx dy; the staged form holds
          // A' = -A log2(e)/2, B' = -B log2(e), C' = -C log2(e)/2
          const float ds = dal * al;
          dA += -0.5f * ds * dx * dx;
          dC += -0.5f * ds * dy * dy;
          dB += -ds * dx * dy;
          dpx += ds * kLn2 * (2.0f * a.z * dx + a.w * dy);
          dpy += ds * kLn2 * (2.0f * bq.x * dy + a.w * dx);
        }
      }
      // wave-level reduction, one atomic per value per wave
      if (__ballot(any) == 0) continue;
      dpx = wave_sum(dpx); dpy = wave_sum(dpy); dA = wave_sum(dA); dB = wave_sum(dB);
      dC = wave_sum(dC); dop = wave_sum(dop); dr = wave_sum(dr); dg = wave_sum(dg);
      db = wave_sum(db); dz = wave_sum(dz);
      if ((tid & 63) == 0) {
        float* G = g2d + ((int64_t)v * n + s_id[k]) * kG2d;
        atomicAdd(G + 0, dpx); atomicAdd(G + 1, dpy); atomicAdd(G + 2, dA);
        atomicAdd(G + 3, dB); atomicAdd(G + 4, dC); atomicAdd(G + 5, dop);
        atomicAdd(G + 6, dr); atomicAdd(G + 7, dg); atomicAdd(G + 8, db);
        atomicAdd(G + 9, dz);
      }
    }
  }
}

// derivatives of the SH basis with respect to the (unnormalised) direction
// components, contracted with dY: returns dL/d(x, y, z)
__device__ inline void sh_grad_dir(int deg, float x, float y, float z, const float* dY,
                                   float& gx, float& gy, float& gz) {
  gx = gy = gz = 0.0f;
  if (deg < 1) return;
  gy += -ShC::c1 * dY[1];
  gz += ShC::c1 * dY[2];
  gx += -ShC::c1 * dY[3];
  if (deg < 2) return;
  gx += ShC::c2a * y * dY[4];
  gy += ShC::c2a * x * dY[4];
  gy += -ShC::c2a * z * dY[5];
  gz += -ShC::c2a * y * dY[5];
  gx += -2.0f * ShC::c2b * x * dY[6];
  gy += -2.0f * ShC::c2b * y * dY[6];
  gz += 4.0f * ShC::c2b * z * dY[6];
  gx += -ShC::c2a * z * dY[7];
  gz += -ShC::c2a * x * dY[7];
  gx += 2.0f * ShC::c2c * x * dY[8];
  gy += -2.0f * ShC::c2c * y * dY[8];
  if (deg < 3) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  gx += -6.0f * ShC::c3a * x * y * dY[9];
  gy += -ShC::c3a * (3.0f * xx - 3.0f * yy) * dY[9];
  gx += ShC::c3b * y * z * dY[10];
  gy += ShC::c3b * x * z * dY[10];
  gz += ShC::c3b * x * y * dY[10];
  gx += 2.0f * ShC::c3c * x * y * dY[11];
  gy += -ShC::c3c * (4.0f * zz - xx - 3.0f * yy) * dY[11];
  gz += -8.0f * ShC::c3c * y * z * dY[11];
  gx += -6.0f * ShC::c3d * x * z * dY[12];
  gy += -6.0f * ShC::c3d * y * z * dY[12];
  gz += ShC::c3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * dY[12];
  gx += -ShC::c3c * (4.0f * zz - 3.0f * xx - yy) * dY[13];
  gy += 2.0f * ShC::c3c * x * y * dY[13];
  gz += -8.0f * ShC::c3c * x * z * dY[13];
  gx += 2.0f * ShC::c3e * x * z * dY[14];
  gy += -2.0f * ShC::c3e * y * z * dY[14];
  gz += ShC::c3e * (xx - yy) * dY[14];
  gx += -ShC::c3a * (3.0f * xx - 3.0f * yy) * dY[15];
  gy += 6.0f * ShC::c3a * x * y * dY[15];
}

__global__ __launch_bounds__(256) void k_gs_project_bwd(
    const float* __restrict__ mean, const float* __restrict__ cov,
    const float* __restrict__ sh, int deg, int64_t n, KViews views, GsOpt o,
    const float* __restrict__ g2d, float* __restrict__ d_mean, float* __restrict__ d_cov,
    float* __restrict__ d_op, float* __restrict__ d_sh) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float mx = mean[i], my = mean[n + i], mz = mean[2 * n + i];
  float S6[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) S6[k] = cov[k * n + i];
  const int K = (deg + 1) * (deg + 1);
  float dm[3] = {0, 0, 0}, dcv[6] = {0, 0, 0, 0, 0, 0}, dopa = 0.0f;
  float dshv[16][3];
#pragma unroll
  for (int k = 0; k < 16; ++k) dshv[k][0] = dshv[k][1] = dshv[k][2] = 0.0f;
  for (int v = 0; v < views.n; ++v) {
    const float* G = g2d + ((int64_t)v * n + i) * kG2d;
    const float gpx = G[0], gpy = G[1], gA = G[2], gB = G[3], gC = G[4], gop = G[5];
    const float grgb[3] = {G[6], G[7], G[8]};
    const float gz = G[9];
    if (gpx == 0 && gpy == 0 && gA == 0 && gB == 0 && gC == 0 && gop == 0 && grgb[0] == 0 &&
        grgb[1] == 0 && grgb[2] == 0 && gz == 0)
      continue;
    const KView& cv = views.v[v];
    Geom g;
    if (!gs_geom32(cv, mx, my, mz, S6, o.lowpass, o.extent, g)) continue;
    dopa += gop;
    // conic (A, B, C) = inverse of [[a, b], [b, c]]
    const float inv = 1.0f / g.det;
    const float A = g.c * inv, B = -g.b * inv, C = g.a * inv;
    // H = -Q G Q with G = [[gA, gB/2], [gB/2, gC]], Q = [[A, B], [B, C]]
    const float G00 = gA, G01 = 0.5f * gB, G11 = gC;
    const float QG00 = A * G00 + B * G01, QG01 = A * G01 + B * G11;
    const float QG10 = B * G00 + C * G01, QG11 = B * G01 + C * G11;
    const float H00 = -(QG00 * A + QG01 * B), H01 = -(QG00 * B + QG01 * C);
    const float H11 = -(QG10 * B + QG11 * C);
    // dL/dSigma2D as a full symmetric matrix Gs
    const float Gs[2][2] = {{H00, H01}, {H01, H11}};
    // dSigma3D = M^T Gs M ; dM = 2 Gs M Sigma
    const float S[3][3] = {{S6[0], S6[1], S6[2]}, {S6[1], S6[3], S6[4]}, {S6[2], S6[4], S6[5]}};
    float GM[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) GM[a][k] = Gs[a][0] * g.M[0][k] + Gs[a][1] * g.M[1][k];
    float D3[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) D3[r][k] = g.M[0][r] * GM[0][k] + g.M[1][r] * GM[1][k];
    dcv[0] += D3[0][0];
    dcv[1] += D3[0][1] + D3[1][0];
    dcv[2] += D3[0][2] + D3[2][0];
    dcv[3] += D3[1][1];
    dcv[4] += D3[1][2] + D3[2][1];
    dcv[5] += D3[2][2];
    float dM[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        dM[a][k] = 2.0f * (GM[a][0] * S[0][k] + GM[a][1] * S[1][k] + GM[a][2] * S[2][k]);
    // M0k = jx R0k + j02 R2k, M1k = jy R1k + j12 R2k
    float djx = 0, dj02 = 0, djy = 0, dj12 = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      djx += dM[0][k] * cv.R[k];
      dj02 += dM[0][k] * cv.R[6 + k];
      djy += dM[1][k] * cv.R[3 + k];
      dj12 += dM[1][k] * cv.R[6 + k];
    }
    const float tz = g.t[2];
    const float limx = 1.3f * ((0.5f * (float)cv.W) / cv.fx);
    const float limy = 1.3f * ((0.5f * (float)cv.H) / cv.fy);
    const bool inx = g.ux > -limx && g.ux < limx, iny = g.uy > -limy && g.uy < limy;
    const float cxl = clamp_f(g.ux, -limx, limx), cyl = clamp_f(g.uy, -limy, limy);
    // j02 = -jx cxl, j12 = -jy cyl
    djx += -dj02 * cxl;
    djy += -dj12 * cyl;
    float dux = inx ? -dj02 * g.jx : 0.0f;
    float duy = iny ? -dj12 * g.jy : 0.0f;
    // pixel position
    dux += gpx * cv.fx;
    duy += gpy * cv.fy;
    float dt[3];
    dt[0] = dux / tz;
    dt[1] = duy / tz;
    dt[2] = -dux * g.t[0] / (tz * tz) - duy * g.t[1] / (tz * tz) - djx * cv.fx / (tz * tz) -
            djy * cv.fy / (tz * tz) + gz;
    // colour
    float dx = mx - cv.cam[0], dy = my - cv.cam[1], dz = mz - cv.cam[2];
    const float len = sqrtf(dx * dx + dy * dy + dz * dz);
    const float rn = 1.0f / len;
    dx *= rn; dy *= rn; dz *= rn;
    float Y[16];
    sh_eval(deg, dx, dy, dz, Y);
    float dY[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) dY[k] = 0.0f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float pre = 0.5f;
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < K) pre += Y[k] * sh[(k * 3 + ch) * n + i];
      if (pre <= 0.0f || grgb[ch] == 0.0f) continue;  // clamped at zero: no gradient
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < K) {
          dshv[k][ch] += Y[k] * grgb[ch];
          dY[k] += sh[(k * 3 + ch) * n + i] * grgb[ch];
        }
    }
    float gdx, gdy, gdz;
    sh_grad_dir(deg, dx, dy, dz, dY, gdx, gdy, gdz);
    const float dot = gdx * dx + gdy * dy + gdz * dz;
    float dmv[3] = {(gdx - dx * dot) * rn, (gdy - dy * dot) * rn, (gdz - dz * dot) * rn};
    // t = R m + T
#pragma unroll
    for (int k = 0; k < 3; ++k)
      dm[k] += cv.R[k] * dt[0] + cv.R[3 + k] * dt[1] + cv.R[6 + k] * dt[2] + dmv[k];
  }
  d_mean[i] += dm[0];
  d_mean[n + i] += dm[1];
  d_mean[2 * n + i] += dm[2];
#pragma unroll
  for (int k = 0; k < 6; ++k) d_cov[k * n + i] += dcv[k];
  d_op[i] += dopa;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < K)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) d_sh[(k * 3 + ch) * n + i] += dshv[k][ch];
}

template <int TILE>
static void launch_blend_bwd(const RenderWs& L, void* ws, int64_t n, const KViews& kv,
                             const GsOpt& o, const float* tf, const float* d_rgb,
                             const float* d_depth, hipStream_t st) {
  hipLaunchKernelGGL(k_gs_blend_bwd<TILE>, dim3((unsigned)L.tiles_total),
                     dim3(BwdCfg<TILE>::BLOCK), 0, st, at<uint2>(ws, L.ranges),
                     at<uint32_t>(ws, L.ids), at<float4>(ws, L.rec), n,
                     kv, o, L.tiles_x, L.tiles_x * L.tiles_y, at<uint32_t>(ws, L.last), tf, d_rgb,
                     d_depth, at<float>(ws, L.g2d));
}

}  // namespace vrs

using namespace vrs;

extern "C" vrs_status vrs_render_gaussians_backward(
    const float* mean, const float* cov, const float* opacity, const float* sh, int sh_degree,
    int64_t n, const vrs_view* views, int n_views, const vrs_raster_opts* ro,
    const float* t_final, const float* d_rgb, const float* d_depth, float* d_mean, float* d_cov,
    float* d_opacity, float* d_sh, void* ws, size_t ws_bytes, int64_t max_pairs, void* stream) {
  GsOpt o;
  KViews kv;
  RenderWs L;
  if (!ro || !make_views(views, n_views, &kv)) return VRS_EINVAL;
  if (ro->order != VRS_ORDER_PRIMITIVE) return VRS_EUNSUPPORTED;
  o.tile = ro->tile; o.aclamp = ro->alpha_clamp; o.amin = ro->alpha_min; o.tmin = ro->t_min;
  o.order = ro->order;
  o.lowpass = ro->lowpass; o.extent = ro->extent;
  for (int k = 0; k < 3; ++k) o.bg[k] = ro->bg[k];
  for (int i = 1; i < n_views; ++i)
    if (views[i].width != views[0].width || views[i].height != views[0].height) return VRS_EINVAL;
  if (sh_degree < 0 || sh_degree > 3 || n < 0) return VRS_EINVAL;
  if (!render_layout(n, n_views, views, o.tile, opts_radix(ro), max_pairs, &L) || !ws ||
      ws_bytes < L.total)
    return VRS_EINVAL;
  if (!t_final || !d_rgb || (n > 0 && (!mean || !cov || !opacity || !sh || !d_mean || !d_cov ||
                                       !d_opacity || !d_sh)))
    return VRS_EINVAL;
  if (n == 0) return VRS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  VRS_HIP_CHECK(fill_u32(at<uint32_t>(ws, L.g2d), 0u, L.vn * kG2d, st));
  switch (o.tile) {
    case 8: launch_blend_bwd<8>(L, ws, n, kv, o, t_final, d_rgb, d_depth, st); break;
    case 16: launch_blend_bwd<16>(L, ws, n, kv, o, t_final, d_rgb, d_depth, st); break;
    default: launch_blend_bwd<32>(L, ws, n, kv, o, t_final, d_rgb, d_depth, st); break;
  }
  VRS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gs_project_bwd, dim3(div_up(n, 256)), dim3(256), 0, st, mean, cov, sh,
                     sh_degree, n, kv, o, at<float>(ws, L.g2d), d_mean, d_cov, d_opacity, d_sh);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}
