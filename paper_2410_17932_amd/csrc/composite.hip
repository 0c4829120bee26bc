// Combination of the periphery P and the foveal images F (Sec. 3.4,
// Eqs. 2-5), its adjoint, and the L1 photometric term of the fitting loss
// (Sec. 3.5, Eq. 6).
//
// One thread per four full-frame pixels of a row (one per pixel when the
// width is not a multiple of 4): the crop table travels as a kernel argument,
// each pixel walks the crops of its view in index order.  HBM-bound: P is
// read and out written once; F is read only under the crops.  In place (out
// is P) only the four-pixel groups under some crop are read and written.
#include "vrs_common.h"

namespace vrs {

struct CompArgs {
  int n_crops, W, H, nv, mode;
  float ring, m, gamma;
  int view[VRS_MAX_CROPS], x0[VRS_MAX_CROPS], y0[VRS_MAX_CROPS], S[VRS_MAX_CROPS];
  float gx[VRS_MAX_CROPS], gy[VRS_MAX_CROPS];
  long long fbase[VRS_MAX_CROPS];
  const int4* place;   // device crop placement (x0, y0, gaze), or null
};

// Origin and gaze of crop k: the host values, or the device placement
// table's (origins clamped into the view).
// Crop origin and gaze from the host table, or from the device placement
// table `pl` (a.place, or a workgroup's copy of it in LDS).
__device__ inline int cx0(const CompArgs& a, int k, const int4* pl) {
  return pl ? clamp_origin(pl[k].x, a.W - a.S[k]) : a.x0[k];
}
__device__ inline int cy0(const CompArgs& a, int k, const int4* pl) {
  return pl ? clamp_origin(pl[k].y, a.H - a.S[k]) : a.y0[k];
}
__device__ inline float cgx(const CompArgs& a, int k, const int4* pl) {
  return pl ? __int_as_float(pl[k].z) : a.gx[k];
}
__device__ inline float cgy(const CompArgs& a, int k, const int4* pl) {
  return pl ? __int_as_float(pl[k].w) : a.gy[k];
}
__device__ inline int cx0(const CompArgs& a, int k) { return cx0(a, k, a.place); }
__device__ inline int cy0(const CompArgs& a, int k) { return cy0(a, k, a.place); }
__device__ inline float cgx(const CompArgs& a, int k) { return cgx(a, k, a.place); }
__device__ inline float cgy(const CompArgs& a, int k) { return cgy(a, k, a.place); }

__device__ inline float clamp01(float x) { return x < 0.0f ? 0.0f : (x > 1.0f ? 1.0f : x); }

__device__ inline float gray_at(const float* F, int S, int x, int y) {
  x = x < 0 ? 0 : (x > S - 1 ? S - 1 : x);
  y = y < 0 ? 0 : (y > S - 1 ? S - 1 : y);
  const long long pl = (long long)S * S, o = (long long)y * S + x;
  return (F[o] + F[pl + o] + F[2 * pl + o]) * (1.0f / 3.0f);
}

// Sobel gradients of the channel-mean image at (x, y), replicated borders.
__device__ inline void sobel(const float* F, int S, int x, int y, float& gx, float& gy) {
  const float a = gray_at(F, S, x - 1, y - 1), b = gray_at(F, S, x, y - 1),
              c = gray_at(F, S, x + 1, y - 1), d = gray_at(F, S, x - 1, y),
              e = gray_at(F, S, x + 1, y), f = gray_at(F, S, x - 1, y + 1),
              g = gray_at(F, S, x, y + 1), h = gray_at(F, S, x + 1, y + 1);
  gx = (c + 2.0f * e + h) - (a + 2.0f * d + f);
  gy = (f + 2.0f * g + h) - (a + 2.0f * b + c);
}

__device__ inline float smootherstep(float x) { return x * x * x * (x * (6.0f * x - 15.0f) + 10.0f); }
__device__ inline float smootherstep_d(float x) { return 30.0f * x * x * (x - 1.0f) * (x - 1.0f); }

// Blend mask c of crop k at crop pixel (lx, ly); u_out = argument of S2
// (PAPER mode), fe_out = edge term.
__device__ inline float blend_mask(const CompArgs& a, int k, const float* F, int lx, int ly,
                                   float& u_out, float& gx, float& gy, const int4* pl) {
  const float dx = (float)(cx0(a, k, pl) + lx) + 0.5f - cgx(a, k, pl);
  const float dy = (float)(cy0(a, k, pl) + ly) + 0.5f - cgy(a, k, pl);
  const float r = sqrtf(dx * dx + dy * dy);
  const float df = 0.5f * (float)a.S[k];
  if (a.mode == VRS_BLEND_LINEAR) {
    u_out = 0.0f;
    gx = gy = 0.0f;
    return clamp01((df - r) / a.ring);
  }
  const float rn = clamp01(r / df);
  const float fp = (rn - a.m) / (1.0f - a.m);
  // gamma = 0: Eq. 5 without the edge term (Eq. 4), no Sobel work
  gx = gy = 0.0f;
  if (a.gamma != 0.0f) sobel(F, a.S[k], lx, ly, gx, gy);
  const float fe = 0.25f * sqrtf(gx * gx + gy * gy);
  u_out = fp + a.gamma * fe;
  return 1.0f - smootherstep(clamp01(u_out));
}

__global__ __launch_bounds__(256) void k_composite(CompArgs a, const float* P,
                                                   const float* __restrict__ F, float* out) {
  const long long plane = (long long)a.W * a.H;
  const long long total = plane * a.nv;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int v = (int)(i / plane);
    const long long pi = i - v * plane;
    const int y = (int)(pi / a.W), x = (int)(pi - (long long)y * a.W);
    const long long base = (long long)v * 3 * plane + pi;
    float o0 = P[base], o1 = P[base + plane], o2 = P[base + 2 * plane];
    for (int k = 0; k < a.n_crops; ++k) {
      if (a.view[k] != v) continue;
      const int lx = x - cx0(a, k), ly = y - cy0(a, k), S = a.S[k];
      if (lx < 0 || ly < 0 || lx >= S || ly >= S) continue;
      {
        // outside the crop's inscribed circle the mask is 0 in both modes
        const float dx = (float)(cx0(a, k) + lx) + 0.5f - cgx(a, k);
        const float dy = (float)(cy0(a, k) + ly) + 0.5f - cgy(a, k);
        if (!(sqrtf(dx * dx + dy * dy) < 0.5f * (float)S)) continue;
      }
      const float* Fk = F + a.fbase[k];
      float u, gx, gy;
      const float c = blend_mask(a, k, Fk, lx, ly, u, gx, gy, a.place);
      const long long fp = (long long)S * S, fo = (long long)ly * S + lx;
      o0 = (1.0f - c) * o0 + c * Fk[fo];
      o1 = (1.0f - c) * o1 + c * Fk[fp + fo];
      o2 = (1.0f - c) * o2 + c * Fk[2 * fp + fo];
    }
    out[base] = o0;
    out[base + plane] = o1;
    out[base + 2 * plane] = o2;
  }
}

// Same per pixel as k_composite, four consecutive pixels of a row per thread
// (W % 4 == 0): 16-byte loads and stores of P and out, crops rejected once
// per four pixels.
// Four pixels (v, y, x..x+3) of a row: their crop chain from P into out
// (which may be P: every read comes before the writes).
// cand: the crops that may cover the quad (bit k), walked in crop order.
__device__ inline void comp_quad(const CompArgs& a, const float* P, const float* __restrict__ F,
                                 float* out, int v, int y, int x, const int4* pl, uint32_t cand) {
  const long long plane = (long long)a.W * a.H;
  const long long base = (long long)v * 3 * plane + (long long)y * a.W + x;
  float4 c4[3] = {*reinterpret_cast<const float4*>(P + base),
                  *reinterpret_cast<const float4*>(P + base + plane),
                  *reinterpret_cast<const float4*>(P + base + 2 * plane)};
  float o[3][4];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    o[ch][0] = c4[ch].x; o[ch][1] = c4[ch].y; o[ch][2] = c4[ch].z; o[ch][3] = c4[ch].w;
  }
  while (cand) {
    const int k = __builtin_ctz(cand);
    cand &= cand - 1;
    if (a.view[k] != v) continue;
    const int S = a.S[k], ly = y - cy0(a, k, pl);
    if (ly < 0 || ly >= S || x + 3 < cx0(a, k, pl) || x >= cx0(a, k, pl) + S) continue;
    const float* Fk = F + a.fbase[k];
    const long long fp = (long long)S * S;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int lx = x + j - cx0(a, k, pl);
      if (lx < 0 || lx >= S) continue;
      {
        // outside the crop's inscribed circle the mask is 0 in both modes
        // (the same operations as blend_mask): the pixel keeps its value
        const float dx = (float)(cx0(a, k, pl) + lx) + 0.5f - cgx(a, k, pl);
        const float dy = (float)(cy0(a, k, pl) + ly) + 0.5f - cgy(a, k, pl);
        if (!(sqrtf(dx * dx + dy * dy) < 0.5f * (float)S)) continue;
      }
      float u, gx, gy;
      const float c = blend_mask(a, k, Fk, lx, ly, u, gx, gy, pl);
      const long long fo = (long long)ly * S + lx;
      o[0][j] = (1.0f - c) * o[0][j] + c * Fk[fo];
      o[1][j] = (1.0f - c) * o[1][j] + c * Fk[fp + fo];
      o[2][j] = (1.0f - c) * o[2][j] + c * Fk[2 * fp + fo];
    }
  }
#pragma unroll
  for (int ch = 0; ch < 3; ++ch)
    *reinterpret_cast<float4*>(out + base + ch * plane) =
        make_float4(o[ch][0], o[ch][1], o[ch][2], o[ch][3]);
}

__global__ __launch_bounds__(256) void k_composite4(CompArgs a, const float* __restrict__ P,
                                                    const float* __restrict__ F,
                                                    float* __restrict__ out) {
  const long long plane = (long long)a.W * a.H, qplane = plane / 4;
  const long long total = qplane * a.nv;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const int v = (int)(q / qplane);
    const long long pi = (q - v * qplane) * 4;
    const int y = (int)(pi / a.W), x = (int)(pi - (long long)y * a.W);
    comp_quad(a, P, F, out, v, y, x, a.place, a.n_crops >= 32 ? ~0u : (1u << a.n_crops) - 1u);
  }
}

// In place: workgroup (b, k) takes crop k's four-pixel groups [256 b,
// 256 b + 256) in row order over the crop's rows and the groups its columns
// touch; a group under several crops is done once, by the first of them,
// with the whole crop chain.  Pixels under no crop are not touched.
__global__ __launch_bounds__(256) void k_composite4_inplace(CompArgs a, float* io,
                                                            const float* __restrict__ F) {
  // the device placement table read once per workgroup: every pixel walks
  // the crop chain, which would otherwise wait on a load per crop
  __shared__ int4 s_pl[VRS_MAX_CROPS];
  __shared__ uint32_t s_near;
  const int4* pl = nullptr;
  if (a.place) {   // uniform
    if (threadIdx.x < a.n_crops) s_pl[threadIdx.x] = a.place[threadIdx.x];
    __syncthreads();
    pl = s_pl;
  }
  const int kc = blockIdx.y;
  const int S = a.S[kc], v = a.view[kc];
  const int gx0 = cx0(a, kc, pl) >> 2, ng = ((cx0(a, kc, pl) + S - 1) >> 2) - gx0 + 1;
  // the crops whose square meets this crop's four-pixel groups: the only
  // ones any of the workgroup's groups can lie under (crop kc among them)
  if (threadIdx.x < 64) {
    const int k = threadIdx.x;
    bool near = false;
    if (k < a.n_crops && a.view[k] == v) {
      const int kx = cx0(a, k, pl), ky = cy0(a, k, pl), ks = a.S[k];
      const int ky0 = cy0(a, kc, pl);
      near = kx < (gx0 + ng) * 4 && kx + ks > gx0 * 4 && ky < ky0 + S && ky + ks > ky0;
    }
    const uint64_t m = __ballot(near);
    if (threadIdx.x == 0) s_near = (uint32_t)m;
  }
  __syncthreads();
  const uint32_t near = s_near;
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= (long long)S * ng) return;
  const int ly = (int)(i / ng);
  const int y = cy0(a, kc, pl) + ly, x = (gx0 + (int)(i - (long long)ly * ng)) * 4;
  for (uint32_t e = near & ((1u << kc) - 1u); e; e &= e - 1) {
    const int k = __builtin_ctz(e);
    if (a.view[k] == v && y >= cy0(a, k, pl) && y < cy0(a, k, pl) + a.S[k] &&
        x + 3 >= cx0(a, k, pl) && x < cx0(a, k, pl) + a.S[k])
      return;   // an earlier crop's group
  }
  comp_quad(a, io, F, io, v, y, x, pl, near);
}

// Adjoint.  Per pixel the crop chain is replayed forward to recover the
// intermediate images, then walked backwards:
//   dF_k += c_k g,  dc_k = <g, F_k - out_{k-1}>,  g <- (1 - c_k) g,  dP += g.
// In PAPER mode dc_k also flows into F_k through the Sobel edge term
// (scattered to the 3x3 neighbourhood with atomics).
__global__ __launch_bounds__(256) void k_composite_bwd(CompArgs a, const float* __restrict__ P,
                                                       const float* __restrict__ F,
                                                       const float* __restrict__ dout,
                                                       float* __restrict__ dP,
                                                       float* __restrict__ dF) {
  const long long plane = (long long)a.W * a.H;
  const long long total = plane * a.nv;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int v = (int)(i / plane);
    const long long pi = i - v * plane;
    const int y = (int)(pi / a.W), x = (int)(pi - (long long)y * a.W);
    const long long base = (long long)v * 3 * plane + pi;
    int ks[VRS_MAX_CROPS];
    int nk = 0;
    for (int k = 0; k < a.n_crops; ++k) {
      if (a.view[k] != v) continue;
      const int lx = x - cx0(a, k), ly = y - cy0(a, k);
      if (lx < 0 || ly < 0 || lx >= a.S[k] || ly >= a.S[k]) continue;
      ks[nk++] = k;
    }
    float g0 = dout[base], g1 = dout[base + plane], g2 = dout[base + 2 * plane];
    if (nk > 0) {
      // forward replay: o_j = image after crop j
      float o[VRS_MAX_CROPS + 1][3];
      float cs[VRS_MAX_CROPS], us[VRS_MAX_CROPS], gxs[VRS_MAX_CROPS], gys[VRS_MAX_CROPS];
      o[0][0] = P[base]; o[0][1] = P[base + plane]; o[0][2] = P[base + 2 * plane];
      for (int j = 0; j < nk; ++j) {
        const int k = ks[j], S = a.S[k];
        const int lx = x - cx0(a, k), ly = y - cy0(a, k);
        const float* Fk = F + a.fbase[k];
        cs[j] = blend_mask(a, k, Fk, lx, ly, us[j], gxs[j], gys[j], a.place);
        const long long fp = (long long)S * S, fo = (long long)ly * S + lx;
        for (int ch = 0; ch < 3; ++ch)
          o[j + 1][ch] = (1.0f - cs[j]) * o[j][ch] + cs[j] * Fk[ch * fp + fo];
      }
      for (int j = nk - 1; j >= 0; --j) {
        const int k = ks[j], S = a.S[k];
        const int lx = x - cx0(a, k), ly = y - cy0(a, k);
        const float* Fk = F + a.fbase[k];
        const long long fp = (long long)S * S, fo = (long long)ly * S + lx;
        const float c = cs[j];
        const float f0 = Fk[fo], f1 = Fk[fp + fo], f2 = Fk[2 * fp + fo];
        const float dc = g0 * (f0 - o[j][0]) + g1 * (f1 - o[j][1]) + g2 * (f2 - o[j][2]);
        if (dF) {
          float* dFk = dF + a.fbase[k];
          if (a.mode == VRS_BLEND_PAPER) {
            // neighbours scatter into this crop pixel too (edge term)
            atomicAdd(&dFk[fo], c * g0);
            atomicAdd(&dFk[fp + fo], c * g1);
            atomicAdd(&dFk[2 * fp + fo], c * g2);
          } else {
            dFk[fo] += c * g0;
            dFk[fp + fo] += c * g1;
            dFk[2 * fp + fo] += c * g2;
          }
          const float u = us[j];
          if (a.mode == VRS_BLEND_PAPER && u > 0.0f && u < 1.0f) {
            // c = 1 - S2(u), u = fp + gamma |grad|/4
            const float mag = sqrtf(gxs[j] * gxs[j] + gys[j] * gys[j]);
            if (mag > 0.0f) {
              const float dfe = -smootherstep_d(u) * a.gamma * dc;
              const float s = dfe * 0.25f / mag / 3.0f;  // d|g|/dg = g/|g|; gray = mean/3
              const float wx = s * gxs[j], wy = s * gys[j];
              // Sobel taps: gx weights (+1,+2,+1 on x+1; -1,-2,-1 on x-1),
              // gy weights (+1,+2,+1 on y+1; -1,-2,-1 on y-1)
              for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                  const float kx = (float)ox * (oy == 0 ? 2.0f : 1.0f);
                  const float ky = (float)oy * (ox == 0 ? 2.0f : 1.0f);
                  const float wgt = kx * wx + ky * wy;
                  if (wgt == 0.0f) continue;
                  int sx = lx + ox, sy = ly + oy;
                  sx = sx < 0 ? 0 : (sx > S - 1 ? S - 1 : sx);
                  sy = sy < 0 ? 0 : (sy > S - 1 ? S - 1 : sy);
                  const long long so = (long long)sy * S + sx;
                  atomicAdd(&dFk[so], wgt);
                  atomicAdd(&dFk[fp + so], wgt);
                  atomicAdd(&dFk[2 * fp + so], wgt);
                }
            }
          }
        }
        g0 *= 1.0f - c;
        g1 *= 1.0f - c;
        g2 *= 1.0f - c;
      }
    }
    if (dP) {
      dP[base] += g0;
      dP[base + plane] += g1;
      dP[base + 2 * plane] += g2;
    }
  }
}

// L1: block partial sums of |pred - target| atomically added to loss[0]
// (zeroed by the preceding fill), gradient scale*sign(pred - target)/n.
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ pred,
                                            const float* __restrict__ target, long long n,
                                            float* loss, float* __restrict__ dpred, float scale) {
  __shared__ float s_part[4];
  float acc = 0.0f;
  const float inv = 1.0f / (float)n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float d = pred[i] - target[i];
    acc += fabsf(d);
    if (dpred) dpred[i] += d > 0.0f ? scale * inv : (d < 0.0f ? -scale * inv : 0.0f);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s_part[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, (s_part[0] + s_part[1] + s_part[2] + s_part[3]) * inv);
}

__global__ void k_zero1(float* p) { *p = 0.0f; }

static bool comp_args(int nv, int W, int H, const vrs_crop* crops, int n_crops, int mode,
                      float ring, float m, float gamma, const vrs_crop_place* place,
                      CompArgs* a) {
  if (nv < 1 || nv > VRS_MAX_VIEWS || W < 1 || H < 1 || n_crops < 0 || n_crops > VRS_MAX_CROPS ||
      (n_crops > 0 && !crops))
    return false;
  if (mode != VRS_BLEND_LINEAR && mode != VRS_BLEND_PAPER) return false;
  if (mode == VRS_BLEND_LINEAR && !(ring > 0)) return false;
  if (mode == VRS_BLEND_PAPER && !(m < 1.0f)) return false;
  a->n_crops = n_crops;
  a->W = W;
  a->H = H;
  a->nv = nv;
  a->mode = mode;
  a->ring = ring;
  a->m = m;
  a->gamma = gamma;
  a->place = reinterpret_cast<const int4*>(place);
  long long fb = 0;
  for (int k = 0; k < n_crops; ++k) {
    const vrs_crop& c = crops[k];
    if (c.view < 0 || c.view >= nv || c.size < 1 || c.size > W || c.size > H) return false;
    if (!place && (c.x0 < 0 || c.y0 < 0 || c.x0 + c.size > W || c.y0 + c.size > H)) return false;
    a->view[k] = c.view;
    a->x0[k] = c.x0;
    a->y0[k] = c.y0;
    a->S[k] = c.size;
    a->gx[k] = c.gaze_x;
    a->gy[k] = c.gaze_y;
    a->fbase[k] = fb;
    fb += 3LL * c.size * c.size;
  }
  return true;
}

}  // namespace vrs

using namespace vrs;

namespace vrs {
vrs_status composite_impl(const float* rgb_periphery, int n_views, int width, int height,
                          const float* fovea_rgb, const vrs_crop* crops, int n_crops,
                          const vrs_crop_place* place, int mode, float ring, float m, float gamma,
                          float* out, void* stream, const Trace* tr) {
  CompArgs a;
  if (!comp_args(n_views, width, height, crops, n_crops, mode, ring, m, gamma, place, &a))
    return VRS_EINVAL;
  if (!rgb_periphery || !out || (n_crops > 0 && !fovea_rgb)) return VRS_EINVAL;
  const long long total = (long long)width * height * n_views;
  trace_begin(tr, VRS_TRACE_COMPOSITE, static_cast<hipStream_t>(stream));
  const bool vec4 = width % 4 == 0 && (reinterpret_cast<uintptr_t>(rgb_periphery) & 15) == 0 &&
                    (reinterpret_cast<uintptr_t>(out) & 15) == 0;
  if (vec4 && out == rgb_periphery) {
    // four-pixel groups of the largest crop (for origins read on the
    // device, as many as any origin can give: ((S + 2) >> 2) + 1 per row)
    long long most = 0;
    for (int k = 0; k < n_crops; ++k) {
      const int S = crops[k].size;
      const long long row = place ? ((S + 2) >> 2) + 1
                                  : ((crops[k].x0 + S - 1) >> 2) - (crops[k].x0 >> 2) + 1;
      most = std::max<long long>(most, (long long)S * row);
    }
    if (n_crops > 0)
      hipLaunchKernelGGL(k_composite4_inplace, dim3((unsigned)((most + 255) / 256), n_crops),
                         dim3(256), 0, static_cast<hipStream_t>(stream), a, out, fovea_rgb);
  } else if (vec4) {
    const int blocks = (int)std::min<long long>(16384, (total / 4 + 255) / 256);
    hipLaunchKernelGGL(k_composite4, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                       a, rgb_periphery, fovea_rgb, out);
  } else {
    const int blocks = (int)std::min<long long>(16384, (total + 255) / 256);
    hipLaunchKernelGGL(k_composite, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                       a, rgb_periphery, fovea_rgb, out);
  }
  VRS_LAUNCH_CHECK();
  trace_end(tr, VRS_TRACE_COMPOSITE, static_cast<hipStream_t>(stream));
  return VRS_OK;
}
}  // namespace vrs

extern "C" vrs_status vrs_composite_frame(const float* rgb_periphery, int n_views, int width,
                                          int height, const float* fovea_rgb,
                                          const vrs_crop* crops, int n_crops,
                                          const vrs_crop_place* place, int mode, float ring,
                                          float m, float gamma, float* out, void* stream) {
  return composite_impl(rgb_periphery, n_views, width, height, fovea_rgb, crops, n_crops, place,
                        mode, ring, m, gamma, out, stream, nullptr);
}

extern "C" vrs_status vrs_composite_frame_backward(const float* rgb_periphery, int n_views,
                                                   int width, int height, const float* fovea_rgb,
                                                   const vrs_crop* crops, int n_crops,
                                                   const vrs_crop_place* place, int mode,
                                                   float ring, float m, float gamma,
                                                   const float* d_out, float* d_rgb_periphery,
                                                   float* d_fovea, void* stream) {
  CompArgs a;
  if (!comp_args(n_views, width, height, crops, n_crops, mode, ring, m, gamma, place, &a))
    return VRS_EINVAL;
  if (!rgb_periphery || !d_out || (n_crops > 0 && !fovea_rgb)) return VRS_EINVAL;
  const long long total = (long long)width * height * n_views;
  const int blocks = (int)std::min<long long>(16384, (total + 255) / 256);
  hipLaunchKernelGGL(k_composite_bwd, dim3(blocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), a, rgb_periphery, fovea_rgb, d_out,
                     d_rgb_periphery, d_fovea);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}

extern "C" vrs_status vrs_l1_loss(const float* pred, const float* target, int64_t n, float* loss,
                                  float* d_pred, float scale, void* stream) {
  if (!pred || !target || !loss || n < 1) return VRS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, st, loss);
  const int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_l1, dim3(blocks), dim3(256), 0, st, pred, target, (long long)n, loss,
                     d_pred, scale);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}
