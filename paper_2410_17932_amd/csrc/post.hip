// After the combination: tone mapping (Sec. 3.4, the ADOP camera model, in
// the reading stated in vrsplat.h) and the training objective's kernels
// (Sec. 3.5, Eqs. 6-7): D-SSIM, the regulariser R, and the Adam step.
//
// All of them stream their images once (the SSIM tiles re-read a 5-pixel
// halo), so each is bound by HBM bandwidth.  Sums over an image are
// deterministic (per-block partials reduced in a fixed order), except the
// response-curve gradient, accumulated per block with LDS atomics.
#include <cmath>

#include "vrs_common.h"

namespace vrs {
namespace {

// ------------------------------------------------------------ tone mapping
constexpr int kTmFixed = 7, kTmMaxResp = 256;
constexpr int kTmBlock = 256, kTmBlocksPerView = 1024;

struct TmView {
  float cx, cy, inv_d2;   // principal point, rounded 1 / half-diagonal^2
};
struct TmArgs {
  TmView v[VRS_MAX_VIEWS];
  int nv, W, H, n;        // views, size, response samples
};

bool tm_args(const vrs_view* views, int nv, int n, TmArgs* a) {
  if (!views || nv < 1 || nv > VRS_MAX_VIEWS || n < 2 || n > kTmMaxResp) return false;
  const int W = views[0].width, H = views[0].height;
  if (W < 1 || H < 1) return false;
  for (int i = 0; i < nv; ++i) {
    if (views[i].width != W || views[i].height != H) return false;
    const double hd2 = (W / 2.0) * (W / 2.0) + (H / 2.0) * (H / 2.0);
    a->v[i] = TmView{views[i].cx, views[i].cy, (float)(1.0 / hd2)};
  }
  a->nv = nv;
  a->W = W;
  a->H = H;
  a->n = n;
  return true;
}

// Per-block view constants: 2^-ev rounded from double precision, white
// balance, vignetting coefficients, the response samples in LDS.
struct TmShared {
  float e, wb[3], k[3];
  float resp[kTmMaxResp];
};

__device__ inline void tm_load(TmShared& sh, const float* __restrict__ par, int n) {
  if (threadIdx.x == 0) {
    sh.e = (float)exp2(-(double)par[0]);
    for (int c = 0; c < 3; ++c) {
      sh.wb[c] = par[1 + c];
      sh.k[c] = par[4 + c];
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) sh.resp[i] = par[kTmFixed + i];
  __syncthreads();
}

// Squared normalised radius and vignetting factor of pixel (x, y), in the
// documented single-precision order.
__device__ inline void tm_vig(const TmView& tv, const TmShared& sh, int x, int y, float& r2,
                              float& vig) {
#pragma clang fp contract(off)
  const float dx = ((float)x + 0.5f) - tv.cx, dy = ((float)y + 0.5f) - tv.cy;
  r2 = (dy * dy + dx * dx) * tv.inv_d2;
  vig = ((sh.k[2] * r2 + sh.k[1]) * r2 + sh.k[0]) * r2 + 1.0f;
}

// t, its segment i and fraction f, and whether t is inside (0, 1).
__device__ inline float tm_t(float x, float e, float wb, float vig) {
#pragma clang fp contract(off)
  return ((x * e) * wb) * vig;
}
__device__ inline int tm_seg(float t, int n, float& f) {
#pragma clang fp contract(off)
  const float s = fminf(fmaxf(t, 0.0f), 1.0f) * (float)(n - 1);
  const int i = min((int)floorf(s), n - 2);
  f = s - (float)i;
  return i;
}

__global__ __launch_bounds__(kTmBlock) void k_tonemap(const float* __restrict__ in,
                                                      const float* __restrict__ params, TmArgs a,
                                                      float* __restrict__ out) {
  __shared__ TmShared sh;
  const int v = blockIdx.y;
  const int P = kTmFixed + a.n;
  tm_load(sh, params + (int64_t)v * P, a.n);
  const int64_t plane = (int64_t)a.W * a.H;
  const float* src = in + (int64_t)v * 3 * plane;
  float* dst = out + (int64_t)v * 3 * plane;
  for (int64_t p = blockIdx.x * (int64_t)kTmBlock + threadIdx.x; p < plane;
       p += (int64_t)gridDim.x * kTmBlock) {
    const int y = (int)(p / a.W), x = (int)(p - (int64_t)y * a.W);
    float r2, vig;
    tm_vig(a.v[v], sh, x, y, r2, vig);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float t = tm_t(src[c * plane + p], sh.e, sh.wb[c], vig);
      float f;
      const int i = tm_seg(t, a.n, f);
      dst[c * plane + p] = fmaf(f, sh.resp[i + 1] - sh.resp[i], sh.resp[i]);
    }
  }
}

// Adjoint: d_in written; per block partial sums of the parameters'
// gradients, [view][block][7 + n].
__global__ __launch_bounds__(kTmBlock) void k_tonemap_bwd(
    const float* __restrict__ in, const float* __restrict__ params, TmArgs a,
    const float* __restrict__ d_out, float* __restrict__ d_in, float* __restrict__ partial) {
  __shared__ TmShared sh;
  __shared__ float s_dr[kTmMaxResp];
  __shared__ float s_red[kTmBlock / 64][kTmFixed];
  const int v = blockIdx.y;
  const int P = kTmFixed + a.n;
  for (int i = threadIdx.x; i < a.n; i += kTmBlock) s_dr[i] = 0.0f;
  tm_load(sh, params + (int64_t)v * P, a.n);
  const int64_t plane = (int64_t)a.W * a.H;
  const float* src = in + (int64_t)v * 3 * plane;
  const float* g = d_out + (int64_t)v * 3 * plane;
  float acc[kTmFixed] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t p = blockIdx.x * (int64_t)kTmBlock + threadIdx.x; p < plane;
       p += (int64_t)gridDim.x * kTmBlock) {
    const int y = (int)(p / a.W), x = (int)(p - (int64_t)y * a.W);
    float r2, vig;
    tm_vig(a.v[v], sh, x, y, r2, vig);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float xi = src[c * plane + p];
      const float gi = g[c * plane + p];
      const float t = tm_t(xi, sh.e, sh.wb[c], vig);
      float f;
      const int i = tm_seg(t, a.n, f);
      atomicAdd(&s_dr[i], gi * (1.0f - f));
      atomicAdd(&s_dr[i + 1], gi * f);
      const bool inside = t > 0.0f && t < 1.0f;
      const float dt = inside ? gi * (sh.resp[i + 1] - sh.resp[i]) * (float)(a.n - 1) : 0.0f;
      if (d_in) d_in[(int64_t)v * 3 * plane + c * plane + p] = dt * sh.e * sh.wb[c] * vig;
      acc[0] += dt * t;
      acc[1 + c] += dt * xi * sh.e * vig;
      const float base = dt * xi * sh.e * sh.wb[c];
      acc[4] += base * r2;
      acc[5] += base * r2 * r2;
      acc[6] += base * r2 * r2 * r2;
    }
  }
  acc[0] *= -0.69314718055994531f;   // d t / d ev = -ln 2 t
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kTmFixed; ++q) {
    float s = acc[q];
#pragma unroll
    for (int sh2 = 32; sh2 > 0; sh2 >>= 1) s += __shfl_xor(s, sh2, 64);
    if (lane == 0) s_red[wave][q] = s;
  }
  __syncthreads();
  if (!partial) return;
  float* out = partial + ((int64_t)v * gridDim.x + blockIdx.x) * P;
  if (threadIdx.x < kTmFixed) {
    float s = 0.0f;
    for (int w = 0; w < kTmBlock / 64; ++w) s += s_red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
  for (int i = threadIdx.x; i < a.n; i += kTmBlock) out[kTmFixed + i] = s_dr[i];
}

// d_params[v][q] += sum over blocks of partial[v][b][q], in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_partials(const float* __restrict__ partial,
                                                         int nb, int P,
                                                         float* __restrict__ d_params) {
  __shared__ float s[256];
  const int q = blockIdx.x, v = blockIdx.y;
  float acc = 0.0f;
  for (int b = threadIdx.x; b < nb; b += 256) acc += partial[((int64_t)v * nb + b) * P + q];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) d_params[(int64_t)v * P + q] += s[0];
}

int tm_blocks(const TmArgs& a) {
  return std::max(1, std::min(kTmBlocksPerView, div_up((int64_t)a.W * a.H, kTmBlock)));
}

// ------------------------------------------------------------------- SSIM
constexpr int kSsTile = 32, kSsHalo = 5, kSsIn = kSsTile + 2 * kSsHalo;   // 42
constexpr int kSsBlock = 256;

struct SsArgs {
  int planes, W, H;
  int tiles_x, tiles_y;
  float w[11];   // the window's 1-D taps, rounded from double precision
};

// Separable 11-tap blur of NM maps staged in LDS (in: [NM][42][43]) to the
// tile's 32 x 32 outputs; each thread produces four rows of one column.
// hbuf: [NM][42][33].  Returns the blurred values o[NM][4].
template <int NM>
__device__ inline void ss_blur(const SsArgs& a, float (*in)[kSsIn][kSsIn + 1],
                               float (*hbuf)[kSsIn][kSsTile + 1], float o[NM][4]) {
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  for (int r = ty; r < kSsIn; r += 8) {
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      float s = 0.0f;
#pragma unroll
      for (int j = 0; j < 11; ++j) s = fmaf(a.w[j], in[m][r][tx + j], s);
      hbuf[m][r][tx] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      float s = 0.0f;
#pragma unroll
      for (int j = 0; j < 11; ++j) s = fmaf(a.w[j], hbuf[m][r + j][tx], s);
      o[m][q] = s;
    }
  }
}

// Loads NM planes' halo tiles (zero outside the image) into LDS.
template <int NM>
__device__ inline void ss_stage(const float* const src[NM], const SsArgs& a, int X0, int Y0,
                                float (*in)[kSsIn][kSsIn + 1]) {
  for (int idx = threadIdx.x; idx < kSsIn * kSsIn; idx += kSsBlock) {
    const int r = idx / kSsIn, c = idx - r * kSsIn;
    const int y = Y0 + r - kSsHalo, x = X0 + c - kSsHalo;
    const bool ok = x >= 0 && x < a.W && y >= 0 && y < a.H;
#pragma unroll
    for (int m = 0; m < NM; ++m) in[m][r][c] = ok ? src[m][(int64_t)y * a.W + x] : 0.0f;
  }
  __syncthreads();
}

// SSIM over one tile, from seven blurred moments of x, y and e = x - y
// (mu_x, mu_y, E[x^2], E[y^2], E[xy], D = mu_e, E[e^2]).  With a1 = 2 mu_x
// mu_y + C1, a2 = 2 s_xy + C2, b1 = a1 + D^2 (= mu_x^2 + mu_y^2 + C1),
// b2 = a2 + v_e (= s_xx + s_yy + C2, v_e = E[e^2] - D^2), the map's
// complement is 1 - SSIM = (b1 v_e + D^2 a2) / (b1 b2): no difference of
// nearly equal terms where x and y agree.  MAPS: writes the map's partials
// in (mu_x, E[x^2]) and their combination with E[xy]'s, in the same
// difference form (A, B, C' = C + 2B: A = -2 a2 D (mu_y (mu_x + mu_y) + C1)
// / (b1^2 b2) + 2 a1 (D a2 - mu_y v_e) / (b1 b2^2), B = -SSIM / b2,
// C' = 2 a1 v_e / (b1 b2^2)) to maps [3][planes][H][W]; else the block's sum
// of 1 - SSIM to partial[block].
template <bool MAPS>
__global__ __launch_bounds__(kSsBlock) void k_ssim(const float* __restrict__ x,
                                                   const float* __restrict__ y, SsArgs a,
                                                   float* __restrict__ maps,
                                                   float* __restrict__ partial) {
  __shared__ float s_in[2][kSsIn][kSsIn + 1];
  __shared__ float s_h[7][kSsIn][kSsTile + 1];
  __shared__ float s_red[kSsBlock / 64];
  const int pl = blockIdx.z;
  const int X0 = blockIdx.x * kSsTile, Y0 = blockIdx.y * kSsTile;
  const int64_t plane = (int64_t)a.W * a.H;
  {
    const float* src[2] = {x + pl * plane, y + pl * plane};
    ss_stage<2>(src, a, X0, Y0, s_in);
  }
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // horizontal pass: the seven moments from x and y on the fly
  for (int r = ty; r < kSsIn; r += 8) {
    float h[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 11; ++j) {
      const float w = a.w[j], u = s_in[0][r][tx + j], v = s_in[1][r][tx + j], e = u - v;
      h[0] = fmaf(w, u, h[0]);
      h[1] = fmaf(w, v, h[1]);
      h[2] = fmaf(w, u * u, h[2]);
      h[3] = fmaf(w, v * v, h[3]);
      h[4] = fmaf(w, u * v, h[4]);
      h[5] = fmaf(w, e, h[5]);
      h[6] = fmaf(w, e * e, h[6]);
    }
#pragma unroll
    for (int m = 0; m < 7; ++m) s_h[m][r][tx] = h[m];
  }
  __syncthreads();
  const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
  float sum = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    float o[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      float t = 0.0f;
#pragma unroll
      for (int j = 0; j < 11; ++j) t = fmaf(a.w[j], s_h[m][r + j][tx], t);
      o[m] = t;
    }
    const int gx = X0 + tx, gy = Y0 + r;
    if (gx >= a.W || gy >= a.H) continue;
    const float mx = o[0], my = o[1], D = o[5];
    const float sxy = o[4] - mx * my;
    const float ve = o[6] - D * D;
    const float a1 = 2.0f * mx * my + C1, a2 = 2.0f * sxy + C2;
    const float b1 = a1 + D * D, b2 = a2 + ve;
    const float inv = 1.0f / (b1 * b2);
    if (MAPS) {
      const float s = a1 * a2 * inv;
      const float A = -2.0f * a2 * D * (my * (mx + my) + C1) * inv / b1 +
                      2.0f * a1 * (D * a2 - my * ve) * inv / b2;
      const int64_t o2 = pl * plane + (int64_t)gy * a.W + gx;
      const int64_t all = (int64_t)a.planes * plane;
      maps[o2] = A;
      maps[all + o2] = -s / b2;
      maps[2 * all + o2] = 2.0f * a1 * ve * inv / b2;
    } else {
      sum += (b1 * ve + D * D * a2) * inv;
    }
  }
  if (!MAPS) {
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) sum += __shfl_xor(sum, sh, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = 0.0f;
      for (int w = 0; w < kSsBlock / 64; ++w) t += s_red[w];
      const int64_t b = ((int64_t)pl * a.tiles_y + blockIdx.y) * a.tiles_x + blockIdx.x;
      partial[b] = t;
    }
  }
}

// d_x += scale (blur(A) + 2 (x - y) blur(B) + y blur(C')), scale =
// -d_loss / N (the partials' adjoint: A + 2 x B + y C with C = C' - 2B).
__global__ __launch_bounds__(kSsBlock) void k_ssim_bwd(const float* __restrict__ x,
                                                       const float* __restrict__ y, SsArgs a,
                                                       const float* __restrict__ maps,
                                                       const float* __restrict__ d_loss,
                                                       float inv_n, float* __restrict__ d_x) {
  __shared__ float s_in[3][kSsIn][kSsIn + 1];
  __shared__ float s_h[3][kSsIn][kSsTile + 1];
  const int pl = blockIdx.z;
  const int X0 = blockIdx.x * kSsTile, Y0 = blockIdx.y * kSsTile;
  const int64_t plane = (int64_t)a.W * a.H;
  const int64_t all = (int64_t)a.planes * plane;
  const float* src[3] = {maps + pl * plane, maps + all + pl * plane, maps + 2 * all + pl * plane};
  ss_stage<3>(src, a, X0, Y0, s_in);
  float o[3][4];
  ss_blur<3>(a, s_in, s_h, o);
  const float scale = -(d_loss ? *d_loss : 1.0f) * inv_n;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gx = X0 + tx, gy = Y0 + ty + 8 * q;
    if (gx >= a.W || gy >= a.H) continue;
    const int64_t i = pl * plane + (int64_t)gy * a.W + gx;
    const float yi = y[i];
    const float g = o[0][q] + 2.0f * (x[i] - yi) * o[1][q] + yi * o[2][q];
    d_x[i] += scale * g;
  }
}

// out[0] = sum(partial) / N (the blocks' sums of 1 - SSIM), in a fixed
// order.
__global__ __launch_bounds__(256) void k_dssim_finish(const float* __restrict__ partial,
                                                      int64_t nb, double inv_n,
                                                      float* __restrict__ out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += 256) acc += (double)partial[b];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(s[0] * inv_n);
}

bool ss_args(int planes, int W, int H, SsArgs* a) {
  if (planes < 1 || W < 1 || H < 1 || planes > 65535) return false;
  a->planes = planes;
  a->W = W;
  a->H = H;
  a->tiles_x = div_up(W, kSsTile);
  a->tiles_y = div_up(H, kSsTile);
  double g[11], s = 0.0;
  for (int j = 0; j < 11; ++j) {
    const double u = j - 5;
    g[j] = std::exp(-u * u / (2.0 * 1.5 * 1.5));
    s += g[j];
  }
  for (int j = 0; j < 11; ++j) a->w[j] = (float)(g[j] / s);
  return a->tiles_y <= 65535;
}

// -------------------------------------------------------------- regulariser
struct RegArgs {
  int n, nv, W, H;
  int view[VRS_MAX_CROPS], x0[VRS_MAX_CROPS], y0[VRS_MAX_CROPS], S[VRS_MAX_CROPS];
  long long fbase[VRS_MAX_CROPS], ebase[VRS_MAX_CROPS + 1];   // fovea offsets, element prefix
  const int4* place;
};

__device__ inline void reg_locate(const RegArgs& a, long long e, int& k, int& c, int& yy,
                                  int& xx, int& x0, int& y0) {
  k = 0;
  while (k + 1 < a.n && a.ebase[k + 1] <= e) ++k;
  const long long r = e - a.ebase[k];
  const int S = a.S[k];
  c = (int)(r / ((long long)S * S));
  const long long q = r - (long long)c * S * S;
  yy = (int)(q / S);
  xx = (int)(q - (long long)yy * S);
  if (a.place) {
    x0 = clamp_origin(a.place[k].x, a.W - S);
    y0 = clamp_origin(a.place[k].y, a.H - S);
  } else {
    x0 = a.x0[k];
    y0 = a.y0[k];
  }
}

constexpr int kRegBlock = 256, kRegBlocks = 1024;

__global__ __launch_bounds__(kRegBlock) void k_reg_sums(const float* __restrict__ fovea,
                                                        const float* __restrict__ rgb, RegArgs a,
                                                        double* __restrict__ partial) {
  __shared__ double s_f[kRegBlock / 64], s_p[kRegBlock / 64];
  const long long total = a.ebase[a.n];
  const int64_t plane = (int64_t)a.W * a.H;
  double sf = 0.0, sp = 0.0;
  for (long long e = blockIdx.x * (long long)kRegBlock + threadIdx.x; e < total;
       e += (long long)gridDim.x * kRegBlock) {
    int k, c, yy, xx, x0, y0;
    reg_locate(a, e, k, c, yy, xx, x0, y0);
    const int S = a.S[k];
    sf += (double)fovea[a.fbase[k] + ((long long)c * S + yy) * S + xx];
    sp += (double)rgb[((int64_t)a.view[k] * 3 + c) * plane + (int64_t)(y0 + yy) * a.W + x0 + xx];
  }
#pragma unroll
  for (int sh = 32; sh > 0; sh >>= 1) {
    sf += __shfl_xor(sf, sh, 64);
    sp += __shfl_xor(sp, sh, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_f[threadIdx.x >> 6] = sf;
    s_p[threadIdx.x >> 6] = sp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double f = 0.0, p = 0.0;
    for (int w = 0; w < kRegBlock / 64; ++w) {
      f += s_f[w];
      p += s_p[w];
    }
    partial[2 * blockIdx.x] = f;
    partial[2 * blockIdx.x + 1] = p;
  }
}

__global__ __launch_bounds__(256) void k_reg_finish(const double* __restrict__ partial, int nb,
                                                    double inv_cnt, float* __restrict__ out) {
  __shared__ double s[2][256];
  double f = 0.0, p = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    f += partial[2 * b];
    p += partial[2 * b + 1];
  }
  s[0][threadIdx.x] = f;
  s[1][threadIdx.x] = p;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] += s[0][threadIdx.x + w];
      s[1][threadIdx.x] += s[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double d = (s[0][0] - s[1][0]) * inv_cnt;
    out[0] = (float)fabs(d);
    out[1] = (float)d;
  }
}

// dF += g, dP -= g over the crops, g = d_r sign(diff) / count.
__global__ __launch_bounds__(kRegBlock) void k_reg_bwd(RegArgs a, const float* __restrict__ r,
                                                       const float* __restrict__ d_r,
                                                       float inv_cnt, float* __restrict__ d_fovea,
                                                       float* __restrict__ d_rgb) {
  const float diff = r[1];
  const float sg = diff > 0.0f ? 1.0f : (diff < 0.0f ? -1.0f : 0.0f);
  const float g = (d_r ? *d_r : 1.0f) * sg * inv_cnt;
  if (g == 0.0f) return;
  const long long total = a.ebase[a.n];
  const int64_t plane = (int64_t)a.W * a.H;
  for (long long e = blockIdx.x * (long long)kRegBlock + threadIdx.x; e < total;
       e += (long long)gridDim.x * kRegBlock) {
    int k, c, yy, xx, x0, y0;
    reg_locate(a, e, k, c, yy, xx, x0, y0);
    const int S = a.S[k];
    if (d_fovea) d_fovea[a.fbase[k] + ((long long)c * S + yy) * S + xx] += g;
    if (d_rgb)
      atomicAdd(&d_rgb[((int64_t)a.view[k] * 3 + c) * plane + (int64_t)(y0 + yy) * a.W + x0 + xx],
                -g);
  }
}

bool reg_args(int nv, int W, int H, const vrs_crop* crops, int n, const vrs_crop_place* place,
              RegArgs* a) {
  if (nv < 1 || nv > VRS_MAX_VIEWS || W < 1 || H < 1 || n < 1 || n > VRS_MAX_CROPS || !crops)
    return false;
  a->n = n;
  a->nv = nv;
  a->W = W;
  a->H = H;
  a->place = reinterpret_cast<const int4*>(place);
  long long fb = 0;
  a->ebase[0] = 0;
  for (int k = 0; k < n; ++k) {
    const vrs_crop& c = crops[k];
    if (c.view < 0 || c.view >= nv || c.size < 1 || c.size > W || c.size > H) return false;
    if (!place && (c.x0 < 0 || c.y0 < 0 || c.x0 + c.size > W || c.y0 + c.size > H)) return false;
    a->view[k] = c.view;
    a->x0[k] = c.x0;
    a->y0[k] = c.y0;
    a->S[k] = c.size;
    a->fbase[k] = fb;
    fb += 3LL * c.size * c.size;
    a->ebase[k + 1] = fb;
  }
  return true;
}

// --------------------------------------------------------------------- Adam
constexpr int kAdamBlock = 256;

__device__ inline void adam1(float& p, float g, float& m, float& v, float b1, float b2, float lr,
                             float ibc1, float ibc2, float eps) {
#pragma clang fp contract(off)
  m = b1 * m + (1.0f - b1) * g;
  v = b2 * v + (1.0f - b2) * (g * g);
  const float mh = m * ibc1, vh = v * ibc2;
  p = p - lr * mh / (sqrtf(vh) + eps);
}

__global__ __launch_bounds__(kAdamBlock) void k_adam(float* __restrict__ p,
                                                     const float* __restrict__ g,
                                                     float* __restrict__ m, float* __restrict__ v,
                                                     int64_t n, float b1, float b2, float lr,
                                                     float ibc1, float ibc2, float eps) {
  const int64_t n4 = n >> 2;
  float4* p4 = reinterpret_cast<float4*>(p);
  const float4* g4 = reinterpret_cast<const float4*>(g);
  float4* m4 = reinterpret_cast<float4*>(m);
  float4* v4 = reinterpret_cast<float4*>(v);
  const int64_t stride = (int64_t)gridDim.x * kAdamBlock;
  for (int64_t i = blockIdx.x * (int64_t)kAdamBlock + threadIdx.x; i < n4; i += stride) {
    float4 pp = p4[i], mm = m4[i], vv = v4[i];
    const float4 gg = g4[i];
    adam1(pp.x, gg.x, mm.x, vv.x, b1, b2, lr, ibc1, ibc2, eps);
    adam1(pp.y, gg.y, mm.y, vv.y, b1, b2, lr, ibc1, ibc2, eps);
    adam1(pp.z, gg.z, mm.z, vv.z, b1, b2, lr, ibc1, ibc2, eps);
    adam1(pp.w, gg.w, mm.w, vv.w, b1, b2, lr, ibc1, ibc2, eps);
    p4[i] = pp;
    m4[i] = mm;
    v4[i] = vv;
  }
  for (int64_t i = 4 * n4 + blockIdx.x * (int64_t)kAdamBlock + threadIdx.x; i < n; i += stride) {
    float pp = p[i], mm = m[i], vv = v[i];
    adam1(pp, g[i], mm, vv, b1, b2, lr, ibc1, ibc2, eps);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
  }
}

bool aligned16(const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; }

}  // namespace
}  // namespace vrs

using namespace vrs;

// ------------------------------------------------------------ entry points
extern "C" size_t vrs_tonemap_workspace_size(const vrs_view* views, int n_views, int n_resp) {
  TmArgs a;
  if (!tm_args(views, n_views, n_resp, &a)) return 0;
  return (size_t)n_views * tm_blocks(a) * (kTmFixed + n_resp) * sizeof(float);
}

extern "C" vrs_status vrs_tonemap(const float* in, const vrs_view* views, int n_views,
                                  const float* params, int n_resp, float* out, void* stream) {
  TmArgs a;
  if (!tm_args(views, n_views, n_resp, &a) || !in || !params || !out) return VRS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_tonemap, dim3(tm_blocks(a), n_views), dim3(kTmBlock), 0, st, in, params,
                     a, out);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}

extern "C" vrs_status vrs_tonemap_backward(const float* in, const vrs_view* views, int n_views,
                                           const float* params, int n_resp, const float* d_out,
                                           float* d_in, float* d_params, void* ws,
                                           size_t ws_bytes, void* stream) {
  TmArgs a;
  if (!tm_args(views, n_views, n_resp, &a) || !in || !params || !d_out) return VRS_EINVAL;
  if (d_params && (!ws || ws_bytes < vrs_tonemap_workspace_size(views, n_views, n_resp)))
    return VRS_EINVAL;
  if (!d_in && !d_params) return VRS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nb = tm_blocks(a);
  float* partial = d_params ? static_cast<float*>(ws) : nullptr;
  hipLaunchKernelGGL(k_tonemap_bwd, dim3(nb, n_views), dim3(kTmBlock), 0, st, in, params, a,
                     d_out, d_in, partial);
  VRS_LAUNCH_CHECK();
  if (d_params) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(kTmFixed + n_resp, n_views), dim3(256), 0, st,
                       partial, nb, kTmFixed + n_resp, d_params);
    VRS_LAUNCH_CHECK();
  }
  return VRS_OK;
}

extern "C" size_t vrs_dssim_workspace_size(int planes, int width, int height) {
  SsArgs a;
  if (!ss_args(planes, width, height, &a)) return 0;
  // block partials of the forward, or the three derivative maps of the
  // adjoint (the larger)
  const size_t part = (size_t)planes * a.tiles_x * a.tiles_y * sizeof(float);
  const size_t maps = 3 * (size_t)planes * width * height * sizeof(float);
  return std::max(part, maps);
}

extern "C" vrs_status vrs_dssim(const float* x, const float* y, int planes, int width,
                                int height, float* loss, void* ws, size_t ws_bytes,
                                void* stream) {
  SsArgs a;
  if (!ss_args(planes, width, height, &a) || !x || !y || !loss || !ws ||
      ws_bytes < vrs_dssim_workspace_size(planes, width, height))
    return VRS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* partial = static_cast<float*>(ws);
  hipLaunchKernelGGL(k_ssim<false>, dim3(a.tiles_x, a.tiles_y, planes), dim3(kSsBlock), 0, st, x,
                     y, a, nullptr, partial);
  VRS_LAUNCH_CHECK();
  const int64_t nb = (int64_t)planes * a.tiles_x * a.tiles_y;
  hipLaunchKernelGGL(k_dssim_finish, dim3(1), dim3(256), 0, st, partial, nb,
                     1.0 / ((double)planes * width * height), loss);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}

extern "C" vrs_status vrs_dssim_backward(const float* x, const float* y, int planes, int width,
                                         int height, const float* d_loss, float* d_x, void* ws,
                                         size_t ws_bytes, void* stream) {
  SsArgs a;
  if (!ss_args(planes, width, height, &a) || !x || !y || !d_x || !ws ||
      ws_bytes < vrs_dssim_workspace_size(planes, width, height))
    return VRS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* maps = static_cast<float*>(ws);
  const dim3 grid(a.tiles_x, a.tiles_y, planes);
  hipLaunchKernelGGL(k_ssim<true>, grid, dim3(kSsBlock), 0, st, x, y, a, maps, nullptr);
  VRS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(kSsBlock), 0, st, x, y, a, maps, d_loss,
                     (float)(1.0 / ((double)planes * width * height)), d_x);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}

extern "C" size_t vrs_regulariser_workspace_size(void) {
  return 2 * sizeof(double) * kRegBlocks;
}

extern "C" vrs_status vrs_regulariser(const float* fovea_rgb, const float* rgb, int n_views,
                                      int width, int height, const vrs_crop* crops, int n_crops,
                                      const vrs_crop_place* place, float* r, void* ws,
                                      size_t ws_bytes, void* stream) {
  RegArgs a;
  if (!reg_args(n_views, width, height, crops, n_crops, place, &a) || !fovea_rgb || !rgb || !r ||
      !ws || ws_bytes < vrs_regulariser_workspace_size())
    return VRS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nb = std::max(1, std::min(kRegBlocks, div_up(a.ebase[n_crops], kRegBlock)));
  double* partial = static_cast<double*>(ws);
  hipLaunchKernelGGL(k_reg_sums, dim3(nb), dim3(kRegBlock), 0, st, fovea_rgb, rgb, a, partial);
  VRS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reg_finish, dim3(1), dim3(256), 0, st, partial, nb,
                     1.0 / (double)a.ebase[n_crops], r);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}

extern "C" vrs_status vrs_regulariser_backward(int n_views, int width, int height,
                                               const vrs_crop* crops, int n_crops,
                                               const vrs_crop_place* place, const float* r,
                                               const float* d_r, float* d_fovea, float* d_rgb,
                                               void* stream) {
  RegArgs a;
  if (!reg_args(n_views, width, height, crops, n_crops, place, &a) || !r) return VRS_EINVAL;
  if (!d_fovea && !d_rgb) return VRS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nb = std::max(1, std::min(kRegBlocks, div_up(a.ebase[n_crops], kRegBlock)));
  hipLaunchKernelGGL(k_reg_bwd, dim3(nb), dim3(kRegBlock), 0, st, a, r, d_r,
                     (float)(1.0 / (double)a.ebase[n_crops]), d_fovea, d_rgb);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}

extern "C" vrs_status vrs_adam_step(float* param, const float* grad, float* m, float* v,
                                    int64_t n, int step, float lr, float beta1, float beta2,
                                    float eps, void* stream) {
  if (n < 0 || step < 1 || (n > 0 && (!param || !grad || !m || !v))) return VRS_EINVAL;
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f))
    return VRS_EINVAL;
  if (!aligned16(param) || !aligned16(grad) || !aligned16(m) || !aligned16(v)) return VRS_EINVAL;
  if (n == 0) return VRS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double bc1 = 1.0 - std::pow((double)beta1, step), bc2 = 1.0 - std::pow((double)beta2, step);
  const int blocks = std::max(1, std::min(8192, div_up(std::max<int64_t>(n >> 2, 1), kAdamBlock)));
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(kAdamBlock), 0, st, param, grad, m, v, n, beta1,
                     beta2, lr, (float)(1.0 / bc1), (float)(1.0 / bc2), eps);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}
