// Foveal decoder, forward: the small gated CNN that resolves each crop's
// neural-point pyramid into the foveal image F, with the periphery crop
// injected at the finest level (Sec. 3.3).
//
// Each level is one implicit-GEMM 3x3 convolution on the matrix cores:
//   M = output pixels (a tile of TH rows x 16 columns per workgroup, one
//       16-pixel row segment per MFMA row block),
//   N = 2 * Kp pre-activations, ordered so N-tile 2t holds the feature half
//       and N-tile 2t+1 the gate half of channels [16t, 16t+16): the gated
//       epilogue ELU(f) * sigmoid(g) pairs values held by the same lane,
//   K = 9 taps x Cin8 input channels (Cin padded to 8), padded to the MFMA
//       depth.
// The loader builds the zero-padded (TH+2) x 18 halo tile of the level's
// input in LDS directly from its sources -- pyramid layer, bilinear x2
// upsample of the coarser level's output, periphery crop -- so the
// concatenated input never exists in HBM.  One launch per level covers all
// crops (crops of uneven size are packed back to back in the grid).
// Arithmetic: float operands with v_mfma_f32_16x16x4_f32 (VRS_F32), or
// bfloat16 operands with v_mfma_f32_16x16x32_bf16 and float accumulation
// (VRS_BF16); biases, activations and the RGB head in float.
#include <type_traits>

#include "vrs_common.h"

namespace vrs {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kDecMaxNT = 8;  // widths up to 64 channels

struct DecLevel {
  int C, cin, cin8, kpad, kp, nout, kn, kpn, has_p, n_crops, W, H, width;
  int tile_base[VRS_MAX_CROPS + 1];
  int tiles_x[VRS_MAX_CROPS];
  int S[VRS_MAX_CROPS];
  int view[VRS_MAX_CROPS], x0[VRS_MAX_CROPS], y0[VRS_MAX_CROPS];
  int mx0[VRS_MAX_CROPS], my0[VRS_MAX_CROPS];   // largest origin inside the view
  const int4* place;                 // device crop placement (x0, y0, gaze), or null
  long long pyr_off[VRS_MAX_CROPS];  // float offset of this layer in the pyramid
  long long h_off[VRS_MAX_CROPS];    // element offset of h_l
  long long hn_off[VRS_MAX_CROPS];   // element offset of h_{l+1}
  long long pre_off[VRS_MAX_CROPS];  // float offset of the pre-activations
};

template <typename T>
struct DecTraits;
template <>
struct DecTraits<float> {
  static constexpr int KSTEP = 4;
  static constexpr int TH = 8;
};
template <>
struct DecTraits<__bf16> {
  static constexpr int KSTEP = 32;
  static constexpr int TH = 16;
};

// Origin of crop k in its view: the host value, or the device placement
// table's clamped into the view.
__device__ inline int dec_x0(const DecLevel& d, int k) {
  return d.place ? clamp_origin(d.place[k].x, d.mx0[k]) : d.x0[k];
}
__device__ inline int dec_y0(const DecLevel& d, int k) {
  return d.place ? clamp_origin(d.place[k].y, d.my0[k]) : d.y0[k];
}

__device__ inline float to_f(float x) { return x; }
__device__ inline float to_f(__bf16 x) { return (float)x; }

// Activations of the gated convolution, on the hardware exp2 and reciprocal
// (a few ulp; the reference and the gradients use the library functions).
__device__ inline float elu_f(float x) {
  return x > 0.0f ? x : __builtin_amdgcn_exp2f(x * 1.4426950408889634f) - 1.0f;
}
__device__ inline float sigmoid_f(float x) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-x * 1.4426950408889634f));
}

// value of input channel c of level l at pixel (y, x) of crop k (inside the
// S x S layer)
template <typename T>
__device__ inline float dec_input(const DecLevel& d, int k, int S, int y, int x, int c,
                                  const float* __restrict__ pyr, const float* __restrict__ periph,
                                  const T* __restrict__ hnext) {
  if (c < d.C) return pyr[d.pyr_off[k] + ((long long)y * S + x) * d.C + c];
  c -= d.C;
  if (c < d.kn) {
    const int Sn = S >> 1;
    const float sx = 0.5f * (float)x - 0.25f, sy = 0.5f * (float)y - 0.25f;
    const float fx0 = floorf(sx), fy0 = floorf(sy);
    const float fx = sx - fx0, fy = sy - fy0;
    int xa = (int)fx0, ya = (int)fy0, xb = xa + 1, yb = ya + 1;
    xa = xa < 0 ? 0 : (xa > Sn - 1 ? Sn - 1 : xa);
    xb = xb < 0 ? 0 : (xb > Sn - 1 ? Sn - 1 : xb);
    ya = ya < 0 ? 0 : (ya > Sn - 1 ? Sn - 1 : ya);
    yb = yb < 0 ? 0 : (yb > Sn - 1 ? Sn - 1 : yb);
    const T* h = hnext + d.hn_off[k];
    const float v00 = to_f(h[((long long)ya * Sn + xa) * d.kpn + c]);
    const float v01 = to_f(h[((long long)ya * Sn + xb) * d.kpn + c]);
    const float v10 = to_f(h[((long long)yb * Sn + xa) * d.kpn + c]);
    const float v11 = to_f(h[((long long)yb * Sn + xb) * d.kpn + c]);
    return (1.0f - fy) * ((1.0f - fx) * v00 + fx * v01) + fy * ((1.0f - fx) * v10 + fx * v11);
  }
  c -= d.kn;
  if (d.has_p && c < 3) {
    const long long plane = (long long)d.W * d.H;
    return periph[(long long)d.view[k] * 3 * plane + c * plane +
                  (long long)(dec_y0(d, k) + y) * d.W + (dec_x0(d, k) + x)];
  }
  return 0.0f;
}

// Channel order of the halo tile in LDS (and of the packed weights' K
// dimension): [upsampled coarser output (kn) | pyramid layer (C) | periphery
// crop (3, finest level only) | zero padding], so the upsampled channels form
// aligned 8-channel groups.  Returns the original input channel, or -1 for
// padding.
__device__ __host__ inline int lds_to_orig(int c, int C, int kn, int has_p) {
  if (c < kn) return C + c;
  c -= kn;
  if (c < C) return c;
  c -= C;
  if (has_p && c < 3) return C + kn + c;
  return -1;
}

template <typename T>
__device__ inline void load8(const T* p, float* v);
template <>
__device__ inline void load8<__bf16>(const __bf16* p, float* v) {
  const v8bf a = *reinterpret_cast<const v8bf*>(p);
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (float)a[j];
}
template <>
__device__ inline void load8<float>(const float* p, float* v) {
  const float4 a = *reinterpret_cast<const float4*>(p), b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
template <typename T>
__device__ inline void store8(T* p, const float* v);
template <>
__device__ inline void store8<__bf16>(__bf16* p, const float* v) {
  // one vector conversion: four packed two-value conversions
  typedef float v8f __attribute__((ext_vector_type(8)));
  const v8f f = {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
  *reinterpret_cast<v8bf*>(p) = __builtin_convertvector(f, v8bf);
}
template <>
__device__ inline void store8<float>(float* p, const float* v) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  *reinterpret_cast<float4*>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
}
// eight elements moved as they are
template <typename T>
__device__ inline void copy8(T* dst, const T* src) {
  static_assert(sizeof(T) == 2 || sizeof(T) == 4, "BF16 or float");
  *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(src);
  if constexpr (sizeof(T) == 4)
    *reinterpret_cast<uint4*>(dst + 4) = *reinterpret_cast<const uint4*>(src + 4);
}

// head: optional fused RGB head at the finest level (fovea != null):
// F = W_o h_0 + b_o written straight to the packed foveal image; h_0 is
// then only written when pre-activations are requested (backward).
struct HeadFuse {
  const float* wo;
  const float* bo;
  float* fovea;
  long long out_base[VRS_MAX_CROPS];
};

// Geometry of one workgroup's LDS: halo tile, the coarser level's footprint
// and the weights.  ONE: the whole weight operand (up to 24 KB) is loaded
// once, at the start, overlapping the halo fill; otherwise two chunks of CHS
// k-steps are double-buffered: 8 KB, or 4 KB for two N-tiles, whose level
// (the finest) is bound by the halo fill's latency, so four workgroups per
// CU (40 KB each) beat whole weights at three.
template <typename T, int NT, bool ONE>
struct ConvCfg {
  // 8-row tiles where the accumulators would leave one wave per SIMD
  static constexpr int TH = sizeof(T) == 2 && NT >= 8 ? 8 : DecTraits<T>::TH;
  static constexpr int KSTEP = DecTraits<T>::KSTEP;
  static constexpr int NPIX = (TH + 2) * 18;
  // halo pixel stride: cin8 channels, plus 8 (16 bytes) in the BF16 levels:
  // their strides of an odd number of 16-byte units (80 and 144 bytes) meet
  // more LDS bank conflicts in the fill's 16-byte stores and the A-operand
  // reads than 96 and 160 bytes.  The coarse footprint is then kept in BF16,
  // so the finest level still fits four workgroups per CU (together: LDS
  // conflict cycles -57 %, -49 % and -16 % for 2, 4 and 8 N-tiles).
  static constexpr int CPAD = sizeof(T) == 2 ? 8 : 0;
  static constexpr int CR = TH / 2 + 2, CC = 10;       // coarse rows / columns staged
  static constexpr int NOUT = NT * 16;
  static constexpr int NBUF = ONE ? 1 : 2;
  static constexpr int CBYTES = ONE ? 24576 : (NT <= 2 ? 4096 : 8192);
  static constexpr int CHS = CBYTES / (NOUT * KSTEP * (int)sizeof(T)) > 0
                                 ? CBYTES / (NOUT * KSTEP * (int)sizeof(T)) : 1;
  static constexpr int CK = CHS * KSTEP;                // k per chunk
  static constexpr int BROW = CK + 16 / (int)sizeof(T); // padded LDS row (elements)
  static constexpr int PPR = CK * (int)sizeof(T) / 16;  // 16-byte pieces per row
  static constexpr int PIECES = NOUT * PPR;
  static constexpr int PPT = (PIECES + 255) / 256;
};

// The weight chunks reuse the coarse footprint's LDS (the coarser level's
// output as stored, T) once the halo tile is filled; the per-k-step A
// offsets (int [k-steps][4]) follow.
template <typename T, int NT, bool ONE>
__host__ __device__ inline int conv_region_bytes(int kn) {
  using Cfg = ConvCfg<T, NT, ONE>;
  const int kn8 = (kn + 7) & ~7;
  const int coarse = Cfg::CR * Cfg::CC * kn8 * (int)sizeof(T);
  const int wchunks = Cfg::NBUF * Cfg::NOUT * Cfg::BROW * (int)sizeof(T);
  return coarse > wchunks ? coarse : wchunks;
}
template <typename T, int NT, bool ONE>
__host__ __device__ inline size_t conv_smem_bytes(int cin8, int kn, int kpad) {
  using Cfg = ConvCfg<T, NT, ONE>;
  return (size_t)Cfg::NPIX * (cin8 + Cfg::CPAD) * sizeof(T) + conv_region_bytes<T, NT, ONE>(kn) +
         (size_t)(kpad / Cfg::KSTEP) * 4 * sizeof(int);
}

// One 16-channel slice of the RGB head on the matrix cores: acc += A B with
// A = the head weights (lane (col, kq): W_o[col][4 kq + i]) and B = the
// gated values (lane (col, kq): channels 4 kq + i of pixel col).  BF16
// operands with float accumulation (one 16x16x16 step), or float operands
// (four 16x16x4 steps, the slice's k = 4 kq + i taken as k-index kq of
// step i).
template <typename T>
__device__ inline v4f head_mfma(const float* wa, const float* hv, v4f acc) {
  if constexpr (sizeof(T) == 2) {
    typedef short v4s __attribute__((ext_vector_type(4)));
    v4s a, b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = __builtin_bit_cast(short, (__bf16)wa[i]);
      b[i] = __builtin_bit_cast(short, (__bf16)hv[i]);
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[i], hv[i], acc, 0, 0, 0);
    return acc;
  }
}

// Register budget per N-tile count: the occupancy the accumulators allow
// (4, 3, 2, 2 waves per SIMD for 2, 4, 6, 8 N-tiles; 8 N-tiles use 8-row
// tiles).
template <int NT>
constexpr int conv_waves() { return NT <= 2 ? 4 : (NT <= 4 ? 3 : 2); }
template <typename T, int NT, bool ONE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(conv_waves<NT>())))
void k_dec_conv(DecLevel d, const float* __restrict__ pyr,
                                                  const float* __restrict__ periph,
                                                  const T* __restrict__ hnext,
                                                  const T* __restrict__ wp,
                                                  const float* __restrict__ bp,
                                                  T* __restrict__ hout, float* __restrict__ pre,
                                                  HeadFuse hf) {
  using Cfg = ConvCfg<T, NT, ONE>;
  constexpr int TH = Cfg::TH, RPW = TH / 4, KSTEP = Cfg::KSTEP, NPIX = Cfg::NPIX;
  constexpr int CR = Cfg::CR, CC = Cfg::CC, NOUT = Cfg::NOUT, CHS = Cfg::CHS, CK = Cfg::CK;
  constexpr int BROW = Cfg::BROW;
  extern __shared__ __align__(16) char smem[];
  const int cin8 = d.cin8, kn8 = (d.kn + 7) & ~7;
  const int cs = cin8 + Cfg::CPAD;   // halo pixel stride (elements)
  T* tile = reinterpret_cast<T*>(smem);
  char* region = smem + (size_t)NPIX * cs * sizeof(T);
  T* ctile = reinterpret_cast<T*>(region);
  T* sB = reinterpret_cast<T*>(region);   // after the fill
  int* s_aoff = reinterpret_cast<int*>(region + conv_region_bytes<T, NT, ONE>(d.kn));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int k = 0;
  while (k + 1 < d.n_crops && (int)blockIdx.x >= d.tile_base[k + 1]) ++k;
  const int tl = blockIdx.x - d.tile_base[k];
  const int S = d.S[k];
  const int oy = (tl / d.tiles_x[k]) * TH, ox = (tl % d.tiles_x[k]) * 16;
  const int nsteps = d.kpad / KSTEP;
  const int nchunks = (nsteps + CHS - 1) / CHS;
  // ---- weight chunks: global -> registers -> LDS, one chunk ahead
  uint4 breg[Cfg::PPT];
  auto load_chunk = [&](int c) {
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
      const int pc = tid + q * 256;
      breg[q] = make_uint4(0, 0, 0, 0);
      if (pc < Cfg::PIECES) {
        const int n = pc / Cfg::PPR, kk = (pc - n * Cfg::PPR) * (16 / (int)sizeof(T));
        const int gk = c * CK + kk;
        if (gk < d.kpad) breg[q] = *reinterpret_cast<const uint4*>(wp + (long long)n * d.kpad + gk);
      }
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
      const int pc = tid + q * 256;
      if (pc < Cfg::PIECES) {
        const int n = pc / Cfg::PPR, kk = (pc - n * Cfg::PPR) * (16 / (int)sizeof(T));
        *reinterpret_cast<uint4*>(&sB[(buf * NOUT + n) * BROW + kk]) = breg[q];
      }
    }
  };
  load_chunk(0);
  // ---- the coarser level's output under this tile, clamped at the layer
  // edge, staged once (each coarse pixel feeds up to 16 fine pixels)
  const int Sn = S >> 1;
  const int cy0 = (oy >> 1) - 1, cx0 = (ox >> 1) - 1;
  if (d.kn > 0) {
    // copied as stored (8 channels = one 16-byte piece in BF16)
    const int kg = kn8 >> 3;
    const int nco = CR * CC * kg;
    auto csrc = [&](int e) {
      const int cp = e / kg, g = e - cp * kg;
      const int cyi = cp / CC, cxi = cp - cyi * CC;
      int yy = cy0 + cyi, xx = cx0 + cxi;
      yy = yy < 0 ? 0 : (yy > Sn - 1 ? Sn - 1 : yy);
      xx = xx < 0 ? 0 : (xx > Sn - 1 ? Sn - 1 : xx);
      return hnext + d.hn_off[k] + ((long long)yy * Sn + xx) * d.kpn + g * 8;
    };
    // two items per thread and round, both loads in flight before the stores
    for (int e0 = tid; e0 < nco; e0 += 512) {
      const int e1 = e0 + 256;
      uint4 r0[sizeof(T) / 2], r1[sizeof(T) / 2];
      const T* p0 = csrc(e0);
#pragma unroll
      for (int h = 0; h < (int)sizeof(T) / 2; ++h) r0[h] = reinterpret_cast<const uint4*>(p0)[h];
      if (e1 < nco) {
        const T* p1 = csrc(e1);
#pragma unroll
        for (int h = 0; h < (int)sizeof(T) / 2; ++h) r1[h] = reinterpret_cast<const uint4*>(p1)[h];
      }
#pragma unroll
      for (int h = 0; h < (int)sizeof(T) / 2; ++h) reinterpret_cast<uint4*>(&ctile[e0 * 8])[h] = r0[h];
      if (e1 < nco)
#pragma unroll
        for (int h = 0; h < (int)sizeof(T) / 2; ++h) reinterpret_cast<uint4*>(&ctile[e1 * 8])[h] = r1[h];
    }
    __syncthreads();
  }
  // A-operand offset of each k-step and lane group kq: k = 32 s + 8 kq (BF16,
  // one 8-channel unit) or 4 s + kq (FP32, one channel) is tap * cin8 +
  // channel.  Steps past the 9 taps read tap 8 (their weights are zero).
  {
    const int units = sizeof(T) == 2 ? (cin8 >> 3) : cin8;
    for (int i = tid; i < nsteps * 4; i += 256) {
      const int u = i;   // unit index along K: 4 per k-step
      int tap = u / units, cu = u - tap * units;
      if (tap > 8) {
        tap = 8;
        cu = 0;
      }
      const int ty = tap / 3, tx = tap - 3 * ty;
      s_aoff[i] = (ty * 18 + tx) * cs + cu * (sizeof(T) == 2 ? 8 : 1);
    }
  }
  // ---- halo tile fill.  Upsampled channels: one work item per 2x2 block of
  // fine pixels and 8-channel group -- fine rows 2m+1, 2m+2 (and columns
  // likewise) interpolate the same two coarse rows with weights 3/4, 1/4 and
  // 1/4, 3/4, so four coarse reads serve four pixels.  Other channels
  // (pyramid layer, periphery crop, padding): one item per pixel and group.
  // Pixels outside the layer are zero.
  const int G = cin8 >> 3;
  const int kgf = d.kn >> 3;   // full 8-channel groups of upsampled channels
  constexpr int NB = (TH + 2) / 2 * 9;   // 2x2 blocks of the halo tile
  const bool fast_py = d.C == 4 && (d.kn & 7) == 0 && (reinterpret_cast<uintptr_t>(pyr) & 15) == 0;
  const long long plane = (long long)d.W * d.H;
  const int n_up = NB * kgf, n_items = n_up + NPIX * (G - kgf);
  // this crop's pyramid layer and periphery window (the origin read once)
  const float* pyr_base = pyr + d.pyr_off[k];
  const float* per_base = d.has_p ? periph + (long long)d.view[k] * 3 * plane +
                                        (long long)dec_y0(d, k) * d.W + dec_x0(d, k)
                                  : periph;
  // every halo pixel inside the layer: no zero selects
  const bool interior = oy >= 1 && ox >= 1 && oy + TH + 1 <= S && ox + 17 <= S;
  // upsampled item e = block * kgf + group (groups fastest, so that a wave's
  // coarse reads and tile writes are runs of consecutive 32- and 16-byte
  // pieces), advanced by 256 items per round without divisions
  const int kgf_s = kgf > 0 ? kgf : 1;
  const int up_sb = 256 / kgf_s, up_sg = 256 - up_sb * kgf_s;
  int up_blk = tid / kgf_s, up_g = tid - up_blk * kgf_s;
  for (int e = tid; e < n_items; e += 256) {
    const int blk = up_blk, g = up_g;
    up_blk += up_sb;
    up_g += up_sg;
    if (up_g >= kgf_s) {
      up_g -= kgf_s;
      ++up_blk;
    }
    if (e < n_up) {
      const int bi = blk / 9, bj = blk - bi * 9;
      const T* c00 = &ctile[(bi * CC + bj) * kn8 + g * 8];
      float a00[8], a01[8], a10[8], a11[8];
      load8<T>(c00, a00);
      load8<T>(c00 + kn8, a01);
      load8<T>(c00 + CC * kn8, a10);
      load8<T>(c00 + (CC + 1) * kn8, a11);
      // horizontal: left fine column (3/4 a_0 + 1/4 a_1), right (1/4, 3/4),
      // each pair from the difference: a_0 + d/4 and a_1 - d/4
      float tl[8], tr[8], bl[8], br[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float dt = a01[j] - a00[j], db = a11[j] - a10[j];
        tl[j] = fmaf(0.25f, dt, a00[j]);
        tr[j] = fmaf(-0.25f, dt, a01[j]);
        bl[j] = fmaf(0.25f, db, a10[j]);
        br[j] = fmaf(-0.25f, db, a11[j]);
      }
      auto put = [&](auto inside_tag) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int dy = q >> 1, dx = q & 1;
          const int hy = 2 * bi + dy, hx = 2 * bj + dx;
          const int y = oy + hy - 1, x = ox + hx - 1;
          const bool in = decltype(inside_tag)::value || (y >= 0 && y < S && x >= 0 && x < S);
          float v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            // vertical likewise: top + e/4 (upper fine row), bot - e/4
            const float top = dx ? tr[j] : tl[j], bot = dx ? br[j] : bl[j];
            const float e = bot - top;
            const float val = dy ? fmaf(-0.25f, e, bot) : fmaf(0.25f, e, top);
            v[j] = in ? val : 0.0f;
          }
          store8<T>(&tile[(hy * 18 + hx) * cs + g * 8], v);
        }
      };
      if (interior)
        put(std::true_type{});
      else
        put(std::false_type{});
    } else {
      const int e2 = e - n_up;
      const int g = kgf + e2 / NPIX, pix = e2 - (g - kgf) * NPIX;
      const int hy = pix / 18, hx = pix - hy * 18;
      const int y = oy + hy - 1, x = ox + hx - 1;
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = 0.0f;
      if (y >= 0 && y < S && x >= 0 && x < S) {
        const int c0 = g * 8;
        if (fast_py && c0 == d.kn) {
          // pyramid layer (4 channels, one 16-byte load) and periphery crop
          const float4 pv = *reinterpret_cast<const float4*>(pyr_base + ((long long)y * S + x) * 4);
          v[0] = pv.x; v[1] = pv.y; v[2] = pv.z; v[3] = pv.w;
          if (d.has_p) {
            const float* pp = per_base + (long long)y * d.W + x;
            v[4] = pp[0];
            v[5] = pp[plane];
            v[6] = pp[2 * plane];
          }
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int oc = lds_to_orig(c0 + j, d.C, d.kn, d.has_p);
            if (oc >= 0) v[j] = dec_input<T>(d, k, S, y, x, oc, pyr, periph, hnext);
          }
        }
      }
      store8<T>(&tile[pix * cs + g * 8], v);
    }
  }
  __syncthreads();   // the coarse footprint is dead from here
  store_chunk(0);
  __syncthreads();
  // ---- MFMA main loop over weight chunks
  // the accumulators start from the biases (lane (col, kq) holds channels
  // 4 kq + i of each N-tile), so the epilogue adds nothing
  const int r0 = wave * RPW;
  const int col = lane & 15, kq = lane >> 4;
  v4f acc[RPW][NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const float4 bj = *reinterpret_cast<const float4*>(&bp[j * 16 + 4 * kq]);
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r][j] = v4f{bj.x, bj.y, bj.z, bj.w};
  }
  const int rowbase = (r0 * 18 + col) * cs;
  for (int c = 0; c < nchunks; ++c) {
    if (!ONE && c + 1 < nchunks) load_chunk(c + 1);
    const T* B = sB + (ONE ? 0 : (c & 1)) * NOUT * BROW;
#pragma unroll
    for (int s = 0; s < CHS; ++s) {
      const int ks = c * CHS + s;
      if (ks >= nsteps) break;
      const int abase = rowbase + s_aoff[ks * 4 + kq];
      if constexpr (sizeof(T) == 2) {
        v8bf a[RPW];
#pragma unroll
        for (int r = 0; r < RPW; ++r)
          a[r] = *reinterpret_cast<const v8bf*>(&tile[abase + r * 18 * cs]);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const v8bf b = *reinterpret_cast<const v8bf*>(&B[(j * 16 + col) * BROW + s * KSTEP + kq * 8]);
#pragma unroll
          for (int r = 0; r < RPW; ++r)
            acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a[r], acc[r][j], 0, 0, 0);
        }
      } else {
        float a[RPW];
#pragma unroll
        for (int r = 0; r < RPW; ++r) a[r] = to_f(tile[abase + r * 18 * cs]);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const float b = to_f(B[(j * 16 + col) * BROW + s * KSTEP + kq]);
#pragma unroll
          for (int r = 0; r < RPW; ++r)
            acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b, a[r], acc[r][j], 0, 0, 0);
        }
      }
    }
    if (!ONE) {
      if (c + 1 < nchunks) store_chunk((c + 1) & 1);
      __syncthreads();
    }
  }
  // ---- gated epilogue.  The weights are the MFMA's A operand, so lane
  // (col, kq) holds channels 4 kq + i (i < 4) of N-tile j for the pixel in
  // column col: feature and gate of a channel sit in the same lane, and the
  // lane's four channels are contiguous in h and in the pre-activations.
  const bool write_h = hf.fovea == nullptr || pre != nullptr;
  const int x = ox + col;
  // The fused RGB head F = W_o h + b_o is one small matrix product per row
  // on the matrix cores: the gated values already sit in the layout of the
  // B operand (lane (col, kq): channels 4 kq + i of pixel col), W_o (rows:
  // colour channels, padded to 16) is the A operand, and the result's lanes
  // kq = 0 hold the three colours of pixel col.  Channel pairs outer, rows
  // inner: the head's A operand is built once per pair.
  v4f head[RPW];
  if (hf.fovea) {
    const v4f hb0 = kq == 0 ? v4f{hf.bo[0], hf.bo[1], hf.bo[2], 0.0f} : v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int r = 0; r < RPW; ++r) head[r] = hb0;
  }
#pragma unroll
  for (int t = 0; t < NT / 2; ++t) {
    float wa[4];   // A operand: W_o[col][t 16 + 4 kq + i] (zero beyond 3 colours or the width)
    if (hf.fovea) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ch = t * 16 + 4 * kq + i;
        wa[i] = col < 3 && ch < d.width ? hf.wo[col * d.width + ch] : 0.0f;
      }
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int y = oy + r0 + r;
      if (y >= S) continue;   // uniform over the wave
      const long long p = (long long)y * S + x;
      const float f[4] = {acc[r][2 * t][0], acc[r][2 * t][1], acc[r][2 * t][2],
                          acc[r][2 * t][3]};
      const float g[4] = {acc[r][2 * t + 1][0], acc[r][2 * t + 1][1], acc[r][2 * t + 1][2],
                          acc[r][2 * t + 1][3]};
      float hv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) hv[i] = elu_f(f[i]) * sigmoid_f(g[i]);
      if (hf.fovea) head[r] = head_mfma<T>(wa, hv, head[r]);
      if (x < S) {
        if (write_h) {
          T* hp = hout + d.h_off[k] + p * d.kp + t * 16 + 4 * kq;
          if constexpr (sizeof(T) == 2) {
            typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
            *reinterpret_cast<v4bf*>(hp) = v4bf{(__bf16)hv[0], (__bf16)hv[1], (__bf16)hv[2], (__bf16)hv[3]};
          } else {
            *reinterpret_cast<float4*>(hp) = make_float4(hv[0], hv[1], hv[2], hv[3]);
          }
        }
        if (pre) {
          float* pp = pre + d.pre_off[k] + p * d.nout;
          *reinterpret_cast<float4*>(pp + 2 * t * 16 + 4 * kq) = make_float4(f[0], f[1], f[2], f[3]);
          *reinterpret_cast<float4*>(pp + (2 * t + 1) * 16 + 4 * kq) = make_float4(g[0], g[1], g[2], g[3]);
        }
      }
    }
  }
  if (hf.fovea && kq == 0 && x < S) {
    const long long opl = (long long)S * S;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int y = oy + r0 + r;
      if (y >= S) continue;
      const long long p = (long long)y * S + x;
      hf.fovea[hf.out_base[k] + p] = head[r][0];
      hf.fovea[hf.out_base[k] + opl + p] = head[r][1];
      hf.fovea[hf.out_base[k] + 2 * opl + p] = head[r][2];
    }
  }
}

// Re-order every level's float weights [2K][3][3][Cin] into its GEMM
// operand [nout][kpad] (N-tile pairs of feature/gate halves, k = tap*Cin8 + c
// with c in the LDS channel order, zero padding) and its bias, all levels in
// one launch.
template <typename T>
struct PackArgs {
  int n;
  int K[VRS_MAX_LEVELS], cin[VRS_MAX_LEVELS], cin8[VRS_MAX_LEVELS], kp[VRS_MAX_LEVELS],
      kpad[VRS_MAX_LEVELS], kn[VRS_MAX_LEVELS];
  long long start[VRS_MAX_LEVELS + 1];   // first element of each level
  const float* w[VRS_MAX_LEVELS];
  const float* b[VRS_MAX_LEVELS];
  T* wp[VRS_MAX_LEVELS];
  float* bp[VRS_MAX_LEVELS];
  int C;
};

template <typename T>
__global__ void k_dec_pack(PackArgs<T> a) {
  const long long total = a.start[a.n];
  for (long long e0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; e0 < total;
       e0 += (long long)gridDim.x * blockDim.x) {
    int l = 0;
    while (l + 1 < a.n && e0 >= a.start[l + 1]) ++l;
    const long long e = e0 - a.start[l];
    const int kpad = a.kpad[l], cin8 = a.cin8[l], K = a.K[l];
    const int n = (int)(e / kpad), kk = (int)(e - (long long)n * kpad);
    const int t = n / 32, half = (n % 32) / 16, ch = t * 16 + (n % 16);
    const int tap = kk / cin8, c = kk - tap * cin8;
    const int oc = lds_to_orig(c, a.C, a.kn[l], l == 0 ? 1 : 0);
    float v = 0.0f;
    if (ch < K && tap < 9 && oc >= 0 && oc < a.cin[l]) {
      const int row = half ? K + ch : ch;
      v = a.w[l][((long long)row * 9 + tap) * a.cin[l] + oc];
    }
    a.wp[l][e] = (T)v;
    if (kk == 0) a.bp[l][n] = ch < K ? a.b[l][half ? K + ch : ch] : 0.0f;
  }
}

// RGB head: F = W_o h_0 + b_o, one thread per output pixel of any crop.
struct HeadArgs {
  int n_crops, kp, K0;
  int S[VRS_MAX_CROPS];
  long long pix_base[VRS_MAX_CROPS + 1];
  long long out_base[VRS_MAX_CROPS];
  long long h_off[VRS_MAX_CROPS];
};

template <typename T>
__global__ void k_dec_head(HeadArgs a, const T* __restrict__ h0, const float* __restrict__ wo,
                           const float* __restrict__ bo, float* __restrict__ out) {
  const long long npix = a.pix_base[a.n_crops];
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npix;
       p += (long long)gridDim.x * blockDim.x) {
    int k = 0;
    while (k + 1 < a.n_crops && p >= a.pix_base[k + 1]) ++k;
    const long long q = p - a.pix_base[k];
    const int S = a.S[k];
    const T* h = h0 + a.h_off[k] + q * a.kp;
    float a0 = bo[0], a1 = bo[1], a2 = bo[2];
    for (int c = 0; c < a.K0; ++c) {
      const float v = to_f(h[c]);
      a0 += wo[c] * v;
      a1 += wo[a.K0 + c] * v;
      a2 += wo[2 * a.K0 + c] * v;
    }
    const long long plane = (long long)S * S;
    out[a.out_base[k] + q] = a0;
    out[a.out_base[k] + plane + q] = a1;
    out[a.out_base[k] + 2 * plane + q] = a2;
  }
}

// ------------------------------------------------------------ host side
struct DecPlan {
  int nd, C, dtype;
  int K[VRS_MAX_LEVELS], kp[VRS_MAX_LEVELS], cin[VRS_MAX_LEVELS], cin8[VRS_MAX_LEVELS],
      kpad[VRS_MAX_LEVELS];
  size_t w_off[VRS_MAX_LEVELS], b_off[VRS_MAX_LEVELS];   // offsets into the float weights
  size_t head_w, head_b;
  // workspace (bytes)
  size_t wp[VRS_MAX_LEVELS], bp[VRS_MAX_LEVELS], h[VRS_MAX_LEVELS], pre[VRS_MAX_LEVELS],
      dh[VRS_MAX_LEVELS], total;
  long long h_elems[VRS_MAX_LEVELS], pre_elems[VRS_MAX_LEVELS];
  int n_crops;
  long long head_pix;
};

static int round_up(int a, int b) { return (a + b - 1) / b * b; }

static bool dec_plan(const vrs_decoder_desc* dd, const vrs_crop* crops, int n_crops, DecPlan* P) {
  if (!dd || dd->n_levels < 1 || dd->n_levels > VRS_MAX_LEVELS || dd->in_ch < 1) return false;
  if (dd->dtype != VRS_F32 && dd->dtype != VRS_BF16) return false;
  if (n_crops < 1 || n_crops > VRS_MAX_CROPS || !crops) return false;
  P->nd = dd->n_levels;
  P->C = dd->in_ch;
  P->dtype = dd->dtype;
  P->n_crops = n_crops;
  const int kstep = dd->dtype == VRS_BF16 ? 32 : 4;
  const size_t esz = dd->dtype == VRS_BF16 ? 2 : 4;
  size_t wo = 0;
  for (int l = 0; l < P->nd; ++l) {
    const int K = dd->width[l];
    if (K < 1 || K > 16 * kDecMaxNT / 2) return false;
    P->K[l] = K;
    P->kp[l] = round_up(K, 16);
  }
  for (int l = 0; l < P->nd; ++l) {
    P->cin[l] = P->C + (l + 1 < P->nd ? P->K[l + 1] : 0) + (l == 0 ? 3 : 0);
    P->cin8[l] = round_up(P->cin[l], 8);
    P->kpad[l] = round_up(9 * P->cin8[l], kstep);
    P->w_off[l] = wo;
    wo += (size_t)2 * P->K[l] * 9 * P->cin[l];
    P->b_off[l] = wo;
    wo += 2 * P->K[l];
  }
  P->head_w = wo;
  P->head_b = wo + 3 * P->K[0];
  const int unit = 1 << (P->nd - 1);
  Carver c;
  for (int l = 0; l < P->nd; ++l) {
    long long he = 0;
    for (int k = 0; k < n_crops; ++k) {
      if (crops[k].size < unit || crops[k].size % unit) return false;
      const long long s = crops[k].size >> l;
      he += s * s;
    }
    P->h_elems[l] = he * P->kp[l];
    P->pre_elems[l] = he * 2 * P->kp[l];
    P->wp[l] = c.take((size_t)2 * P->kp[l] * P->kpad[l] * esz);
    P->bp[l] = c.take((size_t)2 * P->kp[l] * 4);
    P->h[l] = c.take((size_t)P->h_elems[l] * esz);
    P->pre[l] = c.take((size_t)P->pre_elems[l] * 4);
    P->dh[l] = c.take((size_t)P->h_elems[l] * 4);
  }
  P->total = c.off;
  return true;
}

static void level_args(const DecPlan& P, int l, const vrs_crop* crops, int n_crops,
                       const KViews& kv, int levels, const vrs_crop_place* place, DecLevel* d,
                       int* blocks) {
  d->place = reinterpret_cast<const int4*>(place);
  const int NT = 2 * P.kp[l] / 16;
  const int TH = P.dtype == VRS_BF16 && NT < 8 ? 16 : 8;   // as ConvCfg
  d->C = P.C;
  d->cin = P.cin[l];
  d->cin8 = P.cin8[l];
  d->kpad = P.kpad[l];
  d->kp = P.kp[l];
  d->nout = 2 * P.kp[l];
  d->kn = l + 1 < P.nd ? P.K[l + 1] : 0;
  d->kpn = l + 1 < P.nd ? P.kp[l + 1] : 0;
  d->has_p = l == 0;
  d->n_crops = n_crops;
  d->W = kv.v[0].W;
  d->H = kv.v[0].H;
  d->width = P.K[l];
  long long pyr = 0, h = 0, hn = 0, pre = 0;
  int tb = 0;
  for (int k = 0; k < n_crops; ++k) {
    const int S = crops[k].size >> l;
    const int tx = (S + 15) / 16, ty = (S + TH - 1) / TH;
    d->tile_base[k] = tb;
    d->tiles_x[k] = tx;
    tb += tx * ty;
    d->S[k] = S;
    d->view[k] = crops[k].view;
    d->x0[k] = crops[k].x0;
    d->y0[k] = crops[k].y0;
    d->mx0[k] = kv.v[crops[k].view].W - crops[k].size;
    d->my0[k] = kv.v[crops[k].view].H - crops[k].size;
    long long lay = pyr;
    for (int q = 0; q < l; ++q) lay += (long long)(crops[k].size >> q) * (crops[k].size >> q);
    d->pyr_off[k] = lay * P.C;
    for (int q = 0; q < levels; ++q) pyr += (long long)(crops[k].size >> q) * (crops[k].size >> q);
    d->h_off[k] = h;
    h += (long long)S * S * P.kp[l];
    d->pre_off[k] = pre;
    pre += (long long)S * S * 2 * P.kp[l];
    if (l + 1 < P.nd) {
      d->hn_off[k] = hn;
      hn += (long long)(S / 2) * (S / 2) * P.kp[l + 1];
    } else {
      d->hn_off[k] = 0;
    }
  }
  d->tile_base[n_crops] = tb;
  *blocks = tb;
}

// LDS a workgroup may allocate on the current device (queried once).
static size_t max_lds_bytes() {
  static size_t cached = 0;
  if (!cached) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
      cached = (size_t)v;
    else
      cached = 64 * 1024;
  }
  return cached;
}

template <typename T, int NT>
static hipError_t launch_nt(const DecLevel& d, int blocks, const float* pyr, const float* periph,
                            const T* hn, const T* wp, const float* bp, T* h, float* pre,
                            const HeadFuse& hf, hipStream_t st) {
  // the whole weight operand in one LDS chunk when it fits (not with two
  // N-tiles: see ConvCfg)
  using One = ConvCfg<T, NT, true>;
  const bool one = NT > 2 && d.kpad <= One::CK;
  const size_t need = one ? conv_smem_bytes<T, NT, true>(d.cin8, d.kn, d.kpad)
                          : conv_smem_bytes<T, NT, false>(d.cin8, d.kn, d.kpad);
  if (need > max_lds_bytes()) return hipErrorInvalidValue;
  if (one)
    hipLaunchKernelGGL((k_dec_conv<T, NT, true>), dim3(blocks), dim3(256), need, st, d, pyr,
                       periph, hn, wp, bp, h, pre, hf);
  else
    hipLaunchKernelGGL((k_dec_conv<T, NT, false>), dim3(blocks), dim3(256), need, st, d, pyr,
                       periph, hn, wp, bp, h, pre, hf);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_conv(const DecLevel& d, int NT, int blocks, const float* pyr,
                              const float* periph, const T* hn, const T* wp, const float* bp, T* h,
                              float* pre, const HeadFuse& hf, hipStream_t st) {
  switch (NT) {
    case 2: return launch_nt<T, 2>(d, blocks, pyr, periph, hn, wp, bp, h, pre, hf, st);
    case 4: return launch_nt<T, 4>(d, blocks, pyr, periph, hn, wp, bp, h, pre, hf, st);
    case 6: return launch_nt<T, 6>(d, blocks, pyr, periph, hn, wp, bp, h, pre, hf, st);
    default: return launch_nt<T, 8>(d, blocks, pyr, periph, hn, wp, bp, h, pre, hf, st);
  }
}

template <typename T>
static vrs_status decode_impl(const DecPlan& P, const float* pyramid, int levels,
                              const float* periph, const KViews& kv, const vrs_crop* crops,
                              int n_crops, const vrs_crop_place* place, const float* weights,
                              float* out, void* ws, bool keep_pre, hipStream_t st) {
  {
    PackArgs<T> pa;
    pa.n = P.nd;
    pa.C = P.C;
    long long s = 0;
    for (int l = 0; l < P.nd; ++l) {
      pa.K[l] = P.K[l];
      pa.cin[l] = P.cin[l];
      pa.cin8[l] = P.cin8[l];
      pa.kp[l] = P.kp[l];
      pa.kpad[l] = P.kpad[l];
      pa.kn[l] = l + 1 < P.nd ? P.K[l + 1] : 0;
      pa.w[l] = weights + P.w_off[l];
      pa.b[l] = weights + P.b_off[l];
      pa.wp[l] = at<T>(ws, P.wp[l]);
      pa.bp[l] = at<float>(ws, P.bp[l]);
      pa.start[l] = s;
      s += (long long)2 * P.kp[l] * P.kpad[l];
    }
    pa.start[P.nd] = s;
    const int blocks = (int)std::min<long long>(1024, (s + 255) / 256);
    hipLaunchKernelGGL(k_dec_pack<T>, dim3(blocks), dim3(256), 0, st, pa);
    VRS_LAUNCH_CHECK();
  }
  DecLevel d;
  for (int l = P.nd - 1; l >= 0; --l) {
    int blocks = 0;
    level_args(P, l, crops, n_crops, kv, levels, place, &d, &blocks);
    const T* hn = l + 1 < P.nd ? at<T>(ws, P.h[l + 1]) : nullptr;
    HeadFuse hf{};
    if (l == 0) {
      // the RGB head runs in the finest level's epilogue
      hf.wo = weights + P.head_w;
      hf.bo = weights + P.head_b;
      hf.fovea = out;
      long long o = 0;
      for (int k = 0; k < n_crops; ++k) {
        hf.out_base[k] = o;
        o += 3LL * crops[k].size * crops[k].size;
      }
    }
    VRS_HIP_CHECK(launch_conv<T>(d, 2 * P.kp[l] / 16, blocks, pyramid, periph, hn,
                                 at<T>(ws, P.wp[l]), at<float>(ws, P.bp[l]), at<T>(ws, P.h[l]),
                                 keep_pre ? at<float>(ws, P.pre[l]) : nullptr, hf, st));
  }
  return VRS_OK;
}

bool dec_plan_public(const vrs_decoder_desc* dd, const vrs_crop* crops, int n_crops, size_t* total) {
  DecPlan P;
  if (!dec_plan(dd, crops, n_crops, &P)) return false;
  *total = P.total;
  return true;
}

}  // namespace vrs

using namespace vrs;

extern "C" size_t vrs_decoder_workspace_size(const vrs_decoder_desc* dd, const vrs_crop* crops,
                                             int n_crops) {
  DecPlan P;
  if (!dec_plan(dd, crops, n_crops, &P)) return 0;
  return P.total;
}

// crops inside their (equally sized) views, sizes multiples of the coarsest
// layer; the origins only when no device placement table overrides them
static bool dec_crops_ok(const vrs_view* views, int n_views, const vrs_crop* crops, int n_crops,
                         int levels, const vrs_crop_place* place) {
  for (int i = 1; i < n_views; ++i)
    if (views[i].width != views[0].width || views[i].height != views[0].height) return false;
  for (int k = 0; k < n_crops; ++k) {
    const vrs_crop& c = crops[k];
    if (c.view < 0 || c.view >= n_views || c.size < 1 || c.size > views[c.view].width ||
        c.size > views[c.view].height || c.size % (1 << (levels - 1)))
      return false;
    if (!place && (c.x0 < 0 || c.y0 < 0 || c.x0 + c.size > views[c.view].width ||
                   c.y0 + c.size > views[c.view].height))
      return false;
  }
  return true;
}

namespace vrs {
vrs_status decode_impl_entry(const float* pyramid, int levels, const float* rgb_periphery,
                             const vrs_view* views, int n_views, const vrs_crop* crops,
                             int n_crops, const vrs_crop_place* place, const float* weights,
                             const vrs_decoder_desc* dd, float* fovea_rgb, void* ws,
                             size_t ws_bytes, void* stream, const Trace* tr) {
  DecPlan P;
  KViews kv;
  if (!make_views(views, n_views, &kv) || !dec_plan(dd, crops, n_crops, &P)) return VRS_EINVAL;
  if (levels < P.nd || levels > VRS_MAX_LEVELS) return VRS_EINVAL;
  if (!pyramid || !rgb_periphery || !weights || !fovea_rgb || !ws || ws_bytes < P.total)
    return VRS_EINVAL;
  if (dd->in_ch != 4) return VRS_EUNSUPPORTED;
  if (!dec_crops_ok(views, n_views, crops, n_crops, levels, place)) return VRS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  trace_begin(tr, VRS_TRACE_DECODER, st);
  vrs_status r;
  if (P.dtype == VRS_BF16)
    r = decode_impl<__bf16>(P, pyramid, levels, rgb_periphery, kv, crops, n_crops, place,
                            weights, fovea_rgb, ws, false, st);
  else
    r = decode_impl<float>(P, pyramid, levels, rgb_periphery, kv, crops, n_crops, place,
                           weights, fovea_rgb, ws, false, st);
  trace_end(tr, VRS_TRACE_DECODER, st);
  return r;
}
}  // namespace vrs

extern "C" vrs_status vrs_decode_fovea(const float* pyramid, int levels,
                                       const float* rgb_periphery, const vrs_view* views,
                                       int n_views, const vrs_crop* crops, int n_crops,
                                       const vrs_crop_place* place, const float* weights,
                                       const vrs_decoder_desc* dd, float* fovea_rgb, void* ws,
                                       size_t ws_bytes, void* stream) {
  return decode_impl_entry(pyramid, levels, rgb_periphery, views, n_views, crops, n_crops, place,
                           weights, dd, fovea_rgb, ws, ws_bytes, stream, nullptr);
}

// ------------------------------------------------------------- backward
namespace vrs {

// head: dh0 = W_o^T dF, dW_o += dF h0^T, db_o += sum dF (block sums, atomics)
template <typename T>
__global__ __launch_bounds__(256) void k_dec_head_bwd(HeadArgs a, const T* __restrict__ h0,
                                                      const float* __restrict__ wo,
                                                      const float* __restrict__ dF,
                                                      float* __restrict__ dh0,
                                                      float* __restrict__ dwo,
                                                      float* __restrict__ dbo) {
  __shared__ float s_acc[3 * 64 + 3];
  for (int e = threadIdx.x; e < 3 * a.K0 + 3; e += blockDim.x) s_acc[e] = 0.0f;
  __syncthreads();
  const long long npix = a.pix_base[a.n_crops];
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p < npix) {
    int k = 0;
    while (k + 1 < a.n_crops && p >= a.pix_base[k + 1]) ++k;
    const long long q = p - a.pix_base[k];
    const long long plane = (long long)a.S[k] * a.S[k];
    const float g[3] = {dF[a.out_base[k] + q], dF[a.out_base[k] + plane + q],
                        dF[a.out_base[k] + 2 * plane + q]};
    const T* h = h0 + a.h_off[k] + q * a.kp;
    float* dh = dh0 + a.h_off[k] + q * a.kp;
    for (int c = 0; c < a.K0; ++c) {
      const float hv = to_f(h[c]);
      dh[c] += wo[c] * g[0] + wo[a.K0 + c] * g[1] + wo[2 * a.K0 + c] * g[2];
      if (dwo) {
        atomicAdd(&s_acc[c], g[0] * hv);
        atomicAdd(&s_acc[a.K0 + c], g[1] * hv);
        atomicAdd(&s_acc[2 * a.K0 + c], g[2] * hv);
      }
    }
    if (dbo)
      for (int ch = 0; ch < 3; ++ch) atomicAdd(&s_acc[3 * a.K0 + ch], g[ch]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 3 * a.K0 + 3; e += blockDim.x) {
    if (e < 3 * a.K0 && dwo) atomicAdd(&dwo[e], s_acc[e]);
    if (e >= 3 * a.K0 && dbo) atomicAdd(&dbo[e - 3 * a.K0], s_acc[e]);
  }
}

// gate: h = ELU(f) sigmoid(g); pre-activations overwritten by their grads
__global__ void k_dec_gate_bwd(float* __restrict__ pre, const float* __restrict__ dh,
                               long long npix, int kp, int K) {
  const long long total = npix * kp;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long p = e / kp;
    const int ch = (int)(e - p * kp);
    const int t = ch / 16, j = ch % 16;
    float* pf = pre + p * 2 * kp + t * 32 + j;
    float* pg = pf + 16;
    if (ch >= K) { *pf = 0.0f; *pg = 0.0f; continue; }
    const float f = *pf, g = *pg, d = dh[p * kp + ch];
    const float sg = 1.0f / (1.0f + expf(-g));
    const float el = f > 0.0f ? f : expm1f(f);
    const float del = f > 0.0f ? 1.0f : el + 1.0f;
    *pf = d * sg * del;
    *pg = d * el * sg * (1.0f - sg);
  }
}

// transposed convolution: gradient of level l's input, routed to its
// sources (pyramid layer, upsampled coarser output, periphery crop)
template <typename T>
__global__ __launch_bounds__(256) void k_dec_dgrad(DecLevel d, const float* __restrict__ dpre,
                                                   const float* __restrict__ w, float* __restrict__ dpyr,
                                                   float* __restrict__ dhn, float* __restrict__ dper) {
  const int cin = d.cin;
  // global pixel index over all crops of this level
  long long pbase[VRS_MAX_CROPS + 1];
  pbase[0] = 0;
  for (int k = 0; k < d.n_crops; ++k) pbase[k + 1] = pbase[k] + (long long)d.S[k] * d.S[k];
  const long long n_elem = pbase[d.n_crops] * cin;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n_elem;
       e += (long long)gridDim.x * blockDim.x) {
    const long long p = e / cin;
    const int c = (int)(e - p * cin);
    int k = 0;
    while (k + 1 < d.n_crops && p >= pbase[k + 1]) ++k;
    const int S = d.S[k];
    const long long q = p - pbase[k];
    const int y = (int)(q / S), x = (int)(q - (long long)y * S);
    const float* dp = dpre + d.pre_off[k];
    float acc = 0.0f;
    for (int ky = 0; ky < 3; ++ky) {
      const int oy = y - ky + 1;
      if (oy < 0 || oy >= S) continue;
      for (int kx = 0; kx < 3; ++kx) {
        const int ox = x - kx + 1;
        if (ox < 0 || ox >= S) continue;
        const float* g = dp + ((long long)oy * S + ox) * d.nout;
        const int tap = ky * 3 + kx;
        for (int ch = 0; ch < d.width; ++ch) {
          const int t = ch / 16, j = ch % 16;
          acc += g[t * 32 + j] * w[((long long)ch * 9 + tap) * cin + c];
          acc += g[t * 32 + 16 + j] * w[((long long)(d.width + ch) * 9 + tap) * cin + c];
        }
      }
    }
    if (c < d.C) {
      if (dpyr) dpyr[d.pyr_off[k] + q * d.C + c] += acc;
    } else if (c < d.C + d.kn) {
      const int cc = c - d.C;
      const int Sn = S >> 1;
      const float sx = 0.5f * (float)x - 0.25f, sy = 0.5f * (float)y - 0.25f;
      const float fx0 = floorf(sx), fy0 = floorf(sy);
      const float fx = sx - fx0, fy = sy - fy0;
      int xa = (int)fx0, ya = (int)fy0, xb = xa + 1, yb = ya + 1;
      xa = xa < 0 ? 0 : (xa > Sn - 1 ? Sn - 1 : xa);
      xb = xb < 0 ? 0 : (xb > Sn - 1 ? Sn - 1 : xb);
      ya = ya < 0 ? 0 : (ya > Sn - 1 ? Sn - 1 : ya);
      yb = yb < 0 ? 0 : (yb > Sn - 1 ? Sn - 1 : yb);
      float* h = dhn + d.hn_off[k];
      atomicAdd(&h[((long long)ya * Sn + xa) * d.kpn + cc], acc * (1.0f - fy) * (1.0f - fx));
      atomicAdd(&h[((long long)ya * Sn + xb) * d.kpn + cc], acc * (1.0f - fy) * fx);
      atomicAdd(&h[((long long)yb * Sn + xa) * d.kpn + cc], acc * fy * (1.0f - fx));
      atomicAdd(&h[((long long)yb * Sn + xb) * d.kpn + cc], acc * fy * fx);
    } else if (d.has_p && dper) {
      const int cc = c - d.C - d.kn;
      const long long plane = (long long)d.W * d.H;
      atomicAdd(&dper[(long long)d.view[k] * 3 * plane + cc * plane +
                      (long long)(dec_y0(d, k) + y) * d.W + (dec_x0(d, k) + x)],
                acc);
    }
  }
}

// weight gradient over 8x8 output tiles: dW[row][tap][c] += sum_p dpre[p][row] x[p+tap][c]
template <typename T>
__global__ __launch_bounds__(256) void k_dec_wgrad(DecLevel d, const float* __restrict__ pyr,
                                                   const float* __restrict__ periph,
                                                   const T* __restrict__ hnext,
                                                   const float* __restrict__ dpre,
                                                   float* __restrict__ dw, float* __restrict__ db) {
  extern __shared__ __align__(16) char smem[];
  const int cin = d.cin, K = d.width;
  float* sx = reinterpret_cast<float*>(smem);          // [10*10][cin]
  float* sg = sx + 100 * cin;                          // [64][2K]
  int b = blockIdx.x, k = 0;
  while (k + 1 < d.n_crops && b >= d.tile_base[k + 1]) ++k;
  const int S = d.S[k];
  const int tl = b - d.tile_base[k], tpr = (S + 7) / 8;
  const int oy = (tl / tpr) * 8, ox = (tl % tpr) * 8;
  for (int e = threadIdx.x; e < 100 * cin; e += blockDim.x) {
    const int pix = e / cin, c = e - pix * cin;
    const int y = oy + pix / 10 - 1, x = ox + pix % 10 - 1;
    float v = 0.0f;
    if (y >= 0 && y < S && x >= 0 && x < S) v = dec_input<T>(d, k, S, y, x, c, pyr, periph, hnext);
    sx[e] = v;
  }
  for (int e = threadIdx.x; e < 64 * 2 * K; e += blockDim.x) {
    const int pix = e / (2 * K), r = e - pix * 2 * K;
    const int y = oy + pix / 8, x = ox + pix % 8;
    float v = 0.0f;
    if (y < S && x < S) {
      const int ch = r < K ? r : r - K, half = r < K ? 0 : 1;
      v = dpre[d.pre_off[k] + ((long long)y * S + x) * d.nout + (ch / 16) * 32 + half * 16 + ch % 16];
    }
    sg[e] = v;
  }
  __syncthreads();
  const int nw = 2 * K * 9 * cin;
  for (int e = threadIdx.x; e < nw; e += blockDim.x) {
    const int row = e / (9 * cin), rem = e - row * 9 * cin;
    const int tap = rem / cin, c = rem - tap * cin;
    const int ky = tap / 3, kx = tap - ky * 3;
    float acc = 0.0f;
    for (int pix = 0; pix < 64; ++pix) {
      const int py = pix / 8, px = pix % 8;
      acc += sg[pix * 2 * K + row] * sx[((py + ky) * 10 + px + kx) * cin + c];
    }
    if (acc != 0.0f) atomicAdd(&dw[e], acc);
  }
  for (int r = threadIdx.x; r < 2 * K; r += blockDim.x) {
    float acc = 0.0f;
    for (int pix = 0; pix < 64; ++pix) acc += sg[pix * 2 * K + r];
    if (acc != 0.0f) atomicAdd(&db[r], acc);
  }
}

template <typename T>
static vrs_status decode_bwd_impl(const DecPlan& P, const float* pyramid, int levels,
                                  const float* periph, const KViews& kv, const vrs_crop* crops,
                                  int n_crops, const vrs_crop_place* place,
                                  const float* weights, const float* d_fovea,
                                  float* d_pyr, float* d_per, float* d_w, void* ws,
                                  hipStream_t st) {
  // recompute every level's pre-activations (the forward's h_l stay valid)
  for (int l = P.nd - 1; l >= 0; --l) {
    DecLevel d;
    int blocks = 0;
    level_args(P, l, crops, n_crops, kv, levels, place, &d, &blocks);
    const T* hn = l + 1 < P.nd ? at<T>(ws, P.h[l + 1]) : nullptr;
    VRS_HIP_CHECK(launch_conv<T>(d, 2 * P.kp[l] / 16, blocks, pyramid, periph, hn,
                                 at<T>(ws, P.wp[l]), at<float>(ws, P.bp[l]), at<T>(ws, P.h[l]),
                                 at<float>(ws, P.pre[l]), HeadFuse{}, st));
    VRS_HIP_CHECK(fill_u32(at<uint32_t>(ws, P.dh[l]), 0u, P.h_elems[l], st));
  }
  // head
  {
    HeadArgs ha;
    ha.n_crops = n_crops;
    ha.kp = P.kp[0];
    ha.K0 = P.K[0];
    long long p = 0, o = 0;
    DecLevel d0;
    int b0 = 0;
    level_args(P, 0, crops, n_crops, kv, levels, place, &d0, &b0);
    for (int k = 0; k < n_crops; ++k) {
      ha.S[k] = crops[k].size;
      ha.pix_base[k] = p;
      ha.out_base[k] = o;
      ha.h_off[k] = d0.h_off[k];
      p += (long long)crops[k].size * crops[k].size;
      o += 3LL * crops[k].size * crops[k].size;
    }
    ha.pix_base[n_crops] = p;
    hipLaunchKernelGGL(k_dec_head_bwd<T>, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, ha,
                       at<T>(ws, P.h[0]), weights + P.head_w, d_fovea, at<float>(ws, P.dh[0]),
                       d_w ? d_w + P.head_w : nullptr, d_w ? d_w + P.head_b : nullptr);
    VRS_LAUNCH_CHECK();
  }
  for (int l = 0; l < P.nd; ++l) {
    DecLevel d;
    int blocks = 0;
    level_args(P, l, crops, n_crops, kv, levels, place, &d, &blocks);
    long long npix = 0;
    for (int k = 0; k < n_crops; ++k) npix += (long long)d.S[k] * d.S[k];
    const int gb = (int)std::min<long long>(16384, (npix * P.kp[l] + 255) / 256);
    hipLaunchKernelGGL(k_dec_gate_bwd, dim3(gb), dim3(256), 0, st, at<float>(ws, P.pre[l]),
                       at<float>(ws, P.dh[l]), npix, P.kp[l], P.K[l]);
    VRS_LAUNCH_CHECK();
    const int dbk = (int)std::min<long long>(16384, (npix * P.cin[l] + 255) / 256);
    hipLaunchKernelGGL(k_dec_dgrad<T>, dim3(dbk), dim3(256), 0, st, d, at<float>(ws, P.pre[l]),
                       weights + P.w_off[l], d_pyr,
                       l + 1 < P.nd ? at<float>(ws, P.dh[l + 1]) : nullptr, d_per);
    VRS_LAUNCH_CHECK();
    if (d_w) {
      DecLevel dw8 = d;
      int tb = 0;
      for (int k = 0; k < n_crops; ++k) {
        dw8.tile_base[k] = tb;
        const int t = (d.S[k] + 7) / 8;
        tb += t * t;
      }
      dw8.tile_base[n_crops] = tb;
      const size_t smem = (size_t)(100 * P.cin[l] + 64 * 2 * P.K[l]) * 4;
      if (smem > 64 * 1024) return VRS_EUNSUPPORTED;
      const T* hn = l + 1 < P.nd ? at<T>(ws, P.h[l + 1]) : nullptr;
      hipLaunchKernelGGL(k_dec_wgrad<T>, dim3(tb), dim3(256), smem, st, dw8, pyramid, periph, hn,
                         at<float>(ws, P.pre[l]), d_w + P.w_off[l], d_w + P.b_off[l]);
      VRS_LAUNCH_CHECK();
    }
  }
  return VRS_OK;
}

}  // namespace vrs

extern "C" vrs_status vrs_decode_fovea_backward(const float* pyramid, int levels,
                                                const float* rgb_periphery, const vrs_view* views,
                                                int n_views, const vrs_crop* crops, int n_crops,
                                                const vrs_crop_place* place,
                                                const float* weights, const vrs_decoder_desc* dd,
                                                const float* d_fovea, float* d_pyramid,
                                                float* d_rgb_periphery, float* d_weights,
                                                void* ws, size_t ws_bytes, void* stream) {
  DecPlan P;
  KViews kv;
  if (!make_views(views, n_views, &kv) || !dec_plan(dd, crops, n_crops, &P)) return VRS_EINVAL;
  if (levels < P.nd || levels > VRS_MAX_LEVELS || !pyramid || !rgb_periphery || !weights ||
      !d_fovea || !ws || ws_bytes < P.total)
    return VRS_EINVAL;
  if (dd->in_ch != 4) return VRS_EUNSUPPORTED;
  if (!dec_crops_ok(views, n_views, crops, n_crops, levels, place)) return VRS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (P.dtype == VRS_BF16)
    return decode_bwd_impl<__bf16>(P, pyramid, levels, rgb_periphery, kv, crops, n_crops, place,
                                   weights, d_fovea, d_pyramid, d_rgb_periphery, d_weights, ws,
                                   st);
  return decode_bwd_impl<float>(P, pyramid, levels, rgb_periphery, kv, crops, n_crops, place,
                                weights, d_fovea, d_pyramid, d_rgb_periphery, d_weights, ws, st);
}
