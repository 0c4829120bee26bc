// Peripheral 3D Gaussian splatting, forward (Sec. 3.2 of VR-Splatting: the
// full image P and the approximate depth of Eq. 1).
//
// Pipeline per call, all views in the same launches:
//   k_gs_preprocess   one thread per Gaussian, attributes read once for all
//                     views; EWA projection, SH colour, 48-byte record,
//                     depth key and tile count per (view, Gaussian)
//   radix sort        (depth bits) of all (view, Gaussian) entries
//   scan              tile counts in depth order -> pair offsets (device)
//   k_gs_emit         output-parallel: each thread writes one (tile, id)
//                     pair, so stores are fully coalesced
//   radix sort        (tile id) of the pairs, stable: keeps depth order
//   k_gs_ranges       [begin, end) per tile from the sorted keys
//   k_gs_blend        one workgroup per tile, batches of records staged in
//                     LDS, front-to-back blend with a block-wide early exit
#include "gs_layout.h"

namespace vrs {

bool gs_render_layout(int64_t n, int nv, const vrs_view* views, int tile, int64_t max_pairs,
                      size_t* rec, size_t* ranges, size_t* sorted_ids, size_t* last,
                      size_t* pair_count, int64_t* tiles_x, int64_t* tiles_y, size_t* total) {
  RenderWs L;
  if (!render_layout(n, nv, views, tile, max_pairs, &L)) return false;
  *rec = L.rec;
  *ranges = L.ranges;
  *sorted_ids = L.pairs_in_1 ? L.pval1 : L.pval0;
  *last = L.last;
  *pair_count = L.pair_count;
  *tiles_x = L.tiles_x;
  *tiles_y = L.tiles_y;
  *total = L.total;
  return true;
}

// ------------------------------------------------------------ preprocess
__global__ __launch_bounds__(256) void k_gs_preprocess(
    const float* __restrict__ mean, const float* __restrict__ cov,
    const float* __restrict__ opacity, const float* __restrict__ sh, int deg, int64_t n,
    KViews views, GsOpt o, float4* __restrict__ rec, uint32_t* __restrict__ dkey,
    uint32_t* __restrict__ dval, uint32_t* __restrict__ ntiles) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float mx = mean[i], my = mean[n + i], mz = mean[2 * n + i];
  float S6[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) S6[k] = cov[k * n + i];
  const float op = opacity[i];
  const int K = (deg + 1) * (deg + 1);
  float coef[16][3];
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < K)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) coef[k][ch] = sh[(k * 3 + ch) * n + i];
  for (int v = 0; v < views.n; ++v) {
    const KView& cv = views.v[v];
    const int64_t e = v * n + i;
    Geom g;
    const bool ok = gs_geom32(cv, mx, my, mz, S6, o.lowpass, o.extent, g);
    dval[e] = (uint32_t)e;
    if (!ok) {
      dkey[e] = 0xffffffffu;
      ntiles[e] = 0;
      rec[3 * e + 0] = make_float4(0, 0, 0, 0);
      rec[3 * e + 1] = make_float4(0, 0, 0, 0);
      rec[3 * e + 2] = make_float4(0, 0, __uint_as_float(0xffffffffu), 0);
      continue;
    }
    const float inv = 1.0f / g.det;
    const float A = g.c * inv, B = -g.b * inv, C = g.a * inv;
    // view-dependent colour
    float dx = mx - cv.cam[0], dy = my - cv.cam[1], dz = mz - cv.cam[2];
    const float rn = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= rn; dy *= rn; dz *= rn;
    float Y[16];
    sh_eval(deg, dx, dy, dz, Y);
    float col[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float acc = 0.5f;
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < K) acc += Y[k] * coef[k][ch];
      col[ch] = acc > 0.0f ? acc : 0.0f;
    }
    const int tile = o.tile;
    const int tx0 = g.x0 / tile, tx1 = g.x1 / tile, ty0 = g.y0 / tile, ty1 = g.y1 / tile;
    dkey[e] = __float_as_uint(g.t[2]);
    ntiles[e] = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    rec[3 * e + 0] = make_float4(g.px, g.py, A, B);
    rec[3 * e + 1] = make_float4(C, op, col[0], col[1]);
    rec[3 * e + 2] = make_float4(col[2], g.t[2], __uint_as_float(pack_xy(g.x0, g.y0)),
                                 __uint_as_float(pack_xy(g.x1, g.y1)));
  }
}

// ------------------------------------------------------------------ emit
// Output-parallel pair emission: pair p belongs to the depth-ordered entry
// j with offs[j] <= p < offs[j] + ntiles[j] (last such j, found by binary
// search within the block's window).  key = view*tiles_per_view + tile,
// value = Gaussian index.
constexpr int kEmitPerThread = 4;
__global__ __launch_bounds__(256) void k_gs_emit(
    const uint32_t* __restrict__ offs, const uint32_t* __restrict__ sorted_e,
    const float4* __restrict__ rec, const uint32_t* __restrict__ total_p, int64_t vn,
    int64_t n, int64_t max_pairs, int tile, int64_t tiles_x, int64_t tiles_per_view,
    uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval, int32_t* status) {
  __shared__ int64_t s_lo, s_hi;
  const int64_t total = *total_p;
  const int64_t cap = std::min<int64_t>(total, max_pairs);
  if (blockIdx.x == 0 && threadIdx.x == 0 && total > max_pairs) set_status(status, VRS_ECAPACITY);
  const int64_t p0 = blockIdx.x * (int64_t)blockDim.x * kEmitPerThread;
  if (p0 >= cap) return;
  const int64_t p1 = std::min<int64_t>(p0 + (int64_t)blockDim.x * kEmitPerThread, cap) - 1;
  if (threadIdx.x < 2) {
    // last j with offs[j] <= target
    const int64_t target = threadIdx.x == 0 ? p0 : p1;
    int64_t lo = 0, hi = vn - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) >> 1;
      if ((int64_t)offs[mid] <= target) lo = mid;
      else hi = mid - 1;
    }
    if (threadIdx.x == 0) s_lo = lo;
    else s_hi = lo;
  }
  __syncthreads();
  const int64_t wlo = s_lo, whi = s_hi;
  for (int r = 0; r < kEmitPerThread; ++r) {
    const int64_t p = p0 + r * (int64_t)blockDim.x + threadIdx.x;
    if (p > p1) break;
    int64_t lo = wlo, hi = whi;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) >> 1;
      if ((int64_t)offs[mid] <= p) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t e = sorted_e[lo];
    const int64_t v = e / n, gi = e - v * n;
    const float4 r2 = rec[3 * (int64_t)e + 2];
    const uint32_t lo_xy = __float_as_uint(r2.z), hi_xy = __float_as_uint(r2.w);
    const int tx0 = (int)(lo_xy & 0xffffu) / tile, ty0 = (int)(lo_xy >> 16) / tile;
    const int tx1 = (int)(hi_xy & 0xffffu) / tile;
    const int w = tx1 - tx0 + 1;
    const int k = (int)(p - (int64_t)offs[lo]);
    const int ty = ty0 + k / w, tx = tx0 + k % w;
    pkey[p] = (uint32_t)(v * tiles_per_view + (int64_t)ty * tiles_x + tx);
    pval[p] = (uint32_t)gi;
  }
}

// ---------------------------------------------------------------- ranges
__global__ void k_gs_ranges(const uint32_t* __restrict__ key, const uint32_t* total_p,
                            int64_t max_pairs, int64_t tiles_total, uint2* __restrict__ ranges) {
  const int64_t cnt = std::min<int64_t>(*total_p, max_pairs);
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < cnt;
       p += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = key[p];
    if (k >= (uint64_t)tiles_total) continue;   // never for a well-formed list
    if (p == 0 || key[p - 1] != k) ranges[k].x = (uint32_t)p;
    if (p == cnt - 1 || key[p + 1] != k) ranges[k].y = (uint32_t)(p + 1);
  }
}

// ----------------------------------------------------------------- blend
// One workgroup per (view, tile).  BLOCK threads, PPT pixels per thread.
// Records of the tile list are staged in LDS in batches of BLOCK; every
// pixel evaluates the batch in list order; the block leaves the list as
// soon as all its pixels have stopped (block-wide vote).
template <int TILE>
struct BlendCfg {
  static constexpr int PIX = TILE * TILE;
  static constexpr int BLOCK = PIX < 256 ? PIX : 256;
  static constexpr int PPT = PIX / BLOCK;
};

template <int TILE>
__global__ __launch_bounds__(BlendCfg<TILE>::BLOCK) void k_gs_blend(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids,
    const float4* __restrict__ rec, int64_t n, KViews views, GsOpt o, int64_t tiles_x,
    int64_t tiles_per_view, float* __restrict__ out_rgb, float* __restrict__ out_depth,
    float* __restrict__ out_t, int32_t* __restrict__ out_n, uint32_t* __restrict__ out_last,
    uint32_t* __restrict__ out_evals) {
  using Cfg = BlendCfg<TILE>;
  constexpr int BLOCK = Cfg::BLOCK, PPT = Cfg::PPT;
  __shared__ float4 s_a[BLOCK], s_b[BLOCK], s_c[BLOCK];
  const int64_t tglob = blockIdx.x;
  const int v = (int)(tglob / tiles_per_view);
  const int64_t tl = tglob - (int64_t)v * tiles_per_view;
  const int ty = (int)(tl / tiles_x), tx = (int)(tl - (int64_t)ty * tiles_x);
  const KView& cv = views.v[v];
  const int W = cv.W, H = cv.H;
  const int tid = threadIdx.x;
  int px[PPT], py[PPT];
  float T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT];
  int cnt[PPT];
  uint32_t last[PPT], evals[PPT];
  bool done[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int l = tid + q * BLOCK;
    px[q] = tx * TILE + (l % TILE);
    py[q] = ty * TILE + (l / TILE);
    T[q] = 1.0f; C0[q] = C1[q] = C2[q] = D[q] = 0.0f;
    cnt[q] = 0;
    last[q] = 0;
    evals[q] = 0;
    done[q] = px[q] >= W || py[q] >= H;
  }
  const uint2 rg = ranges[tglob];
  const uint32_t begin = rg.x, end = rg.y > rg.x ? rg.y : rg.x;
  const float aclamp = o.aclamp, amin = o.amin, tmin = o.tmin;
  for (uint32_t b0 = begin; b0 < end; b0 += BLOCK) {
    bool mine_done = true;
#pragma unroll
    for (int q = 0; q < PPT; ++q) mine_done &= done[q];
    if (__syncthreads_count(mine_done) == BLOCK) break;
    const uint32_t j = b0 + tid;
    if (j < end) {
      const uint32_t id = ids[j];
      const int64_t e = (int64_t)v * n + (id < (uint64_t)n ? id : 0);
      s_a[tid] = rec[3 * e + 0];
      s_b[tid] = rec[3 * e + 1];
      s_c[tid] = rec[3 * e + 2];
    }
    __syncthreads();
    const int cntb = (int)min((uint32_t)BLOCK, end - b0);
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      if (done[q]) continue;
      const float xc = (float)px[q] + 0.5f, yc = (float)py[q] + 0.5f;
      const uint32_t pxy = pack_xy(px[q], py[q]);
      const uint32_t pxl = pxy & 0xffffu, pyl = pxy >> 16;
      for (int k = 0; k < cntb; ++k) {
        const float4 c = s_c[k];
        const uint32_t lo = __float_as_uint(c.z), hi = __float_as_uint(c.w);
        if (pxl < (lo & 0xffffu) || pxl > (hi & 0xffffu) || pyl < (lo >> 16) || pyl > (hi >> 16))
          continue;
        ++evals[q];
        const float4 a = s_a[k];
        const float4 bq = s_b[k];
        float dx, dy, eq, al;
        if (!gs_alpha(a, bq, xc, yc, aclamp, dx, dy, eq, al)) continue;
        if (al < amin) continue;
        const float Tn = T[q] * (1.0f - al);
        if (Tn < tmin) {
          done[q] = true;
          break;
        }
        const float wgt = al * T[q];
        C0[q] += bq.z * wgt;
        C1[q] += bq.w * wgt;
        C2[q] += c.x * wgt;
        D[q] += c.y * wgt;
        T[q] = Tn;
        ++cnt[q];
        last[q] = b0 + k + 1 - begin;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    if (px[q] >= W || py[q] >= H) continue;
    const int64_t pix = (int64_t)v * W * H + (int64_t)py[q] * W + px[q];
    const int64_t plane = (int64_t)W * H;
    out_rgb[(int64_t)v * 3 * plane + 0 * plane + (int64_t)py[q] * W + px[q]] = C0[q] + T[q] * o.bg[0];
    out_rgb[(int64_t)v * 3 * plane + 1 * plane + (int64_t)py[q] * W + px[q]] = C1[q] + T[q] * o.bg[1];
    out_rgb[(int64_t)v * 3 * plane + 2 * plane + (int64_t)py[q] * W + px[q]] = C2[q] + T[q] * o.bg[2];
    out_depth[pix] = D[q];
    out_t[pix] = T[q];
    out_n[pix] = cnt[q];
    out_last[pix] = last[q];
    out_evals[pix] = evals[q];
  }
}

}  // namespace vrs

using namespace vrs;

static bool read_opts(const vrs_raster_opts* ro, GsOpt* o) {
  if (!ro) return false;
  o->tile = ro->tile;
  o->aclamp = ro->alpha_clamp;
  o->amin = ro->alpha_min;
  o->tmin = ro->t_min;
  o->lowpass = ro->lowpass;
  o->extent = ro->extent;
  for (int k = 0; k < 3; ++k) o->bg[k] = ro->bg[k];
  return (o->tile == 8 || o->tile == 16 || o->tile == 32) && o->extent > 0 && o->lowpass >= 0;
}

static bool same_dims(const vrs_view* views, int nv) {
  for (int i = 1; i < nv; ++i)
    if (views[i].width != views[0].width || views[i].height != views[0].height) return false;
  return true;
}

extern "C" size_t vrs_render_workspace_size(int64_t n, int n_views, const vrs_view* views,
                                            const vrs_raster_opts* opts, int64_t max_pairs) {
  RenderWs L;
  if (!opts || !render_layout(n, n_views, views, opts->tile, max_pairs, &L)) return 0;
  return L.total;
}

extern "C" vrs_status vrs_render_workspace_layout(int64_t n, int n_views, const vrs_view* views,
                                                  const vrs_raster_opts* opts,
                                                  int64_t max_pairs, vrs_render_layout* out) {
  RenderWs L;
  if (!opts || !out || !render_layout(n, n_views, views, opts->tile, max_pairs, &L))
    return VRS_EINVAL;
  out->pair_count = L.pair_count;
  out->sorted_ids = L.pairs_in_1 ? L.pval1 : L.pval0;
  out->tile_ranges = L.ranges;
  out->tiles_x = L.tiles_x;
  out->tiles_y = L.tiles_y;
  out->tiles_total = L.tiles_total;
  out->pixel_evals = L.evals;
  return VRS_OK;
}

template <int TILE>
static void launch_blend(const RenderWs& L, void* ws, int64_t n, const KViews& kv, const GsOpt& o,
                         float* rgb, float* depth, float* tf, int32_t* nc, hipStream_t st) {
  const uint2* ranges = at<uint2>(ws, L.ranges);
  const uint32_t* ids = at<uint32_t>(ws, L.pairs_in_1 ? L.pval1 : L.pval0);
  hipLaunchKernelGGL(k_gs_blend<TILE>, dim3((unsigned)L.tiles_total), dim3(BlendCfg<TILE>::BLOCK),
                     0, st, ranges, ids, at<float4>(ws, L.rec), n, kv, o, L.tiles_x,
                     L.tiles_x * L.tiles_y, rgb, depth, tf, nc, at<uint32_t>(ws, L.last),
                     at<uint32_t>(ws, L.evals));
}

extern "C" vrs_status vrs_render_gaussians(const float* mean, const float* cov,
                                           const float* opacity, const float* sh, int sh_degree,
                                           int64_t n, const vrs_view* views, int n_views,
                                           const vrs_raster_opts* opts, float* rgb, float* depth,
                                           float* t_final, int32_t* n_contrib, void* ws,
                                           size_t ws_bytes, int64_t max_pairs,
                                           int32_t* dev_status, void* stream) {
  GsOpt o;
  KViews kv;
  RenderWs L;
  if (!read_opts(opts, &o) || !make_views(views, n_views, &kv) || !same_dims(views, n_views))
    return VRS_EINVAL;
  if (n < 0 || n > (int64_t(1) << 28) || (n > 0 && (!mean || !cov || !opacity || !sh)))
    return VRS_EINVAL;
  if (sh_degree < 0 || sh_degree > 3) return VRS_EINVAL;
  if (!rgb || !depth || !t_final || !n_contrib || !ws) return VRS_EINVAL;
  if (max_pairs < 0 || max_pairs >= (int64_t(1) << 30)) return VRS_EINVAL;
  if (!render_layout(n, n_views, views, o.tile, max_pairs, &L) || ws_bytes < L.total)
    return VRS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t vn = L.vn;
  uint32_t* pair_count = at<uint32_t>(ws, L.pair_count);
  if (vn > 0) {
    trace_begin(VRS_TRACE_GS_PREPROCESS, st);
    hipLaunchKernelGGL(k_gs_preprocess, dim3(div_up(n, 256)), dim3(256), 0, st, mean, cov,
                       opacity, sh, sh_degree, n, kv, o, at<float4>(ws, L.rec),
                       at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0),
                       at<uint32_t>(ws, L.ntiles));
    VRS_LAUNCH_CHECK();
    trace_end(VRS_TRACE_GS_PREPROCESS, st);
    trace_begin(VRS_TRACE_GS_DEPTH_SORT, st);
    bool d1 = false;
    VRS_HIP_CHECK(radix_sort_u32(at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0),
                                 at<uint32_t>(ws, L.dkey1), at<uint32_t>(ws, L.dval1), nullptr, vn,
                                 32, at<void>(ws, L.sort_tmp), dev_status, st, &d1));
    const uint32_t* sorted_e = at<uint32_t>(ws, d1 ? L.dval1 : L.dval0);
    VRS_HIP_CHECK(exclusive_scan_u32(at<uint32_t>(ws, L.ntiles), sorted_e, at<uint32_t>(ws, L.offs),
                                     pair_count, nullptr, vn, at<void>(ws, L.scan_tmp), dev_status,
                                     st));
    trace_end(VRS_TRACE_GS_DEPTH_SORT, st);
    trace_begin(VRS_TRACE_GS_EMIT, st);
    {
      const int blocks = std::max(1, div_up(max_pairs, 256 * kEmitPerThread));
      hipLaunchKernelGGL(k_gs_emit, dim3(blocks), dim3(256), 0, st, at<uint32_t>(ws, L.offs),
                         sorted_e, at<float4>(ws, L.rec), pair_count, vn, n, max_pairs, o.tile,
                         L.tiles_x, L.tiles_x * L.tiles_y, at<uint32_t>(ws, L.pkey0),
                         at<uint32_t>(ws, L.pval0), dev_status);
      VRS_LAUNCH_CHECK();
    }
    trace_end(VRS_TRACE_GS_EMIT, st);
    trace_begin(VRS_TRACE_GS_SORT, st);
    bool p1 = false;
    VRS_HIP_CHECK(radix_sort_u32(at<uint32_t>(ws, L.pkey0), at<uint32_t>(ws, L.pval0),
                                 at<uint32_t>(ws, L.pkey1), at<uint32_t>(ws, L.pval1), pair_count,
                                 max_pairs, L.tile_bits, at<void>(ws, L.sort_tmp), dev_status, st,
                                 &p1));
    trace_end(VRS_TRACE_GS_SORT, st);
  } else {
    VRS_HIP_CHECK(fill_u32(pair_count, 0, 1, st));
  }
  VRS_HIP_CHECK(fill_u32(at<uint32_t>(ws, L.ranges), 0, L.tiles_total * 2, st));
  if (max_pairs > 0) {
    const int blocks = (int)std::min<int64_t>(8192, std::max(1, div_up(max_pairs, 256)));
    hipLaunchKernelGGL(k_gs_ranges, dim3(blocks), dim3(256), 0, st,
                       at<uint32_t>(ws, L.pairs_in_1 ? L.pkey1 : L.pkey0), pair_count, max_pairs,
                       L.tiles_total, at<uint2>(ws, L.ranges));
    VRS_LAUNCH_CHECK();
  }
  trace_begin(VRS_TRACE_GS_BLEND, st);
  switch (o.tile) {
    case 8: launch_blend<8>(L, ws, n, kv, o, rgb, depth, t_final, n_contrib, st); break;
    case 16: launch_blend<16>(L, ws, n, kv, o, rgb, depth, t_final, n_contrib, st); break;
    default: launch_blend<32>(L, ws, n, kv, o, rgb, depth, t_final, n_contrib, st); break;
  }
  VRS_LAUNCH_CHECK();
  trace_end(VRS_TRACE_GS_BLEND, st);
  return VRS_OK;
}
