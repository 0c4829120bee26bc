// Foveal neural-point splat, forward (Sec. 3.3 sub-frustum + depth cull;
// Sec. 4 "Inference": one count, one scan and one fill over all pyramid
// layers and all crops).
//
// Fragments go straight to per-pixel segments: emission counts each layer
// pixel's fragments, a scan turns the counts into segment offsets, and each
// fragment's place in its segment is its rank by (float32 bits of t.z,
// point index) among the segment's fragments -- so the lists come out in
// blend order with no global sort, and deterministically (atomics only
// place survivors and fragments in scratch lists whose order the ranking
// removes).
//   k_pt_prep      per-pixel counters, the survivor and fragment counts and
//                  the pixel scan's temporary zeroed, crop grid
//   k_pt_select    one thread per point, points read once for all crops:
//                  projection, layer, crop footprints, then the depth cull;
//                  survivors (depth key, entry, fragment offset) compacted in
//                  the same pass, one 64-bit atomic per workgroup for the
//                  survivor and fragment bases, and the survivor that opens
//                  each emission chunk
//   k_pt_emit      one workgroup per chunk of 1024 consecutive fragments,
//                  one thread per survivor of the chunk: writes its
//                  fragments (layer pixel, weight | point index, depth key),
//                  counts them per pixel and takes each one a free place in
//                  its pixel's segment (the counting atomics' old values)
//   scan           per-pixel counts -> segment offsets
//   k_pt_scatter   each fragment's record (point index, depth key, weight,
//                  pixel) to its segment place: no atomics
//   k_pt_rank      one thread per segment place: the record's rank in its
//                  segment -> its final place (the lanes of one segment
//                  read the same records)
//   k_pt_blend     one thread per layer pixel walks its list front to back
#include <hip/hip_fp16.h>

#include "pt_device.h"

namespace vrs {

struct SplatWs {
  size_t surv, ctr, live, frag_count,   // survivors: (entry, depth key, fragment offset, 0)
      chunk_first,                 // per emission chunk: the survivor holding its first fragment
      fkey0, fval0, fdep, fslot,   // fragments in emission order, place in segment
      seg,                         // (point index, depth key, weight, pixel) per segment place
      fkey1, fval1,                // fragments in blend order
      pcnt, poff,                  // per layer pixel: fragment count, segment offsets [P + 1]
      grid, scan_tmp, total;
  int gx, gy;   // crop-lookup grid cells per view row / column
  int64_t vn, pix_total;
};

constexpr int kSelBlock = 256;
// Fragments per emission workgroup (one chunk of the fragment range).
constexpr int kEmitFrags = 1024;

static int64_t pyramid_pixels(const vrs_crop* crops, int n_crops, int levels) {
  int64_t s = 0;
  for (int k = 0; k < n_crops; ++k)
    for (int l = 0; l < levels; ++l) {
      int64_t e = crops[k].size >> l;
      s += e * e;
    }
  return s;
}

// Crop-lookup grid: cells of kGridCell x kGridCell view pixels, per view.
constexpr int kGridCell = 32;

static bool splat_layout(int64_t np, int nv, int W, int H, const vrs_crop* crops, int n_crops,
                         int levels, int64_t max_frags, SplatWs* L) {
  if (np < 0 || nv < 1 || nv > VRS_MAX_VIEWS || n_crops < 0 || n_crops > VRS_MAX_CROPS ||
      levels < 1 || levels > VRS_MAX_LEVELS || max_frags < 0 || (n_crops > 0 && !crops) ||
      W < 1 || H < 1)
    return false;
  L->gx = (W + kGridCell - 1) / kGridCell;
  L->gy = (H + kGridCell - 1) / kGridCell;
  L->vn = np * nv;
  L->pix_total = pyramid_pixels(crops, n_crops, levels);
  const int64_t vn = std::max<int64_t>(L->vn, 1), mf = std::max<int64_t>(max_frags, 1);
  const int64_t pt = std::max<int64_t>(L->pix_total, 1);
  Carver c;
  L->surv = c.take(vn * 16);
  L->ctr = c.take(8);   // survivors in the low word, fragments in the high word
  L->live = L->ctr;
  L->frag_count = L->ctr + 4;
  L->chunk_first = c.take((mf / kEmitFrags + 2) * 4);
  L->fkey0 = c.take(mf * 4);
  L->fval0 = c.take(mf * 8);
  L->fdep = c.take(mf * 4);
  L->fslot = c.take(mf * 4);
  L->seg = c.take(mf * 16);
  L->fkey1 = c.take(mf * 4);
  L->fval1 = c.take(mf * 8);
  L->pcnt = c.take(pt * 4);
  L->poff = c.take((pt + 1) * 4);
  L->grid = c.take((size_t)nv * L->gx * L->gy * 4);
  L->scan_tmp = c.take(scan_tmp_bytes(pt));
  L->total = c.off;
  return true;
}

static bool splat_layout_for(int64_t np, int n_views, const vrs_view* views, const vrs_crop* crops,
                             int n_crops, int levels, int64_t max_frags, SplatWs* L) {
  if (!views || n_views < 1) return false;
  return splat_layout(np, n_views, views[0].width, views[0].height, crops, n_crops, levels,
                      max_frags, L);
}

// host: crop table with packed-pyramid and packed-output bases; with a
// device placement table the host origins are not used (nor checked)
bool make_crops(const vrs_crop* crops, int n_crops, int levels, const KViews& kv, KCrops* out,
                const vrs_crop_place* place, bool check_origins = true) {
  if (n_crops < 0 || n_crops > VRS_MAX_CROPS || levels < 1 || levels > VRS_MAX_LEVELS)
    return false;
  if (n_crops > 0 && !crops) return false;
  out->n = n_crops;
  out->place = reinterpret_cast<const int4*>(place);
  int64_t pb = 0, ob = 0;
  const int unit = 1 << (levels - 1);
  for (int k = 0; k < n_crops; ++k) {
    const vrs_crop& c = crops[k];
    if (c.view < 0 || c.view >= kv.n) return false;
    if (c.size < unit || c.size % unit != 0) return false;
    const KView& v = kv.v[c.view];
    if (c.size > v.W || c.size > v.H) return false;
    if (!place && check_origins &&
        (c.x0 < 0 || c.y0 < 0 || c.x0 + c.size > v.W || c.y0 + c.size > v.H))
      return false;
    KCrop& d = out->c[k];
    d.view = c.view; d.x0 = c.x0; d.y0 = c.y0; d.size = c.size;
    d.gx = c.gaze_x; d.gy = c.gaze_y;
    d.mx0 = v.W - c.size;
    d.my0 = v.H - c.size;
    d.pix_base = (int)pb;
    d.out_base = (int)ob;
    for (int l = 0; l < levels; ++l) pb += (int64_t)(c.size >> l) * (c.size >> l);
    ob += (int64_t)3 * c.size * c.size;
    if (pb > (int64_t(1) << 30) || ob > (int64_t(1) << 30)) return false;
  }
  return true;
}

struct PtArgs {
  float cov_min, slack;
  int levels;
  uint32_t view_mask;  // views that own at least one crop
};

// ---------------------------------------------------------------- select
// Crop-lookup grid: per view and cell, the bit set of crops that a point
// whose pixel lies in the cell may reach.  A footprint at layer l < levels
// reaches at most 2^(l-1) + 1 view pixels beyond its crop, so crop k is
// listed in every cell that meets [x0 - 2^levels - 2, x0 + size + 2^levels + 2)
// (likewise y); border cells extend to infinity so that lookups of pixels
// outside the view clamp to them.
// ox, oy: the crops' origins (a workgroup's copy in LDS).
__device__ inline void pt_cropgrid_cell(const KCrops& crops, int levels, int gx, int gy,
                                        int64_t idx, const int* ox, const int* oy,
                                        uint32_t* __restrict__ grid) {
  const int v = (int)(idx / ((int64_t)gx * gy));
  const int cell = (int)(idx - (int64_t)v * gx * gy);
  const int cy = cell / gx, cx = cell - cy * gx;
  const int M = (1 << levels) + 2;
  const int64_t lo_x = cx == 0 ? INT32_MIN : (int64_t)cx * kGridCell;
  const int64_t hi_x = cx == gx - 1 ? INT32_MAX : (int64_t)(cx + 1) * kGridCell;
  const int64_t lo_y = cy == 0 ? INT32_MIN : (int64_t)cy * kGridCell;
  const int64_t hi_y = cy == gy - 1 ? INT32_MAX : (int64_t)(cy + 1) * kGridCell;
  uint32_t mask = 0;
  for (int k = 0; k < crops.n; ++k) {
    const KCrop& c = crops.c[k];
    if (c.view != v) continue;
    const int cx0 = ox[k], cy0 = oy[k];
    const int64_t x0 = (int64_t)cx0 - M, x1 = (int64_t)cx0 + c.size + M;
    const int64_t y0 = (int64_t)cy0 - M, y1 = (int64_t)cy0 + c.size + M;
    if (x0 < hi_x && x1 > lo_x && y0 < hi_y && y1 > lo_y) mask |= 1u << k;
  }
  grid[idx] = mask;
}

// Crop k placed on its gaze point g: the crop of size S centred on the gaze,
// x0 = clamp(rint(g.x - S/2), 0, W - S) (ties to even), y0 likewise; the
// gaze itself in the last two words.
__device__ inline int4 place_crop(const KCrops& kc, int k, float2 g) {
  const float h = 0.5f * (float)kc.c[k].size;
  const float fx = rintf(g.x - h), fy = rintf(g.y - h);
  // clamp in float first: a non-finite or huge gaze gives a valid origin
  const float cx = fminf(fmaxf(fx, 0.0f), (float)kc.c[k].mx0);
  const float cy = fminf(fmaxf(fy, 0.0f), (float)kc.c[k].my0);
  return make_int4(cx == cx ? (int)cx : 0, cy == cy ? (int)cy : 0, __float_as_int(g.x),
                   __float_as_int(g.y));
}

// Crop origins from gaze points on the device (Sec. 4 "Inference": the eye
// tracker is read after the periphery is rendered), one thread per crop.
__global__ void k_place_crops(const float2* __restrict__ gaze, KCrops kc, int4* __restrict__ out) {
  const int k = threadIdx.x;
  if (k >= kc.n) return;
  out[k] = place_crop(kc, k, gaze[k]);
}

// Per-call set-up in one launch: the per-pixel fragment counters, the
// survivor and fragment counts and the pixel scan's temporary zeroed, and
// the crop-lookup grid.
// With gaze, the crops are placed here as well (what the placement entry
// point computes): every workgroup places them for its own cells, the first
// one writes the placement table that the later kernels read.
__global__ void k_pt_prep(uint32_t* __restrict__ pcnt, int64_t pix_total,
                          uint64_t* __restrict__ ctr, uint32_t* __restrict__ scan_tmp,
                          int64_t scan_words, KCrops crops, int nv, int levels, int gx, int gy,
                          uint32_t* __restrict__ grid, const float2* __restrict__ gaze,
                          int4* __restrict__ place_out) {
  const int64_t cells = (int64_t)nv * gx * gy;
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  // crop origins read once per workgroup (from the device placement table
  // when there is one): a cell's crop loop would otherwise wait on each
  __shared__ int s_ox[VRS_MAX_CROPS], s_oy[VRS_MAX_CROPS];
  if (threadIdx.x < crops.n) {
    if (gaze) {
      const int4 pl = place_crop(crops, threadIdx.x, gaze[threadIdx.x]);
      s_ox[threadIdx.x] = pl.x;
      s_oy[threadIdx.x] = pl.y;
      if (blockIdx.x == 0) place_out[threadIdx.x] = pl;
    } else {
      s_ox[threadIdx.x] = crop_x0(crops, threadIdx.x);
      s_oy[threadIdx.x] = crop_y0(crops, threadIdx.x);
    }
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // the counters in 16-byte stores (the workspace's sub-buffers are 256-byte
  // aligned), the tail word by word
  uint4* p4 = reinterpret_cast<uint4*>(pcnt);
  for (int64_t q = gt; q < pix_total / 4; q += stride) p4[q] = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t i = (pix_total & ~int64_t(3)) + gt; i < pix_total; i += stride) pcnt[i] = 0u;
  for (int64_t i = gt; i < scan_words; i += stride) scan_tmp[i] = 0u;
  if (gt == 0) *ctr = 0ull;
  for (int64_t i = gt; i < cells; i += stride)
    pt_cropgrid_cell(crops, levels, gx, gy, i, s_ox, s_oy, grid);
}

// Candidate crops of one point in view v: the crop-lookup grid cell of a
// reciprocal-based pixel estimate (within 1e-2 px of the exact one, well
// inside the grid's slack).  A non-positive or non-finite estimate gives
// every crop.
__device__ inline uint32_t pt_candidates(const KView& cv, int v, int n_crops,
                                         const uint32_t* __restrict__ grid, int gx, int gy,
                                         float x, float y, float z) {
  uint32_t cand = n_crops >= 32 ? 0xffffffffu : ((1u << n_crops) - 1u);
  const float tx = cv.R[0] * x + cv.R[1] * y + cv.R[2] * z + cv.t[0];
  const float ty = cv.R[3] * x + cv.R[4] * y + cv.R[5] * z + cv.t[1];
  const float tz = cv.R[6] * x + cv.R[7] * y + cv.R[8] * z + cv.t[2];
  if (tz > 0.0f) {
    const float rz = __builtin_amdgcn_rcpf(tz);
    const float ex = (cv.fx * (tx * rz) + cv.cx) * (1.0f / kGridCell);
    const float ey = (cv.fy * (ty * rz) + cv.cy) * (1.0f / kGridCell);
    if (isfinite(ex) && isfinite(ey)) {
      const float fx = fminf(fmaxf(floorf(ex), 0.0f), (float)(gx - 1));
      const float fy = fminf(fmaxf(floorf(ey), 0.0f), (float)(gy - 1));
      cand = grid[((int64_t)v * gy + (int)fy) * gx + (int)fx];
    }
  }
  return cand;
}

// Footprint targets of a projected point over the candidate crops of view v
// and the point's one or two pyramid layers; cview, csize, ox, oy: the
// crops' views, sizes and origins (a workgroup's copy in LDS: a lane's crop
// index is its own, so a read from the kernel arguments would be a vector
// load and a wait per crop).
__device__ inline uint32_t pt_targets_over(const PtGeom& g, int v, uint32_t cand, int levels,
                                           const int* cview, const int* csize, const int* ox,
                                           const int* oy) {
  uint32_t cnt = 0;
  const float M = (float)(1 << levels);
  while (cand) {
    const int k = __builtin_ctz(cand);
    cand &= cand - 1;
    if (cview[k] != v) continue;
    const int cx0 = ox[k], cy0 = oy[k], size = csize[k];
    const float ax = g.px - (float)cx0, ay = g.py - (float)cy0, lim = (float)size + M;
    if (!(ax >= -M && ax < lim && ay >= -M && ay < lim)) continue;
    for (int li = 0; li < (g.two ? 2 : 1); ++li) {
      const int l = g.l0 + li, Sl = size >> l;
      float xl, yl;
      int ix, iy;
      if (pt_layer32(g, cx0, cy0, l, Sl, xl, yl, ix, iy)) cnt += pt_targets(ix, iy, Sl);
    }
  }
  return cnt;
}

// Workgroup b holds points [1024b, 1024b+1024), handled in four rounds of
// 256.  Per round and view each lane's fragment count and depth key go to
// LDS and each wave ballots its survivors; a scan over the (view, round,
// wave) slots places them and their fragments within the workgroup, and one
// 64-bit atomic on the (survivor, fragment) counts gives the workgroup's
// output bases, so no separate scan of fragment counts is needed.  The
// compacted order is
// therefore arbitrary across workgroups, which nothing downstream sees: each
// fragment's final place is its rank by (depth key, point index) in its
// pixel.  One atomic per 1024 points: a single counter address serialises
// its atomics, so workgroups are kept large.
constexpr int kSelRounds = 4, kSelPart = kSelBlock * kSelRounds;

__global__ __launch_bounds__(kSelBlock) void k_pt_select(
    const float* __restrict__ pos, const float* __restrict__ radius, int64_t np, KViews views,
    KCrops crops, PtArgs a, const float* __restrict__ depth, const float* __restrict__ tfinal,
    const uint32_t* __restrict__ grid, int gx, int gy, uint4* __restrict__ surv,
    uint64_t* __restrict__ ctr, uint32_t* __restrict__ chunk_first, int64_t max_frags,
    int32_t* status) {
  constexpr int NW = kSelBlock / 64;
  constexpr int NSLOT = kSelRounds * VRS_MAX_VIEWS * NW;   // (view, round, wave), view-major
  static_assert(NSLOT <= kSelBlock, "one slot per thread in the slot scan");
  __shared__ uint32_t s_base, s_fbase;
  __shared__ uint64_t s_mask[NSLOT];
  __shared__ uint32_t s_pre[NSLOT], s_fsum[NSLOT], s_fpre[NSLOT];
  __shared__ uint32_t s_wsum[NW], s_wfsum[NW];
  // crop origins (from the device placement table when there is one),
  // views and sizes read once: a survivor's crop loop would otherwise wait
  // on loads per crop
  __shared__ int s_ox[VRS_MAX_CROPS], s_oy[VRS_MAX_CROPS], s_cv[VRS_MAX_CROPS], s_cs[VRS_MAX_CROPS];
  extern __shared__ __align__(16) char s_dyn[];
  const int nv = views.n;
  float* s_zd = reinterpret_cast<float*>(s_dyn);                               // [round][view][tid]
  uint32_t* s_cnt = reinterpret_cast<uint32_t*>(s_dyn) + kSelRounds * nv * kSelBlock;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < NSLOT; e += kSelBlock) {
    s_mask[e] = 0;
    s_fsum[e] = 0;
  }
  if (tid < crops.n) {
    s_ox[tid] = crop_x0(crops, tid);
    s_oy[tid] = crop_y0(crops, tid);
    s_cv[tid] = crops.c[tid].view;
    s_cs[tid] = crops.c[tid].size;
  }
  __syncthreads();
  const int64_t part = blockIdx.x;
  // ---- counts of every (round, view, point), in stages so that each
  // stage's loads (positions; grid cells; T' and depth under the points) are
  // in flight together: a point's fragment count is its footprint targets
  // over the candidate crops, zero if the depth cull hides it.  The cull
  // runs before the targets (the result is the same: a hidden point counts
  // zero either way) because it removes most points that reach a crop.
  float px[kSelRounds], py[kSelRounds], pz[kSelRounds], pr[kSelRounds];
  bool pin[kSelRounds];
#pragma unroll
  for (int j = 0; j < kSelRounds; ++j) {
    const int64_t i = part * kSelPart + (int64_t)j * kSelBlock + tid;
    pin[j] = i < np;
    px[j] = py[j] = pz[j] = pr[j] = 0.0f;
    if (pin[j]) { px[j] = pos[i]; py[j] = pos[np + i]; pz[j] = pos[2 * np + i]; pr[j] = radius[i]; }
  }
  for (int v = 0; v < nv; ++v) {
    const KView& cv = views.v[v];
    const bool vm = (a.view_mask >> v) & 1u;
    const int64_t plane = (int64_t)cv.W * cv.H;
    uint32_t cand[kSelRounds];
#pragma unroll
    for (int j = 0; j < kSelRounds; ++j)
      cand[j] = pin[j] && vm ? pt_candidates(cv, v, crops.n, grid, gx, gy, px[j], py[j], pz[j]) : 0u;
    bool ok[kSelRounds], cull[kSelRounds];
    float tz[kSelRounds], tf[kSelRounds], dp[kSelRounds];
#pragma unroll
    for (int j = 0; j < kSelRounds; ++j) {
      ok[j] = cull[j] = false;
      tz[j] = tf[j] = dp[j] = 0.0f;
      if (cand[j]) {
        PtGeom g;
        ok[j] = pt_geom32(cv, px[j], py[j], pz[j], pr[j], a.levels, g);
        tz[j] = g.t[2];
        int64_t pi;
        cull[j] = ok[j] && tfinal && pt_cull_pixel(cv, g, pi);
        if (cull[j]) {
          tf[j] = tfinal[v * plane + pi];
          dp[j] = depth[v * plane + pi];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kSelRounds; ++j) {
      uint32_t cnt = 0;
      if (ok[j] && !(cull[j] && pt_hidden(tz[j], tf[j], dp[j], a.cov_min, a.slack))) {
        PtGeom g;   // recomputed for the few points the cull keeps
        pt_geom32(cv, px[j], py[j], pz[j], pr[j], a.levels, g);
        cnt = pt_targets_over(g, v, cand[j], a.levels, s_cv, s_cs, s_ox, s_oy);
      }
      s_zd[(j * nv + v) * kSelBlock + tid] = tz[j];
      s_cnt[(j * nv + v) * kSelBlock + tid] = cnt;
      const uint64_t m = __ballot(cnt != 0);
      if (m) {   // the slot's fragment total
        uint32_t fs = cnt;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) fs += __shfl_xor(fs, o, 64);
        if (lane == 0) {
          s_mask[(v * kSelRounds + j) * NW + wave] = m;
          s_fsum[(v * kSelRounds + j) * NW + wave] = fs;
        }
      }
    }
  }
  __syncthreads();
  // ---- exclusive scans of the slot survivor and fragment counts in output
  // order, then the workgroup's bases
  {
    const uint32_t c = tid < NSLOT ? (uint32_t)__popcll(s_mask[tid]) : 0u;
    const uint32_t f = tid < NSLOT ? s_fsum[tid] : 0u;
    uint32_t ic = c, jf = f;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(ic, o, 64), z = __shfl_up(jf, o, 64);
      if (lane >= o) {
        ic += y;
        jf += z;
      }
    }
    if (lane == 63) {
      s_wsum[wave] = ic;
      s_wfsum[wave] = jf;
    }
    __syncthreads();
    uint32_t woff = 0, wfoff = 0, total = 0, ftotal = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      if (w < wave) {
        woff += s_wsum[w];
        wfoff += s_wfsum[w];
      }
      total += s_wsum[w];
      ftotal += s_wfsum[w];
    }
    if (tid < NSLOT) {
      s_pre[tid] = woff + ic - c;
      s_fpre[tid] = wfoff + jf - f;
    }
    if (tid == 0) {
      const uint64_t old = total ? atomicAdd(ctr, ((uint64_t)ftotal << 32) | total) : 0ull;
      s_base = (uint32_t)old;
      s_fbase = (uint32_t)(old >> 32);
      // the fragment count wraps only far beyond any capacity
      if ((old >> 32) + ftotal > 0xffffffffull) set_status(status, VRS_ECAPACITY);
    }
  }
  __syncthreads();
  // ---- survivors to their positions, with their fragment offsets
  const uint32_t base = s_base, fbase = s_fbase;
  for (int j = 0; j < kSelRounds; ++j) {
    const int64_t i = part * kSelPart + (int64_t)j * kSelBlock + tid;
    for (int v = 0; v < nv; ++v) {
      const int slot = (v * kSelRounds + j) * NW + wave;
      const uint64_t m = s_mask[slot];
      if (!m) continue;   // uniform
      const uint32_t cnt = s_cnt[(j * nv + v) * kSelBlock + tid];
      uint32_t fi = cnt;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(fi, o, 64);
        if (lane >= o) fi += y;
      }
      if (!cnt) continue;
      const uint32_t below = __builtin_amdgcn_mbcnt_hi(
          (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      const uint32_t p = base + s_pre[slot] + below;
      const uint32_t fo = fbase + s_fpre[slot] + fi - cnt;
      surv[p] = make_uint4((uint32_t)(v * np + i),
                           __float_as_uint(s_zd[(j * nv + v) * kSelBlock + tid]), fo, 0u);
      // the emission chunks whose first fragment is one of this survivor's
      for (uint64_t c = ((uint64_t)fo + kEmitFrags - 1) / kEmitFrags;
           c * kEmitFrags < (uint64_t)fo + cnt && c * kEmitFrags < (uint64_t)max_frags; ++c)
        chunk_first[c] = p;
    }
  }
}

// ------------------------------------------------------------------ emit
// Per-workgroup pixel table in LDS: open addressing with a short linear
// probe.  Device-scope atomics on one address serialise, so fragment counts
// (and segment places) are gathered per workgroup first and the table's
// entries go out as one atomic each; a fragment whose probe finds no place
// falls back to its own atomic.
constexpr int kPixProbe = 8;
constexpr uint32_t kPixEmpty = 0xffffffffu;
template <int N>   // places, a power of two
struct PixHash {
  static constexpr int kBits = N == 4096 ? 12 : (N == 2048 ? 11 : (N == 1024 ? 10 : 9));
  static_assert((1 << kBits) == N, "PixHash size");
  uint32_t key[N], cnt[N];
  __device__ void clear() {
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      key[i] = kPixEmpty;
      cnt[i] = 0u;
    }
  }
  // one more fragment of pixel px: its table place (or -1) and its rank
  // among the table's fragments of px
  __device__ int add(uint32_t px, uint32_t& rank) {
    uint32_t s = (px * 2654435761u) >> (32 - kBits);
    for (int q = 0; q < kPixProbe; ++q) {
      const uint32_t k = atomicCAS(&key[s], kPixEmpty, px);
      if (k == kPixEmpty || k == px) {
        rank = atomicAdd(&cnt[s], 1u);
        return (int)s;
      }
      s = (s + 1) & (N - 1);
    }
    return -1;
  }
};

// One workgroup per chunk of kEmitFrags consecutive fragments (the chunks'
// first survivors are recorded by k_pt_select), one thread per survivor of
// the chunk: its fragments that fall in the chunk, each with its layer
// pixel, weight | point index, depth key and place in the pixel's segment.
// Places come from the pixel counters' old values: the workgroup gathers
// its fragments per pixel in the LDS table (at most half full: a chunk
// holds kEmitFrags fragments), each table entry adds its count with one
// atomic whose old value is the entry's first place, and a fragment's
// place is that plus its rank in the entry.  The chunk is staged in LDS
// and goes out as coalesced stores once the places are known.  Balanced by
// construction: every workgroup emits one chunk, however the fragments
// spread over survivors.
constexpr int kEmitPlaces = 2 * kEmitFrags, kEmitBlock = 256;
constexpr uint32_t kSlotRef = 0x80000000u;   // tag | table place << kRankBits | rank
constexpr int kRankBits = 19;
static_assert(kEmitPlaces <= (1 << (31 - kRankBits)) && kEmitFrags < (1 << kRankBits),
              "table place and rank fit the tag");
static_assert(kEmitPlaces % kEmitBlock == 0 && kEmitFrags % kEmitBlock == 0,
              "table entries and staged fragments per thread");
__global__ __launch_bounds__(kEmitBlock) void k_pt_emit(
    const float* __restrict__ pos, const float* __restrict__ radius, int64_t np, KViews views,
    KCrops crops, PtArgs a, const uint4* __restrict__ surv, const uint32_t* __restrict__ live_p,
    const uint32_t* __restrict__ chunk_first, const uint32_t* __restrict__ total_p,
    int64_t max_frags, uint32_t* __restrict__ fkey, uint64_t* __restrict__ fval,
    uint32_t* __restrict__ fdep, uint32_t* __restrict__ fslot, uint32_t* __restrict__ pcnt,
    const uint32_t* __restrict__ grid, int gx, int gy, int32_t* status) {
  __shared__ PixHash<kEmitPlaces> h;
  // staged fragments: layer pixel, weight bits, place (or tag), owning
  // survivor slot; per survivor slot its point index and depth key
  __shared__ uint32_t s_spx[kEmitFrags], s_sw[kEmitFrags], s_stag[kEmitFrags];
  __shared__ uint16_t s_sown[kEmitFrags];
  __shared__ uint32_t s_pi[kEmitFrags + 1], s_dz[kEmitFrags + 1];
  __shared__ int s_cx0[VRS_MAX_CROPS], s_cy0[VRS_MAX_CROPS], s_cs[VRS_MAX_CROPS],
      s_pb[VRS_MAX_CROPS];
  // crop origins (from the device placement table when there is one), sizes
  // and pyramid bases read once: the crop loop below would otherwise wait on
  // loads per crop
  if (threadIdx.x < crops.n) {
    s_cx0[threadIdx.x] = crop_x0(crops, threadIdx.x);
    s_cy0[threadIdx.x] = crop_y0(crops, threadIdx.x);
    s_cs[threadIdx.x] = crops.c[threadIdx.x].size;
    s_pb[threadIdx.x] = crops.c[threadIdx.x].pix_base;
  }
  __syncthreads();
  const int64_t live = *live_p;
  const int64_t total = *total_p;
  if (blockIdx.x == 0 && threadIdx.x == 0 && total > max_frags) set_status(status, VRS_ECAPACITY);
  if (total > max_frags) return;   // uniform
  const int64_t nchunks = (total + kEmitFrags - 1) / kEmitFrags;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int64_t f0 = ch * kEmitFrags, f1 = std::min<int64_t>(f0 + kEmitFrags, total);
    const int64_t s0 = chunk_first[ch];
    h.clear();
    __syncthreads();
    // survivors s0, s0 + 1, ... while their fragments start before f1 (at
    // most kEmitFrags + 1 of them: each has at least one fragment)
    for (int64_t j = s0 + threadIdx.x; j < live; j += kEmitBlock) {
      const uint4 sv = surv[j];
      const int64_t lo = sv.z;
      if (lo >= f1) break;   // offsets ascend with j
      const int slot = (int)(j - s0);
      const uint32_t e = sv.x;
      const int v = (int)(e / np);
      const int64_t i = e - (int64_t)v * np;
      s_pi[slot] = (uint32_t)i;
      s_dz[slot] = sv.y;
      const KView& cv = views.v[v];
      PtGeom g;
      // the depth cull already passed in k_pt_select; the same single-precision
      // sequence gives identical geometry here
      const float x = pos[i], y = pos[np + i], z = pos[2 * np + i];
      if (!pt_geom32(cv, x, y, z, radius[i], a.levels, g)) continue;
      float f = 0.0f;
      if (g.two) f = log2f(g.s) - (float)g.l0;
      FF ux, uy;   // the weights' position, compensated
      pt_plane_ff(cv, x, y, z, ux, uy);
      int64_t o = lo;
      // the crops the selection counted this point's fragments over (its
      // crop-grid candidates: the other crops give it none), in crop order
      for (uint32_t cand = pt_candidates(cv, v, crops.n, grid, gx, gy, x, y, z); cand && o < f1;
           cand &= cand - 1) {
        const int k = __builtin_ctz(cand);
        const int cx0 = s_cx0[k], cy0 = s_cy0[k], size = s_cs[k];
        int lb = s_pb[k];
        int l = 0;
        for (; l < g.l0; ++l) lb += (size >> l) * (size >> l);
        for (int li = 0; li < (g.two ? 2 : 1); ++li, ++l) {
          const int Sl = size >> l;
          const float wl = g.two ? (li == 0 ? 1.0f - f : f) : 1.0f;
          float xl, yl;
          int ix, iy;
          if (pt_layer32(g, cx0, cy0, l, Sl, xl, yl, ix, iy)) {
            const float bx = pt_frac_ff(cv.fx, ux, cv.cx, cx0, l, ix);
            const float by = pt_frac_ff(cv.fy, uy, cv.cy, cy0, l, iy);
            for (int dy = 0; dy < 2; ++dy)
              for (int dx = 0; dx < 2; ++dx) {
                const int xx = ix + dx, yy = iy + dy;
                if (xx < 0 || xx >= Sl || yy < 0 || yy >= Sl) continue;
                if (o >= f0 && o < f1) {
                  const int local = (int)(o - f0);
                  const uint32_t px = (uint32_t)(lb + yy * Sl + xx);
                  // a point reaches a pixel once, so a pixel's rank in the
                  // table is below the chunk's fragment count
                  uint32_t r;
                  const int hs = h.add(px, r);
                  s_spx[local] = px;
                  s_sw[local] = __float_as_uint(wl * (dx ? bx : 1.0f - bx) * (dy ? by : 1.0f - by));
                  s_stag[local] = hs >= 0 ? (kSlotRef | (uint32_t)hs << kRankBits | r)
                                          : atomicAdd(&pcnt[px], 1u);
                  s_sown[local] = (uint16_t)slot;
                }
                ++o;
              }
          }
          lb += Sl * Sl;
        }
      }
    }
    __syncthreads();
    {
      // every entry's atomic issued before any result is awaited (device-
      // scope atomics take about a microsecond each); the old values
      // replace the counts
      constexpr int kPer = kEmitPlaces / kEmitBlock;
      uint32_t first[kPer];
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        const int q = threadIdx.x + r * kEmitBlock;
        const uint32_t key = h.key[q];
        first[r] = key != kPixEmpty ? atomicAdd(&pcnt[key], h.cnt[q]) : 0u;
      }
#pragma unroll
      for (int r = 0; r < kPer; ++r) h.cnt[threadIdx.x + r * kEmitBlock] = first[r];
    }
    __syncthreads();
    // the chunk out, coalesced, with its places
    for (int q = threadIdx.x; q < (int)(f1 - f0); q += kEmitBlock) {
      const uint32_t t = s_stag[q];
      const int own = s_sown[q];
      fkey[f0 + q] = s_spx[q];
      fval[f0 + q] = ((uint64_t)s_sw[q] << 32) | (uint64_t)s_pi[own];
      fdep[f0 + q] = s_dz[own];
      fslot[f0 + q] = (t & kSlotRef)
                          ? h.cnt[(t & ~kSlotRef) >> kRankBits] + (t & ((1u << kRankBits) - 1u))
                          : t;
    }
    __syncthreads();   // the stage is reused by the next chunk
  }
}

// Each fragment's record (point index, depth key, weight, pixel) to its
// segment place (checked against the segment, so an unresolved place can
// never write outside it).
__global__ __launch_bounds__(256) void k_pt_scatter(const uint32_t* __restrict__ fkey,
                                                    const uint64_t* __restrict__ fval,
                                                    const uint32_t* __restrict__ fdep,
                                                    const uint32_t* __restrict__ fslot,
                                                    const uint32_t* __restrict__ poff,
                                                    const uint32_t* __restrict__ total_p,
                                                    int64_t max_frags, uint4* __restrict__ seg) {
  const int64_t total = *total_p;
  if (total > max_frags) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t px = fkey[i];
    const uint64_t v = fval[i];
    const uint32_t at = poff[px] + fslot[i];
    if (at < poff[px + 1]) seg[at] = make_uint4((uint32_t)v, fdep[i], (uint32_t)(v >> 32), px);
  }
}

// One thread per segment place: the record's final place is its segment's
// offset plus the number of the segment's records before it in (depth key,
// point id) order, the id being the point's index in the caller's numbering
// (ids[i] for stored point i when a numbering is given, else i; a point
// reaches a layer pixel at most once, so the pairs are distinct).  Equal
// depth keys are rare, so the numbering is looked up only for them.
// Consecutive places share segments, so the lanes of a segment read the
// same records; places go in reverse, so that the long segments of each
// crop's coarse layers start early.
__global__ __launch_bounds__(256) void k_pt_rank(const uint4* __restrict__ seg,
                                                 const uint32_t* __restrict__ poff,
                                                 const uint32_t* __restrict__ total_p,
                                                 int64_t max_frags, int64_t pix_total,
                                                 const uint32_t* __restrict__ ids,
                                                 uint32_t* __restrict__ okey,
                                                 uint64_t* __restrict__ oval) {
  const int64_t total = *total_p;
  if (total > max_frags) return;
  const uint64_t* key = reinterpret_cast<const uint64_t*>(seg);   // depth key << 32 | index
  for (int64_t sr = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; sr < total;
       sr += (int64_t)gridDim.x * blockDim.x) {
    const uint4 rec = seg[total - 1 - sr];
    if (rec.w >= pix_total) continue;   // every place is filled; never taken
    const uint64_t own = ((uint64_t)rec.y << 32) | rec.x;
    const uint32_t start = poff[rec.w], n = poff[rec.w + 1] - start;
    uint32_t rank = 0;
    if (ids) {
      // keys in groups of kRankBatch, every group's loads in flight before
      // the comparisons; equal depth keys (rare) are settled after the
      // group by the original indices, so no index load sits between the
      // key loads and their use
      const uint32_t own_id = ids[rec.x];
      constexpr int kRankBatch = 8;
      for (uint32_t j0 = 0; j0 < n; j0 += kRankBatch) {
        uint64_t kk[kRankBatch];
#pragma unroll
        for (int q = 0; q < kRankBatch; ++q)
          kk[q] = j0 + q < n ? key[2 * (int64_t)(start + j0 + q)] : 0ull;
        uint32_t ties = 0;
#pragma unroll
        for (int q = 0; q < kRankBatch; ++q) {
          if (j0 + q >= n) continue;
          const uint32_t kd = (uint32_t)(kk[q] >> 32);
          rank += kd < rec.y ? 1u : 0u;
          if (kd == rec.y && kk[q] != own) ties |= 1u << q;
        }
        while (ties) {
          const int q = __builtin_ctz(ties);
          ties &= ties - 1;
          rank += ids[(uint32_t)kk[q]] < own_id ? 1u : 0u;
        }
      }
    } else {
#pragma unroll 8
      for (uint32_t j = 0; j < n; ++j) rank += key[2 * (int64_t)(start + j)] < own ? 1u : 0u;
    }
    okey[start + rank] = rec.w;
    oval[start + rank] = ((uint64_t)rec.z << 32) | rec.x;
  }
}

// ----------------------------------------------------------------- blend
// One thread per layer pixel: its list front to back (zero where empty).
// Pixels go in reverse pyramid order: each crop's coarse layers (the long
// lists) come after its finest layer in the pyramid, so in reverse the
// long lists start early and the finest layers' short lists fill the end.
__global__ __launch_bounds__(256) void k_pt_blend(const uint64_t* __restrict__ fval,
                                                  const uint32_t* __restrict__ poff,
                                                  const uint32_t* __restrict__ total_p,
                                                  int64_t max_frags,
                                                  const uint16_t* __restrict__ feat,
                                                  const float* __restrict__ opacity, int64_t np,
                                                  int64_t pix_total, float4* __restrict__ pyr) {
  const bool over = (int64_t)*total_p > max_frags;
  for (int64_t kr = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; kr < pix_total;
       kr += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = pix_total - 1 - kr;
    float T = 1.0f;
    float4 F = make_float4(0, 0, 0, 0);
    const uint32_t start = over ? 0u : poff[k], n = over ? 0u : poff[k + 1] - start;
    // fragments in groups of kPtBatch, every group's loads in flight before
    // its (sequential) compositing: long lists are otherwise one load
    // latency per fragment
    constexpr int kPtBatch = 8;
    for (uint32_t j0 = 0; j0 < n; j0 += kPtBatch) {
      uint64_t vv[kPtBatch];
      float op[kPtBatch];
      uint2 hb[kPtBatch];
#pragma unroll
      for (int q = 0; q < kPtBatch; ++q)
        vv[q] = j0 + q < n ? fval[start + j0 + q] : ~0ull;
#pragma unroll
      for (int q = 0; q < kPtBatch; ++q) {
        const uint32_t id = (uint32_t)vv[q];
        const bool ok = id < (uint64_t)np;
        op[q] = ok && opacity ? opacity[id] : 1.0f;
        hb[q] = ok ? *reinterpret_cast<const uint2*>(feat + (int64_t)id * 4) : make_uint2(0, 0);
      }
#pragma unroll
      for (int q = 0; q < kPtBatch; ++q) {
        if (j0 + q >= n || (uint32_t)vv[q] >= (uint64_t)np) continue;
        const float w = __uint_as_float((uint32_t)(vv[q] >> 32));
        const float al = opacity ? w * op[q] : w;
        const float aT = al * T;
        F.x += h2f((uint16_t)(hb[q].x & 0xffffu)) * aT;
        F.y += h2f((uint16_t)(hb[q].x >> 16)) * aT;
        F.z += h2f((uint16_t)(hb[q].y & 0xffffu)) * aT;
        F.w += h2f((uint16_t)(hb[q].y >> 16)) * aT;
        T = T * (1.0f - al);
      }
    }
    pyr[k] = F;
  }
}

__global__ void k_zero4(float4* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

}  // namespace vrs

using namespace vrs;

static bool check_views(const vrs_view* views, int nv, KViews* kv) {
  if (!make_views(views, nv, kv)) return false;
  for (int i = 1; i < nv; ++i)
    if (views[i].width != views[0].width || views[i].height != views[0].height) return false;
  return true;
}

extern "C" size_t vrs_splat_workspace_size(int64_t np, int n_views, const vrs_view* views,
                                           const vrs_crop* crops, int n_crops, int levels,
                                           int64_t max_frags) {
  SplatWs L;
  KViews kv;
  KCrops kc;
  if (!check_views(views, n_views, &kv) ||
      !make_crops(crops, n_crops, levels, kv, &kc, nullptr, false))
    return 0;
  if (!splat_layout_for(np, n_views, views, crops, n_crops, levels, max_frags, &L)) return 0;
  return L.total;
}

extern "C" vrs_status vrs_splat_workspace_layout(int64_t np, int n_views, const vrs_view* views,
                                                 const vrs_crop* crops, int n_crops, int levels,
                                                 int64_t max_frags, vrs_splat_layout* out) {
  SplatWs L;
  if (!out || !splat_layout_for(np, n_views, views, crops, n_crops, levels, max_frags, &L))
    return VRS_EINVAL;
  out->frag_count = L.frag_count;
  out->sorted_keys = L.fkey1;
  out->sorted_ids = L.fval1;   // low 32 bits of each 64-bit value
  out->pyramid_pixels = L.pix_total;
  return VRS_OK;
}

namespace vrs {
vrs_status splat_impl(const float* pos, const float* radius, const uint16_t* feat,
                      const float* opacity, int64_t np, int channels, int levels,
                      const vrs_view* views, int n_views, const vrs_crop* crops, int n_crops,
                      const vrs_crop_place* place, const float* depth, const float* t_final,
                      float cov_min, float slack, const uint32_t* point_ids, float* pyramid,
                      void* ws, size_t ws_bytes, int64_t max_frags, int32_t* dev_status,
                      void* stream, const Trace* tr, const float* gaze) {
  KViews kv;
  KCrops kc;
  SplatWs L;
  if (gaze && !place) return VRS_EINVAL;
  if (channels != 4) return channels > 0 ? VRS_EUNSUPPORTED : VRS_EINVAL;
  if (!check_views(views, n_views, &kv) || !make_crops(crops, n_crops, levels, kv, &kc, place))
    return VRS_EINVAL;
  if (np < 0 || np * n_views >= (int64_t(1) << 30) ||
      (np > 0 && (!pos || !radius || !feat)))
    return VRS_EINVAL;
  if ((depth == nullptr) != (t_final == nullptr)) return VRS_EINVAL;
  if (!pyramid || !ws || max_frags < 0 || max_frags >= (int64_t(1) << 30)) return VRS_EINVAL;
  if (!splat_layout_for(np, n_views, views, crops, n_crops, levels, max_frags, &L) || ws_bytes < L.total)
    return VRS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  PtArgs a;
  a.cov_min = cov_min;
  a.slack = slack;
  a.levels = levels;
  a.view_mask = 0;
  for (int k = 0; k < n_crops; ++k) a.view_mask |= 1u << crops[k].view;
  const int64_t vn = L.vn;
  uint32_t* frag_count = at<uint32_t>(ws, L.frag_count);
  trace_begin(tr, VRS_TRACE_SPLAT, st);
  if (vn == 0 || n_crops == 0) {
    if (gaze && n_crops > 0) {   // the crops are still placed for the later stages
      hipLaunchKernelGGL(k_place_crops, dim3(1), dim3(64), 0, st,
                         reinterpret_cast<const float2*>(gaze), kc,
                         reinterpret_cast<int4*>(const_cast<vrs_crop_place*>(place)));
      VRS_LAUNCH_CHECK();
    }
    if (L.pix_total > 0) {
      const int blocks = (int)std::min<int64_t>(4096, div_up(L.pix_total, 256));
      hipLaunchKernelGGL(k_zero4, dim3(blocks), dim3(256), 0, st,
                         reinterpret_cast<float4*>(pyramid), L.pix_total);
      VRS_LAUNCH_CHECK();
    }
    VRS_HIP_CHECK(fill_u32(frag_count, 0, 1, st));
    trace_end(tr, VRS_TRACE_SPLAT, st);
    return VRS_OK;
  }
  uint32_t* live = at<uint32_t>(ws, L.live);
  const int sel_parts = div_up(np, kSelPart);
  const size_t sel_lds = (size_t)kSelRounds * n_views * kSelBlock * 8;
  uint32_t* grid = at<uint32_t>(ws, L.grid);
  {
    const int64_t cells = (int64_t)n_views * L.gx * L.gy;
    const int64_t scan_words = (int64_t)(scan_tmp_bytes(L.pix_total) / 4);
    const int64_t most = std::max(std::max<int64_t>(L.pix_total, scan_words), cells);
    hipLaunchKernelGGL(k_pt_prep, dim3((unsigned)std::min<int64_t>(4096, div_up(most, 256))),
                       dim3(256), 0, st, at<uint32_t>(ws, L.pcnt), L.pix_total,
                       at<uint64_t>(ws, L.ctr), at<uint32_t>(ws, L.scan_tmp), scan_words, kc,
                       n_views, levels, L.gx, L.gy, grid, reinterpret_cast<const float2*>(gaze),
                       reinterpret_cast<int4*>(const_cast<vrs_crop_place*>(place)));
    VRS_LAUNCH_CHECK();
  }
  // survivors with their fragment offsets (compaction order), then emission
  hipLaunchKernelGGL(k_pt_select, dim3(sel_parts), dim3(kSelBlock), sel_lds, st, pos, radius, np, kv,
                     kc, a, depth, t_final, grid, L.gx, L.gy, at<uint4>(ws, L.surv),
                     at<uint64_t>(ws, L.ctr), at<uint32_t>(ws, L.chunk_first), max_frags,
                     dev_status);
  VRS_LAUNCH_CHECK();
  uint32_t* pcnt = at<uint32_t>(ws, L.pcnt);
  uint32_t* poff = at<uint32_t>(ws, L.poff);
  // one workgroup per chunk of the capacity's fragment range (grid-stride
  // beyond 8192 chunks); workgroups past the counted chunks leave at once
  const int64_t emit_blocks =
      std::min<int64_t>(8192, std::max<int64_t>(1, div_up(max_frags, kEmitFrags)));
  hipLaunchKernelGGL(k_pt_emit, dim3((unsigned)emit_blocks), dim3(kEmitBlock), 0, st, pos, radius,
                     np, kv, kc, a, at<uint4>(ws, L.surv), live, at<uint32_t>(ws, L.chunk_first),
                     frag_count, max_frags, at<uint32_t>(ws, L.fkey0), at<uint64_t>(ws, L.fval0),
                     at<uint32_t>(ws, L.fdep), at<uint32_t>(ws, L.fslot), pcnt, grid, L.gx, L.gy,
                     dev_status);
  VRS_LAUNCH_CHECK();
  // per-pixel segments, then each fragment to its place in blend order
  VRS_HIP_CHECK(exclusive_scan_u32(pcnt, nullptr, poff, poff + L.pix_total, nullptr, L.pix_total,
                                   at<void>(ws, L.scan_tmp), dev_status, st, true));
  const unsigned fb = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, div_up(max_frags, 256)));
  hipLaunchKernelGGL(k_pt_scatter, dim3(fb), dim3(256), 0, st, at<uint32_t>(ws, L.fkey0),
                     at<uint64_t>(ws, L.fval0), at<uint32_t>(ws, L.fdep),
                     at<uint32_t>(ws, L.fslot), poff, frag_count, max_frags,
                     at<uint4>(ws, L.seg));
  VRS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_pt_rank, dim3(fb), dim3(256), 0, st, at<uint4>(ws, L.seg), poff,
                     frag_count, max_frags, L.pix_total, point_ids, at<uint32_t>(ws, L.fkey1),
                     at<uint64_t>(ws, L.fval1));
  VRS_LAUNCH_CHECK();
  const unsigned pb = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, div_up(L.pix_total, 256)));
  hipLaunchKernelGGL(k_pt_blend, dim3(pb), dim3(256), 0, st, at<uint64_t>(ws, L.fval1), poff,
                     frag_count, max_frags, feat, opacity, np, L.pix_total,
                     reinterpret_cast<float4*>(pyramid));
  VRS_LAUNCH_CHECK();
  trace_end(tr, VRS_TRACE_SPLAT, st);
  return VRS_OK;
}
}  // namespace vrs

extern "C" vrs_status vrs_splat_points(const float* pos, const float* radius,
                                       const uint16_t* feat, const float* opacity, int64_t np,
                                       int channels, int levels, const vrs_view* views,
                                       int n_views, const vrs_crop* crops, int n_crops,
                                       const vrs_crop_place* place, const float* depth,
                                       const float* t_final, float cov_min, float slack,
                                       const uint32_t* point_ids, float* pyramid, void* ws,
                                       size_t ws_bytes, int64_t max_frags, int32_t* dev_status,
                                       void* stream) {
  return splat_impl(pos, radius, feat, opacity, np, channels, levels, views, n_views, crops,
                    n_crops, place, depth, t_final, cov_min, slack, point_ids, pyramid, ws,
                    ws_bytes, max_frags, dev_status, stream, nullptr);
}

// ------------------------------------------------------------- backward
namespace vrs {

// Segment heads replay their pixel's list: a forward walk finds the final
// transmittance (and the first fully opaque fragment, after which nothing is
// visible), then a backward walk recovers T before each fragment as
// T / (1 - alpha) and accumulates
//   dfeat = alpha T dF,  dalpha = T (feat - acc) . dF,  acc = feat alpha + (1 - alpha) acc
// Fragment weights are recomputed from the point to carry dalpha into the
// position and radius (trilinear weight = layer weight x bilinear weight).
__global__ __launch_bounds__(256) void k_pt_blend_bwd(
    const uint32_t* __restrict__ fkey, const uint64_t* __restrict__ fval,
    const uint32_t* __restrict__ total_p, int64_t max_frags, const float* __restrict__ pos,
    const float* __restrict__ radius, const uint16_t* __restrict__ feat,
    const float* __restrict__ opacity, int64_t np, KViews views, KCrops crops, PtArgs a,
    int64_t pix_total, const float4* __restrict__ dpyr, float* __restrict__ d_feat,
    float* __restrict__ d_pos, float* __restrict__ d_radius, float* __restrict__ d_opacity) {
  const int64_t cnt = std::min<int64_t>(*total_p, max_frags);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t key = fkey[i];
    if (i > 0 && fkey[i - 1] == key) continue;
    if (key >= (uint64_t)pix_total) continue;
    const float4 g = dpyr[key];
    // locate crop, layer and pixel of this key
    int k = 0;
    while (k + 1 < crops.n && (int)key >= crops.c[k + 1].pix_base) ++k;
    const KCrop& c = crops.c[k];
    int l = 0, lb = c.pix_base;
    while (l + 1 < a.levels && (int)key >= lb + (c.size >> l) * (c.size >> l)) {
      lb += (c.size >> l) * (c.size >> l);
      ++l;
    }
    const int Sl = c.size >> l;
    const int xx = ((int)key - lb) % Sl, yy = ((int)key - lb) / Sl;
    // forward walk
    int64_t j = i, jend = i;
    float T = 1.0f;
    while (jend < cnt && fkey[jend] == key) {
      const uint64_t vv = fval[jend];
      const uint32_t id = (uint32_t)vv;
      const float w = __uint_as_float((uint32_t)(vv >> 32));
      const float al = opacity && id < (uint64_t)np ? w * opacity[id] : w;
      ++jend;
      if (al >= 1.0f) { T = 0.0f; break; }   // fully opaque: nothing behind is visible
      T = T * (1.0f - al);
    }
    // backward walk over [i, jend)
    float acc[4] = {0, 0, 0, 0};
    bool opaque_end = T == 0.0f;
    for (j = jend - 1; j >= i; --j) {
      const uint64_t vv = fval[j];
      const uint32_t id = (uint32_t)vv;
      if (id >= (uint64_t)np) continue;
      const float w = __uint_as_float((uint32_t)(vv >> 32));
      const float o = opacity ? opacity[id] : 1.0f;
      const float al = w * o;
      float Tb;
      if ((opaque_end && j == jend - 1) || !(1.0f - al >= 0.5f)) {
        // T before an opaque or nearly opaque fragment: the product of the
        // ones in front (dividing by a small 1 - alpha would amplify error)
        Tb = 1.0f;
        for (int64_t q = i; q < j; ++q) {
          const uint64_t u = fval[q];
          const uint32_t iq = (uint32_t)u;
          const float wq = __uint_as_float((uint32_t)(u >> 32));
          Tb *= 1.0f - (opacity && iq < (uint64_t)np ? wq * opacity[iq] : wq);
        }
      } else {
        Tb = T / (1.0f - al);
      }
      const uint2 hb = *reinterpret_cast<const uint2*>(feat + (int64_t)id * 4);
      const float f[4] = {h2f((uint16_t)(hb.x & 0xffffu)), h2f((uint16_t)(hb.x >> 16)),
                          h2f((uint16_t)(hb.y & 0xffffu)), h2f((uint16_t)(hb.y >> 16))};
      const float gg[4] = {g.x, g.y, g.z, g.w};
      float dal = 0.0f;
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        if (d_feat) atomicAdd(&d_feat[(int64_t)id * 4 + ch], al * Tb * gg[ch]);
        dal += Tb * (f[ch] - acc[ch]) * gg[ch];
        acc[ch] = f[ch] * al + (1.0f - al) * acc[ch];
      }
      T = Tb;
      if (d_opacity && opacity) atomicAdd(&d_opacity[id], dal * w);
      const float dw = dal * o;
      if ((d_pos || d_radius) && dw != 0.0f) {
        const KView& cv = views.v[c.view];
        PtGeom pg;
        if (!pt_geom32(cv, pos[id], pos[np + id], pos[2 * np + id], radius[id], a.levels, pg))
          continue;
        float xl, yl;
        int ix, iy;
        const int cx0 = crop_x0(crops, k), cy0 = crop_y0(crops, k);
        if (!pt_layer32(pg, cx0, cy0, l, Sl, xl, yl, ix, iy)) continue;
        FF ux, uy;
        pt_plane_ff(cv, pos[id], pos[np + id], pos[2 * np + id], ux, uy);
        const float bx = pt_frac_ff(cv.fx, ux, cv.cx, cx0, l, ix);
        const float by = pt_frac_ff(cv.fy, uy, cv.cy, cy0, l, iy);
        const int dx = xx - ix, dy = yy - iy;
        const float wx = dx ? bx : 1.0f - bx, wy = dy ? by : 1.0f - by;
        float f2 = 0.0f, wl = 1.0f;
        if (pg.two) {
          f2 = log2f(pg.s) - (float)pg.l0;
          wl = l == pg.l0 ? 1.0f - f2 : f2;
        }
        const float dwl = dw * wx * wy;
        const float sc = ldexpf(1.0f, -l);
        const float dpx = dw * wl * wy * (dx ? 1.0f : -1.0f) * sc;
        const float dpy = dw * wl * wx * (dy ? 1.0f : -1.0f) * sc;
        float ds = 0.0f;
        if (pg.two) ds = (l == pg.l0 ? -dwl : dwl) / (pg.s * 0.69314718055994531f);
        const float tz = pg.t[2];
        const float dr = ds * 2.0f * cv.fx / tz;
        float dt0 = dpx * cv.fx / tz, dt1 = dpy * cv.fy / tz;
        float dt2 = -dpx * cv.fx * pg.t[0] / (tz * tz) - dpy * cv.fy * pg.t[1] / (tz * tz) -
                    ds * pg.s / tz;
        if (d_radius) atomicAdd(&d_radius[id], dr);
        if (d_pos)
#pragma unroll
          for (int q = 0; q < 3; ++q)
            atomicAdd(&d_pos[q * np + id], cv.R[q] * dt0 + cv.R[3 + q] * dt1 + cv.R[6 + q] * dt2);
      }
    }
  }
}

}  // namespace vrs

extern "C" vrs_status vrs_splat_points_backward(const float* pos, const float* radius,
                                                const uint16_t* feat, const float* opacity,
                                                int64_t np, int channels, int levels,
                                                const vrs_view* views, int n_views,
                                                const vrs_crop* crops, int n_crops,
                                                const vrs_crop_place* place,
                                                const float* d_pyramid, float* d_feat,
                                                float* d_pos, float* d_radius, float* d_opacity,
                                                void* ws, size_t ws_bytes, int64_t max_frags,
                                                void* stream) {
  KViews kv;
  KCrops kc;
  SplatWs L;
  if (channels != 4) return channels > 0 ? VRS_EUNSUPPORTED : VRS_EINVAL;
  if (!check_views(views, n_views, &kv) || !make_crops(crops, n_crops, levels, kv, &kc, place))
    return VRS_EINVAL;
  if (!splat_layout_for(np, n_views, views, crops, n_crops, levels, max_frags, &L) || !ws ||
      ws_bytes < L.total || !d_pyramid)
    return VRS_EINVAL;
  if (np > 0 && (!pos || !radius || !feat)) return VRS_EINVAL;
  if (np == 0 || n_crops == 0) return VRS_OK;
  PtArgs a;
  a.cov_min = 0.5f;
  a.slack = 1.05f;
  a.levels = levels;
  a.view_mask = 0;
  for (int k = 0; k < n_crops; ++k) a.view_mask |= 1u << crops[k].view;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int bb = (int)std::min<int64_t>(8192, std::max(1, div_up(max_frags, 256)));
  hipLaunchKernelGGL(k_pt_blend_bwd, dim3(bb), dim3(256), 0, st,
                     at<uint32_t>(ws, L.fkey1), at<uint64_t>(ws, L.fval1),
                     at<uint32_t>(ws, L.frag_count), max_frags, pos, radius, feat, opacity, np, kv,
                     kc, a, L.pix_total, reinterpret_cast<const float4*>(d_pyramid), d_feat, d_pos,
                     d_radius, d_opacity);
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}

// ------------------------------------------------------- crop placement

extern "C" vrs_status vrs_place_crops(const float* gaze, const vrs_view* views, int n_views,
                                      const vrs_crop* crops, int n_crops, vrs_crop_place* place,
                                      void* stream) {
  KViews kv;
  KCrops kc;
  if (!gaze || !place || n_crops < 1 || !check_views(views, n_views, &kv) ||
      !make_crops(crops, n_crops, 1, kv, &kc, nullptr, false))
    return VRS_EINVAL;
  hipLaunchKernelGGL(k_place_crops, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const float2*>(gaze), kc, reinterpret_cast<int4*>(place));
  VRS_LAUNCH_CHECK();
  return VRS_OK;
}
