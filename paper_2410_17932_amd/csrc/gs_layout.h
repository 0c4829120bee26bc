// Workspace layout of the periphery (shared by its forward and backward).
#pragma once
#include "gs_device.h"

namespace vrs {

// ---------------------------------------------------------------- layout
// Tiles are grouped in super-tiles of kSuper x kSuper tiles (one tile per
// lane of a wave) for binning.
constexpr int kSuper = 8;
// Tile schedule words: [0, 256) length-bucket histogram, 256 the count of
// finished prefix workgroups (both zeroed before the binning), [320, 576)
// the bucket cursors.
constexpr int kSchedHist = 0, kSchedDone = 256, kSchedCursor = 320, kSchedWords = 576;

struct RenderWs {
  size_t rec, rect, dkey0, dval0, dkey1, dval1, nsup, nsorted, soffs, psum, pair_count, super_count,
      skey0, sval0, skey1, sval1,   // (super-tile, Gaussian) pairs
      srange, ubase, nunits,        // per super-tile run and first work unit
      ucnt, tcnt, toff,             // per (unit, tile) and per tile counts, tile offsets
      ids,                          // tile lists (Gaussian indices), super-tile order
      order,                        // tile schedule: tile ids, longest list first
      ranges, last, evals, g2d, sort_tmp, scan_tmp,
      sched,                        // length-bucket histogram, done count, bucket cursors
      stot, sbase,                  // per super-tile: tile pairs, list base
      pcoef, fix_list, fix_count,   // per-pixel order: key coefficients, exact-pass queue
      tkey,                         // per-pixel order: tile-list bound words
      total;
  int64_t vn, tiles_x, tiles_y, tiles_total, npix, sxn, syn, spv, st_total;
  int st_bits;
  int radix;   // digit width of the sorts
};

inline int bits_for(int64_t n) {
  int b = 1;
  while (b < 32 && (int64_t(1) << b) < n) ++b;
  return b;
}

// Binning work unit: up to kBinUnit consecutive pairs of one super-tile's
// run (one wave, kBinUnit / 64 rounds of one pair per lane).
constexpr int kBinUnit = 256;
inline int64_t bin_units_max(int64_t max_pairs, int64_t st_total) {
  return (std::max<int64_t>(max_pairs, 1) + kBinUnit - 1) / kBinUnit + st_total;
}

// Digit width of the periphery's radix sorts from the options (0: 8 bits).
inline int opts_radix(const vrs_raster_opts* o) { return o->radix_bits == 0 ? 8 : o->radix_bits; }

inline bool render_layout(int64_t n, int nv, const vrs_view* views, int tile, int radix,
                          int64_t max_pairs, RenderWs* L, int order = VRS_ORDER_PRIMITIVE) {
  if (order != VRS_ORDER_PRIMITIVE && order != VRS_ORDER_PIXEL) return false;
  if (n < 0 || nv < 1 || nv > VRS_MAX_VIEWS || !views || max_pairs < 0) return false;
  if (tile != 8 && tile != 16 && tile != 32) return false;
  if (!radix_bits_ok(radix)) return false;
  L->radix = radix;
  const int W = views[0].width, H = views[0].height;
  L->vn = n * nv;
  L->tiles_x = (W + tile - 1) / tile;
  L->tiles_y = (H + tile - 1) / tile;
  L->tiles_total = L->tiles_x * L->tiles_y * nv;
  L->npix = (int64_t)W * H * nv;
  L->sxn = (L->tiles_x + kSuper - 1) / kSuper;
  L->syn = (L->tiles_y + kSuper - 1) / kSuper;
  L->spv = L->sxn * L->syn;
  L->st_total = L->spv * nv;
  L->st_bits = bits_for(L->st_total);
  const int64_t vn = std::max<int64_t>(L->vn, 1);
  const int64_t mp = std::max<int64_t>(max_pairs, 1);
  Carver c;
  L->rec = c.take((size_t)vn * 48);
  L->rect = c.take((size_t)vn * 8);   // per (view, Gaussian): its rectangle alone (record word 2.zw)
  L->dkey0 = c.take(vn * 4);
  L->dval0 = c.take(vn * 4);
  L->dkey1 = c.take(vn * 4);
  L->dval1 = c.take(vn * 4);
  L->nsup = c.take(vn * 4);
  L->nsorted = c.take(vn * 4);   // nsup in depth order
  L->soffs = c.take(vn * 4);
  L->psum = c.take((size_t)(vn + 255) / 256 * 8);   // per preprocess block: tile pairs
  L->pair_count = c.take(4);
  L->super_count = c.take(4);
  L->skey0 = c.take(mp * 4);
  L->sval0 = c.take(mp * 8);
  L->skey1 = c.take(mp * 4);
  L->sval1 = c.take(mp * 8);
  L->srange = c.take((size_t)L->st_total * 8);
  L->ubase = c.take((size_t)(L->st_total + 1) * 4);
  L->nunits = c.take(4);
  L->ucnt = c.take((size_t)bin_units_max(mp, L->st_total) * 64 * 4);
  L->tcnt = c.take((size_t)L->tiles_total * 4);
  L->toff = c.take((size_t)L->tiles_total * 4);
  L->ids = c.take(mp * 4);
  L->ranges = c.take((size_t)L->tiles_total * 8);
  L->order = c.take((size_t)L->tiles_total * 4);
  L->last = c.take((size_t)std::max<int64_t>(L->npix, 1) * 4);
  L->evals = c.take((size_t)std::max<int64_t>(L->npix, 1) * 4);
  L->g2d = c.take((size_t)vn * 10 * 4);   // per (view, Gaussian) screen-space gradients
  L->sort_tmp = c.take(std::max(sort_tmp_bytes(vn, 32, radix), sort_tmp_bytes(mp, L->st_bits, radix)));
  L->scan_tmp = c.take(std::max(scan_tmp_bytes(vn), scan_tmp_bytes(L->tiles_total)));
  L->sched = c.take((size_t)kSchedWords * 4);   // follows scan_tmp: cleared together
  L->stot = c.take((size_t)L->st_total * 4);
  L->sbase = c.take((size_t)L->st_total * 4);
  L->pcoef = L->fix_list = L->fix_count = L->tkey = 0;
  if (order == VRS_ORDER_PIXEL) {
    // the tile lists' bound words (64-bit): the pair sort's value buffer,
    // free once the binning has scattered it
    L->tkey = L->sval0;
    L->pcoef = c.take((size_t)vn * 48);
    L->fix_list = c.take((size_t)std::max<int64_t>(L->npix, 1) * 4);
    L->fix_count = c.take(4);
  }
  L->total = c.off;
  return true;
}

// Per-pixel order (gs_pixel.hip): key coefficients and sort keys after the
// preprocess, the tile lists sorted by per-tile bound after the binning, and
// the blend with its exact pass for unresolved pixels.
void launch_gs_pixdepth(const RenderWs& L, void* ws, const float* mean, const float* cov,
                        int64_t n, const KViews& kv, hipStream_t st);
void launch_gs_tile_zsort(const RenderWs& L, void* ws, int64_t n, const KViews& kv, int tile,
                         hipStream_t st);
void launch_gs_blend_px(const RenderWs& L, void* ws, int64_t n, const uint32_t* order,
                        const KViews& kv, const GsOpt& o, float* rgb, float* depth, float* tf,
                        int32_t* nc, hipStream_t st);

// The blend kernel of the tile size in o.tile (stats: also the adjoint's
// last positions and the evaluation counts), gs_blend.hip.
void launch_gs_blend(bool stats, const RenderWs& L, void* ws, int64_t n, const uint32_t* order,
                     const KViews& kv, const GsOpt& o, float* rgb, float* depth, float* tf,
                     int32_t* nc, hipStream_t st);

}  // namespace vrs
