// Workspace layout of the periphery (shared by its forward and backward).
#pragma once
#include "gs_device.h"

namespace vrs {

// ---------------------------------------------------------------- layout
struct RenderWs {
  size_t rec, dkey0, dval0, dkey1, dval1, ntiles, offs, pair_count, pkey0, pval0, pkey1, pval1,
      okey0, oval0, okey1, oval1,   // tile schedule (length bucket, tile), sorted once
      ranges, last, evals, g2d, sort_tmp, scan_tmp, total;
  int64_t vn, tiles_x, tiles_y, tiles_total, npix;
  int tile_bits;
  bool pairs_in_1;
};

inline int bits_for(int64_t n) {
  int b = 1;
  while (b < 32 && (int64_t(1) << b) < n) ++b;
  return b;
}

inline bool render_layout(int64_t n, int nv, const vrs_view* views, int tile, int64_t max_pairs,
                          RenderWs* L) {
  if (n < 0 || nv < 1 || nv > VRS_MAX_VIEWS || !views || max_pairs < 0) return false;
  if (tile != 8 && tile != 16 && tile != 32) return false;
  const int W = views[0].width, H = views[0].height;
  L->vn = n * nv;
  L->tiles_x = (W + tile - 1) / tile;
  L->tiles_y = (H + tile - 1) / tile;
  L->tiles_total = L->tiles_x * L->tiles_y * nv;
  L->npix = (int64_t)W * H * nv;
  L->tile_bits = bits_for(L->tiles_total);
  const int tile_passes = (L->tile_bits + 7) / 8;
  L->pairs_in_1 = (tile_passes & 1) != 0;
  const int64_t vn = std::max<int64_t>(L->vn, 1);
  const int64_t mp = std::max<int64_t>(max_pairs, 1);
  Carver c;
  L->rec = c.take((size_t)vn * 48);
  L->dkey0 = c.take(vn * 4);
  L->dval0 = c.take(vn * 4);
  L->dkey1 = c.take(vn * 4);
  L->dval1 = c.take(vn * 4);
  L->ntiles = c.take(vn * 4);
  L->offs = c.take(vn * 4);
  L->pair_count = c.take(4);
  L->pkey0 = c.take(mp * 4);
  L->pval0 = c.take(mp * 4);
  L->pkey1 = c.take(mp * 4);
  L->pval1 = c.take(mp * 4);
  L->ranges = c.take((size_t)L->tiles_total * 8);
  L->okey0 = c.take((size_t)L->tiles_total * 4);
  L->oval0 = c.take((size_t)L->tiles_total * 4);
  L->okey1 = c.take((size_t)L->tiles_total * 4);
  L->oval1 = c.take((size_t)L->tiles_total * 4);
  L->last = c.take((size_t)std::max<int64_t>(L->npix, 1) * 4);
  L->evals = c.take((size_t)std::max<int64_t>(L->npix, 1) * 4);
  L->g2d = c.take((size_t)vn * 10 * 4);   // per (view, Gaussian) screen-space gradients
  L->sort_tmp = c.take(std::max(std::max(sort_tmp_bytes(vn, 32), sort_tmp_bytes(mp, L->tile_bits)),
                                sort_tmp_bytes(L->tiles_total, 8)));
  L->scan_tmp = c.take(scan_tmp_bytes(vn));
  L->total = c.off;
  return true;
}

}  // namespace vrs
