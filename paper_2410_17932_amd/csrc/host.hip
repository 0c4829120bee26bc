// Host-side helpers of the C-ABI: descriptor conversion and status strings.
#include <cmath>

#include "vrs_common.h"

namespace vrs {

bool make_views(const vrs_view* views, int n, KViews* out) {
  if (!views || n < 1 || n > VRS_MAX_VIEWS) return false;
  out->n = n;
  for (int i = 0; i < n; ++i) {
    const vrs_view& s = views[i];
    KView& d = out->v[i];
    if (s.width <= 0 || s.height <= 0 || s.width > 65535 || s.height > 65535) return false;
    if (!(s.fx > 0) || !(s.fy > 0)) return false;
    d.fx = s.fx; d.fy = s.fy; d.cx = s.cx; d.cy = s.cy;
    for (int k = 0; k < 9; ++k) d.R[k] = s.rot[k];
    for (int k = 0; k < 3; ++k) d.t[k] = s.trans[k];
    d.znear = s.znear;
    d.W = s.width; d.H = s.height;
    // camera centre o = -R^T t (double precision, rounded once)
    for (int k = 0; k < 3; ++k) {
      double acc = 0;
      for (int j = 0; j < 3; ++j) acc -= (double)s.rot[3 * j + k] * (double)s.trans[j];
      d.cam[k] = (float)acc;
    }
  }
  return true;
}

}  // namespace vrs

extern "C" const char* vrs_status_string(vrs_status s) {
  switch (s) {
    case VRS_OK: return "ok";
    case VRS_EINVAL: return "invalid argument";
    case VRS_ECAPACITY: return "workspace capacity exceeded";
    case VRS_EHIP: return "HIP runtime error";
    case VRS_EUNSUPPORTED: return "unsupported configuration";
    case VRS_ETIMEOUT: return "device-side wait expired";
  }
  return "unknown status";
}

extern "C" const char* vrs_version(void) { return "vrsplat 0.1 gfx950"; }
