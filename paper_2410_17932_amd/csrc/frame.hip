// Per-frame runtime of the foveated renderer (Fig. 5 of the paper): the
// plan object holding everything fixed across frames (views, crop sizes,
// the autotuned tile size and sort radix, capacities, decoder shape,
// combination mode) and vrs_render_frame, which enqueues one whole frame:
// periphery with Eq. 1 depth (Sec. 3.2) -> crops placed from the gaze read
// on the device after the periphery (Sec. 4 "Inference") -> depth-culled
// point splat (Sec. 3.3) -> decoder -> combination in place (Sec. 3.4).
// Host code only: every stage is one of the library's entry points, the
// frame adds no kernel of its own.  Nothing synchronises the host, so the
// call is capturable into one HIP graph; a new gaze is a new device-buffer
// content, not a new graph.
#include <new>
#include <vector>

#include "vrs_common.h"

struct vrs_plan {
  vrs_plan_desc d;   // pointer fields point into the vectors below
  std::vector<vrs_view> views;
  std::vector<vrs_crop> crops;
  vrs::Trace trace;
  size_t ws[3];
};

namespace {

bool decoder_ok(const vrs_decoder_desc& dd, int levels) {
  return dd.n_levels >= 1 && dd.n_levels <= levels && dd.in_ch == 4 &&
         (dd.dtype == VRS_F32 || dd.dtype == VRS_BF16);
}

}  // namespace

extern "C" vrs_status vrs_plan_create(const vrs_plan_desc* desc, vrs_plan** out) {
  if (!desc || !out) return VRS_EINVAL;
  *out = nullptr;
  const vrs_plan_desc& d = *desc;
  if (d.n_views < 1 || d.n_views > VRS_MAX_VIEWS || !d.views) return VRS_EINVAL;
  if (d.n_crops < 0 || d.n_crops > VRS_MAX_CROPS || (d.n_crops > 0 && !d.crops))
    return VRS_EINVAL;
  if (d.n_gaussians < 0 || d.n_points < 0 || d.sh_degree < 0 || d.sh_degree > 3)
    return VRS_EINVAL;
  if (d.levels < 1 || d.levels > VRS_MAX_LEVELS || !decoder_ok(d.decoder, d.levels))
    return VRS_EINVAL;
  if (d.point_channels != 4) return VRS_EUNSUPPORTED;
  if (d.max_pairs < 0 || d.max_frags < 0) return VRS_EINVAL;
  if (d.blend_mode != VRS_BLEND_LINEAR && d.blend_mode != VRS_BLEND_PAPER) return VRS_EINVAL;
  vrs_plan* p = new (std::nothrow) vrs_plan();
  if (!p) return VRS_EINVAL;
  p->d = d;
  p->views.assign(d.views, d.views + d.n_views);
  if (d.n_crops > 0) p->crops.assign(d.crops, d.crops + d.n_crops);
  p->d.views = p->views.data();
  p->d.crops = p->crops.data();
  for (int s = 0; s < vrs::kTraceStages; ++s) p->trace.start[s] = p->trace.stop[s] = nullptr;
  // every size query validates its part of the plan (views, tile and sort
  // radix, crop sizes against the views and the pyramid depth, decoder)
  p->ws[VRS_WS_RENDER] = vrs_render_workspace_size(d.n_gaussians, d.n_views, p->d.views,
                                                   &d.raster, d.max_pairs);
  // (a plan without crops renders the periphery alone: no foveal workspaces)
  const bool fovea = d.n_crops > 0;
  p->ws[VRS_WS_SPLAT] = fovea ? vrs_splat_workspace_size(d.n_points, d.n_views, p->d.views,
                                                         p->d.crops, d.n_crops, d.levels,
                                                         d.max_frags)
                              : 0;
  p->ws[VRS_WS_DECODER] = fovea ? vrs_decoder_workspace_size(&d.decoder, p->d.crops, d.n_crops)
                                : 0;
  if (!p->ws[0] || (fovea && (!p->ws[1] || !p->ws[2]))) {
    delete p;
    return VRS_EINVAL;
  }
  *out = p;
  return VRS_OK;
}

extern "C" void vrs_plan_destroy(vrs_plan* plan) { delete plan; }

extern "C" size_t vrs_workspace_size(const vrs_plan* plan, int which) {
  if (!plan || which < VRS_WS_RENDER || which > VRS_WS_DECODER) return 0;
  return plan->ws[which];
}

extern "C" vrs_status vrs_plan_describe(const vrs_plan* plan, vrs_plan_desc* out) {
  if (!plan || !out) return VRS_EINVAL;
  *out = plan->d;
  return VRS_OK;
}

extern "C" vrs_status vrs_plan_trace(vrs_plan* plan, int stage, void* start_event,
                                     void* stop_event) {
  if (!plan || stage < VRS_TRACE_OFF || stage > VRS_TRACE_GS_DEPTH_SORT) return VRS_EINVAL;
  if (stage == VRS_TRACE_OFF) {
    for (int s = 0; s < vrs::kTraceStages; ++s)
      plan->trace.start[s] = plan->trace.stop[s] = nullptr;
    return VRS_OK;
  }
  if ((start_event == nullptr) != (stop_event == nullptr)) return VRS_EINVAL;
  plan->trace.start[stage] = static_cast<hipEvent_t>(start_event);
  plan->trace.stop[stage] = static_cast<hipEvent_t>(stop_event);
  return VRS_OK;
}

extern "C" vrs_status vrs_render_frame(const vrs_plan* plan, const vrs_scene* scene,
                                       const float* gaze, const vrs_frame_buffers* b,
                                       int32_t flags, void* stream) {
  if (!plan || !scene || !b) return VRS_EINVAL;
  if (flags & ~VRS_FRAME_STATS) return VRS_EINVAL;
  const vrs_plan_desc& d = plan->d;
  if (gaze && !b->place) return VRS_EINVAL;
  const bool fovea = d.n_crops > 0;
  if (!b->ws_render ||
      (fovea && (!b->ws_splat || !b->ws_decoder || !b->pyramid || !b->fovea_rgb)))
    return VRS_EINVAL;
  const vrs::Trace* tr = &plan->trace;
  const int W = d.views[0].width, H = d.views[0].height;
  vrs_status r = vrs::render_impl(scene->mean, scene->cov, scene->opacity, scene->sh, d.sh_degree,
                                  d.n_gaussians, d.views, d.n_views, &d.raster, b->rgb, b->depth,
                                  b->t_final, b->n_contrib, b->ws_render, plan->ws[VRS_WS_RENDER],
                                  d.max_pairs, b->status_render, stream,
                                  (flags & VRS_FRAME_STATS) ? vrs::kRenderStats : 0, tr);
  if (r != VRS_OK || !fovea) return r;
  // the gaze is read here, after the periphery: the splat's set-up launch
  // places the crops (as vrs_place_crops would) and writes b->place, which
  // every later stage reads
  const vrs_crop_place* place = gaze ? b->place : nullptr;
  r = vrs::splat_impl(scene->pos, scene->radius, scene->feat, scene->point_opacity, d.n_points,
                      d.point_channels, d.levels, d.views, d.n_views, d.crops, d.n_crops, place,
                      d.depth_cull ? b->depth : nullptr, d.depth_cull ? b->t_final : nullptr,
                      d.cov_min, d.slack, scene->point_ids, b->pyramid, b->ws_splat,
                      plan->ws[VRS_WS_SPLAT], d.max_frags, b->status_splat, stream, tr, gaze);
  if (r != VRS_OK) return r;
  r = vrs::decode_impl_entry(b->pyramid, d.levels, b->rgb, d.views, d.n_views, d.crops,
                             d.n_crops, place, scene->decoder_weights, &d.decoder, b->fovea_rgb,
                             b->ws_decoder, plan->ws[VRS_WS_DECODER], stream, tr);
  if (r != VRS_OK) return r;
  return vrs::composite_impl(b->rgb, d.n_views, W, H, b->fovea_rgb, d.crops, d.n_crops, place,
                             d.blend_mode, d.ring, d.m, d.gamma, b->rgb, stream, tr);
}
