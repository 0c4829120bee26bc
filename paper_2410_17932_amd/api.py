"""Thin ctypes binding of libvrsplat.so (include/vrsplat.h).

Argument marshalling only: every step of the renderer runs in the HIP
library.  torch provides device memory and the current stream.  If the
library is missing, every call raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvrsplat.so")
_lib = None

VRS_OK, VRS_EINVAL, VRS_ECAPACITY, VRS_EHIP, VRS_EUNSUPPORTED, VRS_ETIMEOUT = range(6)
VRS_F32, VRS_BF16 = 0, 1
BLEND_LINEAR, BLEND_PAPER = 0, 1
MAX_VIEWS, MAX_CROPS, MAX_LEVELS = 8, 32, 8


class VrsError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {status_string(code)} ({code})")
        self.code = code


class View(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("rot", ctypes.c_float * 9),
                ("trans", ctypes.c_float * 3), ("znear", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class Crop(ctypes.Structure):
    _fields_ = [("view", ctypes.c_int32), ("x0", ctypes.c_int32), ("y0", ctypes.c_int32),
                ("size", ctypes.c_int32), ("gaze_x", ctypes.c_float), ("gaze_y", ctypes.c_float)]


class RasterOpts(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("radix_bits", ctypes.c_int32),
                ("order", ctypes.c_int32), ("alpha_clamp", ctypes.c_float),
                ("alpha_min", ctypes.c_float), ("t_min", ctypes.c_float),
                ("lowpass", ctypes.c_float), ("extent", ctypes.c_float),
                ("bg", ctypes.c_float * 3)]


class DecoderDesc(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("width", ctypes.c_int32 * MAX_LEVELS),
                ("in_ch", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class RenderLayout(ctypes.Structure):
    _fields_ = [("pair_count", ctypes.c_size_t), ("sorted_ids", ctypes.c_size_t),
                ("tile_ranges", ctypes.c_size_t), ("pixel_evals", ctypes.c_size_t),
                ("tiles_x", ctypes.c_int64),
                ("tiles_y", ctypes.c_int64), ("tiles_total", ctypes.c_int64),
                ("super_pair_count", ctypes.c_size_t), ("exact_pass_count", ctypes.c_size_t),
                ("tile_words", ctypes.c_size_t)]


class SplatLayout(ctypes.Structure):
    _fields_ = [("frag_count", ctypes.c_size_t), ("sorted_keys", ctypes.c_size_t),
                ("sorted_ids", ctypes.c_size_t), ("pyramid_pixels", ctypes.c_int64)]


_vp, _i64, _int, _flt, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_size_t
_P = ctypes.POINTER


class PlanDesc(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("views", _P(View)),
                ("n_gaussians", ctypes.c_int64), ("sh_degree", ctypes.c_int32),
                ("n_points", ctypes.c_int64), ("point_channels", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("n_crops", ctypes.c_int32), ("crops", _P(Crop)),
                ("raster", RasterOpts), ("decoder", DecoderDesc),
                ("depth_cull", ctypes.c_int32), ("cov_min", ctypes.c_float),
                ("slack", ctypes.c_float), ("blend_mode", ctypes.c_int32),
                ("ring", ctypes.c_float), ("m", ctypes.c_float), ("gamma", ctypes.c_float),
                ("max_pairs", ctypes.c_int64), ("max_frags", ctypes.c_int64)]


class Scene(ctypes.Structure):
    _fields_ = [(k, _vp) for k in ("mean", "cov", "opacity", "sh", "pos", "radius", "feat",
                                   "point_opacity", "point_ids", "decoder_weights")]


class FrameBuffers(ctypes.Structure):
    _fields_ = [(k, _vp) for k in ("rgb", "depth", "t_final", "n_contrib", "pyramid",
                                   "fovea_rgb", "place", "ws_render", "ws_splat", "ws_decoder",
                                   "status_render", "status_splat")]

# (name, restype, argtypes) of every exported entry point
SIGNATURES = {
    "vrs_status_string": (ctypes.c_char_p, [_int]),
    "vrs_version": (ctypes.c_char_p, []),
    "vrs_bake_gaussians": (_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "vrs_spatial_order_workspace_size": (_sz, [_i64]),
    "vrs_spatial_order": (_int, [_vp, _i64, _vp, _vp, _sz, _vp]),
    "vrs_spatial_order_noalloc": (_int, [_vp, _i64, _vp, _vp]),
    "vrs_bake_gaussians_backward": (_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "vrs_render_workspace_size": (_sz, [_i64, _int, _P(View), _P(RasterOpts), _i64]),
    "vrs_render_workspace_layout": (_int, [_i64, _int, _P(View), _P(RasterOpts), _i64,
                                           _P(RenderLayout)]),
    "vrs_render_gaussians": (_int, [_vp, _vp, _vp, _vp, _int, _i64, _P(View), _int,
                                    _P(RasterOpts), _vp, _vp, _vp, _vp, _vp, _sz, _i64, _vp,
                                    _vp]),
    "vrs_render_gaussians_backward": (_int, [_vp, _vp, _vp, _vp, _int, _i64, _P(View), _int,
                                             _P(RasterOpts), _vp, _vp, _vp, _vp, _vp, _vp,
                                             _vp, _vp, _sz, _i64, _vp]),
    "vrs_splat_workspace_size": (_sz, [_i64, _int, _P(View), _P(Crop), _int, _int, _i64]),
    "vrs_splat_workspace_layout": (_int, [_i64, _int, _P(View), _P(Crop), _int, _int, _i64,
                                          _P(SplatLayout)]),
    "vrs_splat_points": (_int, [_vp, _vp, _vp, _vp, _i64, _int, _int, _P(View), _int,
                                _P(Crop), _int, _vp, _vp, _vp, _flt, _flt, _vp, _vp, _vp,
                                _sz, _i64, _vp, _vp]),
    "vrs_splat_points_backward": (_int, [_vp, _vp, _vp, _vp, _i64, _int, _int, _P(View), _int,
                                         _P(Crop), _int, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                         _sz, _i64, _vp]),
    "vrs_place_crops": (_int, [_vp, _P(View), _int, _P(Crop), _int, _vp, _vp]),
    "vrs_decoder_workspace_size": (_sz, [_P(DecoderDesc), _P(Crop), _int]),
    "vrs_decode_fovea": (_int, [_vp, _int, _vp, _P(View), _int, _P(Crop), _int, _vp, _vp,
                                _P(DecoderDesc), _vp, _vp, _sz, _vp]),
    "vrs_decode_fovea_backward": (_int, [_vp, _int, _vp, _P(View), _int, _P(Crop), _int, _vp,
                                         _vp, _P(DecoderDesc), _vp, _vp, _vp, _vp, _vp, _sz,
                                         _vp]),
    "vrs_composite_frame": (_int, [_vp, _int, _int, _int, _vp, _P(Crop), _int, _vp, _int,
                                   _flt, _flt, _flt, _vp, _vp]),
    "vrs_composite_frame_backward": (_int, [_vp, _int, _int, _int, _vp, _P(Crop), _int, _vp,
                                            _int, _flt, _flt, _flt, _vp, _vp, _vp, _vp]),
    "vrs_l1_loss": (_int, [_vp, _vp, _i64, _vp, _vp, _flt, _vp]),
    "vrs_tonemap": (_int, [_vp, _P(View), _int, _vp, _int, _vp, _vp]),
    "vrs_tonemap_workspace_size": (_sz, [_P(View), _int, _int]),
    "vrs_tonemap_backward": (_int, [_vp, _P(View), _int, _vp, _int, _vp, _vp, _vp, _vp, _sz,
                                    _vp]),
    "vrs_dssim_workspace_size": (_sz, [_int, _int, _int]),
    "vrs_dssim": (_int, [_vp, _vp, _int, _int, _int, _vp, _vp, _sz, _vp]),
    "vrs_dssim_backward": (_int, [_vp, _vp, _int, _int, _int, _vp, _vp, _vp, _sz, _vp]),
    "vrs_regulariser_workspace_size": (_sz, []),
    "vrs_regulariser": (_int, [_vp, _vp, _int, _int, _int, _P(Crop), _int, _vp, _vp, _vp, _sz,
                               _vp]),
    "vrs_regulariser_backward": (_int, [_int, _int, _int, _P(Crop), _int, _vp, _vp, _vp, _vp,
                                        _vp, _vp]),
    "vrs_adam_step": (_int, [_vp, _vp, _vp, _vp, _i64, _int, _flt, _flt, _flt, _flt, _vp]),
    "vrs_plan_create": (_int, [_P(PlanDesc), _P(_vp)]),
    "vrs_plan_destroy": (None, [_vp]),
    "vrs_workspace_size": (_sz, [_vp, _int]),
    "vrs_plan_describe": (_int, [_vp, _P(PlanDesc)]),
    "vrs_plan_trace": (_int, [_vp, _int, _vp, _vp]),
    "vrs_render_frame": (_int, [_vp, _P(Scene), _vp, _P(FrameBuffers), ctypes.c_int32, _vp]),
}
WS_RENDER, WS_SPLAT, WS_DECODER = 0, 1, 2
FRAME_STATS = 1

TRACE = dict(off=0, gs_blend=1, gs_sort=2, gs_preprocess=3, gs_emit=4, splat=5, decoder=6,
             composite=7, gs_depth_sort=8)


def lib():
    """Load the HIP library (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: build it with paper_2410_17932_amd/build.py")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if hasattr(l, name):
                fn = getattr(l, name)
                fn.restype = res
                fn.argtypes = args
        _lib = l
    return _lib


def status_string(code: int) -> str:
    try:
        return lib().vrs_status_string(code).decode()
    except Exception:  # pragma: no cover - only for messages
        return str(code)


def _check(code, where):
    if code != VRS_OK:
        raise VrsError(code, where)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def ptr(t, dtype=None):
    """Device pointer of a contiguous GPU tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------ descriptors
def make_views(views) -> ctypes.Array:
    """views: list of objects with fx, fy, cx, cy, width, height, rot, trans,
    znear (see synth.View)."""
    arr = (View * len(views))()
    for i, v in enumerate(views):
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = v.fx, v.fy, v.cx, v.cy
        for k, x in enumerate(np.asarray(v.rot, np.float32).ravel()):
            arr[i].rot[k] = float(x)
        for k, x in enumerate(np.asarray(v.trans, np.float32).ravel()):
            arr[i].trans[k] = float(x)
        arr[i].znear = v.znear
        arr[i].width, arr[i].height = v.width, v.height
    return arr


def make_crops(crops) -> ctypes.Array:
    arr = (Crop * max(len(crops), 1))()
    for i, c in enumerate(crops):
        arr[i].view, arr[i].x0, arr[i].y0, arr[i].size = c.view, c.x0, c.y0, c.size
        arr[i].gaze_x, arr[i].gaze_y = c.gaze_x, c.gaze_y
    return arr


ORDER_PRIMITIVE, ORDER_PIXEL = 0, 1


def make_opts(tile=16, alpha_clamp=0.99, alpha_min=1 / 255, t_min=1e-4, lowpass=0.3, extent=3.0,
              bg=(0.0, 0.0, 0.0), radix_bits=8, order=ORDER_PRIMITIVE, **_) -> RasterOpts:
    o = RasterOpts()
    o.tile, o.radix_bits, o.order = tile, radix_bits, order
    o.alpha_clamp, o.alpha_min, o.t_min = alpha_clamp, alpha_min, t_min
    o.lowpass, o.extent = lowpass, extent
    for k in range(3):
        o.bg[k] = bg[k]
    return o


def make_decoder_desc(widths, in_ch=4, dtype=VRS_F32) -> DecoderDesc:
    d = DecoderDesc()
    d.n_levels = len(widths)
    for k, w in enumerate(widths):
        d.width[k] = w
    d.in_ch, d.dtype = in_ch, dtype
    return d


# ------------------------------------------------------------------ bake
def bake_gaussians(logscale, quat, logit):
    n = logit.shape[0]
    cov = torch.empty((6, n), device=logit.device, dtype=torch.float32)
    op = torch.empty(n, device=logit.device, dtype=torch.float32)
    _check(lib().vrs_bake_gaussians(ptr(logscale, torch.float32), ptr(quat, torch.float32),
                                    ptr(logit, torch.float32), n, ptr(cov), ptr(op), _stream()),
           "vrs_bake_gaussians")
    return cov, op


def bake_gaussians_backward(logscale, quat, logit, d_cov, d_opacity, d_logscale, d_quat, d_logit):
    _check(lib().vrs_bake_gaussians_backward(
        ptr(logscale, torch.float32), ptr(quat, torch.float32), ptr(logit, torch.float32),
        logit.shape[0], ptr(d_cov, torch.float32), ptr(d_opacity, torch.float32),
        ptr(d_logscale, torch.float32), ptr(d_quat, torch.float32), ptr(d_logit, torch.float32),
        _stream()), "vrs_bake_gaussians_backward")


def spatial_order(pos):
    """Morton-order permutation of pos [3][n] (device int32 tensor of point
    indices); a load-time storage step for static scenes."""
    n = pos.shape[1]
    size = lib().vrs_spatial_order_workspace_size(n)
    if size == 0:
        raise VrsError(VRS_EINVAL, "vrs_spatial_order_workspace_size")
    ws = torch.empty(size, dtype=torch.uint8, device=pos.device)
    perm = torch.empty(n, dtype=torch.int32, device=pos.device)
    _check(lib().vrs_spatial_order(ptr(pos, torch.float32), n, ptr(perm), ptr(ws), size, _stream()),
           "vrs_spatial_order")
    return perm


NOALLOC_MAX_POINTS = 1 << 20


def spatial_order_noalloc(pos):
    """vrs_spatial_order_noalloc: the same permutation with no workspace
    (the library's fixed scratch; at most NOALLOC_MAX_POINTS points)."""
    n = pos.shape[1]
    perm = torch.empty(n, dtype=torch.int32, device=pos.device)
    _check(lib().vrs_spatial_order_noalloc(ptr(pos, torch.float32), n, ptr(perm), _stream()),
           "vrs_spatial_order_noalloc")
    return perm


# ------------------------------------------------------------- periphery
class RenderWorkspace:
    """Caller-owned workspace of one render call (kept for its backward).
    A backward call replays the lists of the workspace's last forward call:
    `generation` counts forward calls so that a backward can check that no
    other forward has run through the workspace since its own."""

    def __init__(self, n, views, opts, max_pairs, device="cuda"):
        self.generation = 0
        self.n, self.views, self.opts, self.max_pairs = n, views, opts, int(max_pairs)
        self.cviews = make_views(views)
        size = lib().vrs_render_workspace_size(n, len(views), self.cviews, ctypes.byref(opts),
                                               self.max_pairs)
        if size == 0:
            raise VrsError(VRS_EINVAL, "vrs_render_workspace_size")
        self.buf = torch.empty(size, dtype=torch.uint8, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        lay = RenderLayout()
        _check(lib().vrs_render_workspace_layout(n, len(views), self.cviews, ctypes.byref(opts),
                                                 self.max_pairs, ctypes.byref(lay)),
               "vrs_render_workspace_layout")
        self.layout = lay

    def u32(self, off, count):
        return self.buf[off:off + 4 * count].view(torch.int32)

    def pair_count(self) -> int:
        return int(self.u32(self.layout.pair_count, 1).item())

    def super_pair_count(self) -> int:
        return int(self.u32(self.layout.super_pair_count, 1).item())

    def exact_pass_count(self) -> int:
        """Pixels of the last per-pixel-order render resolved by the exact
        pass (0 in per-primitive order)."""
        if self.layout.exact_pass_count == 0:
            return 0
        return int(self.u32(self.layout.exact_pass_count, 1).item())

    def tile_words(self):
        """Per-pixel order: the blend's tile lists as uint64 words
        (z_t bits << 32 | index), int64-viewed on the host, over the ranges
        of tile_lists."""
        if self.layout.tile_words == 0:
            raise ValueError("tile words exist in per-pixel order only")
        cnt = min(self.pair_count(), self.max_pairs)
        off = self.layout.tile_words
        w = self.buf[off:off + 8 * max(cnt, 1)].view(torch.int64)[:cnt]
        return w.cpu().numpy().view(np.uint64)

    def pixel_evals(self, npix):
        """Per-pixel evaluation counts of the last blend (device tensor)."""
        return self.u32(self.layout.pixel_evals, npix)

    def tile_lists(self):
        """(ranges [tiles][2] int64, sorted ids int64) on the host."""
        ranges = self.u32(self.layout.tile_ranges, 2 * self.layout.tiles_total)
        ranges = ranges.view(-1, 2).cpu().numpy().astype(np.int64)
        cnt = min(self.pair_count(), self.max_pairs)
        ids = self.u32(self.layout.sorted_ids, max(cnt, 1))[:cnt].cpu().numpy().astype(np.int64)
        return ranges, ids


def render_gaussians(mean, cov, opacity, sh, sh_degree, views, opts, ws: RenderWorkspace,
                     outputs=None):
    nv = len(views)
    W, H = views[0].width, views[0].height
    dev = mean.device
    if outputs is None:
        outputs = dict(rgb=torch.empty((nv, 3, H, W), device=dev),
                       depth=torch.empty((nv, H, W), device=dev),
                       tfinal=torch.empty((nv, H, W), device=dev),
                       ncontrib=torch.empty((nv, H, W), device=dev, dtype=torch.int32))
    n = mean.shape[1]
    code = lib().vrs_render_gaussians(
        ptr(mean, torch.float32), ptr(cov, torch.float32), ptr(opacity, torch.float32),
        ptr(sh, torch.float32), sh_degree, n, ws.cviews, nv, ctypes.byref(opts),
        ptr(outputs["rgb"]), ptr(outputs["depth"]), ptr(outputs["tfinal"]),
        ptr(outputs["ncontrib"]), ptr(ws.buf), ws.buf.numel(), ws.max_pairs, ptr(ws.status),
        _stream())
    _check(code, "vrs_render_gaussians")
    ws.generation += 1
    return outputs


def render_gaussians_backward(mean, cov, opacity, sh, sh_degree, views, opts, ws, tfinal, d_rgb,
                              d_depth, d_mean, d_cov, d_opacity, d_sh):
    n = mean.shape[1]
    code = lib().vrs_render_gaussians_backward(
        ptr(mean, torch.float32), ptr(cov, torch.float32), ptr(opacity, torch.float32),
        ptr(sh, torch.float32), sh_degree, n, ws.cviews, len(views), ctypes.byref(opts),
        ptr(tfinal, torch.float32), ptr(d_rgb, torch.float32), ptr(d_depth, torch.float32),
        ptr(d_mean, torch.float32), ptr(d_cov, torch.float32), ptr(d_opacity, torch.float32),
        ptr(d_sh, torch.float32), ptr(ws.buf), ws.buf.numel(), ws.max_pairs, _stream())
    _check(code, "vrs_render_gaussians_backward")


# ----------------------------------------------------------------- fovea
def pyramid_pixels(crops, levels) -> int:
    return int(sum(sum((c.size >> l) ** 2 for l in range(levels)) for c in crops))


class SplatWorkspace:
    """Caller-owned workspace of one splat call (fragment lists kept for the
    backward; `generation` as for RenderWorkspace)."""

    def __init__(self, np_, views, crops, levels, max_frags, device="cuda"):
        self.generation = 0
        self.np, self.views, self.crops, self.levels = np_, views, crops, levels
        self.max_frags = int(max_frags)
        self.cviews, self.ccrops = make_views(views), make_crops(crops)
        size = lib().vrs_splat_workspace_size(np_, len(views), self.cviews, self.ccrops,
                                              len(crops), levels, self.max_frags)
        if size == 0:
            raise VrsError(VRS_EINVAL, "vrs_splat_workspace_size")
        self.buf = torch.empty(size, dtype=torch.uint8, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        lay = SplatLayout()
        _check(lib().vrs_splat_workspace_layout(np_, len(views), self.cviews, self.ccrops,
                                                len(crops), levels, self.max_frags,
                                                ctypes.byref(lay)), "vrs_splat_workspace_layout")
        self.layout = lay

    def u32(self, off, count):
        return self.buf[off:off + 4 * count].view(torch.int32)

    def frag_count(self) -> int:
        return int(self.u32(self.layout.frag_count, 1).item())

    def lists(self):
        """(layer-pixel keys, point ids) of every fragment in blend order."""
        cnt = min(self.frag_count(), self.max_frags)
        keys = self.u32(self.layout.sorted_keys, max(cnt, 1))[:cnt].cpu().numpy().astype(np.int64)
        vals = self.u32(self.layout.sorted_ids, 2 * max(cnt, 1))[:2 * cnt].cpu().numpy()
        return keys, vals[0::2].astype(np.int64)   # low word of each 64-bit value


def crop_places(n_crops, device="cuda"):
    """Device table of vrs_crop_place records [n][4] (int32 x0, y0 and the
    float32 gaze bits), filled by place_crops."""
    return torch.zeros((max(n_crops, 1), 4), dtype=torch.int32, device=device)


def place_crops(gaze, views, crops, place):
    """vrs_place_crops: gaze [n][2] float32 device tensor -> place table."""
    _check(lib().vrs_place_crops(ptr(gaze, torch.float32), make_views(views), len(views),
                                 make_crops(crops), len(crops), ptr(place, torch.int32),
                                 _stream()), "vrs_place_crops")
    return place


def splat_points(pos, radius, feat, opacity, views, crops, levels, depth, tfinal, ws,
                 cov_min=0.5, slack=1.05, pyramid=None, point_ids=None, place=None):
    """vrs_splat_points; point_ids (int32 device tensor [np], optional): the
    caller's index of each stored point, which orders fragments of equal
    depth; place (crop_places table, optional): crop origins and gazes read
    on the device."""
    P = pyramid_pixels(crops, levels)
    C = feat.shape[1]
    if pyramid is None:
        pyramid = torch.empty((P, C), device=pos.device, dtype=torch.float32)
    code = lib().vrs_splat_points(
        ptr(pos, torch.float32), ptr(radius, torch.float32), ptr(feat), ptr(opacity),
        pos.shape[1], C, levels, ws.cviews, len(views), ws.ccrops, len(crops),
        ptr(place, torch.int32), ptr(depth), ptr(tfinal), cov_min, slack,
        ptr(point_ids, torch.int32), ptr(pyramid), ptr(ws.buf),
        ws.buf.numel(), ws.max_frags, ptr(ws.status), _stream())
    _check(code, "vrs_splat_points")
    ws.generation += 1
    return pyramid


def splat_points_backward(pos, radius, feat, opacity, views, crops, levels, d_pyramid, ws,
                          d_feat=None, d_pos=None, d_radius=None, d_opacity=None, place=None):
    code = lib().vrs_splat_points_backward(
        ptr(pos, torch.float32), ptr(radius, torch.float32), ptr(feat), ptr(opacity),
        pos.shape[1], feat.shape[1], levels, ws.cviews, len(views), ws.ccrops, len(crops),
        ptr(place, torch.int32), ptr(d_pyramid, torch.float32), ptr(d_feat), ptr(d_pos), ptr(d_radius), ptr(d_opacity),
        ptr(ws.buf), ws.buf.numel(), ws.max_frags, _stream())
    _check(code, "vrs_splat_points_backward")


# --------------------------------------------------------------- decoder
class DecoderWorkspace:
    """Caller-owned workspace of one decoder call (activations kept for the
    backward; `generation` as for RenderWorkspace)."""

    def __init__(self, widths, crops, dtype=VRS_F32, in_ch=4, device="cuda"):
        self.generation = 0
        self.desc = make_decoder_desc(widths, in_ch, dtype)
        self.crops = crops
        self.ccrops = make_crops(crops)
        size = lib().vrs_decoder_workspace_size(ctypes.byref(self.desc), self.ccrops, len(crops))
        if size == 0:
            raise VrsError(VRS_EINVAL, "vrs_decoder_workspace_size")
        self.buf = torch.empty(size, dtype=torch.uint8, device=device)


def fovea_elements(crops) -> int:
    return int(sum(3 * c.size * c.size for c in crops))


def decode_fovea(pyramid, levels, periphery, views, crops, weights, ws: DecoderWorkspace,
                 out=None, place=None):
    if out is None:
        out = torch.empty(fovea_elements(crops), device=pyramid.device, dtype=torch.float32)
    cviews = make_views(views)
    code = lib().vrs_decode_fovea(ptr(pyramid, torch.float32), levels,
                                  ptr(periphery, torch.float32), cviews, len(views), ws.ccrops,
                                  len(crops), ptr(place, torch.int32),
                                  ptr(weights, torch.float32), ctypes.byref(ws.desc),
                                  ptr(out), ptr(ws.buf), ws.buf.numel(), _stream())
    _check(code, "vrs_decode_fovea")
    ws.generation += 1
    return out


def decode_fovea_backward(pyramid, levels, periphery, views, crops, weights, ws, d_fovea,
                          d_pyramid=None, d_periphery=None, d_weights=None, place=None):
    cviews = make_views(views)
    code = lib().vrs_decode_fovea_backward(
        ptr(pyramid, torch.float32), levels, ptr(periphery, torch.float32), cviews, len(views),
        ws.ccrops, len(crops), ptr(place, torch.int32), ptr(weights, torch.float32),
        ctypes.byref(ws.desc),
        ptr(d_fovea, torch.float32), ptr(d_pyramid), ptr(d_periphery), ptr(d_weights),
        ptr(ws.buf), ws.buf.numel(), _stream())
    _check(code, "vrs_decode_fovea_backward")


# ------------------------------------------------------------- combine
def composite_frame(periphery, fovea, crops, mode=BLEND_LINEAR, ring=64.0, m=0.75, gamma=0.2,
                    out=None, place=None):
    """vrs_composite_frame; out may be `periphery` itself (in place: only the
    pixels under the crops are read and written)."""
    V, _, H, W = periphery.shape
    if out is None:
        out = torch.empty_like(periphery)
    code = lib().vrs_composite_frame(ptr(periphery, torch.float32), V, W, H,
                                     ptr(fovea, torch.float32), make_crops(crops), len(crops),
                                     ptr(place, torch.int32), mode, ring, m, gamma, ptr(out),
                                     _stream())
    _check(code, "vrs_composite_frame")
    return out


def composite_frame_backward(periphery, fovea, crops, d_out, d_periphery=None, d_fovea=None,
                             mode=BLEND_LINEAR, ring=64.0, m=0.75, gamma=0.2, place=None):
    V, _, H, W = periphery.shape
    code = lib().vrs_composite_frame_backward(
        ptr(periphery, torch.float32), V, W, H, ptr(fovea, torch.float32), make_crops(crops),
        len(crops), ptr(place, torch.int32), mode, ring, m, gamma, ptr(d_out, torch.float32), ptr(d_periphery),
        ptr(d_fovea), _stream())
    _check(code, "vrs_composite_frame_backward")


# ------------------------------------------------------------ tone mapping
def tonemap_params(n_views, n_resp=32, gamma=1.0 / 2.2, device="cuda"):
    """Neutral camera model (ev 0, unit white balance, no vignetting) with a
    gamma response: float32 [V][7 + n_resp]."""
    p = torch.zeros((n_views, 7 + n_resp), dtype=torch.float32)
    p[:, 1:4] = 1.0
    p[:, 7:] = torch.linspace(0.0, 1.0, n_resp, dtype=torch.float64).pow(gamma).float()
    return p.to(device)


def tonemap(img, views, params, out=None):
    """vrs_tonemap: img [V][3][H][W] -> out (may be img)."""
    V = img.shape[0]
    n = params.shape[1] - 7
    if out is None:
        out = torch.empty_like(img)
    _check(lib().vrs_tonemap(ptr(img, torch.float32), make_views(views), V,
                             ptr(params, torch.float32), n, ptr(out), _stream()), "vrs_tonemap")
    return out


def tonemap_backward(img, views, params, d_out, d_img=None, d_params=None):
    """vrs_tonemap_backward: d_img written (may be None), d_params
    accumulated (may be None)."""
    V = img.shape[0]
    n = params.shape[1] - 7
    cv = make_views(views)
    ws = None
    if d_params is not None:
        size = lib().vrs_tonemap_workspace_size(cv, V, n)
        ws = torch.empty(max(size, 1), dtype=torch.uint8, device=img.device)
    _check(lib().vrs_tonemap_backward(ptr(img, torch.float32), cv, V, ptr(params, torch.float32),
                                      n, ptr(d_out, torch.float32), ptr(d_img), ptr(d_params),
                                      ptr(ws), 0 if ws is None else ws.numel(), _stream()),
           "vrs_tonemap_backward")


# --------------------------------------------------------- training loss
class DssimWorkspace:
    def __init__(self, planes, width, height, device="cuda"):
        self.shape = (planes, height, width)
        size = lib().vrs_dssim_workspace_size(planes, width, height)
        if size == 0:
            raise VrsError(VRS_EINVAL, "vrs_dssim_workspace_size")
        self.buf = torch.empty(size, dtype=torch.uint8, device=device)


def dssim(x, y, ws: DssimWorkspace, loss=None):
    """vrs_dssim over x, y viewed as [planes][H][W]: device scalar."""
    P, H, W = ws.shape
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(lib().vrs_dssim(ptr(x, torch.float32), ptr(y, torch.float32), P, W, H, ptr(loss),
                           ptr(ws.buf), ws.buf.numel(), _stream()), "vrs_dssim")
    return loss


def dssim_backward(x, y, ws: DssimWorkspace, d_x, d_loss=None):
    P, H, W = ws.shape
    _check(lib().vrs_dssim_backward(ptr(x, torch.float32), ptr(y, torch.float32), P, W, H,
                                    ptr(d_loss, torch.float32), ptr(d_x), ptr(ws.buf),
                                    ws.buf.numel(), _stream()), "vrs_dssim_backward")


def regulariser(fovea, periphery, crops, place=None, r=None):
    """vrs_regulariser: device [2] = (R, mean F - mean crop(P))."""
    V, _, H, W = periphery.shape
    if r is None:
        r = torch.empty(2, dtype=torch.float32, device=periphery.device)
    ws = torch.empty(lib().vrs_regulariser_workspace_size(), dtype=torch.uint8,
                     device=periphery.device)
    _check(lib().vrs_regulariser(ptr(fovea, torch.float32), ptr(periphery, torch.float32), V, W,
                                 H, make_crops(crops), len(crops), ptr(place, torch.int32),
                                 ptr(r), ptr(ws), ws.numel(), _stream()), "vrs_regulariser")
    return r


def regulariser_backward(periphery_shape, crops, r, d_r=None, d_fovea=None, d_periphery=None,
                         place=None):
    V, _, H, W = periphery_shape
    _check(lib().vrs_regulariser_backward(V, W, H, make_crops(crops), len(crops),
                                          ptr(place, torch.int32), ptr(r, torch.float32),
                                          ptr(d_r, torch.float32), ptr(d_fovea),
                                          ptr(d_periphery), _stream()),
           "vrs_regulariser_backward")


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """vrs_adam_step in place on float32 tensors of one size."""
    n = param.numel()
    _check(lib().vrs_adam_step(ptr(param, torch.float32), ptr(grad, torch.float32),
                               ptr(m, torch.float32), ptr(v, torch.float32), n, step, lr, beta1,
                               beta2, eps, _stream()), "vrs_adam_step")


# ------------------------------------------------------------ frame plan
class Plan:
    """vrs_plan: views, crop views and sizes, the tuned tile size and sort
    radix, capacities, decoder shape, depth cull and combination of one
    scene and rig (host memory; destroyed with this object)."""

    def __init__(self, views, crops, n_gaussians, sh_degree, n_points, levels, opts, widths,
                 decoder_dtype, max_pairs, max_frags, cull=True, cov_min=0.5, slack=1.05,
                 mode=BLEND_LINEAR, ring=64.0, m=0.75, gamma=0.2):
        self.cviews, self.ccrops = make_views(views), make_crops(crops)
        d = PlanDesc()
        d.n_views, d.views = len(views), self.cviews
        d.n_gaussians, d.sh_degree = int(n_gaussians), sh_degree
        d.n_points, d.point_channels, d.levels = int(n_points), 4, levels
        d.n_crops, d.crops = len(crops), self.ccrops
        d.raster = opts
        d.decoder = make_decoder_desc(widths, 4, decoder_dtype)
        d.depth_cull, d.cov_min, d.slack = int(bool(cull)), cov_min, slack
        d.blend_mode, d.ring, d.m, d.gamma = mode, ring, m, gamma
        d.max_pairs, d.max_frags = int(max_pairs), int(max_frags)
        self.desc = d
        h = ctypes.c_void_p()
        _check(lib().vrs_plan_create(ctypes.byref(d), ctypes.byref(h)), "vrs_plan_create")
        self.handle = h

    def workspace_size(self, which) -> int:
        return int(lib().vrs_workspace_size(self.handle, which))

    def trace(self, stage: str, start=None, stop=None):
        """Record torch.cuda.Event start/stop around stage `stage` of every
        frame of this plan ("off" clears)."""
        code = TRACE[stage]
        for e in (start, stop):
            if e is not None and e.cuda_event == 0:
                e.record()   # torch creates the HIP event on first record
        a = ctypes.c_void_p(start.cuda_event) if start is not None else None
        b = ctypes.c_void_p(stop.cuda_event) if stop is not None else None
        _check(lib().vrs_plan_trace(self.handle, code, a, b), "vrs_plan_trace")

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.vrs_plan_destroy(self.handle)
            self.handle = None


def render_frame(plan: Plan, scene: Scene, gaze, buffers: FrameBuffers, stats=False):
    """vrs_render_frame on the current stream."""
    _check(lib().vrs_render_frame(plan.handle, ctypes.byref(scene), ptr(gaze, torch.float32),
                                  ctypes.byref(buffers), FRAME_STATS if stats else 0, _stream()),
           "vrs_render_frame")


def l1_loss(pred, target, d_pred=None, scale=1.0):
    loss = torch.empty(1, device=pred.device, dtype=torch.float32)
    _check(lib().vrs_l1_loss(ptr(pred, torch.float32), ptr(target, torch.float32), pred.numel(),
                             ptr(loss), ptr(d_pred), scale, _stream()), "vrs_l1_loss")
    return loss
