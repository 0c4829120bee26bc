"""Per-frame runtime of the foveated hybrid renderer (Fig. 5 of the paper):
periphery P and depth (Sec. 3.2) -> gaze crops -> neural-point pyramid with
depth culling (Sec. 3.3) -> decoder -> combination (Sec. 3.4).

Two forms of the same frame:
  * batched: both eyes in one periphery call, every crop of both eyes in one
    splat call and one decoder launch per level, BF16 decoder; the whole
    frame is captured once into a HIP graph and replayed;
  * plain: eager, one periphery call per eye, one splat and one FP32 decoder
    call per crop.
Workspaces are sized once by a counting pass (no host read-back inside a
frame); device-side overflow is reported through the status words.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


class Frame:
    """The batched frame on a plan (vrs_plan_create) with one
    vrs_render_frame call per frame: the periphery's rgb image receives the
    combined frame in place."""

    def __init__(self, scene: dict, decoder_dtype: int = api.VRS_BF16, tile: int = 16,
                 radix_bits: int = 8, mode: int = api.BLEND_LINEAR, ring: float = 64.0,
                 m: float = 0.75, gamma: float = 0.2, cull: bool = True,
                 pair_margin: float = 1.10, frag_margin: float = 1.25,
                 spatial_order: bool = True, order: int = api.ORDER_PRIMITIVE):
        g, p = scene["gaussians"], scene["points"]
        self.views, self.crops, self.levels = scene["views"], scene["crops"], scene["levels"]
        # without points or crops the frame is the periphery alone
        self.fovea_on = bool(self.crops) and p is not None
        if not self.fovea_on:
            self.crops = []
        self.sh_degree = g["sh_degree"]
        self.mode, self.ring, self.m, self.gamma, self.cull = mode, ring, m, gamma, cull
        self.decoder_dtype = decoder_dtype
        self.widths = scene["decoder"]["widths"] if scene.get("decoder") else (16, 32, 64, 64)
        self.raster = dict(scene["raster"], tile=tile, radix_bits=radix_bits, order=order)
        # primitives resident in HBM; attributes baked once (Sec. 4 "Inference")
        self.mean = _dev(g["mean"])
        self.sh = _dev(g["sh"])
        self.cov, self.opacity = api.bake_gaussians(_dev(g["logscale"]), _dev(g["quat"]),
                                                    _dev(g["logit"]))
        self.pos = self.radius = self.feat = self.point_ids = self.weights = None
        self.n, self.np = g["n"], p["n"] if self.fovea_on else 0
        self.pair_margin, self.frag_margin = pair_margin, frag_margin
        self.gaze = self.place = None
        if not self.fovea_on:
            self._plan(tile, radix_bits)
            return
        self.pos, self.radius = _dev(p["pos"]), _dev(p["radius"])
        self.feat = _dev(p["feat"].view(np.int16))
        if spatial_order:
            # storage layout of the static point cloud: Morton order, so the
            # depth cull's per-point reads of depth and T' share cache lines;
            # the input index of each stored point still orders fragments of
            # equal depth
            perm = api.spatial_order(self.pos)
            self.point_ids = perm
            perm = perm.long()
            self.pos = self.pos[:, perm].contiguous()
            self.radius = self.radius[perm].contiguous()
            self.feat = self.feat[perm].contiguous()
        from .synth import pack_decoder
        self.weights = _dev(pack_decoder(scene["decoder"]))
        # fixation points in device memory: each frame places its crops from
        # them on the device, after the periphery (Sec. 4 "Inference"), so a
        # captured frame follows set_gaze() without being captured again
        self.gaze = _dev(np.array([[c.gaze_x, c.gaze_y] for c in self.crops], np.float32))
        self.place = api.crop_places(len(self.crops))
        self._plan(tile, radix_bits)

    # ------------------------------------------------------------ planning
    def _plan(self, tile, radix_bits=None):
        """Counting passes (capacity 1: the totals are computed on the
        device) size the tile-pair and fragment capacities, then the plan and
        its workspaces."""
        if radix_bits is None:
            radix_bits = self.raster["radix_bits"]
        self.raster.update(tile=tile, radix_bits=radix_bits)
        self.opts = api.make_opts(**self.raster)
        V, H, W = len(self.views), self.views[0].height, self.views[0].width
        dev = self.mean.device
        self.rgb = torch.empty((V, 3, H, W), device=dev)
        self.depth = torch.empty((V, H, W), device=dev)
        self.tfinal = torch.empty((V, H, W), device=dev)
        self.ncontrib = torch.empty((V, H, W), device=dev, dtype=torch.int32)
        self.out = self.rgb
        r_out = dict(rgb=self.rgb, depth=self.depth, tfinal=self.tfinal, ncontrib=self.ncontrib)
        self.plan = self.rws = self.sws = self.dws = None
        ws = api.RenderWorkspace(self.n, self.views, self.opts, 1)
        api.render_gaussians(self.mean, self.cov, self.opacity, self.sh, self.sh_degree,
                             self.views, self.opts, ws, r_out)
        self.pairs = ws.pair_count()
        del ws
        self.rws = api.RenderWorkspace(self.n, self.views, self.opts,
                                       int(self.pairs * self.pair_margin) + 4096)
        api.render_gaussians(self.mean, self.cov, self.opacity, self.sh, self.sh_degree,
                             self.views, self.opts, self.rws, r_out)
        self.frags = 0
        self.pyramid = self.fovea = None
        if self.fovea_on:
            self._plan_fovea(dev)
        self.plan = api.Plan(self.views, self.crops, self.n, self.sh_degree, self.np,
                             self.levels, self.opts, self.widths, self.decoder_dtype,
                             self.rws.max_pairs, self.sws.max_frags if self.sws else 0, self.cull,
                             mode=self.mode, ring=self.ring, m=self.m, gamma=self.gamma)
        for which, w in ((api.WS_RENDER, self.rws), (api.WS_SPLAT, self.sws),
                         (api.WS_DECODER, self.dws)):
            assert self.plan.workspace_size(which) == (w.buf.numel() if w else 0)
        ptr = lambda t: None if t is None else t.data_ptr()
        self.c_scene = api.Scene(
            mean=ptr(self.mean), cov=ptr(self.cov), opacity=ptr(self.opacity), sh=ptr(self.sh),
            pos=ptr(self.pos), radius=ptr(self.radius), feat=ptr(self.feat), point_opacity=None,
            point_ids=ptr(self.point_ids), decoder_weights=ptr(self.weights))
        self.c_buf = api.FrameBuffers(
            rgb=ptr(self.rgb), depth=ptr(self.depth), t_final=ptr(self.tfinal),
            n_contrib=ptr(self.ncontrib), pyramid=ptr(self.pyramid), fovea_rgb=ptr(self.fovea),
            place=ptr(self.place), ws_render=ptr(self.rws.buf),
            ws_splat=ptr(self.sws.buf) if self.sws else None,
            ws_decoder=ptr(self.dws.buf) if self.dws else None,
            status_render=ptr(self.rws.status),
            status_splat=ptr(self.sws.status) if self.sws else None)
        torch.cuda.synchronize()
        self.graph = None

    def _plan_fovea(self, dev):
        P = api.pyramid_pixels(self.crops, self.levels)
        self.pyramid = torch.empty((P, 4), device=dev)
        sws = api.SplatWorkspace(self.np, self.views, self.crops, self.levels, 1)
        api.place_crops(self.gaze, self.views, self.crops, self.place)
        api.splat_points(self.pos, self.radius, self.feat, None, self.views, self.crops,
                         self.levels, self.depth if self.cull else None,
                         self.tfinal if self.cull else None, sws, pyramid=self.pyramid,
                         point_ids=self.point_ids, place=self.place)
        self.frags = sws.frag_count()
        del sws
        self.sws = api.SplatWorkspace(self.np, self.views, self.crops, self.levels,
                                      int(self.frags * self.frag_margin) + 4096)
        self.dws = api.DecoderWorkspace(self.widths, self.crops, self.decoder_dtype)
        self.fovea = torch.empty(api.fovea_elements(self.crops), device=dev)

    def set_gaze(self, gaze):
        """New fixation points [n_crops][2] (view pixels) for the next frames:
        written into the device buffer the frame reads (a captured graph
        picks them up on its next replay)."""
        self.gaze.copy_(torch.as_tensor(np.asarray(gaze, np.float32)).reshape(-1, 2))

    def trace(self, stage, start=None, stop=None):
        self.plan.trace(stage, start, stop)

    # --------------------------------------------------------------- frame
    def run(self, stats: bool = False):
        """Enqueue one batched frame on the current stream (stats: also keep
        the periphery's per-pixel evaluation counts and last positions)."""
        api.render_frame(self.plan, self.c_scene, self.gaze, self.c_buf, stats)
        return self.out

    def capture(self):
        """Capture run() into a HIP graph (warm-up on a side stream first)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        torch.cuda.synchronize()
        return self.graph

    def replay(self):
        self.graph.replay()
        return self.out

    def status(self) -> int:
        return max(int(self.rws.status.item()), int(self.sws.status.item()) if self.sws else 0)

    # ----------------------------------------------------------- autotune
    def autotune(self, tiles=(8, 16, 32), radix=(4, 6, 8, 11), reps: int = 5) -> dict:
        """Time the frame for every tile size and sort radix on the live
        scene and keep the fastest (neither changes a result; per-pixel
        order takes tiles of 8 and 16)."""
        if self.raster["order"] == api.ORDER_PIXEL:
            tiles = tuple(t for t in tiles if t <= 16)
        times = {}
        for t in tiles:
            for r in radix:
                self._plan(t, r)
                for _ in range(2):
                    self.run()
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(reps):
                    self.run()
                b.record()
                torch.cuda.synchronize()
                times[(t, r)] = a.elapsed_time(b) / reps
        best = min(times, key=times.get)
        self._plan(*best)
        return dict(tile=best[0], radix_bits=best[1],
                    ms={f"{t}/{r}": round(v, 4) for (t, r), v in times.items()})


class PlainFrame:
    """The plain FP32 form of the same frame: eager, one periphery call per
    eye, one splat and one FP32 decoder call per crop, one combination."""

    def __init__(self, batched: Frame):
        b = batched
        self.b = b
        dev = b.mean.device
        self.opts = b.opts
        self.rws, self.sws, self.dws, self.pyr, self.fov = [], [], [], [], []
        H, W = b.views[0].height, b.views[0].width
        self.rgb = torch.empty_like(b.rgb)
        self.depth = torch.empty_like(b.depth)
        self.tfinal = torch.empty_like(b.tfinal)
        self.nc = torch.empty_like(b.ncontrib)
        for v in range(len(b.views)):
            ws = api.RenderWorkspace(b.n, [b.views[v]], self.opts, 1)
            o = dict(rgb=self.rgb[v:v + 1], depth=self.depth[v:v + 1],
                     tfinal=self.tfinal[v:v + 1], ncontrib=self.nc[v:v + 1])
            api.render_gaussians(b.mean, b.cov, b.opacity, b.sh, b.sh_degree, [b.views[v]],
                                 self.opts, ws, o)
            self.rws.append(api.RenderWorkspace(b.n, [b.views[v]], self.opts,
                                                int(ws.pair_count() * 1.1) + 4096))
        for c in b.crops:
            self.pyr.append(torch.empty((api.pyramid_pixels([c], b.levels), 4), device=dev))
            self.sws.append(api.SplatWorkspace(b.np, b.views, [c], b.levels,
                                               int(b.frags * 1.25) + 4096))
            self.dws.append(api.DecoderWorkspace(b.widths, [c], api.VRS_F32))
            self.fov.append(torch.empty(3 * c.size * c.size, device=dev))
        self.fovea = torch.empty_like(b.fovea)
        self.out = torch.empty_like(b.out)

    def run(self):
        b = self.b
        for v in range(len(b.views)):
            o = dict(rgb=self.rgb[v:v + 1], depth=self.depth[v:v + 1],
                     tfinal=self.tfinal[v:v + 1], ncontrib=self.nc[v:v + 1])
            api.render_gaussians(b.mean, b.cov, b.opacity, b.sh, b.sh_degree, [b.views[v]],
                                 self.opts, self.rws[v], o)
        off = 0
        for k, c in enumerate(b.crops):
            api.splat_points(b.pos, b.radius, b.feat, None, b.views, [c], b.levels,
                             self.depth if b.cull else None, self.tfinal if b.cull else None,
                             self.sws[k], pyramid=self.pyr[k], point_ids=b.point_ids)
            api.decode_fovea(self.pyr[k], b.levels, self.rgb, b.views, [c], b.weights,
                             self.dws[k], out=self.fovea[off:off + 3 * c.size * c.size])
            off += 3 * c.size * c.size
        api.composite_frame(self.rgb, self.fovea, b.crops, b.mode, b.ring, b.m, b.gamma,
                            out=self.out)
        return self.out


class FitStep:
    """One differentiable fitting step (Sec. 3.5): bake -> periphery ->
    depth-culled point splat -> decoder -> combination [-> tone mapping] ->
    loss against a target, then the hand-written adjoints of every stage
    through torch.autograd.  Parameters live in HBM as leaf tensors with
    .grad.  loss "l1": L1; "paper": Eq. 6 without the VGG term,
    (1 - lam) L1 + lam D-SSIM + beta R (lam = 0.2, beta = 1e-5; R of Eq. 7
    over the crops).  tonemap: the camera model's parameters (float32
    [V][7 + n]) join the fitted parameters and map the combined image before
    the loss.  step(): plain gradient descent, or Adam (vrs_adam_step) with
    optimizer="adam"."""

    def __init__(self, scene: dict, target, decoder_dtype: int = api.VRS_BF16, tile: int = 16,
                 ring: float = 64.0, cull: bool = True, pair_margin: float = 1.5,
                 frag_margin: float = 2.0, mask=None, loss: str = "l1", lam: float = 0.2,
                 beta: float = 1e-5, tonemap=None):
        if loss not in ("l1", "paper"):
            raise ValueError("loss must be 'l1' or 'paper'")
        self.loss_kind, self.lam, self.beta = loss, lam, beta
        self.adam_state = {}
        self.adam_t = 0
        self.mask = None if mask is None else (mask if torch.is_tensor(mask) else _dev(mask))
        g, p = scene["gaussians"], scene["points"]
        self.views, self.crops, self.levels = scene["views"], scene["crops"], scene["levels"]
        self.deg, self.ring, self.cull = g["sh_degree"], ring, cull
        self.opts = api.make_opts(**dict(scene["raster"], tile=tile))
        from .synth import pack_decoder
        self.params = dict(
            mean=_dev(g["mean"]), logscale=_dev(g["logscale"]), quat=_dev(g["quat"]),
            logit=_dev(g["logit"]), sh=_dev(g["sh"]), pos=_dev(p["pos"]),
            radius=_dev(p["radius"]),
            feat=_dev(p["feat"].view(np.float16).astype(np.float32)),
            weights=_dev(pack_decoder(scene["decoder"])))
        if tonemap is not None:
            self.params["tonemap"] = (tonemap.detach().clone().float().contiguous()
                                      if torch.is_tensor(tonemap) else _dev(tonemap))
        for t in self.params.values():
            t.requires_grad_(True)
        self.target = None if target is None else (target if torch.is_tensor(target) else _dev(target))
        if self.target is not None:
            V, H, W = len(self.views), self.views[0].height, self.views[0].width
            if tuple(self.target.shape) != (V, 3, H, W):
                raise ValueError(f"target must be [{V}][3][{H}][{W}]")
        self.widths = scene["decoder"]["widths"]
        self.n, self.np = g["n"], p["n"]
        # size the workspaces with counting passes at the initial parameters
        with torch.no_grad():
            cov, op = api.bake_gaussians(self.params["logscale"], self.params["quat"],
                                         self.params["logit"])
            ws = api.RenderWorkspace(self.n, self.views, self.opts, 1)
            r = api.render_gaussians(self.params["mean"], cov, op, self.params["sh"], self.deg,
                                     self.views, self.opts, ws)
            self.rws = api.RenderWorkspace(self.n, self.views, self.opts,
                                           int(ws.pair_count() * pair_margin) + 4096)
            sws = api.SplatWorkspace(self.np, self.views, self.crops, self.levels, 1)
            feat_h = self.params["feat"].to(torch.float16).view(torch.int16)
            api.splat_points(self.params["pos"], self.params["radius"], feat_h, None, self.views,
                             self.crops, self.levels, r["depth"] if cull else None,
                             r["tfinal"] if cull else None, sws)
            self.sws = api.SplatWorkspace(self.np, self.views, self.crops, self.levels,
                                          int(sws.frag_count() * frag_margin) + 4096)
        self.dws = api.DecoderWorkspace(self.widths, self.crops, decoder_dtype)

    def forward(self):
        from .autograd import (BakeGaussians, CompositeFrame, DecodeFovea, Dssim, L1Loss,
                               Regulariser, RenderGaussians, SplatPoints, Tonemap)
        P = self.params
        cov, op = BakeGaussians.apply(P["logscale"], P["quat"], P["logit"])
        rgb, depth, tfinal = RenderGaussians.apply(P["mean"], cov, op, P["sh"], self.deg,
                                                   self.views, self.opts, self.rws)
        pyr = SplatPoints.apply(P["pos"], P["radius"], P["feat"], None, self.views, self.crops,
                                self.levels, depth.detach() if self.cull else None,
                                tfinal if self.cull else None, self.sws)
        fovea = DecodeFovea.apply(pyr, rgb, P["weights"], self.levels, self.views, self.crops,
                                  self.dws)
        out = CompositeFrame.apply(rgb, fovea, self.crops, api.BLEND_LINEAR, self.ring, 0.75, 0.2)
        if "tonemap" in P:
            out = Tonemap.apply(out, P["tonemap"], self.views)
        self.last = dict(out=out, fovea=fovea, rgb=rgb)
        if self.target is None:
            return out, None
        pred, tgt = out, self.target
        if self.mask is not None:
            pred, tgt = out * self.mask, self.target * self.mask
        l1 = L1Loss.apply(pred, tgt)
        if self.loss_kind == "l1":
            return out, l1
        loss = (1.0 - self.lam) * l1 + self.lam * Dssim.apply(pred, tgt)
        if self.crops:
            loss = loss + self.beta * Regulariser.apply(fovea, rgb, self.crops)
        return out, loss

    def step(self, lr: float = 0.0, optimizer: str = "sgd"):
        for t in self.params.values():
            t.grad = None
        out, loss = self.forward()
        loss.backward()
        if lr and optimizer == "adam":
            self.adam_t += 1
            for k, t in self.params.items():
                if k not in self.adam_state:
                    self.adam_state[k] = (torch.zeros_like(t), torch.zeros_like(t))
                m, v = self.adam_state[k]
                api.adam_step(t.data, t.grad.contiguous(), m, v, self.adam_t, lr)
        elif lr:
            with torch.no_grad():
                for t in self.params.values():
                    t -= lr * t.grad
        return loss

    def status(self) -> int:
        return max(int(self.rws.status.item()), int(self.sws.status.item()))
