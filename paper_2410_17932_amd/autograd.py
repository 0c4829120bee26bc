"""torch.autograd.Function wrappers over the C-ABI, so the Gaussians, the
neural points and the decoder can be fitted end to end (Sec. 3.5).  Each
forward and each backward is one call into the HIP library; gradients land
in fresh zeroed tensors (the library accumulates into them).

A backward replays what its forward left in the caller's workspace (tile
lists, stop positions, fragment segments, activations): one forward per
workspace and backward.  The workspaces count their forward calls, and a
backward raises if another forward has run through its workspace since."""
from __future__ import annotations

import torch

from . import api


def _check_generation(ws, gen, what):
    if ws.generation != gen:
        raise RuntimeError(f"{what} backward: its workspace was overwritten by another forward "
                           f"call (use one workspace per forward kept for backward)")


class BakeGaussians(torch.autograd.Function):
    @staticmethod
    def forward(ctx, logscale, quat, logit):
        cov, op = api.bake_gaussians(logscale, quat, logit)
        ctx.save_for_backward(logscale, quat, logit)
        return cov, op

    @staticmethod
    def backward(ctx, d_cov, d_op):
        ls, q, lo = ctx.saved_tensors
        d_ls, d_q, d_lo = torch.zeros_like(ls), torch.zeros_like(q), torch.zeros_like(lo)
        d_op = torch.zeros_like(lo) if d_op is None else d_op.contiguous()
        api.bake_gaussians_backward(ls, q, lo, d_cov.contiguous(), d_op, d_ls, d_q, d_lo)
        return d_ls, d_q, d_lo


class RenderGaussians(torch.autograd.Function):
    """(mean, cov, opacity, sh) -> (rgb [V][3][H][W], depth, T_final)."""

    @staticmethod
    def forward(ctx, mean, cov, opacity, sh, sh_degree, views, opts, ws):
        out = api.render_gaussians(mean, cov, opacity, sh, sh_degree, views, opts, ws)
        ctx.save_for_backward(mean, cov, opacity, sh, out["tfinal"])
        ctx.meta = (sh_degree, views, opts, ws, ws.generation)
        ctx.mark_non_differentiable(out["tfinal"])
        return out["rgb"], out["depth"], out["tfinal"]

    @staticmethod
    def backward(ctx, d_rgb, d_depth, _d_t):
        mean, cov, op, sh, tf = ctx.saved_tensors
        deg, views, opts, ws, gen = ctx.meta
        _check_generation(ws, gen, "RenderGaussians")
        g = [torch.zeros_like(t) for t in (mean, cov, op, sh)]
        d_rgb = torch.zeros_like(tf).unsqueeze(1).expand(-1, 3, -1, -1).contiguous() \
            if d_rgb is None else d_rgb.contiguous()
        api.render_gaussians_backward(mean, cov, op, sh, deg, views, opts, ws, tf, d_rgb,
                                      None if d_depth is None else d_depth.contiguous(), *g)
        return (*g, None, None, None, None)


class SplatPoints(torch.autograd.Function):
    """(pos, radius, feat_f32, opacity) -> pyramid.  The half-precision
    feature bits are re-derived from feat_f32 (exactly representable values
    are expected); depth culling is a non-differentiable mask."""

    @staticmethod
    def forward(ctx, pos, radius, feat, opacity, views, crops, levels, depth, tfinal, ws):
        feat_h = feat.to(torch.float16).view(torch.int16).contiguous()
        pyr = api.splat_points(pos, radius, feat_h, opacity, views, crops, levels, depth, tfinal, ws)
        ctx.save_for_backward(pos, radius, opacity if opacity is not None else pos.new_empty(0))
        ctx.meta = (feat_h, views, crops, levels, ws, opacity is not None, ws.generation)
        return pyr

    @staticmethod
    def backward(ctx, d_pyr):
        pos, radius, op = ctx.saved_tensors
        feat_h, views, crops, levels, ws, has_op, gen = ctx.meta
        _check_generation(ws, gen, "SplatPoints")
        d_pos, d_r = torch.zeros_like(pos), torch.zeros_like(radius)
        d_feat = torch.zeros((pos.shape[1], 4), device=pos.device)
        d_op = torch.zeros_like(op) if has_op else None
        api.splat_points_backward(pos, radius, feat_h, op if has_op else None, views, crops,
                                  levels, d_pyr.contiguous(), ws, d_feat=d_feat, d_pos=d_pos,
                                  d_radius=d_r, d_opacity=d_op)
        return d_pos, d_r, d_feat, d_op, None, None, None, None, None, None


class DecodeFovea(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pyramid, periphery, weights, levels, views, crops, ws):
        out = api.decode_fovea(pyramid, levels, periphery, views, crops, weights, ws)
        ctx.save_for_backward(pyramid, periphery, weights)
        ctx.meta = (levels, views, crops, ws, ws.generation)
        return out

    @staticmethod
    def backward(ctx, d_out):
        pyr, per, w = ctx.saved_tensors
        levels, views, crops, ws, gen = ctx.meta
        _check_generation(ws, gen, "DecodeFovea")
        g = [torch.zeros_like(t) for t in (pyr, per, w)]
        api.decode_fovea_backward(pyr, levels, per, views, crops, w, ws, d_out.contiguous(), *g)
        return (*g, None, None, None, None)


class CompositeFrame(torch.autograd.Function):
    @staticmethod
    def forward(ctx, periphery, fovea, crops, mode, ring, m, gamma):
        out = api.composite_frame(periphery, fovea, crops, mode, ring, m, gamma)
        ctx.save_for_backward(periphery, fovea)
        ctx.meta = (crops, mode, ring, m, gamma)
        return out

    @staticmethod
    def backward(ctx, d_out):
        P, F = ctx.saved_tensors
        crops, mode, ring, m, gamma = ctx.meta
        dP, dF = torch.zeros_like(P), torch.zeros_like(F)
        api.composite_frame_backward(P, F, crops, d_out.contiguous(), dP, dF, mode, ring, m, gamma)
        return dP, dF, None, None, None, None, None


class L1Loss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pred, target):
        ctx.save_for_backward(pred, target)
        return api.l1_loss(pred.contiguous(), target.contiguous())[0]

    @staticmethod
    def backward(ctx, g):
        pred, target = ctx.saved_tensors
        d = torch.zeros_like(pred)
        api.l1_loss(pred.contiguous(), target.contiguous(), d_pred=d, scale=float(g))
        return d, None


class Tonemap(torch.autograd.Function):
    """vrs_tonemap with its adjoint (image and camera-model parameters)."""

    @staticmethod
    def forward(ctx, img, params, views):
        img, params = img.contiguous(), params.contiguous()
        ctx.save_for_backward(img, params)
        ctx.views = views
        return api.tonemap(img, views, params)

    @staticmethod
    def backward(ctx, g):
        img, params = ctx.saved_tensors
        d_img = torch.empty_like(img) if ctx.needs_input_grad[0] else None
        d_par = torch.zeros_like(params) if ctx.needs_input_grad[1] else None
        if d_img is not None or d_par is not None:
            api.tonemap_backward(img, ctx.views, params, g.contiguous(), d_img=d_img,
                                 d_params=d_par)
        return d_img, d_par, None


_DSSIM_WS = {}


def _dssim_ws(planes, W, H, device):
    key = (planes, W, H, str(device))
    if key not in _DSSIM_WS:
        _DSSIM_WS[key] = api.DssimWorkspace(planes, W, H, device)
    return _DSSIM_WS[key]


class Dssim(torch.autograd.Function):
    """D-SSIM (Eq. 6, as in 3DGS) of pred against target over [..][H][W]
    planes; the gradient flows to pred.  Scalar (0-d) result."""

    @staticmethod
    def forward(ctx, pred, target):
        pred, target = pred.contiguous(), target.contiguous()
        H, W = pred.shape[-2:]
        planes = pred.numel() // (H * W)
        ws = _dssim_ws(planes, W, H, pred.device)
        ctx.save_for_backward(pred, target)
        return api.dssim(pred, target, ws)[0].clone()

    @staticmethod
    def backward(ctx, g):
        pred, target = ctx.saved_tensors
        H, W = pred.shape[-2:]
        ws = _dssim_ws(pred.numel() // (H * W), W, H, pred.device)
        d = torch.zeros_like(pred)
        api.dssim_backward(pred, target, ws, d, d_loss=g.reshape(1).contiguous())
        return d, None


class Regulariser(torch.autograd.Function):
    """R of Eq. 7 (|mean F - mean crop(P)|) with its adjoint."""

    @staticmethod
    def forward(ctx, fovea, periphery, crops):
        fovea, periphery = fovea.contiguous(), periphery.contiguous()
        r = api.regulariser(fovea, periphery, crops)
        ctx.save_for_backward(r)
        ctx.crops, ctx.shape = crops, tuple(periphery.shape)
        ctx.fshape = fovea.shape
        return r[0].clone()

    @staticmethod
    def backward(ctx, g):
        (r,) = ctx.saved_tensors
        d_f = torch.zeros(ctx.fshape, device=r.device) if ctx.needs_input_grad[0] else None
        d_p = torch.zeros(ctx.shape, device=r.device) if ctx.needs_input_grad[1] else None
        api.regulariser_backward(ctx.shape, ctx.crops, r, d_r=g.reshape(1).contiguous(),
                                 d_fovea=d_f, d_periphery=d_p)
        return d_f, d_p, None
