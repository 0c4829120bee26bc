"""GPU adjoint kernels against the analytic FP64 gradients of the
differentiable reference (oracle/diff.py, itself pinned by central
differences).  Error measure per element:
    rel = |g - g_ref| / max(|g_ref|, 1e-3 max|g_ref|)
float32 adjoints within 1e-3 (bake, periphery, splat, decoder FP32,
combination), the BF16 decoder within 2e-2 of the largest magnitude."""
import numpy as np
import pytest
import torch

import oracle
from oracle import diff
from paper_2410_17932_amd import api, synth
from paper_2410_17932_amd.autograd import (BakeGaussians, CompositeFrame, DecodeFovea, L1Loss,
                                           RenderGaussians, SplatPoints)

from gpu_helpers import baked, dev, oracle_render, pair_total

pytestmark = pytest.mark.gpu
DT = torch.float64


def _rel(g, ref, floor=1e-3):
    g, ref = np.asarray(g, np.float64), np.asarray(ref, np.float64)
    den = np.maximum(np.abs(ref), floor * max(np.abs(ref).max(), 1e-30))
    return float((np.abs(g - ref) / den).max())


def _p(a):
    return torch.tensor(np.asarray(a), dtype=DT, requires_grad=True)


def test_bake_backward():
    rng = np.random.default_rng(2)
    g = synth.gaussians(rng, 3000, 0)
    P = [_p(g["logscale"]), _p(g["quat"]), _p(g["logit"])]
    cov, op = diff.bake(*P)
    wc, wo = rng.normal(size=cov.shape), rng.normal(size=op.shape)
    ((cov * torch.tensor(wc)).sum() * 100 + (op * torch.tensor(wo)).sum()).backward()
    T = [dev(g["logscale"]).requires_grad_(), dev(g["quat"]).requires_grad_(),
         dev(g["logit"]).requires_grad_()]
    c2, o2 = BakeGaussians.apply(*T)
    ((c2 * dev(wc, torch.float32)).sum() * 100 + (o2 * dev(wo, torch.float32)).sum()).backward()
    for a, b in zip(T, P):
        assert _rel(a.grad.cpu().numpy(), b.grad.numpy()) <= 1e-3


@pytest.mark.parametrize("deg,tile", [(0, 16), (3, 16), (1, 8)])
def test_render_backward(deg, tile):
    sc = synth.small_scene(51 + deg, n_gauss=400, width=72, height=56, f=64.0, sh_degree=deg,
                           n_views=2)
    g, views = sc["gaussians"], sc["views"]
    raster = dict(sc["raster"], tile=tile)
    cov, op = baked(g)
    o, rect, zb = oracle_render(g, cov, op, views, raster)
    V, D = synth.views_array(views), synth.views_dims(views)
    rng = np.random.default_rng(3)
    ok = o["margin"] >= 1e-4                    # unambiguous pixels only
    cr = rng.normal(size=o["rgb"].shape) * ok[:, None]
    cd = rng.normal(size=o["depth"].shape) * ok * 0.1
    # reference
    pix = np.array([(v, x, y) for v in range(2) for y in range(56) for x in range(72)])
    P = dict(mean=_p(g["mean"]), cov=_p(cov), op=_p(op), sh=_p(g["sh"]))
    out = diff.render(P["mean"], P["cov"], P["op"], P["sh"], deg, V, D, pix, raster)
    crt = torch.tensor(cr.transpose(0, 2, 3, 1).reshape(-1, 3))
    cdt = torch.tensor(cd.reshape(-1))
    ((out["rgb"] * crt).sum() + (out["depth"] * cdt).sum()).backward()
    # GPU
    opts = api.make_opts(**raster)
    ws = api.RenderWorkspace(g["n"], views, opts, pair_total(rect, D, tile) + 64)
    T = dict(mean=dev(g["mean"]).requires_grad_(), cov=dev(cov).requires_grad_(),
             op=dev(op).requires_grad_(), sh=dev(g["sh"]).requires_grad_())
    rgb, depth, _ = RenderGaussians.apply(T["mean"], T["cov"], T["op"], T["sh"], deg, views, opts, ws)
    ((rgb * dev(cr, torch.float32)).sum() + (depth * dev(cd, torch.float32)).sum()).backward()
    for k in P:
        r = _rel(T[k].grad.cpu().numpy(), P[k].grad.numpy())
        print(f"render deg {deg} tile {tile} d_{k}: rel {r:.2e}")
        assert r <= 1e-3, k


@pytest.mark.parametrize("rotated,with_op", [(False, True), (True, False)])
def test_splat_backward(rotated, with_op):
    rng = np.random.default_rng(6)
    rot = synth.yaw_pitch(8.0, -6.0) if rotated else None
    views = [synth.pinhole(96, 80, 90.0, rot=rot),
             synth.pinhole(96, 80, 90.0, (0.05, 0.1, -0.2), rot=rot)]
    V, D = synth.views_array(views), synth.views_dims(views)
    p = synth.points(rng, 1500, "uniform")
    p["radius"] = (p["radius"] * 2.5).astype(np.float32)
    crops = [synth.crop_at(0, 40.0, 40.0, 32, 96, 80), synth.crop_at(1, 60.0, 30.0, 48, 96, 80),
             synth.crop_at(0, 50.0, 45.0, 64, 96, 80)]
    ci, _ = synth.crops_array(crops)
    op = rng.uniform(0.3, 1.0, 1500).astype(np.float32)
    L = 3
    feat = p["feat"].view(np.float16).astype(np.float64)
    P = dict(pos=_p(p["pos"]), r=_p(p["radius"]), feat=_p(feat))
    if with_op:
        P["op"] = _p(op)
    pyr = diff.splat(P["pos"], P["r"], P["feat"], P.get("op"), V, D, ci, L)
    cot = rng.normal(size=tuple(pyr.shape))
    (pyr * torch.tensor(cot)).sum().backward()
    nf = len(oracle.point_frags(p["pos"], p["radius"], V, D, ci, L))
    ws = api.SplatWorkspace(1500, views, crops, L, nf + 64)
    T = dict(pos=dev(p["pos"]).requires_grad_(), r=dev(p["radius"]).requires_grad_(),
             feat=dev(feat, torch.float32).requires_grad_())
    if with_op:
        T["op"] = dev(op).requires_grad_()
    out = SplatPoints.apply(T["pos"], T["r"], T["feat"], T.get("op"), views, crops, L, None, None, ws)
    np.testing.assert_allclose(out.detach().cpu().numpy(), pyr.detach().numpy(), atol=1e-4)
    (out * dev(cot, torch.float32)).sum().backward()
    for k in P:
        r = _rel(T[k].grad.cpu().numpy(), P[k].grad.numpy())
        print(f"splat d_{k}: rel {r:.2e}")
        assert r <= 1e-3, k


@pytest.mark.parametrize("widths,L", [((16, 32), 3), ((16, 32, 64, 64), 4)])
@pytest.mark.parametrize("dtype,tol", [(api.VRS_F32, 1e-3), (api.VRS_BF16, 2e-2)])
def test_decoder_backward(dtype, tol, widths, L):
    rng = np.random.default_rng(8)
    dw = synth.decoder_weights(rng, widths, 4)
    packed = synth.pack_decoder(dw)
    packed = (packed + rng.normal(0, 0.05, packed.shape)).astype(np.float32)
    W, H = 120, 100
    views = [synth.pinhole(W, H, 100.0), synth.pinhole(W, H, 100.0, (0.05, 0, 0))]
    crops = [synth.crop_at(0, 40.0, 40.0, 32, W, H), synth.crop_at(1, 70.0, 50.0, 48, W, H)]
    if L == 4:
        crops = [synth.crop_at(0, 40.0, 40.0, 32, W, H), synth.crop_at(1, 70.0, 50.0, 64, W, H)]
    ci, _ = synth.crops_array(crops)
    pyr = rng.normal(size=(oracle.pyramid_pixels(ci, L), 4)).astype(np.float32)
    per = rng.uniform(size=(2, 3, H, W)).astype(np.float32)
    P = dict(pyr=_p(pyr), per=_p(per), w=_p(packed))
    lv, hd = diff.unpack_decoder(P["w"], widths)
    out = diff.decode(P["pyr"], P["per"], ci, L, widths, lv, hd)
    cot = rng.normal(size=tuple(out.shape))
    (out * torch.tensor(cot)).sum().backward()
    ws = api.DecoderWorkspace(widths, crops, dtype)
    T = dict(pyr=dev(pyr).requires_grad_(), per=dev(per).requires_grad_(),
             w=dev(packed).requires_grad_())
    o2 = DecodeFovea.apply(T["pyr"], T["per"], T["w"], L, views, crops, ws)
    (o2 * dev(cot, torch.float32)).sum().backward()
    for k in P:
        g, ref = T[k].grad.cpu().numpy(), P[k].grad.numpy()
        if dtype == api.VRS_F32:
            r = _rel(g, ref)
        else:
            r = float(np.abs(g - ref).max() / np.abs(ref).max())
        print(f"decoder dtype {dtype} d_{k}: err {r:.2e}")
        assert r <= tol, k


@pytest.mark.parametrize("mode", [api.BLEND_LINEAR, api.BLEND_PAPER])
def test_composite_and_l1_backward(mode):
    rng = np.random.default_rng(9)
    W, H = 90, 70
    crops = [synth.crop_at(0, 30.3, 30.1, 32, W, H), synth.crop_at(0, 40.0, 36.0, 48, W, H),
             synth.crop_at(1, 60.0, 20.0, 16, W, H)]
    ci, cf = synth.crops_array(crops)
    P0 = rng.uniform(size=(2, 3, H, W))
    F0 = rng.uniform(size=sum(3 * c.size ** 2 for c in crops))
    tgt = rng.uniform(size=P0.shape)
    P = dict(P=_p(P0), F=_p(F0))
    out = diff.composite(P["P"], P["F"], ci, cf, mode=mode, ring=8.0)
    diff.l1(out, torch.tensor(tgt)).backward()
    T = dict(P=dev(P0, torch.float32).requires_grad_(), F=dev(F0, torch.float32).requires_grad_())
    o2 = CompositeFrame.apply(T["P"], T["F"], crops, mode, 8.0, 0.75, 0.2)
    loss = L1Loss.apply(o2, dev(tgt, torch.float32))
    assert abs(float(loss) - float(diff.l1(out, torch.tensor(tgt)))) < 1e-5
    loss.backward()
    for k in P:
        r = _rel(T[k].grad.cpu().numpy(), P[k].grad.numpy())
        print(f"composite mode {mode} d_{k}: rel {r:.2e}")
        assert r <= 1e-3, k


def test_backward_detects_overwritten_workspace():
    """A second forward through the same workspace before the first one's
    backward would leave the backward replaying the wrong lists: it raises."""
    sc = synth.small_scene(52, n_gauss=200, width=48, height=40, f=48.0)
    g, views = sc["gaussians"], sc["views"]
    cov, op = baked(g)
    opts = api.make_opts(**sc["raster"])
    V, D = synth.views_array(views), synth.views_dims(views)
    rect, _ = oracle.gauss_geom32(g["mean"], cov, V, D)
    ws = api.RenderWorkspace(g["n"], views, opts, pair_total(rect, D, 16) + 64)
    m = dev(g["mean"]).requires_grad_()
    args = (dev(cov), dev(op), dev(g["sh"]), 0, views, opts, ws)
    rgb1, _, _ = RenderGaussians.apply(m, *args)
    rgb2, _, _ = RenderGaussians.apply(m, *args)
    rgb2.sum().backward(retain_graph=True)       # the latest forward: fine
    with pytest.raises(RuntimeError, match="overwritten"):
        rgb1.sum().backward()
