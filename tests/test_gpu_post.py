"""Tone mapping (Sec. 3.4, ADOP camera model as read in oracle/post.py) and
the training objective's kernels (Sec. 3.5, Eqs. 6-7: D-SSIM, the
regulariser R, Adam) against the FP64 reference, through the C-ABI."""
import numpy as np
import pytest
import torch

from oracle import post
from paper_2410_17932_amd import api, synth

from gpu_helpers import dev

pytestmark = pytest.mark.gpu


def _views(W, H, nv=2):
    return [synth.pinhole(W, H, 150.0, (0.03 * i, 0, 0)) for i in range(nv)]


def _params(rng, nv, n):
    p = post.gamma_params(nv, n)
    p[:, 0] = rng.uniform(-0.6, 0.6, nv)
    p[:, 1:4] = rng.uniform(0.7, 1.3, (nv, 3))
    p[:, 4:7] = rng.uniform(-0.3, 0.3, (nv, 3))
    p[:, 7:] = np.sort(rng.uniform(0, 1, (nv, n)), axis=1)
    return p.astype(np.float32)


def _principal(views):
    return np.array([[v.cx, v.cy] for v in views], np.float64)


@pytest.mark.parametrize("W,H,n", [(200, 136, 32), (37, 23, 2), (64, 48, 256)])
def test_tonemap_forward(W, H, n):
    rng = np.random.default_rng(W + n)
    views = _views(W, H)
    x = rng.uniform(-0.2, 1.4, (2, 3, H, W)).astype(np.float32)
    p = _params(rng, 2, n)
    want, _ = post.tonemap(x, p, _principal(views))
    got = api.tonemap(dev(x), views, dev(p)).cpu().numpy()
    assert np.abs(got - want).max() < 2e-6
    # in place
    xi = dev(x)
    api.tonemap(xi, views, dev(p), out=xi)
    assert np.array_equal(xi.cpu().numpy(), got)


def test_tonemap_backward():
    rng = np.random.default_rng(3)
    W, H, n = 200, 136, 32
    views = _views(W, H)
    x = rng.uniform(-0.2, 1.4, (2, 3, H, W)).astype(np.float32)
    p = _params(rng, 2, n)
    g = rng.normal(0, 1, x.shape).astype(np.float32)
    d_img, d_par = post.tonemap_backward(x, p, _principal(views), g)
    di = torch.full(x.shape, 7.0, device="cuda")          # written, not accumulated
    dp = dev(np.full(p.shape, 0.5, np.float32))           # accumulated
    api.tonemap_backward(dev(x), views, dev(p), dev(g), d_img=di, d_params=dp)
    di, dp = di.cpu().numpy(), dp.cpu().numpy() - 0.5
    assert np.abs(di - d_img).max() < 1e-5 * max(1.0, np.abs(d_img).max())
    scale = np.abs(d_par).max(axis=1, keepdims=True)
    assert np.abs(dp - d_par).max() < 2e-4 * scale.max()
    # each gradient alone
    di2 = torch.zeros_like(torch.as_tensor(x, device="cuda"))
    api.tonemap_backward(dev(x), views, dev(p), dev(g), d_img=di2)
    assert np.array_equal(di2.cpu().numpy(), di)
    dp2 = torch.zeros(p.shape, device="cuda")
    api.tonemap_backward(dev(x), views, dev(p), dev(g), d_params=dp2)
    assert np.abs(dp2.cpu().numpy() - d_par).max() < 2e-4 * scale.max()


def test_tonemap_full_frame():
    """The stereo frame (2 x 2016 x 2240) with the gamma initialisation and
    a non-trivial exposure, vignetting and white balance."""
    rng = np.random.default_rng(4)
    views = synth.stereo_rig(2016, 2240, 1100.0)
    x = rng.uniform(0, 1.2, (2, 3, 2240, 2016)).astype(np.float32)
    p = post.gamma_params(2, 32)
    p[:, 0] = 0.3
    p[:, 1:4] = [1.1, 0.95, 0.9]
    p[:, 4:7] = [-0.2, 0.05, -0.01]
    p = p.astype(np.float32)
    want, _ = post.tonemap(x, p, _principal(views))
    got = api.tonemap(dev(x), views, dev(p)).cpu().numpy()
    assert np.abs(got - want).max() < 2e-6


@pytest.mark.parametrize("planes,H,W", [(6, 70, 90), (1, 5, 7), (3, 64, 32)])
def test_dssim_forward_and_backward(planes, H, W):
    rng = np.random.default_rng(planes * 100 + W)
    x = rng.uniform(0, 1, (planes, H, W)).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.15, x.shape), 0, 1).astype(np.float32)
    ws = api.DssimWorkspace(planes, W, H)
    loss = api.dssim(dev(x), dev(y), ws).item()
    assert abs(loss - post.dssim(x, y)) < 2e-6
    want = post.dssim_backward(x, y) * 2.5
    dx = torch.full(x.shape, 0.25, device="cuda")
    api.dssim_backward(dev(x), dev(y), ws, dx, d_loss=torch.tensor([2.5], device="cuda"))
    got = dx.cpu().numpy() - 0.25
    assert np.abs(got - want).max() < 1e-3 * np.abs(want).max() + 1e-12


def test_dssim_fitting_views():
    """Four 1024^2 RGB views (the fitting step's cameras)."""
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, (12, 1024, 1024)).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1).astype(np.float32)
    ws = api.DssimWorkspace(12, 1024, 1024)
    loss = api.dssim(dev(x), dev(y), ws).item()
    assert abs(loss - post.dssim(x, y)) < 2e-6
    dx = torch.zeros(x.shape, device="cuda")
    api.dssim_backward(dev(x), dev(y), ws, dx)
    got = dx.cpu().numpy()
    # sampled: the gradient at a pixel depends on x and y within 10 pixels
    # (two blurs of radius 5), so the reference over a 64 x 64 window whose
    # cut edges are 32 pixels away gives it exactly (rescaled from the
    # window's element count to the whole input's)
    for (c, i, j) in [(0, 0, 0), (5, 500, 700), (11, 1023, 1023), (7, 30, 1000)]:
        i0, j0 = max(0, i - 32), max(0, j - 32)
        xs = x[c, i0:i0 + 64, j0:j0 + 64][None]
        ys = y[c, i0:i0 + 64, j0:j0 + 64][None]
        full = post.dssim_backward(xs, ys) * xs.size / x.size
        assert abs(got[c, i, j] - full[0, i - i0, j - j0]) < 1e-3 * np.abs(full).max()


def test_regulariser_forward_and_backward():
    rng = np.random.default_rng(6)
    V, H, W = 2, 136, 200
    P = rng.uniform(0, 1, (V, 3, H, W)).astype(np.float32)
    spec = [(0, 10, 20, 64), (0, 40, 30, 32), (1, 100, 50, 64)]   # the first two overlap
    crops = [synth.Crop(v, x0, y0, s, x0 + s / 2, y0 + s / 2) for (v, x0, y0, s) in spec]
    F = [rng.uniform(0, 1, (3, s, s)).astype(np.float32) for (_, _, _, s) in spec]
    Fp = np.concatenate([f.ravel() for f in F])
    want, diff = post.regulariser(F, P, spec)
    r = api.regulariser(dev(Fp), dev(P), crops)
    rr = r.cpu().numpy()
    assert abs(rr[0] - want) < 1e-6 and abs(rr[1] - diff) < 1e-6
    dF, dP = post.regulariser_backward(F, P, spec, d_r=3.0)
    dfo = torch.zeros(Fp.shape, device="cuda")
    dpe = torch.ones(P.shape, device="cuda")
    api.regulariser_backward(P.shape, crops, r, d_r=torch.tensor([3.0], device="cuda"),
                             d_fovea=dfo, d_periphery=dpe)
    assert np.abs(dfo.cpu().numpy() - np.concatenate([f.ravel() for f in dF])).max() < 1e-9
    # accumulated into 1.0 in single precision: within half an ulp of 1
    assert np.abs(dpe.cpu().numpy() - 1.0 - dP).max() < 6e-8
    # origins from a device placement table
    place = torch.tensor([[12, 22, 0, 0], [40, 30, 0, 0], [100, 50, 0, 0]], dtype=torch.int32,
                         device="cuda")
    spec2 = [(0, 12, 22, 64), (0, 40, 30, 32), (1, 100, 50, 64)]
    want2, _ = post.regulariser(F, P, spec2)
    r2 = api.regulariser(dev(Fp), dev(P), crops, place=place).cpu().numpy()
    assert abs(r2[0] - want2) < 1e-6


def test_adam_steps():
    rng = np.random.default_rng(7)
    n = 1_000_003    # a tail past the four-wide body
    p = rng.normal(0, 1, n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    tp, tm, tv = dev(p), dev(m), dev(v)
    rp, rm, rv = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 6):
        g = rng.normal(0, 1e-2, n).astype(np.float32)
        api.adam_step(tp, dev(g), tm, tv, step, lr=1e-3, eps=1e-8)
        rp, rm, rv = post.adam(rp, g, rm, rv, step, lr=1e-3, eps=1e-8)
    assert np.abs(tp.cpu().numpy() - rp).max() < 1e-6
    assert np.abs(tm.cpu().numpy() - rm).max() < 1e-8
    assert np.abs(tv.cpu().numpy() - rv).max() < 1e-10
