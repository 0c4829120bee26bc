"""Pins of the differentiable FP64 reference (oracle/diff.py): each forward
equals the C++ reference's forward, and each autograd gradient equals FP64
central differences of that forward (coordinates whose discrete decisions
flip inside the difference interval are skipped and counted)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import diff
from paper_2410_17932_amd import synth

DT = torch.float64


def _fd_check(fn, params, n_coords=24, seed=0, rtol=1e-6, max_skip=0.3):
    """fn(params) -> (loss, decisions); compares autograd with central
    differences on random coordinates of every parameter."""
    loss, dec0 = fn(params)
    grads = torch.autograd.grad(loss, list(params.values()), allow_unused=True)
    rng = np.random.default_rng(seed)
    tested = skipped = 0
    for (name, p), g in zip(params.items(), grads):
        g = torch.zeros_like(p) if g is None else g
        flat = p.detach().reshape(-1)
        gflat = g.reshape(-1)
        scale = float(gflat.abs().max())
        idx = rng.choice(flat.numel(), size=min(n_coords, flat.numel()), replace=False)
        for i in idx:
            th = float(flat[i])
            h = 1e-6 * max(1.0, abs(th))
            vals = []
            decs = []
            for sgn in (1, -1):
                q = {k: v.detach().clone() for k, v in params.items()}
                q[name].reshape(-1)[i] = th + sgn * h
                l, d = fn(q)
                vals.append(float(l))
                decs.append(d)
            if not (_same(decs[0], dec0) and _same(decs[1], dec0)):
                skipped += 1
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            ref = float(gflat[i])
            denom = max(abs(ref), 1e-3 * scale, 1e-300)
            # rounding of the loss itself bounds what a difference can resolve
            fd_noise = 8 * np.finfo(np.float64).eps * max(abs(vals[0]), abs(vals[1])) / h
            assert abs(fd - ref) <= rtol * denom + fd_noise, f"{name}[{i}]: fd {fd} vs autograd {ref}"
            tested += 1
    assert tested > 0 and skipped <= max_skip * (tested + skipped), (tested, skipped)
    return tested, skipped


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def _params(**kw):
    return {k: torch.tensor(np.asarray(v), dtype=DT, requires_grad=True) for k, v in kw.items()}


# ------------------------------------------------------------------ bake
def test_bake_forward_and_gradient():
    rng = np.random.default_rng(1)
    g = synth.gaussians(rng, 50, 0)
    cov_c, op_c = oracle.bake(g["logscale"], g["quat"], g["logit"])
    P = _params(ls=g["logscale"], q=g["quat"], lo=g["logit"])
    cov, op = diff.bake(P["ls"], P["q"], P["lo"])
    np.testing.assert_allclose(cov.detach().numpy(), cov_c, rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(op.detach().numpy(), op_c, rtol=1e-12)
    wc = torch.tensor(rng.normal(size=cov.shape))
    wo = torch.tensor(rng.normal(size=op.shape))

    def fn(p):
        c, o = diff.bake(p["ls"], p["q"], p["lo"])
        return (c * wc).sum() * 1e4 + (o * wo).sum(), ()
    _fd_check(fn, P)


# --------------------------------------------------------------- render
def _render_setup(seed, n=120, W=40, H=32, f=40.0, deg=1, nv=2):
    sc = synth.small_scene(seed, n_gauss=n, width=W, height=H, f=f, sh_degree=deg, n_views=nv)
    g = sc["gaussians"]
    cov, op = oracle.bake(g["logscale"], g["quat"], g["logit"])
    V, D = synth.views_array(sc["views"]), synth.views_dims(sc["views"])
    return sc, g, cov.astype(np.float32), op.astype(np.float32), V, D


def test_render_forward_matches_cpp():
    sc, g, cov, op, V, D = _render_setup(2)
    raster = sc["raster"]
    rect, zb = oracle.gauss_geom32(g["mean"], cov, V, D)
    rec = oracle.gauss_project64(g["mean"], cov, op, g["sh"], 1, V, D)
    ref = oracle.render(rect, zb, rec, D)
    pix = np.array([(v, x, y) for v in range(2) for y in range(32) for x in range(40)])
    P = _params(mean=g["mean"], cov=cov, op=op, sh=g["sh"])
    out = diff.render(P["mean"], P["cov"], P["op"], P["sh"], 1, V, D, pix, raster)
    np.testing.assert_allclose(out["rgb"].detach().numpy().reshape(2, 32, 40, 3),
                               ref["rgb"].transpose(0, 2, 3, 1), atol=1e-12)
    np.testing.assert_allclose(out["depth"].detach().numpy().reshape(2, 32, 40), ref["depth"], atol=1e-11)
    np.testing.assert_allclose(out["tfinal"].detach().numpy().reshape(2, 32, 40), ref["tfinal"], atol=1e-12)


def test_render_cut_at_reach_is_identical():
    """Cutting each pixel's list after its evaluation count (the entries past
    the stop are never reached) leaves the forward and its gradient as they
    are; an opaque scene makes most pixels stop early."""
    sc, g, cov, op, V, D = _render_setup(4, n=500)
    op = np.full_like(op, 0.99)
    cov = (cov * 8).astype(np.float32)
    raster = sc["raster"]
    rect, zb = oracle.gauss_geom32(g["mean"], cov, V, D)
    rec = oracle.gauss_project64(g["mean"], cov, op, g["sh"], 1, V, D)
    ref = oracle.render(rect, zb, rec, D)
    pix = np.array([(v, x, y) for v in range(2) for y in range(32) for x in range(40)])
    reach = ref["evals"][pix[:, 0], pix[:, 2], pix[:, 1]]
    full_len = diff.pixel_lists(rect, zb, pix)[1].sum(1)
    assert (reach < full_len).mean() > 0.3
    rng = np.random.default_rng(1)
    cr = torch.tensor(rng.normal(size=(len(pix), 3)))
    grads = []
    for r in (None, reach):
        P = _params(mean=g["mean"], cov=cov, op=op, sh=g["sh"])
        out = diff.render(P["mean"], P["cov"], P["op"], P["sh"], 1, V, D, pix, raster, reach=r)
        (out["rgb"] * cr).sum().backward()
        grads.append((out, {k: v.grad.clone() for k, v in P.items()}))
    (a, ga), (b, gb) = grads
    for k in ("rgb", "depth", "tfinal"):
        assert torch.equal(a[k], b[k]), k
    for k in ga:
        torch.testing.assert_close(ga[k], gb[k], rtol=1e-12, atol=1e-15)


def test_render_gradient_central_differences():
    sc, g, cov, op, V, D = _render_setup(3, n=60, W=24, H=20, f=24.0, deg=2, nv=1)
    raster = sc["raster"]
    pix = np.array([(0, x, y) for y in range(20) for x in range(24)])
    rng = np.random.default_rng(0)
    cr = torch.tensor(rng.normal(size=(len(pix), 3)))
    cd = torch.tensor(rng.normal(size=len(pix)))

    def fn(p):
        out = diff.render(p["mean"], p["cov"], p["op"], p["sh"], 2, V, D, pix, raster)
        rect, zb = oracle.gauss_geom32(diff._f32(p["mean"]), diff._f32(p["cov"]), V, D)
        idx, valid = diff.pixel_lists(rect, zb, pix)
        # threshold decisions at the float64 values
        with torch.no_grad():
            dec = (idx, valid, np.round(out["tfinal"].numpy() * 0, 0))
        return (out["rgb"] * cr).sum() + (out["depth"] * cd).sum(), dec + _blend_decisions(p, pix, raster, V, D)

    P = _params(mean=g["mean"], cov=cov, op=op, sh=g["sh"])
    tested, skipped = _fd_check(fn, P, n_coords=16)
    print("render coords tested", tested, "skipped", skipped)


def _blend_decisions(p, pix, raster, V, D):
    """Skip / stop masks of every pixel list at the current parameters."""
    with torch.no_grad():
        rect, zb = oracle.gauss_geom32(diff._f32(p["mean"]), diff._f32(p["cov"]), V, D)
        rec = oracle.gauss_project64(diff._f32(p["mean"]), diff._f32(p["cov"]),
                                     diff._f32(p["op"]), diff._f32(p["sh"]), 2, V, D)
        o = oracle.render(rect, zb, rec, D, pix=pix.astype(np.int32))
    return (o["ncontrib"], o["evals"])


# ---------------------------------------------------------------- splat
def _splat_setup(seed, n=150):
    rng = np.random.default_rng(seed)
    cam = synth.pinhole(48, 40, 48.0)
    V, D = synth.views_array([cam]), synth.views_dims([cam])
    p = synth.points(rng, n, "uniform")
    p["radius"] = (p["radius"] * 3).astype(np.float32)
    crops = np.array([[0, 4, 2, 32], [0, 10, 8, 24]], np.int32)
    op = rng.uniform(0.3, 1.0, n).astype(np.float32)
    return p, V, D, crops, op


def test_splat_forward_matches_cpp():
    p, V, D, crops, op = _splat_setup(4)
    ref = oracle.splat_points(p["pos"], p["radius"], p["feat"], V, D, crops, 3, opacity=op)
    P = _params(pos=p["pos"], r=p["radius"], op=op,
                feat=p["feat"].view(np.float16).astype(np.float64))
    out = diff.splat(P["pos"], P["r"], P["feat"], P["op"], V, D, crops, 3)
    np.testing.assert_allclose(out.detach().numpy(), ref, atol=1e-12)


def test_splat_gradient_central_differences():
    p, V, D, crops, op = _splat_setup(5, n=80)
    P = _params(pos=p["pos"], r=p["radius"], op=op,
                feat=p["feat"].view(np.float16).astype(np.float64))
    cot = torch.tensor(np.random.default_rng(1).normal(size=(oracle.pyramid_pixels(crops, 3), 4)))

    def fn(q):
        out = diff.splat(q["pos"], q["r"], q["feat"], q["op"], V, D, crops, 3)
        fr = oracle.point_frags(diff._f32(q["pos"]), diff._f32(q["r"]), V, D, crops, 3)
        return (out * cot).sum(), (fr,)
    tested, skipped = _fd_check(fn, P, n_coords=20)
    print("splat coords tested", tested, "skipped", skipped)


# -------------------------------------------------------------- decoder
def test_decoder_forward_and_gradient():
    rng = np.random.default_rng(6)
    widths, L = (6, 5), 3
    dw = synth.decoder_weights(rng, widths, 4)
    packed = synth.pack_decoder(dw).astype(np.float64)
    packed += rng.normal(0, 0.05, packed.shape)          # non-zero biases too
    crops = np.array([[0, 2, 3, 16], [0, 0, 0, 8]], np.int32)
    Ppix = oracle.pyramid_pixels(crops, L)
    pyr = rng.normal(size=(Ppix, 4))
    periph = rng.uniform(size=(1, 3, 24, 24))
    ref = oracle.decode(crops, L, 4, pyr, periph, np.array([[24, 24]], np.int32), widths, packed)
    P = _params(pyr=pyr, per=periph, w=packed)
    lv, hd = diff.unpack_decoder(P["w"], widths)
    out = diff.decode(P["pyr"], P["per"], crops, L, widths, lv, hd)
    np.testing.assert_allclose(out.detach().numpy(), ref, atol=1e-12)
    cot = torch.tensor(rng.normal(size=out.shape))

    def fn(q):
        lv, hd = diff.unpack_decoder(q["w"], widths)
        return (diff.decode(q["pyr"], q["per"], crops, L, widths, lv, hd) * cot).sum(), ()
    _fd_check(fn, P, n_coords=16)


# ------------------------------------------------------------ composite
@pytest.mark.parametrize("mode", [0, 1])
def test_composite_forward_and_gradient(mode):
    rng = np.random.default_rng(7)
    W, H = 40, 36
    crops = [synth.crop_at(0, 14.3, 15.1, 16, W, H), synth.crop_at(0, 20.0, 18.0, 24, W, H),
             synth.crop_at(1, 30.0, 10.0, 8, W, H)]
    ci, cf = synth.crops_array(crops)
    P0 = rng.uniform(size=(2, 3, H, W))
    F0 = rng.uniform(size=sum(3 * c.size ** 2 for c in crops))
    ref = oracle.composite(P0, np.array([[W, H], [W, H]], np.int32), ci, cf, F0, mode=mode,
                           ring=6.0)
    P = _params(P=P0, F=F0)
    out = diff.composite(P["P"], P["F"], ci, cf, mode=mode, ring=6.0)
    np.testing.assert_allclose(out.detach().numpy(), ref, atol=1e-12)
    cot = torch.tensor(rng.normal(size=out.shape))

    def fn(q):
        o = diff.composite(q["P"], q["F"], ci, cf, mode=mode, ring=6.0)
        return (o * cot).sum(), ()
    _fd_check(fn, P, n_coords=30)
