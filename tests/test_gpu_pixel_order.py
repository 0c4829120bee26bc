"""The periphery in per-pixel order (Sec. 3.2, the popping fix) against the
reference's exact per-pixel sort: images within 1e-4, contributor counts
exact, near-threshold pixels equal to one of the reference's branch
results; tiles 8 and 16 and every digit width; a scene built to overflow the
per-pixel windows, so that the exact pass runs; and the full stereo frame on
sampled pixels."""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_17932_amd import api, synth

from gpu_helpers import baked, check_render, dev, gpu_render, oracle_render, pair_total

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case,tile,radix", [("tiny", 8, 8), ("ragged_stereo", 16, 8),
                                             ("sh3", 16, 11), ("sh3", 8, 4)])
def test_pixel_order_parity(case, tile, radix):
    if case == "tiny":
        sc = synth.config(0)
    elif case == "ragged_stereo":
        sc = synth.small_scene(21, n_gauss=3000, width=200, height=136, f=150.0, n_views=2)
    else:
        sc = synth.small_scene(22, n_gauss=2500, width=176, height=120, f=140.0, sh_degree=3,
                               n_views=2)
    g, views = sc["gaussians"], sc["views"]
    raster = dict(sc["raster"], tile=tile, radix_bits=radix, order=api.ORDER_PIXEL)
    cov, op = baked(g)
    o, rect, zb = oracle_render(g, cov, op, views, raster)
    total = pair_total(rect, synth.views_dims(views), tile)
    gpu, ws = gpu_render(g, cov, op, views, raster, max_pairs=total + 1000)
    assert int(ws.status.item()) == 0
    print(case, "ambiguous pixels:", check_render(o, gpu), "exact pass:", ws.exact_pass_count())
    # the per-pixel order changes the image somewhere
    prim, _, _ = oracle_render(g, cov, op, views, dict(raster, order=api.ORDER_PRIMITIVE))
    assert np.abs(prim["rgb"] - o["rgb"]).max() > 1e-3


def test_pixel_order_window_overflow_takes_the_exact_pass():
    """Wide, thin, tilted Gaussians stacked over a narrow depth range: every
    pixel sees hundreds of candidates whose key bounds overlap, so the
    per-pixel windows overflow and those pixels are resolved by the exact
    pass; the result is still the reference's."""
    rng = np.random.default_rng(14)
    n = 400
    sc = synth.small_scene(14, n_gauss=n, width=96, height=80, f=90.0)
    g = sc["gaussians"]
    g["mean"][0] = rng.uniform(-0.3, 0.3, n)
    g["mean"][1] = rng.uniform(-0.3, 0.3, n)
    g["mean"][2] = rng.uniform(3.0, 3.3, n)
    g["logscale"] = np.stack([np.full(n, np.log(0.25)), np.full(n, np.log(0.25)),
                              np.full(n, np.log(0.004))]).astype(np.float32)
    g["logit"] = np.full(n, -2.5, np.float32)        # faint: long lists per pixel
    for tile in (8, 16):
        raster = dict(sc["raster"], tile=tile, order=api.ORDER_PIXEL)
        cov, op = baked(g)
        o, rect, zb = oracle_render(g, cov, op, sc["views"], raster)
        total = pair_total(rect, synth.views_dims(sc["views"]), tile)
        gpu, ws = gpu_render(g, cov, op, sc["views"], raster, max_pairs=total + 64)
        assert int(ws.status.item()) == 0
        nfix = ws.exact_pass_count()
        print(f"tile {tile}: exact pass for {nfix} of {96 * 80} pixels")
        assert nfix > 100
        check_render(o, gpu, max_ambiguous=0.01)


def test_pixel_order_rejects_tile_32_and_backward():
    sc = synth.config(0)
    g, views = sc["gaussians"], sc["views"]
    cov, op = baked(g)
    opts = api.make_opts(**dict(sc["raster"], tile=32, order=api.ORDER_PIXEL))
    ws = api.RenderWorkspace(g["n"], views, opts, 100000)
    with pytest.raises(api.VrsError) as e:
        api.render_gaussians(dev(g["mean"]), dev(cov), dev(op), dev(g["sh"]), 0, views, opts, ws)
    assert e.value.code == api.VRS_EUNSUPPORTED


def test_fullsize_pixel_order_sampled():
    """The full stereo frame's periphery (2 x 2016x2240, 500k Gaussians SH3)
    in per-pixel order at tile 16, on 4,000 sampled pixels."""
    sc = synth.config(3)
    g, views = sc["gaussians"], sc["views"]
    raster = dict(sc["raster"], tile=16, order=api.ORDER_PIXEL)
    cov, op = baked(g)
    V, D = synth.views_array(views), synth.views_dims(views)
    rect, zb = oracle.gauss_geom32(g["mean"], cov, V, D)
    opts = api.make_opts(**raster)
    ws = api.RenderWorkspace(g["n"], views, opts, pair_total(rect, D, 16) + 1024)
    out = api.render_gaussians(dev(g["mean"]), dev(cov), dev(op), dev(g["sh"]), 3, views, opts, ws)
    torch.cuda.synchronize()
    assert int(ws.status.item()) == 0
    print("full size: exact pass for", ws.exact_pass_count(), "pixels")
    rng = np.random.default_rng(16)
    pix = np.stack([rng.integers(0, 2, 4000), rng.integers(0, 2016, 4000),
                    rng.integers(0, 2240, 4000)], 1).astype(np.int32)
    o, _, _ = oracle_render(g, cov, op, views, raster, pix=pix)
    v, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    gpu = dict(rgb=out["rgb"].cpu().numpy()[v, :, y, x], depth=out["depth"].cpu().numpy()[v, y, x],
               tfinal=out["tfinal"].cpu().numpy()[v, y, x],
               ncontrib=out["ncontrib"].cpu().numpy()[v, y, x])
    check_render(o, gpu, max_ambiguous=0.005)
