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


def _ord_bits(x):
    u = np.asarray(x, np.float32).view(np.uint32)
    return np.where(u & np.uint32(0x80000000), ~u, u | np.uint32(0x80000000))


PREFIX = 4096   # records per tile list sorted by the per-tile bound


def check_tile_words(ws, g, cov, views, tile):
    """The blend's tile lists: per tile, the sorted prefix (first 4096
    positions) holds the binning's first records in another order with a
    non-decreasing bound, and the bound of every prefix position is at most
    the single-precision key (its operation order retyped in numpy float32)
    of every record at that position or later (the rest of the list in the
    binning's order), at every pixel of the tile inside the record's
    rectangle.  Returns the longest list."""
    V, D = synth.views_array(views), synth.views_dims(views)
    rect, _ = oracle.gauss_geom32(g["mean"], cov, V, D)
    c32, _ = oracle.gauss_pixdepth(g["mean"], cov, V, D)
    ranges, ids = ws.tile_lists()
    words = ws.tile_words()
    W, H = int(D[0][0]), int(D[0][1])
    tx_n, ty_n = -(-W // tile), -(-H // tile)
    tv, gis, beta, longest = [], [], [], 0
    for t, (b, e) in enumerate(ranges):
        if e <= b:
            continue
        m = min(e - b, PREFIX)
        w = words[b:b + m]
        hi = (w >> np.uint64(32)).astype(np.uint32)
        assert np.all(hi[1:] >= hi[:-1]), f"tile {t}: bounds decrease"
        wid = (w & np.uint64(0xffffffff)).astype(np.int64)
        assert np.array_equal(np.sort(wid), np.sort(ids[b:b + m])), f"tile {t}: prefix differs"
        tv.append(np.full(e - b, t))
        gis.append(np.concatenate([wid, ids[b + m:e]]))
        beta.append(np.concatenate([hi, np.zeros(e - b - m, np.uint32)]))
        longest = max(longest, e - b)
    t = np.concatenate(tv)
    gi = np.concatenate(gis)
    beta = np.concatenate(beta)
    v = t // (tx_n * ty_n)
    tl = t % (tx_n * ty_n)
    ty, tx = tl // tx_n, tl % tx_n
    r = rect[v, gi]
    x0, x1 = np.maximum(tx * tile, r[:, 0]), np.minimum(np.minimum(tx * tile + tile - 1, r[:, 2]), W - 1)
    y0, y1 = np.maximum(ty * tile, r[:, 1]), np.minimum(np.minimum(ty * tile + tile - 1, r[:, 3]), H - 1)
    k = c32[v, gi].T.astype(np.float32)
    cam = V[v]
    f32 = np.float32
    kmin = np.full(len(t), 0xffffffff, np.uint32)
    for dy in range(tile):
        for dx in range(tile):
            px, py = tx * tile + dx, ty * tile + dy
            m = (px >= x0) & (px <= x1) & (py >= y0) & (py <= y1)
            if not m.any():
                continue
            u = ((px[m].astype(f32) + f32(0.5)) - cam[m, 2]) / cam[m, 0]
            vv = ((py[m].astype(f32) + f32(0.5)) - cam[m, 3]) / cam[m, 1]
            km = k[:, m]
            num = km[6] * u
            num = num + km[7] * vv
            num = num + km[8]
            a = km[0] * u
            a = a + km[1] * vv
            a = a + km[2]
            bq = km[3] * vv
            bq = bq + km[4]
            den = a * u
            den = den + bq * vv
            den = den + km[5]
            with np.errstate(all="ignore"):
                key = num / den
            kmin[m] = np.minimum(kmin[m], _ord_bits(key))
    # suffix minimum of the records' least keys along each list
    start = np.r_[0, np.flatnonzero(np.diff(t)) + 1]
    stop = np.r_[start[1:], len(t)]
    suf = np.empty_like(kmin)
    for s0, s1 in zip(start, stop):
        suf[s0:s1] = np.minimum.accumulate(kmin[s0:s1][::-1])[::-1]
    bad = suf < beta
    assert not bad.any(), f"a bound above a later key at {int(bad.sum())} positions"
    return longest


@pytest.mark.parametrize("n", [5000, 9000])
def test_pixel_order_long_tile_lists(n):
    """Thousands of small Gaussians over a few tiles: lists far longer than
    the sorted prefix, so blending and the exact pass read past it (in the
    binning's order, with looser bounds); the bounds hold and the image is
    the reference's."""
    rng = np.random.default_rng(30 + n)
    sc = synth.small_scene(31, n_gauss=n, width=40, height=32, f=60.0)
    g = sc["gaussians"]
    g["mean"][0] = rng.uniform(-0.05, 0.05, n)
    g["mean"][1] = rng.uniform(-0.05, 0.05, n)
    g["mean"][2] = rng.uniform(3.0, 4.0, n)
    g["logscale"] = np.log(rng.uniform(0.004, 0.02, (3, n))).astype(np.float32)
    g["logit"] = np.full(n, -3.0, np.float32)
    raster = dict(sc["raster"], tile=8, order=api.ORDER_PIXEL)
    cov, op = baked(g)
    o, rect, zb = oracle_render(g, cov, op, sc["views"], raster)
    total = pair_total(rect, synth.views_dims(sc["views"]), 8)
    gpu, ws = gpu_render(g, cov, op, sc["views"], raster, max_pairs=total + 64)
    assert int(ws.status.item()) == 0
    longest = check_tile_words(ws, g, cov, sc["views"], 8)
    print(f"n {n}: longest list {longest}, exact pass {ws.exact_pass_count()}")
    assert longest > PREFIX
    check_render(o, gpu)


def test_tile_words_bound_the_keys():
    """The per-tile bound on a general scene (stereo, ragged edges, tiles 8
    and 16)."""
    sc = synth.small_scene(21, n_gauss=3000, width=200, height=136, f=150.0, n_views=2)
    g, views = sc["gaussians"], sc["views"]
    cov, op = baked(g)
    for tile in (8, 16):
        raster = dict(sc["raster"], tile=tile, order=api.ORDER_PIXEL)
        V, D = synth.views_array(views), synth.views_dims(views)
        rect, _ = oracle.gauss_geom32(g["mean"], cov, V, D)
        _, ws = gpu_render(g, cov, op, views, raster, max_pairs=pair_total(rect, D, tile) + 64)
        assert int(ws.status.item()) == 0
        check_tile_words(ws, g, cov, views, tile)


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
