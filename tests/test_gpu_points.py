"""GPU parity of the foveal neural-point splat (vrs_splat_points) against
the CPU reference: per-layer-pixel fragment lists bit-exact (same points in
the same order), pyramid features within 1e-4, with and without the depth
cull, several crops of uneven size on two views, crops at image borders."""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_17932_amd import api, synth

from gpu_helpers import baked, dev, oracle_render

pytestmark = pytest.mark.gpu


def _depth_buffers(sc):
    g, views, raster = sc["gaussians"], sc["views"], sc["raster"]
    cov, op = baked(g)
    o, _, _ = oracle_render(g, cov, op, views, raster)
    return o["depth"].astype(np.float32), o["tfinal"].astype(np.float32)


def _run(sc, cull, levels=None, opacity=None):
    p, views, crops = sc["points"], sc["views"], sc["crops"]
    L = levels or sc["levels"]
    V, D = synth.views_array(views), synth.views_dims(views)
    ci, _ = synth.crops_array(crops)
    depth = tf = None
    if cull:
        depth, tf = _depth_buffers(sc)
    off, oids = oracle.point_lists(p["pos"], p["radius"], V, D, ci, L, depth, tf)
    pyr_o = oracle.splat_points(p["pos"], p["radius"], p["feat"], V, D, ci, L, depth, tf,
                                opacity=opacity)
    ws = api.SplatWorkspace(p["n"], views, crops, L, max(len(oids), 1) + 100)
    pyr = api.splat_points(dev(p["pos"]), dev(p["radius"]), dev(p["feat"].view(np.int16)),
                           None if opacity is None else dev(opacity), views, crops, L,
                           None if depth is None else dev(depth),
                           None if tf is None else dev(tf), ws)
    torch.cuda.synchronize()
    assert int(ws.status.item()) == 0
    keys, ids = ws.lists()
    counts = np.bincount(keys, minlength=len(off) - 1)
    assert np.array_equal(counts, np.diff(off)), "fragment counts per layer pixel differ"
    assert np.array_equal(ids, oids), "fragment order differs"
    err = np.abs(pyr.cpu().numpy() - pyr_o).max(initial=0)
    assert err <= 1e-4, f"pyramid max err {err}"
    return len(oids)


@pytest.mark.parametrize("cull", [False, True])
def test_points_tiny(cull):
    sc = synth.config(0)
    nf = _run(sc, cull)
    assert nf > 1000 if not cull else nf >= 0


def test_points_multi_crop_stereo():
    crops = ((40.0, 30.0, 64), (150.0, 90.0, 96), (10.0, 120.0, 32), (100.0, 60.0, 128))
    sc = synth.small_scene(31, n_gauss=1500, n_points=6000, width=200, height=136, f=150.0,
                           n_views=2, crops=crops, crop_views=[0, 1, 1, 0], radius="lognormal")
    sc["points"]["radius"] *= 4.0
    _run(sc, cull=False)
    _run(sc, cull=True)


def test_points_stacked_crops():
    """Five crops around one gaze point: a survivor reaches every crop and
    emits up to 40 fragments, so emission chunks hold few survivors and a
    survivor's fragments often span two chunks."""
    crops = ((100.0, 80.0, 64), (101.0, 79.0, 64), (99.0, 81.0, 96), (100.0, 80.0, 96),
             (98.0, 82.0, 128))
    sc = synth.small_scene(33, n_gauss=500, n_points=20000, width=200, height=160, f=150.0,
                           crops=crops, radius="lognormal")
    sc["points"]["radius"] *= 4.0
    nf = _run(sc, cull=False)
    assert nf > 4 * 2048


def test_points_many_survivors():
    """About 300k survivors and 2.4M fragments: some 2,400 emission chunks,
    each opened by the survivor the selection recorded for it."""
    sc = synth.small_scene(35, n_gauss=200, n_points=300000, width=512, height=384, f=300.0,
                           crops=((256.0, 192.0, 256), (200.0, 150.0, 128)), radius="lognormal")
    nf = _run(sc, cull=False)
    assert nf > 2_000_000


def test_points_with_opacity_and_levels():
    sc = synth.small_scene(32, n_points=4000, crops=((64.0, 64.0, 64), (20.0, 20.0, 32)))
    op = np.random.default_rng(0).uniform(0.2, 1.0, sc["points"]["n"]).astype(np.float32)
    _run(sc, cull=False, opacity=op)
    _run(sc, cull=False, levels=2)


def test_points_capacity_flag():
    sc = synth.config(0)
    p, views, crops = sc["points"], sc["views"], sc["crops"]
    ws = api.SplatWorkspace(p["n"], views, crops, 4, 50)
    api.splat_points(dev(p["pos"]), dev(p["radius"]), dev(p["feat"].view(np.int16)), None, views,
                     crops, 4, None, None, ws)
    torch.cuda.synchronize()
    assert int(ws.status.item()) == api.VRS_ECAPACITY


def _morton_reference(pos):
    """30-bit Morton codes from the same float32 quantisation (numpy)."""
    pos = pos.astype(np.float32)
    codes = np.zeros(pos.shape[1], np.uint64)
    for a in range(3):
        v = pos[a]
        lo, hi = v.min(), v.max()
        t = np.zeros_like(v) if not hi > lo else ((v - lo) / np.float32(hi - lo)) * np.float32(1024.0)
        q = np.clip(t, 0.0, 1023.0).astype(np.uint64)
        for b in range(10):
            codes |= ((q >> b) & 1) << (3 * b + a)
    return codes


@pytest.mark.parametrize("n", [1, 1000, 123457])
def test_spatial_order_is_stable_morton_sort(n):
    rng = np.random.default_rng(n)
    pos = np.stack([rng.uniform(-1, 1, n), rng.uniform(-2, 3, n), rng.uniform(2, 6, n)]).astype(np.float32)
    if n > 10:
        pos[:, 5] = pos[:, 7]          # exact duplicates keep index order
    perm = api.spatial_order(dev(pos)).cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    codes = _morton_reference(pos)
    assert np.array_equal(perm, np.argsort(codes, kind="stable"))


def test_spatial_order_degenerate_box():
    pos = np.ones((3, 777), np.float32)
    perm = api.spatial_order(dev(pos)).cpu().numpy()
    assert np.array_equal(perm, np.arange(777))
