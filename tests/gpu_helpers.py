"""Shared helpers of the GPU parity tests: move seeded inputs to the device,
run the CPU reference on the same inputs, compare."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2410_17932_amd import api, synth

DEV = "cuda"


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def baked(g):
    """Float32 covariances and opacities from the CPU reference's bake: the
    renderer's inputs for parity tests of the render entry in isolation."""
    cov, op = oracle.bake(g["logscale"], g["quat"], g["logit"])
    return cov.astype(np.float32), op.astype(np.float32)


def oracle_render(g, cov, op, views, raster, pix=None):
    """The reference's periphery on the same inputs, in the order raster
    asks for (order 1: per pixel)."""
    V, D = synth.views_array(views), synth.views_dims(views)
    rect, zb = oracle.gauss_geom32(g["mean"], cov, V, D, raster["lowpass"], raster["extent"])
    rec = oracle.gauss_project64(g["mean"], cov, op, g["sh"], g["sh_degree"], V, D,
                                 raster["lowpass"])
    per_pixel = None
    if raster.get("order", 0) == 1:
        c32, c64 = oracle.gauss_pixdepth(g["mean"], cov, V, D)
        per_pixel = (c32, c64, V)
    out = oracle.render(rect, zb, rec, D, raster["tile"], raster["alpha_clamp"],
                        raster["alpha_min"], raster["t_min"], raster["bg"], pix=pix,
                        per_pixel=per_pixel)
    # what check_render needs to resolve near-threshold pixels
    out["branches"] = dict(rect=rect, zb=zb, rec=rec, raster=raster, pix=pix,
                           per_pixel=per_pixel)
    return out, rect, zb


def pair_total(rect, dims, tile):
    r = rect[rect[..., 0] >= 0]
    return int(((r[:, 2] // tile - r[:, 0] // tile + 1) * (r[:, 3] // tile - r[:, 1] // tile + 1)).sum())


def super_pair_total(rect, tile, group=8):
    """(super-tile, Gaussian) pairs of the binning: super-tiles of group x
    group tiles reached by each rectangle."""
    r = rect[rect[..., 0] >= 0]
    s = tile * group
    return int(((r[:, 2] // s - r[:, 0] // s + 1) * (r[:, 3] // s - r[:, 1] // s + 1)).sum())


def gpu_render(g, cov, op, views, raster, max_pairs):
    opts = api.make_opts(**raster)
    ws = api.RenderWorkspace(g["n"], views, opts, max_pairs)
    out = api.render_gaussians(dev(g["mean"]), dev(cov), dev(op), dev(g["sh"]), g["sh_degree"],
                               views, opts, ws)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, ws


def tile_counts(rect, dims, tile):
    """Length of every (view, tile) list, tiles in [view][ty][tx] order: the
    number of rectangles whose tile range holds the tile (2-D difference
    array over the tile grid)."""
    W, H = int(dims[0][0]), int(dims[0][1])
    tx_n, ty_n = -(-W // tile), -(-H // tile)
    out = []
    for v in range(rect.shape[0]):
        r = rect[v][rect[v][:, 0] >= 0]
        d = np.zeros((ty_n + 1, tx_n + 1), np.int64)
        x0, y0, x1, y1 = r[:, 0] // tile, r[:, 1] // tile, r[:, 2] // tile + 1, r[:, 3] // tile + 1
        np.add.at(d, (y0, x0), 1)
        np.add.at(d, (y0, x1), -1)
        np.add.at(d, (y1, x0), -1)
        np.add.at(d, (y1, x1), 1)
        out.append(d.cumsum(0).cumsum(1)[:ty_n, :tx_n].ravel())
    return np.concatenate(out)


def check_render(o, gpu, tol=1e-4, margin=1e-4, max_ambiguous=0.002, branches=None):
    """Element-wise comparison on every pixel whose threshold decisions are
    not within `margin` (relative) of their thresholds.  The others may take
    either branch in single precision: with `branches` (dict rect, zb, rec,
    raster and pix, the pixels of o in order, or None for full images) each
    must match one of the results the reference reaches by taking either
    branch at those decisions (contributor count exact, colour, depth and
    transmittance within tol; oracle_render's output carries these inputs);
    without them, only for validity."""
    if branches is None:
        branches = o.get("branches")
    amb = o["margin"] < margin
    ok = ~amb
    assert amb.mean() <= max_ambiguous, f"ambiguous fraction {amb.mean()}"
    full = gpu["rgb"].ndim == 4
    for ch in range(3):
        d = np.abs(gpu["rgb"][:, ch] - o["rgb"][:, ch])[ok]
        assert d.max(initial=0) <= tol, f"rgb ch{ch} max err {d.max()}"
    dscale = max(1.0, float(np.abs(o["depth"]).max()))
    dd = np.abs(gpu["depth"] - o["depth"])[ok]
    assert dd.max(initial=0) <= tol * dscale, f"depth {dd.max()}"
    dt = np.abs(gpu["tfinal"] - o["tfinal"])[ok]
    assert dt.max(initial=0) <= tol, f"T {dt.max()}"
    assert np.array_equal(gpu["ncontrib"][ok], o["ncontrib"][ok])
    # validity everywhere: transmittance in (0, 1], colours finite
    assert np.isfinite(gpu["rgb"]).all() and (gpu["tfinal"] > 0).all() and (gpu["tfinal"] <= 1).all()
    if branches is not None and amb.any():
        b = branches
        if full:
            vv, yy, xx = np.nonzero(amb)
            pix = np.stack([vv, xx, yy], 1)
            g_rgb = gpu["rgb"][vv, :, yy, xx]
            sel = (vv, yy, xx)
        else:
            idx = np.nonzero(amb)[0]
            pix = np.asarray(b["pix"])[idx]
            g_rgb = gpu["rgb"][idx]
            sel = (idx,)
        r = b["raster"]
        alts = oracle.render_branches(b["rect"], b["zb"], b["rec"], pix, r["alpha_clamp"],
                                      r["alpha_min"], r["t_min"], r["bg"], margin,
                                      per_pixel=b.get("per_pixel"))
        for k, alt in enumerate(alts):
            gn, gd, gt = (int(gpu["ncontrib"][sel][k]), float(gpu["depth"][sel][k]),
                          float(gpu["tfinal"][sel][k]))
            hit = any(n == gn and np.abs(g_rgb[k] - c).max() <= tol and abs(gd - d) <= tol * dscale
                      and abs(gt - t) <= tol for n, c, d, t in alt)
            assert hit, (f"ambiguous pixel {pix[k].tolist()}: GPU (n={gn}, rgb={g_rgb[k]}, "
                         f"depth={gd}, T={gt}) is none of {len(alt)} branch results")
    return int(amb.sum())
