#!/usr/bin/env python3
"""Benchmark: stereo foveated frames/s at 2016x2240 per eye on one MI355X.

Workload (the full hybrid stereo frame): 500,000 Gaussians with SH degree 3
for the periphery of both eyes (f = 1100, 64 mm IPD), 5,000,000 neural
points, eight gaze crops per eye of uneven size (256..640 px, 4-layer
pyramids, depth culled against the periphery), a 16/32/64/64 gated decoder
in BF16 on the matrix cores, and the 64 px linear blend ring.  One step =
one whole frame (periphery, splat, decoder, combination) of both eyes,
replayed from a HIP graph with all inputs resident in HBM.

Prints ONE JSON line (rank 0) with the frame rate, the roofline of the
dominant kernel measured live with HIP events, the plain FP32 eager form of
the same frame and the CPU reference timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X fp32 vector, published
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense bf16, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage_ms(frame, stage, steps):
    """Average duration of one stage's kernels over `steps` eager inference
    frames, from HIP events the library records around the stage on the
    frame's stream (the plan's trace table)."""
    import torch
    evs = []
    tot = 0.0
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        frame.trace(stage, a, b)
        frame.run()
        evs.append((a, b))
    frame.trace("off")
    torch.cuda.synchronize()
    for a, b in evs:
        tot += a.elapsed_time(b)
    return tot / steps


def cpu_baseline(scene, budget_s=20.0):
    """The CPU reference timed on the frame, scaled to frames/s.  The
    periphery's per-tile cost is first measured on 256 and 1280 random tiles;
    when the whole frame fits the time budget it is rendered in full
    (periphery of both eyes, then splat, decoder and combination of every
    crop on the reference's own depth), otherwise the tile fit is
    extrapolated and one crop's fovea is scaled by the crop-pixel share."""
    import numpy as np
    import oracle
    from paper_2410_17932_amd import synth
    oracle.build(force=False)
    g, p = scene["gaussians"], scene["points"]
    views, crops, L = scene["views"], scene["crops"], scene["levels"]
    V, D = synth.views_array(views), synth.views_dims(views)
    t0 = time.perf_counter()
    cov, op = oracle.bake(g["logscale"], g["quat"], g["logit"])
    cov, op = cov.astype(np.float32), op.astype(np.float32)
    rect, zb = oracle.gauss_geom32(g["mean"], cov, V, D)
    rec = oracle.gauss_project64(g["mean"], cov, op, g["sh"], 3, V, D)
    t_proj = time.perf_counter() - t0
    W, H = views[0].width, views[0].height
    nv = len(views)
    tx, ty = (W + 15) // 16, (H + 15) // 16
    rng = np.random.default_rng(0)
    n_tiles = nv * tx * ty
    order = rng.permutation(n_tiles)

    def tiles_time(count):
        pix = []
        for s in order[:count]:
            v, t = divmod(int(s), tx * ty)
            x0, y0 = (t % tx) * 16, (t // tx) * 16
            for yy in range(y0, min(y0 + 16, H)):
                for xx in range(x0, min(x0 + 16, W)):
                    pix.append((v, xx, yy))
        t0 = time.perf_counter()
        oracle.render(rect, zb, rec, D, 16, pix=np.array(pix, np.int32))
        return time.perf_counter() - t0

    # the reference bins every Gaussian once per call (fixed cost) and then
    # blends each requested tile: fit t = fixed + per_tile * tiles
    n_small, n_big = 256, 1280
    t_small, t_big = tiles_time(n_small), tiles_time(n_big)
    per_tile = max(t_big - t_small, 0.0) / (n_big - n_small)
    fixed = max(t_small - per_tile * n_small, 0.0)
    est_periph = t_proj + fixed + per_tile * n_tiles
    ci, cf = synth.crops_array(crops)
    decoder_w = synth.pack_decoder(scene["decoder"]).astype(np.float64)
    if est_periph * 1.5 <= budget_s:
        # the whole frame
        t0 = time.perf_counter()
        o = oracle.render(rect, zb, rec, D, 16)
        t_periph = t_proj + time.perf_counter() - t0
        depth = o["depth"].astype(np.float32).reshape(nv, H, W)
        tf = o["tfinal"].astype(np.float32).reshape(nv, H, W)
        rgb = o["rgb"].reshape(nv, 3, H, W)
        t0 = time.perf_counter()
        pyr = oracle.splat_points(p["pos"], p["radius"], p["feat"], V, D, ci, L, depth, tf)
        Fo = oracle.decode(ci, L, 4, pyr, rgb, D, scene["decoder"]["widths"], decoder_w)
        oracle.composite(rgb, D, ci, cf, Fo, mode=0, ring=64.0)
        t_fovea = time.perf_counter() - t0
        t_frame = t_periph + t_fovea
        sample = (f"the whole frame: bake + projection of all Gaussians ({t_proj:.1f} s), periphery "
                  f"of both eyes ({t_periph - t_proj:.1f} s), splat + FP64 decoder + combination of "
                  f"all {len(crops)} crops ({t_fovea:.1f} s); tile-cost probe of {n_small} and "
                  f"{n_big} tiles beforehand")
    else:
        t_periph = est_periph
        c = crops[0]
        c1, _ = synth.crops_array([c])
        cpix = np.array([(c.view, x, y) for y in range(c.y0, c.y0 + c.size)
                         for x in range(c.x0, c.x0 + c.size)], np.int32)
        pr = oracle.render(rect, zb, rec, D, 16, pix=cpix)
        depth = np.zeros((nv, H, W), np.float32)
        tf = np.ones((nv, H, W), np.float32)
        depth[c.view, c.y0:c.y0 + c.size, c.x0:c.x0 + c.size] = pr["depth"].reshape(c.size, c.size)
        tf[c.view, c.y0:c.y0 + c.size, c.x0:c.x0 + c.size] = pr["tfinal"].reshape(c.size, c.size)
        t0 = time.perf_counter()
        pyr = oracle.splat_points(p["pos"], p["radius"], p["feat"], V, D, c1, L, depth, tf)
        oracle.decode(c1, L, 4, pyr, np.zeros((nv, 3, H, W)), D, scene["decoder"]["widths"],
                      decoder_w)
        t_crop = time.perf_counter() - t0
        t_fovea = t_crop * sum(cc.size ** 2 for cc in crops) / (c.size ** 2)
        t_frame = t_periph + t_fovea
        sample = (f"periphery: projection of all Gaussians ({t_proj:.1f} s) + blend of "
                  f"{n_small} and {n_big} of {n_tiles} random 16x16 tiles, linear fit "
                  f"extrapolated to all tiles; fovea: splat + FP64 decoder of crop 0 "
                  f"({c.size}^2, {t_crop:.1f} s) scaled by the crop-pixel share")
    return dict(value=1.0 / t_frame, unit="frames/s", cores=oracle.num_threads(), kind="oracle",
                sample=sample, seconds_per_frame=t_frame)


def measured_traffic(profile, source):
    """HBM bytes per launch from a committed counter summary, or None when
    the kernel's source changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith("|"))
    key = f"source_sha256_16({source})"
    cur = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()[:16]
    if vals.get(key, "").strip() != cur or "traffic_bytes_per_launch" not in vals:
        return None
    return int(vals["traffic_bytes_per_launch"])


def blend_work(frame):
    """Algorithmic floating-point work of the periphery blend: every
    evaluation of a Gaussian at a pixel inside its rectangle costs 14 flops
    (offset, quadratic form, exp, opacity, clamp, transmittance product) and
    each blended contribution 11 more (colour and depth accumulation).  The
    counts come from one instrumented frame (the timed frames do not count)."""
    import torch
    frame.run(stats=True)
    torch.cuda.synchronize()
    npix = frame.depth.numel()
    evals = frame.rws.pixel_evals(npix).to(torch.int64).sum().item()
    contrib = frame.ncontrib.to(torch.int64).sum().item()
    return 14 * evals + 11 * contrib, evals, contrib


def decoder_flops(crops, widths, in_ch=4):
    """Algorithmic flops of the decoder per frame: per crop and level l
    (size S_l = S / 2^l) one 3x3 gated convolution producing 2 K_l channels
    (feature and gate halves) from C_l = in_ch + K_{l+1} (+3 at level 0)
    inputs, 2 * 9 * C_l * 2 K_l flops per output pixel, plus the 1x1 RGB
    head, 2 * 3 * K_0 per pixel."""
    n = len(widths)
    tot = 0
    for c in crops:
        for l in range(n):
            S = c.size >> l
            cin = in_ch + (widths[l + 1] if l + 1 < n else 0) + (3 if l == 0 else 0)
            tot += 2 * 9 * cin * 2 * widths[l] * S * S
        tot += 2 * 3 * widths[0] * c.size * c.size
    return tot


def replay_ms(frame, warmup=3, steps=10):
    """Milliseconds per frame of the captured frame's graph replay."""
    import torch
    frame.capture()
    for _ in range(warmup):
        frame.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        frame.replay()
    torch.cuda.synchronize()
    assert frame.status() == 0, f"device status {frame.status()}"
    return (time.perf_counter() - t0) / steps * 1e3


def free():
    """Return the device memory of frames the caller has dropped."""
    import gc
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def secondary_and_standalone(scene, tile, radix, steps):
    """The paper's own VR setting (one 512 crop per eye at the view centre,
    d_f = 256) on the full-frame scene, and the periphery (config 1) and
    foveal (config 2) workloads on their own."""
    from paper_2410_17932_amd import api, synth
    from paper_2410_17932_amd.frame import Frame
    out = {}
    W, H = scene["views"][0].width, scene["views"][0].height
    vr = dict(scene, crops=[synth.crop_at(v, W / 2, H / 2, 512, W, H) for v in range(2)])
    fr = Frame(vr, decoder_dtype=api.VRS_BF16, tile=tile, radix_bits=radix)
    ms = replay_ms(fr, steps=steps)
    out["secondary_vr_frame"] = dict(workload="one 512 crop per eye (d_f = 256), rest as the "
                                     "full frame", ms_per_frame=round(ms, 4),
                                     frames_per_s=round(1e3 / ms, 1))
    del fr
    free()
    sc1 = synth.config(1)
    fr = Frame(sc1, tile=tile, radix_bits=radix)
    ms = replay_ms(fr, steps=steps)
    out["config1_periphery"] = dict(workload="500k Gaussians SH3, stereo 2016x2240, periphery "
                                    "only", ms_per_frame=round(ms, 4),
                                    frames_per_s=round(1e3 / ms, 1), tile_pairs=fr.pairs)
    del fr
    free()
    # the same periphery in per-pixel order (the paper's popping fix) against
    # the per-primitive order above
    px, exact = {}, {}
    for t in (8, 16):
        fr = Frame(sc1, tile=t, radix_bits=radix, order=api.ORDER_PIXEL)
        px[str(t)] = round(replay_ms(fr, warmup=1, steps=3), 4)
        exact[str(t)] = fr.rws.exact_pass_count()
        del fr
        free()
    best = min(px, key=px.get)
    out["periphery_pixel_order"] = dict(
        workload="config 1 periphery in per-pixel order (exact per-pixel sort)",
        ms_per_frame=px[best], tile=int(best), ms_by_tile=px,
        primitive_order_ms=out["config1_periphery"]["ms_per_frame"],
        exact_pass_pixels=exact[best], exact_pass_pixels_by_tile=exact)
    sc2 = synth.config(2)
    fr = Frame(sc2, decoder_dtype=api.VRS_BF16, tile=tile, radix_bits=radix)
    fr.run()
    st = {k: stage_ms(fr, k, steps) for k in ("splat", "decoder")}
    out["config2_fovea"] = dict(workload="5M points, one 512 crop at the left-eye centre culled "
                                "against the periphery, decoder 16/32/64/64 BF16",
                                splat_ms=round(st["splat"], 4), decoder_ms=round(st["decoder"], 4),
                                fovea_ms=round(st["splat"] + st["decoder"], 4),
                                fragments=fr.frags)
    del fr
    free()
    return out


def _event_ms(fn, steps):
    """Milliseconds per call of fn() (enqueued on the current stream),
    between HIP events, after one untimed call."""
    import torch
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def post_and_training(scene, steps):
    """Tone mapping of the full stereo frame (forward and adjoint), and the
    training objective's kernels at the fitting step's sizes: D-SSIM of four
    1024^2 RGB views (forward and adjoint), the regulariser over this frame's
    crops, and one Adam step over the fitting scene's parameter count (1M
    Gaussians x 59 floats + 2M points x 8 floats).  Each with its
    algorithmic HBM bytes and the fraction of 8 TB/s."""
    import torch
    from paper_2410_17932_amd import api
    out = {}
    g = torch.Generator(device="cuda").manual_seed(9)

    def hbm(ms, nbytes):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return dict(ms=round(ms, 4), bytes=int(nbytes), gb_per_s=round(gbs, 1),
                    frac_of_8tbs=round(gbs / 8000.0, 3))

    views = scene["views"]
    V, H, W = len(views), views[0].height, views[0].width
    img = torch.rand((V, 3, H, W), device="cuda", generator=g)
    par = api.tonemap_params(V)
    par[:, 0] = 0.3
    par[:, 4] = -0.2
    res = torch.empty_like(img)
    nimg = img.numel() * 4
    out["tonemap_frame"] = hbm(_event_ms(lambda: api.tonemap(img, views, par, out=res), steps),
                               2 * nimg)
    d_in = torch.empty_like(img)
    d_par = torch.zeros_like(par)
    out["tonemap_frame_backward"] = hbm(_event_ms(
        lambda: api.tonemap_backward(img, views, par, res, d_img=d_in, d_params=d_par), steps),
        3 * nimg)
    del img, res, d_in
    x = torch.rand((12, 1024, 1024), device="cuda", generator=g)
    y = (x + 0.1 * torch.randn(x.shape, device="cuda", generator=g)).clamp(0, 1)
    ws = api.DssimWorkspace(12, 1024, 1024)
    loss = torch.empty(1, device="cuda")
    nx = x.numel() * 4
    out["dssim_4x1024sq"] = hbm(_event_ms(lambda: api.dssim(x, y, ws, loss=loss), steps), 2 * nx)
    dx = torch.zeros_like(x)
    # maps written and read back (3 planes each), x and y read twice, d_x
    # read and written
    out["dssim_4x1024sq_backward"] = hbm(_event_ms(lambda: api.dssim_backward(x, y, ws, dx),
                                                   steps), 6 * nx + 4 * nx + 2 * nx)
    del x, y, ws, dx
    crops = scene["crops"]
    if crops:
        nf = sum(3 * c.size * c.size for c in crops)
        fov = torch.rand(nf, device="cuda", generator=g)
        per = torch.rand((V, 3, H, W), device="cuda", generator=g)
        r = torch.empty(2, device="cuda")
        out["regulariser_crops"] = hbm(_event_ms(lambda: api.regulariser(fov, per, crops, r=r),
                                                 steps), 2 * nf * 4)
        del fov, per
    n = 1_000_000 * 59 + 2_000_000 * 8
    p_ = torch.zeros(n, device="cuda")
    g_ = torch.randn(n, device="cuda", generator=g) * 1e-3
    m_ = torch.zeros(n, device="cuda")
    v_ = torch.zeros(n, device="cuda")
    out["adam_fit_params"] = hbm(_event_ms(lambda: api.adam_step(p_, g_, m_, v_, 1, 1e-3), steps),
                                 7 * 4 * n)
    out["adam_fit_params"]["params"] = n
    del p_, g_, m_, v_
    free()
    return {"post_and_training": out}


def table3_and_fig2(scene, tile, radix, steps):
    """Synthetic reproductions of the paper's performance ablation (Table 3:
    depth culling off, full-width finest decoder level, combination with and
    without the Sobel edge term) and scaling curves (Fig. 2: periphery time
    against the number of Gaussians, foveal time against the crop size)."""
    import numpy as np
    from paper_2410_17932_amd import api, synth
    from paper_2410_17932_amd.frame import Frame
    t3 = {}
    fr = Frame(scene, decoder_dtype=api.VRS_BF16, tile=tile, radix_bits=radix)
    fr.run()
    base = {k: stage_ms(fr, k, steps) for k in ("splat", "decoder", "composite")}
    frags_on = fr.frags
    del fr
    free()
    fr = Frame(scene, decoder_dtype=api.VRS_BF16, tile=tile, radix_bits=radix, cull=False,
               frag_margin=1.1)
    fr.run()
    t3["depth_cull"] = dict(on_splat_ms=round(base["splat"], 4),
                            off_splat_ms=round(stage_ms(fr, "splat", steps), 4),
                            on_fragments=frags_on, off_fragments=fr.frags)
    del fr
    free()
    wide = dict(scene, decoder=synth.decoder_weights(np.random.default_rng(7), (32, 32, 64, 64), 4))
    fr = Frame(wide, decoder_dtype=api.VRS_BF16, tile=tile, radix_bits=radix)
    fr.run()
    t3["finest_decoder_width"] = dict(width16_ms=round(base["decoder"], 4),
                                      width32_ms=round(stage_ms(fr, "decoder", steps), 4))
    del fr
    free()
    comp = dict(linear_ring_ms=round(base["composite"], 4))
    for name, gamma in (("paper_edge_ms", 0.2), ("paper_no_edge_ms", 0.0)):
        fr = Frame(scene, decoder_dtype=api.VRS_BF16, tile=tile, radix_bits=radix,
                   mode=api.BLEND_PAPER, gamma=gamma)
        fr.run()
        comp[name] = round(stage_ms(fr, "composite", steps), 4)
        del fr
        free()
    t3["combination"] = comp
    # Fig. 2: periphery against the number of Gaussians (stereo 2016x2240)
    views = scene["views"]
    g_sweep = {}
    for n in (100_000, 250_000, 500_000, 1_000_000):
        g = synth.gaussians(np.random.default_rng(n), n, 3)
        sc = dict(gaussians=g, points=None, decoder=None, views=views, crops=[],
                  levels=4, raster=dict(scene["raster"]))
        fr = Frame(sc, tile=tile, radix_bits=radix)
        g_sweep[str(n)] = round(replay_ms(fr, steps=steps), 4)
        del fr
        free()
    # ... and the fovea against the crop size (one crop per eye)
    W, H = views[0].width, views[0].height
    c_sweep = {}
    for S in (256, 512, 768, 1024):
        sc = dict(scene, crops=[synth.crop_at(v, W / 2, H / 2, S, W, H) for v in range(2)])
        fr = Frame(sc, decoder_dtype=api.VRS_BF16, tile=tile, radix_bits=radix)
        fr.run()
        c_sweep[str(S)] = round(stage_ms(fr, "splat", steps) + stage_ms(fr, "decoder", steps), 4)
        del fr
        free()
    return dict(table3=t3, fig2=dict(periphery_ms_by_gaussians=g_sweep,
                                     fovea_ms_by_crop_size=c_sweep))


def profile_pass(args):
    """A short eager run for hardware-counter passes: two inference frames,
    then a plain device copy of known size for the HBM byte-counter
    calibration."""
    import torch
    from paper_2410_17932_amd import api, synth
    from paper_2410_17932_amd.frame import Frame
    scene = synth.config(args.config)
    fr = Frame(scene, decoder_dtype=api.VRS_BF16, tile=args.tile or 32, radix_bits=args.radix)
    for _ in range(2):
        fr.run()
    torch.cuda.synchronize()
    x = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    log("profile pass done: frames 2, calibration copy 256 MiB")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary frame, standalone configs and sweeps")
    ap.add_argument("--tile", type=int, default=0, help="0 = autotune tile and radix")
    ap.add_argument("--radix", type=int, default=8)
    ap.add_argument("--profile-pass", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the frame is measured on one GPU only (asked for --gpus {args.gpus}); "
              "the path has no multi-GPU form", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2410_17932_amd import api, synth
    from paper_2410_17932_amd.frame import Frame, PlainFrame
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    api.lib()
    if args.profile_pass:
        profile_pass(args)
        return
    t0 = time.perf_counter()
    scene = synth.config(args.config)
    log(f"scene generated in {time.perf_counter() - t0:.1f} s")
    fr = Frame(scene, decoder_dtype=api.VRS_BF16)
    if args.tile == 0:
        tune = fr.autotune()
    else:
        fr._plan(args.tile, args.radix)
        tune = dict(tile=args.tile, radix_bits=args.radix)
    tile, radix = tune["tile"], tune["radix_bits"]
    log(f"autotune: {tune}; pairs {fr.pairs}, fragments {fr.frags}")
    fr.capture()
    for _ in range(args.warmup):
        fr.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fr.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    fps = args.steps / dt
    assert fr.status() == 0, f"device status {fr.status()}"
    log(f"graph replay: {ms:.3f} ms/frame, {fps:.1f} frames/s")
    # per-stage kernel time over K eager inference frames (library-recorded
    # HIP events on the frame's stream)
    stages = {}
    for st in ("gs_preprocess", "gs_depth_sort", "gs_emit", "gs_sort", "gs_blend", "splat",
               "decoder", "composite"):
        stages[st] = stage_ms(fr, st, args.steps)
    log("stages ms:", json.dumps({k: round(v, 4) for k, v in stages.items()}))
    flops, evals, contrib = blend_work(fr)
    blend_s = stages["gs_blend"] * 1e-3
    achieved = flops / blend_s / 1e12
    roofline = dict(kernel="k_gs_blend (periphery front-to-back blend)", bound="alu",
                    achieved=round(achieved, 3), peak=FP32_VALU_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / FP32_VALU_PEAK_TFLOPS, 4),
                    traffic=measured_traffic("gs_blend_config3_hbm_counters.md",
                                             "paper_2410_17932_amd/csrc/gs_blend.hip"),
                    work=dict(flops=flops, evaluations=evals, contributions=contrib,
                              ms=round(stages["gs_blend"], 4)))
    # decoder on the matrix cores: algorithmic flops over its stage time
    dflops = decoder_flops(scene["crops"], scene["decoder"]["widths"])
    dtf = dflops / (stages["decoder"] * 1e-3) / 1e12
    decoder_mfma = dict(kernel="k_dec_conv (gated 3x3 conv, BF16 MFMA)", bound="mfma",
                        achieved=round(dtf, 2), peak=BF16_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                        frac=round(dtf / BF16_MFMA_PEAK_TFLOPS, 4), flops_per_frame=dflops,
                        ms=round(stages["decoder"], 4))
    # rasterizer HBM rate: the periphery's tile binning (its HBM-bound stage).
    # Algorithmic bytes: per (super-tile, Gaussian) pair and sort pass 4 B
    # read by the digit count and 2 x 12 B (key + value) by the scatter, then
    # 4 B (run bounds) + 8 B (unit counts) + 8 B (scatter) read; per (tile,
    # Gaussian) pair the 4 B index written to its list.
    supers = fr.rws.super_pair_count()
    sxn, syn = -(-fr.rws.layout.tiles_x // 8), -(-fr.rws.layout.tiles_y // 8)
    st_total = sxn * syn * len(fr.views)
    st_bits = max(1, (st_total - 1).bit_length())
    st_passes = max(1, -(-st_bits // radix))
    bin_bytes = supers * (28 * st_passes + 20) + fr.pairs * 4
    bin_gbs = bin_bytes / (stages["gs_sort"] * 1e-3) / 1e9
    result = dict(metric="stereo foveated frames/s @2016x2240/eye; rasterizer HBM GB/s vs peak",
                  value=round(fps, 3), unit="frames/s", n_gpus=1, steps=args.steps,
                  warmup=args.warmup, ms_per_step=round(ms, 4), higher_is_better=True,
                  scaling="weak", vs_baseline=None, dtype="f32+bf16", data="synthetic",
                  config=dict(workload=f"config {args.config}: stereo 2016x2240/eye, 500k "
                              "Gaussians SH3, 5M neural points, 8 crops/eye 256..640 px, "
                              "decoder 16/32/64/64 BF16, hipGraph replay",
                              tile=tile, radix_bits=radix, pairs=fr.pairs, fragments=fr.frags),
                  roofline=roofline, decoder_mfma=decoder_mfma,
                  rasterizer_hbm=dict(stage="periphery tile binning (super-tile sort, "
                                      "count, scatter)", achieved=round(bin_gbs, 1),
                                      peak=HBM_PEAK_GBS, unit="GB/s",
                                      frac=round(bin_gbs / HBM_PEAK_GBS, 4),
                                      bytes=bin_bytes, super_pairs=supers),
                  stages_ms={k: round(v, 4) for k, v in stages.items()},
                  autotune=tune)
    if not args.no_plain:
        pf = PlainFrame(fr)
        for _ in range(2):
            pf.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = max(3, args.steps // 3)
        for _ in range(k):
            pf.run()
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) / k * 1e3
        result["plain_fp32_eager"] = dict(ms_per_frame=round(pms, 4), frames_per_s=round(1e3 / pms, 3))
        log(f"plain FP32 eager: {pms:.3f} ms/frame")
        del pf
    del fr
    free()
    if not args.no_extras:
        k = max(5, args.steps // 3)
        result.update(secondary_and_standalone(scene, tile, radix, k))
        log("secondary / standalone:", json.dumps({x: result[x] for x in
                                                   ("secondary_vr_frame", "config1_periphery",
                                                    "periphery_pixel_order", "config2_fovea")}))
        result.update(table3_and_fig2(scene, tile, radix, k))
        log("table 3 / fig 2:", json.dumps({x: result[x] for x in ("table3", "fig2")}))
        result.update(post_and_training(scene, k))
        log("post / training:", json.dumps(result["post_and_training"]))
    if not args.no_cpu_baseline:
        cb = cpu_baseline(scene)
        result["cpu_baseline"] = cb
        log(f"cpu baseline: {cb['seconds_per_frame']:.1f} s/frame on {cb['cores']} threads")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
