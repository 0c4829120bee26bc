"""Seeded synthetic inputs for the foveated hybrid renderer.

This module only draws numbers and lays them out.  It holds none of the
renderer's arithmetic: covariances, opacities, projections, colours and
everything downstream are computed by the library (and, in tests, by the
independent CPU reference).  Both sides read the arrays produced here.

The scenes stand in for the paper's captured MipNeRF-360 / Tanks&Temples
scenes (Sec. 4 "Evaluation": 0.3-0.5M Gaussians, about 5M neural points,
2016x2240 pixels per eye, 512 px fovea), which are not available here: the
counts, resolutions and crop sizes match, the content is random.

Draw order for one scene (numpy ``default_rng(seed)``):
  1. Gaussians: means, log-scales, quaternions, opacity logits, SH coefficients
  2. neural points: positions, radii, features
  3. decoder weights (level 0 .. n-1, then the RGB head)
  4. gaze positions and crop sizes
Camera rigs are fixed by the configuration and draw nothing, except the
random fitting cameras, which are drawn after step 4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# The degree-0 real spherical harmonic is the constant 1/(2 sqrt(pi)); a DC
# coefficient k gives colour 0.5 + k/(2 sqrt(pi)).  Drawing k as below makes
# the degree-0 colour uniform in [0, 1].
_DC_SCALE = 2.0 * math.sqrt(math.pi)


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------
def gaussians(rng: np.random.Generator, n: int, sh_degree: int,
              xy=(-1.0, 1.0), z=(2.0, 6.0), logscale=(-3.0, 0.5),
              sh_hi_sigma=0.05) -> dict:
    """Gaussian parameters in structure-of-arrays layout.

    mean [3][n] (x,y uniform in ``xy``, z uniform in ``z``), logscale [3][n]
    ~ N(mu, sigma) per axis, quat [4][n] (w,x,y,z) uniform on S^3 (normalised
    4-D standard normal), logit [n] ~ N(0,1), sh [K][3][n] with K=(deg+1)^2:
    the DC band gives an RGB uniform in [0,1], higher bands ~ N(0, sh_hi_sigma).
    """
    mean = np.empty((3, n), np.float32)
    mean[0] = rng.uniform(xy[0], xy[1], n)
    mean[1] = rng.uniform(xy[0], xy[1], n)
    mean[2] = rng.uniform(z[0], z[1], n)
    ls = rng.normal(logscale[0], logscale[1], (3, n)).astype(np.float32)
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    logit = rng.standard_normal(n).astype(np.float32)
    k = (sh_degree + 1) ** 2
    sh = np.empty((k, 3, n), np.float32)
    sh[0] = (rng.uniform(0.0, 1.0, (3, n)) - 0.5) * _DC_SCALE
    if k > 1:
        sh[1:] = rng.normal(0.0, sh_hi_sigma, (k - 1, 3, n))
    return dict(mean=mean, logscale=ls, quat=q.astype(np.float32), logit=logit,
                sh=sh, sh_degree=sh_degree, n=n)


def points(rng: np.random.Generator, n: int, radius: str = "uniform",
           xy=(-1.0, 1.0), z=(2.0, 6.0), channels: int = 4) -> dict:
    """Neural points: pos [3][n] f32, radius [n] f32 (world units),
    feat [n][channels] IEEE half bits (uint16), features ~ N(0,1).

    ``radius``: "uniform" -> U[0.005, 0.02]; "lognormal" -> ln r ~ N(-5, 0.5).
    """
    pos = np.empty((3, n), np.float32)
    pos[0] = rng.uniform(xy[0], xy[1], n)
    pos[1] = rng.uniform(xy[0], xy[1], n)
    pos[2] = rng.uniform(z[0], z[1], n)
    if radius == "uniform":
        r = rng.uniform(0.005, 0.02, n)
    elif radius == "lognormal":
        r = np.exp(rng.normal(-5.0, 0.5, n))
    else:
        raise ValueError(radius)
    feat = rng.standard_normal((n, channels)).astype(np.float16)
    return dict(pos=pos, radius=r.astype(np.float32),
                feat=np.ascontiguousarray(feat).view(np.uint16), n=n,
                channels=channels)


def decoder_weights(rng: np.random.Generator, widths, in_ch: int,
                    rgb_ch: int = 3, sigma: float = 0.1) -> dict:
    """Gated-conv decoder weights, level 0 = finest.

    Level l takes Cin_l = in_ch (pyramid layer) + widths[l+1] (upsampled
    coarser output, absent at the coarsest level) + rgb_ch (periphery crop,
    level 0 only) channels and produces 2*widths[l] pre-activations (feature
    half then gate half).  Conv weights [2K][3][3][Cin] ~ N(0, sigma), biases
    zero; head [rgb_ch][widths[0]] ~ N(0, sigma), bias zero.
    """
    widths = list(widths)
    n = len(widths)
    levels = []
    for l in range(n):
        cin = in_ch + (widths[l + 1] if l + 1 < n else 0) + (rgb_ch if l == 0 else 0)
        w = rng.normal(0.0, sigma, (2 * widths[l], 3, 3, cin)).astype(np.float32)
        b = np.zeros(2 * widths[l], np.float32)
        levels.append((w, b))
    head_w = rng.normal(0.0, sigma, (rgb_ch, widths[0])).astype(np.float32)
    head_b = np.zeros(rgb_ch, np.float32)
    return dict(widths=widths, in_ch=in_ch, rgb_ch=rgb_ch, levels=levels,
                head=(head_w, head_b))


def pack_decoder(dw: dict) -> np.ndarray:
    """Flatten decoder weights into the packed float32 buffer the library
    takes: for level 0..n-1: W_l then b_l; then head W, head b."""
    parts = []
    for w, b in dw["levels"]:
        parts += [w.ravel(), b.ravel()]
    parts += [dw["head"][0].ravel(), dw["head"][1].ravel()]
    return np.concatenate(parts).astype(np.float32)


# --------------------------------------------------------------------------
# cameras and crops
# --------------------------------------------------------------------------
@dataclass
class View:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    rot: np.ndarray = field(default_factory=lambda: np.eye(3, dtype=np.float32))
    trans: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))
    znear: float = 0.2

    def as_floats(self) -> np.ndarray:
        """[fx, fy, cx, cy, R(9, row-major world->camera), t(3), znear]."""
        return np.concatenate([[self.fx, self.fy, self.cx, self.cy],
                               np.asarray(self.rot, np.float32).ravel(),
                               np.asarray(self.trans, np.float32).ravel(),
                               [self.znear]]).astype(np.float32)


def pinhole(width: int, height: int, f: float, eye=(0.0, 0.0, 0.0),
            rot=None) -> View:
    """Pinhole camera with principal point at the image centre, camera centre
    ``eye`` (world) and world->camera rotation ``rot`` (identity: looks +z)."""
    r = np.eye(3) if rot is None else np.asarray(rot, np.float64)
    t = -r @ np.asarray(eye, np.float64)
    return View(float(f), float(f), width / 2.0, height / 2.0, width, height,
                r.astype(np.float32), t.astype(np.float32))


def stereo_rig(width: int, height: int, f: float, ipd: float = 0.064):
    """Left and right eye, parallel axes looking +z, eyes at x = -+ipd/2."""
    return [pinhole(width, height, f, (-ipd / 2, 0.0, 0.0)),
            pinhole(width, height, f, (+ipd / 2, 0.0, 0.0))]


def yaw_pitch(yaw_deg: float, pitch_deg: float) -> np.ndarray:
    """World->camera rotation of a camera turned by yaw (about y) then pitch
    (about x)."""
    a, b = math.radians(yaw_deg), math.radians(pitch_deg)
    ry = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])
    rx = np.array([[1, 0, 0], [0, math.cos(b), -math.sin(b)], [0, math.sin(b), math.cos(b)]])
    return (ry @ rx).T


@dataclass
class Crop:
    view: int
    x0: int
    y0: int
    size: int
    gaze_x: float
    gaze_y: float

    def as_ints(self):
        return [self.view, self.x0, self.y0, self.size]


def crop_at(view: int, gaze_x: float, gaze_y: float, size: int, width: int,
            height: int) -> Crop:
    """Square crop of ``size`` around the gaze point, integer origin clamped so
    the crop stays inside the image."""
    x0 = int(min(max(round(gaze_x - size / 2), 0), width - size))
    y0 = int(min(max(round(gaze_y - size / 2), 0), height - size))
    return Crop(view, x0, y0, size, float(gaze_x), float(gaze_y))


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
RASTER_DEFAULTS = dict(tile=16, alpha_clamp=0.99, alpha_min=1.0 / 255.0,
                       t_min=1e-4, lowpass=0.3, extent=3.0, bg=(0.0, 0.0, 0.0))


def small_scene(seed: int, n_gauss: int = 1000, n_points: int = 2000,
                width: int = 128, height: int = 128, f: float = 128.0,
                sh_degree: int = 0, n_views: int = 1, crops=((64.0, 64.0, 64),),
                levels: int = 4, widths=(8, 8), radius: str = "uniform",
                crop_views=None) -> dict:
    """A parametrised tiny scene.  The default reproduces the tiny plain
    forward case: 1,000 Gaussians, 128x128, f=128, 2,000 points, one 64x64
    crop at gaze (64, 64), 4-layer pyramid, 2-level 8-channel decoder."""
    rng = np.random.default_rng(seed)
    g = gaussians(rng, n_gauss, sh_degree)
    p = points(rng, n_points, radius)
    dw = decoder_weights(rng, widths, p["channels"])
    if n_views == 1:
        views = [pinhole(width, height, f)]
    elif n_views == 2:
        views = stereo_rig(width, height, f)
    else:
        views = [pinhole(width, height, f, (0.05 * (i - (n_views - 1) / 2), 0, 0))
                 for i in range(n_views)]
    cs = []
    for i, (gx, gy, s) in enumerate(crops):
        v = crop_views[i] if crop_views is not None else 0
        cs.append(crop_at(v, gx, gy, s, width, height))
    return dict(gaussians=g, points=p, decoder=dw, views=views, crops=cs,
                levels=levels, raster=dict(RASTER_DEFAULTS), seed=seed)


def config(idx: int, seed: int | None = None) -> dict:
    """The five workload configurations (seed defaults to the index).

    0: tiny plain forward, 1: VR periphery (500k Gaussians, SH3, stereo
    2016x2240, f=1100), 2: foveal points (5M points, 512 crop at the left-eye
    centre, 16/32/64/64 decoder), 3: full stereo frame (1 + 2, eight crops
    per eye of size 256..640), 4: fitting step (1M Gaussians, 2M points, four
    1024^2 cameras, one 512 crop each)."""
    seed = idx if seed is None else seed
    if idx == 0:
        return small_scene(seed)
    rng = np.random.default_rng(seed)
    W, H, F = 2016, 2240, 1100.0
    if idx in (1, 2, 3):
        g = gaussians(rng, 500_000, 3)
        p = points(rng, 5_000_000, "lognormal") if idx >= 2 else None
        dw = decoder_weights(rng, (16, 32, 64, 64), 4) if idx >= 2 else None
        views = stereo_rig(W, H, F)
        if idx == 1:
            crops = []
        elif idx == 2:
            crops = [crop_at(0, W / 2, H / 2, 512, W, H)]
        else:
            crops = []
            for v in range(2):
                for _ in range(8):
                    s = int(rng.choice(np.arange(256, 641, 32)))
                    gx = rng.uniform(s / 2, W - s / 2)
                    gy = rng.uniform(s / 2, H - s / 2)
                    crops.append(crop_at(v, gx, gy, s, W, H))
        return dict(gaussians=g, points=p, decoder=dw, views=views, crops=crops,
                    levels=4, raster=dict(RASTER_DEFAULTS), seed=seed,
                    composite=dict(mode="linear", ring=64.0))
    if idx == 4:
        g = gaussians(rng, 1_000_000, 3)
        p = points(rng, 2_000_000, "lognormal")
        dw = decoder_weights(rng, (16, 32, 64, 64), 4)
        crops_g = [(rng.uniform(256, 1024 - 256), rng.uniform(256, 1024 - 256))
                   for _ in range(4)]
        views = []
        for _ in range(4):
            eye = (rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), rng.uniform(-1.0, 0.0))
            rot = yaw_pitch(rng.uniform(-10, 10), rng.uniform(-10, 10))
            views.append(pinhole(1024, 1024, 512.0, eye, rot))
        crops = [crop_at(i, gx, gy, 512, 1024, 1024) for i, (gx, gy) in enumerate(crops_g)]
        target = perturbed_copy(g, rng)
        return dict(gaussians=g, points=p, decoder=dw, views=views, crops=crops,
                    levels=4, raster=dict(RASTER_DEFAULTS), seed=seed,
                    target_gaussians=target, composite=dict(mode="linear", ring=64.0))
    raise ValueError(idx)


def perturbed_copy(g: dict, rng: np.random.Generator, mean_sigma=0.01,
                   colour_sigma=0.05) -> dict:
    """Copy of a Gaussian set with means jittered by N(0, mean_sigma) and the
    degree-0 colour jittered by N(0, colour_sigma)."""
    out = dict(g)
    out["mean"] = (g["mean"] + rng.normal(0.0, mean_sigma, g["mean"].shape)).astype(np.float32)
    sh = g["sh"].copy()
    sh[0] += (rng.normal(0.0, colour_sigma, sh[0].shape) * _DC_SCALE).astype(np.float32)
    out["sh"] = sh
    return out


def views_array(views) -> np.ndarray:
    return np.stack([v.as_floats() for v in views]).astype(np.float32)


def views_dims(views) -> np.ndarray:
    return np.array([[v.width, v.height] for v in views], np.int32)


def crops_array(crops) -> tuple[np.ndarray, np.ndarray]:
    """(ints [n][4] = view, x0, y0, size ; floats [n][2] = gaze x, y)."""
    ci = np.array([c.as_ints() for c in crops], np.int32).reshape(-1, 4)
    cf = np.array([[c.gaze_x, c.gaze_y] for c in crops], np.float32).reshape(-1, 2)
    return ci, cf
