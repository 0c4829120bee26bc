"""FP64 CPU reference of the foveated hybrid renderer -- test infrastructure.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the library never does.  The arithmetic lives in
``oracle.cpp`` (C++17, OpenMP, built with g++ -O2 -ffp-contract=off, no
fast-math); this module compiles it and wraps it with numpy.

Parity pins (see tests/test_oracle_*.py): brute-force per-pixel evaluation,
closed forms for single isotropic / anisotropic Gaussians and single points,
the A + T = 1 invariant, permutation invariance, SH orthonormality, the
Eq. 2-5 special values, and an independent float64 convolution.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_F = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_D = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_U = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_L = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_H = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")
_i64, _int, _flt, _dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_double
_vp = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile liboracle.so (g++, OpenMP, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        l = ctypes.CDLL(_LIB)
        l.orc_num_threads.restype = _int
        l.orc_sh_basis.argtypes = [_int, _i64, _D, _D]
        l.orc_bake.argtypes = [_i64, _F, _F, _F, _D, _D]
        l.orc_gauss_geom32.argtypes = [_i64, _F, _F, _int, _F, _I, _flt, _flt, _I, _U]
        l.orc_gauss_project64.argtypes = [_i64, _F, _F, _F, _F, _int, _int, _F, _I, _dbl, _D]
        l.orc_tile_lists.argtypes = [_i64, _int, _I, _int, _I, _U, _i64, _I, _L, _vp]
        l.orc_tile_lists.restype = _i64
        l.orc_render.argtypes = [_i64, _int, _I, _int, _I, _U, _D, _D, _i64, _vp,
                                 _D, _D, _D, _I, _D, _I, _vp, _vp, _vp]
        l.orc_gauss_pixdepth32.argtypes = [_i64, _F, _F, _int, _F, _I, _F]
        l.orc_gauss_pixdepth64.argtypes = [_i64, _F, _F, _int, _F, _I, _D]
        l.orc_pyramid_pixels.argtypes = [_int, _I, _int]
        l.orc_pyramid_pixels.restype = _i64
        l.orc_point_lists.argtypes = [_i64, _F, _F, _int, _F, _I, _int, _I, _int, _vp, _vp,
                                      _flt, _flt, _L, _vp]
        l.orc_point_lists.restype = _i64
        l.orc_point_frags.argtypes = [_i64, _F, _F, _int, _F, _I, _int, _I, _int, _vp, _vp,
                                      _flt, _flt, _vp]
        l.orc_point_frags.restype = _i64
        l.orc_splat_points.argtypes = [_i64, _F, _F, _H, _vp, _int, _int, _F, _I, _int, _I,
                                       _int, _vp, _vp, _flt, _flt, _D]
        l.orc_decode.argtypes = [_int, _I, _int, _int, _D, _D, _I, _int, _I, _D, _D]
        l.orc_composite.argtypes = [_int, _I, _D, _int, _I, _F, _D, _int, _dbl, _dbl, _dbl, _D]
        _lib = l
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return lib().orc_num_threads()


# ------------------------------------------------------------------ pieces
def sh_basis(deg: int, dirs: np.ndarray) -> np.ndarray:
    """Real SH basis values [n][(deg+1)^2] at unit directions [n][3]."""
    dirs = _c(dirs, np.float64)
    out = np.zeros((dirs.shape[0], (deg + 1) ** 2))
    lib().orc_sh_basis(deg, dirs.shape[0], dirs, out)
    return out


def bake(logscale, quat, logit):
    """(cov [6][n] float64, opacity [n] float64) -- Sigma = R diag(s^2) R^T,
    opacity = sigmoid(logit)."""
    n = logit.shape[0]
    cov = np.zeros((6, n))
    op = np.zeros(n)
    lib().orc_bake(n, _c(logscale, np.float32), _c(quat, np.float32), _c(logit, np.float32),
                   cov, op)
    return cov, op


def gauss_geom32(mean, cov, views, dims, lowpass=0.3, extent=3.0):
    """Single-precision decisions: (rect [v][n][4] int32, zbits [v][n] uint32)."""
    n = mean.shape[1]
    nv = views.shape[0]
    rect = np.zeros((nv, n, 4), np.int32)
    zb = np.zeros((nv, n), np.uint32)
    lib().orc_gauss_geom32(n, _c(mean, np.float32), _c(cov, np.float32), nv,
                           _c(views, np.float32), _c(dims, np.int32), lowpass, extent, rect, zb)
    return rect, zb


def gauss_project64(mean, cov, opacity, sh, deg, views, dims, lowpass=0.3):
    """Double-precision projected records [v][n][10]
    (px, py, A, B, C, opacity, r, g, b, tz)."""
    n = mean.shape[1]
    nv = views.shape[0]
    rec = np.zeros((nv, n, 10))
    lib().orc_gauss_project64(n, _c(mean, np.float32), _c(cov, np.float32),
                              _c(opacity, np.float32), _c(sh, np.float32), deg, nv,
                              _c(views, np.float32), _c(dims, np.int32), lowpass, rec)
    return rec


def tile_lists(rect, zbits, dims, tile, sel):
    """Sorted Gaussian lists of the selected (view, tile) pairs:
    (offsets [nsel+1] int64, ids int32)."""
    nv, n = zbits.shape
    sel = _c(sel, np.int32).reshape(-1, 2)
    off = np.zeros(sel.shape[0] + 1, np.int64)
    l = lib()
    l.orc_tile_lists(n, nv, _c(dims, np.int32), tile, _c(rect, np.int32), _c(zbits, np.uint32),
                     sel.shape[0], sel, off, None)
    ids = np.zeros(max(int(off[-1]), 1), np.int32)
    l.orc_tile_lists(n, nv, _c(dims, np.int32), tile, _c(rect, np.int32), _c(zbits, np.uint32),
                     sel.shape[0], sel, off, _ptr(ids))
    return off, ids[:off[-1]]


def gauss_pixdepth(mean, cov, views, dims):
    """Per-pixel depth coefficients of every (view, Gaussian) for the
    per-pixel order (Sec. 3.2): (single-precision [v][n][9] decision mirror,
    double-precision [v][n][9] values), see orc_gauss_pixdepth32."""
    n = mean.shape[1]
    nv = views.shape[0]
    c32 = np.zeros((nv, n, 9), np.float32)
    c64 = np.zeros((nv, n, 9))
    args = (n, _c(mean, np.float32), _c(cov, np.float32), nv, _c(views, np.float32),
            _c(dims, np.int32))
    lib().orc_gauss_pixdepth32(*args, c32)
    lib().orc_gauss_pixdepth64(*args, c64)
    return c32, c64


def render(rect, zbits, rec, dims, tile=16, alpha_clamp=0.99, alpha_min=1 / 255, t_min=1e-4,
           bg=(0.0, 0.0, 0.0), pix=None, per_pixel=None):
    """Blend.  With ``pix`` None: dict of full images rgb [v][3][H][W],
    depth/tfinal/margin [v][H][W], ncontrib [v][H][W]; else per-pixel arrays
    for pix [n][3] = (view, x, y).  per_pixel = (coef32, coef64, views):
    the per-pixel order (gauss_pixdepth's coefficients, the views array)."""
    nv, n = zbits.shape
    dims = _c(dims, np.int32)
    pp = (None, None, None)
    if per_pixel is not None:
        c32, c64, vw = per_pixel
        keep = (_c(c32, np.float32), _c(c64, np.float64), _c(vw, np.float32))
        pp = tuple(_ptr(a) for a in keep)
    opts = np.array([alpha_clamp, alpha_min, t_min, *bg], np.float64)
    if pix is None:
        npix = int(sum(int(w) * int(h) for w, h in dims))
        pixarr = None
    else:
        pixarr = _c(pix, np.int32).reshape(-1, 3)
        npix = pixarr.shape[0]
    rgb = np.zeros((npix, 3))
    depth = np.zeros(npix)
    tf = np.zeros(npix)
    nc = np.zeros(npix, np.int32)
    mg = np.zeros(npix)
    ev = np.zeros(npix, np.int32)
    lib().orc_render(n, nv, dims, tile, _c(rect, np.int32), _c(zbits, np.uint32),
                     _c(rec, np.float64), opts, npix, _ptr(pixarr), rgb, depth, tf, nc, mg, ev,
                     *pp)
    if pix is not None:
        return dict(rgb=rgb, depth=depth, tfinal=tf, ncontrib=nc, margin=mg, evals=ev)
    out = dict(rgb=[], depth=[], tfinal=[], ncontrib=[], margin=[], evals=[])
    o = 0
    for w, h in dims:
        k = int(w) * int(h)
        out["rgb"].append(rgb[o:o + k].reshape(h, w, 3).transpose(2, 0, 1))
        for name, arr in (("depth", depth), ("tfinal", tf), ("ncontrib", nc), ("margin", mg),
                          ("evals", ev)):
            out[name].append(arr[o:o + k].reshape(h, w))
        o += k
    return {k: np.stack(v) for k, v in out.items()}


def _pix_order(c32, c64, view_row, x, y, ids):
    """Per-pixel order of ids at pixel (x, y) (see orc_gauss_pixdepth32):
    (ids sorted by (order-preserving bits of the single-precision key,
    index), their double-precision z*)."""
    f = np.float32
    fx, fy, cx, cy = (f(view_row[k]) for k in range(4))
    u = (f(x) + f(0.5) - cx) / fx
    v = (f(y) + f(0.5) - cy) / fy
    k = c32[ids]
    num = (k[:, 6] * u + k[:, 7] * v) + k[:, 8]
    den = ((k[:, 0] * u + k[:, 1] * v + k[:, 2]) * u + (k[:, 3] * v + k[:, 4]) * v) + k[:, 5]
    bits = (num / den).astype(np.float32).view(np.uint32)
    ordk = np.where(bits >> 31 == 1, ~bits, bits | np.uint32(0x80000000))
    ids = ids[np.lexsort((ids, ordk))]
    ud = (x + 0.5 - float(view_row[2])) / float(view_row[0])
    vd = (y + 0.5 - float(view_row[3])) / float(view_row[1])
    k = c64[ids]
    z = (k[:, 6] * ud + k[:, 7] * vd + k[:, 8]) / (k[:, 0] * ud * ud + k[:, 1] * ud * vd +
                                                   k[:, 2] * ud + k[:, 3] * vd * vd +
                                                   k[:, 4] * vd + k[:, 5])
    return ids, z


def render_branches(rect, zbits, rec, pix, alpha_clamp=0.99, alpha_min=1 / 255, t_min=1e-4,
                    bg=(0.0, 0.0, 0.0), margin=1e-4, max_alt=64, per_pixel=None):
    """Every result a pixel may legitimately take when single precision
    decides its blend thresholds (Sec. 3.2 blend; the thresholds alpha_min
    and t_min are the rasteriser options): the per-pixel blend of ``render``
    walked again in float64, but wherever a decision (alpha against
    alpha_min, the next transmittance against t_min) lies within ``margin``
    (relative) of its threshold, both branches are followed.  Returns, per
    pixel of pix [n][3] = (view, x, y), a list of (ncontrib, rgb[3], depth,
    tfinal) tuples, at most max_alt of them (the first one follows the
    float64 decisions).  Plain per-pixel Python: for the few pixels whose
    decisions are that close.  per_pixel = (coef32, coef64, views): the
    per-pixel order, as for render."""
    bg = np.asarray(bg, np.float64)
    out = []
    for v, x, y in np.asarray(pix, np.int64).reshape(-1, 3):
        r = rect[v]
        m = (r[:, 0] >= 0) & (r[:, 0] <= x) & (x <= r[:, 2]) & (r[:, 1] <= y) & (y <= r[:, 3])
        ids = np.nonzero(m)[0]
        if per_pixel is None:
            ids = ids[np.lexsort((ids, zbits[v, ids]))]
            g = rec[v, ids]
            depth = g[:, 9]
        else:
            c32, c64, vw = per_pixel
            ids, depth = _pix_order(c32[v], c64[v], np.asarray(vw)[v], x, y, ids)
            g = rec[v, ids]
        dx, dy = g[:, 0] - (x + 0.5), g[:, 1] - (y + 0.5)
        q = -0.5 * (g[:, 2] * dx * dx + g[:, 4] * dy * dy) - g[:, 3] * dx * dy
        a = np.minimum(alpha_clamp, g[:, 5] * np.exp(q))
        alts = []
        # states (list position, T, C, D, count, forced alpha decision,
        # forced stop decision at that position); the float64 path first
        stack = [(0, 1.0, np.zeros(3), 0.0, 0, None, None)]
        while stack and len(alts) < max_alt:
            k, T, C, D, cnt, fa, fs = stack.pop()
            while True:
                if k >= len(ids):
                    alts.append((cnt, C + T * bg, D, T))
                    break
                if q[k] > 0:
                    k, fa, fs = k + 1, None, None
                    continue
                take = bool(a[k] >= alpha_min) if fa is None else fa
                if fa is None and abs(a[k] - alpha_min) / alpha_min < margin:
                    stack.append((k, T, C.copy(), D, cnt, not take, None))
                if not take:
                    k, fa, fs = k + 1, None, None
                    continue
                Tn = T * (1 - a[k])
                stop = bool(Tn < t_min) if fs is None else fs
                if fs is None and abs(Tn - t_min) / t_min < margin:
                    stack.append((k, T, C.copy(), D, cnt, True, not stop))
                if stop:
                    alts.append((cnt, C + T * bg, D, T))
                    break
                C = C + g[k, 6:9] * a[k] * T
                D = D + depth[k] * a[k] * T
                T, cnt, k, fa, fs = Tn, cnt + 1, k + 1, None, None
        out.append(alts)
    return out


def pyramid_pixels(crops_i, levels) -> int:
    return int(lib().orc_pyramid_pixels(crops_i.shape[0], _c(crops_i, np.int32), levels))


def point_lists(pos, radius, views, dims, crops_i, levels, depth=None, tfinal=None,
                cov_min=0.5, slack=1.05):
    """Per layer pixel fragment lists: (offsets [P+1] int64, point ids)."""
    np_ = pos.shape[1]
    crops_i = _c(crops_i, np.int32)
    P = pyramid_pixels(crops_i, levels)
    off = np.zeros(P + 1, np.int64)
    d = None if depth is None else _c(depth, np.float32)
    t = None if tfinal is None else _c(tfinal, np.float32)
    l = lib()
    args = (np_, _c(pos, np.float32), _c(radius, np.float32), views.shape[0],
            _c(views, np.float32), _c(dims, np.int32), crops_i.shape[0], crops_i, levels,
            _ptr(d), _ptr(t), cov_min, slack, off)
    cnt = l.orc_point_lists(*args, None)
    ids = np.zeros(max(cnt, 1), np.int32)
    l.orc_point_lists(*args, _ptr(ids))
    return off, ids[:cnt]


def point_frags(pos, radius, views, dims, crops_i, levels, depth=None, tfinal=None,
                cov_min=0.5, slack=1.05):
    """Fragments in blend order with their integer decisions:
    int64 [nfrag][8] = key, point id, crop, layer, ix, iy, l0, two."""
    crops_i = _c(crops_i, np.int32)
    d = None if depth is None else _c(depth, np.float32)
    t = None if tfinal is None else _c(tfinal, np.float32)
    args = (pos.shape[1], _c(pos, np.float32), _c(radius, np.float32), views.shape[0],
            _c(views, np.float32), _c(dims, np.int32), crops_i.shape[0], crops_i, levels,
            _ptr(d), _ptr(t), cov_min, slack)
    l = lib()
    cnt = l.orc_point_frags(*args, None)
    out = np.zeros((max(cnt, 1), 8), np.int64)
    l.orc_point_frags(*args, _ptr(out))
    return out[:cnt]


def splat_points(pos, radius, feat, views, dims, crops_i, levels, depth=None, tfinal=None,
                 opacity=None, cov_min=0.5, slack=1.05):
    """Packed pyramid [P][C] float64 (layer pixels of all crops and layers)."""
    np_ = pos.shape[1]
    C = feat.shape[1]
    crops_i = _c(crops_i, np.int32)
    P = pyramid_pixels(crops_i, levels)
    out = np.zeros((P, C))
    d = None if depth is None else _c(depth, np.float32)
    t = None if tfinal is None else _c(tfinal, np.float32)
    o = None if opacity is None else _c(opacity, np.float32)
    lib().orc_splat_points(np_, _c(pos, np.float32), _c(radius, np.float32),
                           _c(feat, np.uint16), _ptr(o), C, views.shape[0],
                           _c(views, np.float32), _c(dims, np.int32), crops_i.shape[0], crops_i,
                           levels, _ptr(d), _ptr(t), cov_min, slack, out)
    return out


def decode(crops_i, levels, channels, pyramid, periph, dims, widths, weights):
    """Foveal RGB, packed [sum_k 3 S_k^2] float64."""
    crops_i = _c(crops_i, np.int32)
    tot = int(sum(3 * int(s) ** 2 for s in crops_i[:, 3]))
    out = np.zeros(tot)
    w = np.asarray(widths, np.int32)
    lib().orc_decode(crops_i.shape[0], crops_i, levels, channels, _c(pyramid, np.float64),
                     _c(periph, np.float64), _c(dims, np.int32), len(w), w,
                     _c(weights, np.float64), out)
    return out


def composite(P, dims, crops_i, gaze, F, mode=0, ring=64.0, m=0.75, gamma=0.2):
    """Combined frame [v][3][H][W] float64 (mode 0 linear ring, 1 Eqs. 2-5)."""
    crops_i = _c(crops_i, np.int32)
    out = np.zeros(np.shape(P), np.float64)
    lib().orc_composite(len(dims), _c(dims, np.int32), _c(P, np.float64), crops_i.shape[0],
                        crops_i, _c(gaze, np.float32).reshape(-1, 2), _c(F, np.float64), mode,
                        ring, m, gamma, out)
    return out
