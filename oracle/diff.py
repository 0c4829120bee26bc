"""Differentiable FP64 reference -- test infrastructure, like the rest of
``oracle``: only tests, the smoke check and the benchmark's CPU leg use it.

The renderer's definitions written once more as plain torch CPU float64 ops,
so that autograd yields the analytic gradients the HIP adjoint kernels are
checked against (Sec. 3.5: the pipeline is optimised end to end).  The
integer decisions (culling, pixel rectangles, depth order, pyramid layer and
target pixels) are taken exactly as in ``oracle.cpp`` (single precision,
documented order) and are constants of the differentiation; the
floating-point thresholds of the blend (alpha below alpha_min, the
transmittance stop) are decided on the float64 values, as in ``oracle.cpp``.

Pins (tests/test_oracle_grad.py): every forward here equals the
corresponding ``oracle.cpp`` forward to 1e-10; every gradient equals FP64
central differences (h = 1e-6 max(1, |theta|)) of the same forward, with
coordinates whose discrete decisions flip inside [theta - h, theta + h]
skipped and counted.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as Fnn

from . import gauss_geom32, point_frags

DT = torch.float64


def _t(a):
    return a if torch.is_tensor(a) else torch.as_tensor(np.asarray(a), dtype=DT)


def _f32(t):
    return np.ascontiguousarray(t.detach().cpu().numpy().astype(np.float32))


def camera(view_row, dims_row):
    """float64 camera from the 17-float view record (fx, fy, cx, cy, R, t,
    znear) and (W, H)."""
    v = np.asarray(view_row, np.float32).astype(np.float64)
    R = torch.tensor(v[4:13].reshape(3, 3), dtype=DT)
    t = torch.tensor(v[13:16], dtype=DT)
    return dict(fx=float(v[0]), fy=float(v[1]), cx=float(v[2]), cy=float(v[3]), R=R, t=t,
                znear=float(v[16]), W=int(dims_row[0]), H=int(dims_row[1]), o=-(R.T @ t))


# ------------------------------------------------------------------- bake
def bake(logscale, quat, logit):
    """Sigma = R(q/|q|) diag(exp(2 logscale)) R^T (6-vector), sigmoid(logit)."""
    q = quat / quat.norm(dim=0, keepdim=True)
    w, x, y, z = q
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)])])
    s2 = torch.exp(2 * logscale)                  # [3][n]
    S = torch.einsum("ikn,kn,jkn->ijn", R, s2, R)
    cov = torch.stack([S[0, 0], S[0, 1], S[0, 2], S[1, 1], S[1, 2], S[2, 2]])
    return cov, torch.sigmoid(logit)


# ---------------------------------------------------------------- periphery
def sh_basis(deg, d):
    """Real SH (graphics sign convention, degree <= 3) at unit rows of d."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    c0 = 0.5 * math.sqrt(1 / math.pi)
    out = [torch.full_like(x, c0)]
    if deg >= 1:
        c1 = math.sqrt(3 / (4 * math.pi))
        out += [-c1 * y, c1 * z, -c1 * x]
    if deg >= 2:
        a, b, c = 0.5 * math.sqrt(15 / math.pi), 0.25 * math.sqrt(5 / math.pi), 0.25 * math.sqrt(15 / math.pi)
        out += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z, c * (x * x - y * y)]
    if deg >= 3:
        a = 0.25 * math.sqrt(35 / (2 * math.pi))
        b = 0.5 * math.sqrt(105 / math.pi)
        c = 0.25 * math.sqrt(21 / (2 * math.pi))
        dd = 0.25 * math.sqrt(7 / math.pi)
        e = 0.25 * math.sqrt(105 / math.pi)
        out += [-a * y * (3 * x * x - y * y), b * x * y * z, -c * y * (4 * z * z - x * x - y * y),
                dd * z * (2 * z * z - 3 * x * x - 3 * y * y), -c * x * (4 * z * z - x * x - y * y),
                e * z * (x * x - y * y), -a * x * (x * x - 3 * y * y)]
    return torch.stack(out, 1)


def project(mean, cov, opacity, sh, deg, cam, lowpass=0.3):
    """EWA projection of every Gaussian into one camera: dict of [n] tensors
    px, py, A, B, C (conic), op, z and rgb [n][3]."""
    R, tv = cam["R"], cam["t"]
    t = R @ mean + tv[:, None]
    tz = t[2]
    ux, uy = t[0] / tz, t[1] / tz
    limx = 1.3 * (0.5 * cam["W"] / cam["fx"])
    limy = 1.3 * (0.5 * cam["H"] / cam["fy"])
    jx, jy = cam["fx"] / tz, cam["fy"] / tz
    j02 = -jx * torch.clamp(ux, -limx, limx)
    j12 = -jy * torch.clamp(uy, -limy, limy)
    M0 = jx[:, None] * R[0][None] + j02[:, None] * R[2][None]      # [n][3]
    M1 = jy[:, None] * R[1][None] + j12[:, None] * R[2][None]
    S = torch.stack([torch.stack([cov[0], cov[1], cov[2]], 1),
                     torch.stack([cov[1], cov[3], cov[4]], 1),
                     torch.stack([cov[2], cov[4], cov[5]], 1)], 1)   # [n][3][3]
    M = torch.stack([M0, M1], 1)                                    # [n][2][3]
    C2 = M @ S @ M.transpose(1, 2)
    a = C2[:, 0, 0] + lowpass
    b = C2[:, 0, 1]
    c = C2[:, 1, 1] + lowpass
    det = a * c - b * b
    d = mean.T - cam["o"][None]
    d = d / d.norm(dim=1, keepdim=True)
    Y = sh_basis(deg, d)                                            # [n][K]
    K = Y.shape[1]
    rgb = torch.clamp(0.5 + torch.einsum("nk,kcn->nc", Y, sh[:K]), min=0.0)
    return dict(px=cam["fx"] * ux + cam["cx"], py=cam["fy"] * uy + cam["cy"], A=c / det,
                B=-b / det, C=a / det, op=opacity, z=tz, rgb=rgb)


def pixel_lists(rect, zbits, pix, reach=None):
    """Padded per-pixel candidate lists in (depth bits, index) order:
    (idx [P][L] int64, valid [P][L] bool).  reach [P] (optional): pixel k
    evaluates only the first reach[k] entries of its list (the blend stops
    there), so the list is cut after them."""
    lists = []
    for k, (v, x, y) in enumerate(pix):
        r = rect[v]
        m = (r[:, 0] >= 0) & (r[:, 0] <= x) & (x <= r[:, 2]) & (r[:, 1] <= y) & (y <= r[:, 3])
        ids = np.nonzero(m)[0]
        ids = ids[np.lexsort((ids, zbits[v, ids]))]
        lists.append(ids if reach is None else ids[:int(reach[k])])
    L = max([len(l) for l in lists] + [1])
    idx = np.zeros((len(lists), L), np.int64)
    valid = np.zeros((len(lists), L), bool)
    for i, l in enumerate(lists):
        idx[i, :len(l)] = l
        valid[i, :len(l)] = True
    return idx, valid


def render(mean, cov, opacity, sh, deg, views, dims, pix, raster, reach=None):
    """Blend the requested pixels pix [P][3] = (view, x, y): dict rgb [P][3],
    depth [P], tfinal [P] (differentiable w.r.t. mean, cov, opacity, sh).
    reach: see pixel_lists (entries past a pixel's stop never contribute)."""
    pix = np.asarray(pix, np.int64).reshape(-1, 3)
    rect, zb = gauss_geom32(_f32(mean), _f32(cov), views, dims, raster["lowpass"],
                            raster["extent"])
    n = mean.shape[1]
    projs = [project(mean, cov, opacity, sh, deg, camera(views[v], dims[v]), raster["lowpass"])
             for v in range(len(views))]
    cat = {k: torch.cat([p[k] for p in projs]) for k in projs[0]}
    idx, valid = pixel_lists(rect, zb, pix, reach)
    gidx = torch.as_tensor(idx + pix[:, :1] * n)
    validt = torch.as_tensor(valid)
    xc = torch.as_tensor(pix[:, 1:2] + 0.5, dtype=DT)
    yc = torch.as_tensor(pix[:, 2:3] + 0.5, dtype=DT)
    dx = cat["px"][gidx] - xc
    dy = cat["py"][gidx] - yc
    q = -0.5 * (cat["A"][gidx] * dx * dx + cat["C"][gidx] * dy * dy) - cat["B"][gidx] * dx * dy
    alpha = torch.minimum(torch.full_like(q, raster["alpha_clamp"]), cat["op"][gidx] * torch.exp(q))
    with torch.no_grad():
        skip = (~validt) | (q > 0) | (alpha < raster["alpha_min"])
    a_eff = torch.where(skip, torch.zeros_like(alpha), alpha)
    Tn = torch.cumprod(1 - a_eff, 1)
    Tb = torch.cat([torch.ones_like(Tn[:, :1]), Tn[:, :-1]], 1)
    with torch.no_grad():
        stop = (~skip) & (Tn < raster["t_min"])
        first = torch.where(stop.any(1), stop.float().argmax(1), torch.full((len(pix),), Tn.shape[1]))
        keep = torch.arange(Tn.shape[1])[None] < first[:, None]
    w = a_eff * Tb * keep
    rgb = (w[..., None] * cat["rgb"][gidx]).sum(1)
    depth = (w * cat["z"][gidx]).sum(1)
    Tfull = torch.cat([torch.ones_like(Tn[:, :1]), Tn], 1)
    tfinal = Tfull.gather(1, first[:, None]).squeeze(1)
    rgb = rgb + tfinal[:, None] * torch.as_tensor(np.asarray(raster["bg"], np.float64))[None]
    return dict(rgb=rgb, depth=depth, tfinal=tfinal)


# -------------------------------------------------------------------- fovea
def _layer_table(crops_i, L):
    base, o = {}, 0
    for k, (_, _, _, S) in enumerate(crops_i):
        for l in range(L):
            s = int(S) >> l
            base[(k, l)] = (o, s)
            o += s * s
    return base, o


def splat(pos, radius, feat, opacity, views, dims, crops_i, L, depth=None, tfinal=None,
          cov_min=0.5, slack=1.05):
    """Pyramid [P][C] (differentiable w.r.t. pos, radius, feat, opacity)."""
    crops_i = np.asarray(crops_i, np.int32).reshape(-1, 4)
    fr = point_frags(_f32(pos), _f32(radius), views, dims, crops_i, L, depth, tfinal, cov_min,
                     slack)
    base, P = _layer_table(crops_i, L)
    C = feat.shape[1]
    if len(fr) == 0:
        return torch.zeros((P, C), dtype=DT) + 0 * feat.sum()
    key, pid, crop, layer, ix, iy, l0, two = (fr[:, j] for j in range(8))
    view = crops_i[crop, 0]
    cams = [camera(views[v], dims[v]) for v in range(len(views))]
    Rs = torch.stack([c["R"] for c in cams])[view]                  # [f][3][3]
    ts = torch.stack([c["t"] for c in cams])[view]
    fx = torch.as_tensor([cams[v]["fx"] for v in view], dtype=DT)
    fy = torch.as_tensor([cams[v]["fy"] for v in view], dtype=DT)
    cx = torch.as_tensor([cams[v]["cx"] for v in view], dtype=DT)
    cy = torch.as_tensor([cams[v]["cy"] for v in view], dtype=DT)
    pid_t = torch.as_tensor(pid)
    t = torch.einsum("fij,jf->fi", Rs, pos[:, pid_t]) + ts
    px = fx * t[:, 0] / t[:, 2] + cx
    py = fy * t[:, 1] / t[:, 2] + cy
    s = 2 * fx * radius[pid_t] / t[:, 2]
    l0t = torch.as_tensor(l0, dtype=DT)
    f = torch.log2(s) - l0t
    layer_t = torch.as_tensor(layer)
    wl = torch.where(torch.as_tensor(two) == 1,
                     torch.where(layer_t == torch.as_tensor(l0), 1 - f, f), torch.ones_like(f))
    sc = torch.as_tensor(np.ldexp(1.0, -layer), dtype=DT)
    x0 = torch.as_tensor(crops_i[crop, 1], dtype=DT)
    y0 = torch.as_tensor(crops_i[crop, 2], dtype=DT)
    xl = (px - x0) * sc - 0.5
    yl = (py - y0) * sc - 0.5
    bx = xl - torch.as_tensor(ix, dtype=DT)
    by = yl - torch.as_tensor(iy, dtype=DT)
    local = key - np.array([base[(int(k), int(l))][0] for k, l in zip(crop, layer)])
    Sl = np.array([base[(int(k), int(l))][1] for k, l in zip(crop, layer)])
    xx, yy = local % Sl, local // Sl
    dxs = torch.as_tensor(xx - ix)
    dys = torch.as_tensor(yy - iy)
    wb = torch.where(dxs == 1, bx, 1 - bx) * torch.where(dys == 1, by, 1 - by)
    w = wl * wb
    alpha = w * (opacity[pid_t] if opacity is not None else 1.0)
    # segments (fragments are already in blend order, grouped by key)
    ukeys, start, counts = np.unique(key, return_index=True, return_counts=True)
    Lmax = int(counts.max())
    seg = np.repeat(np.arange(len(ukeys)), counts)
    pos_in = np.arange(len(key)) - start[seg]
    A = torch.zeros((len(ukeys), Lmax), dtype=DT)
    A = A.index_put((torch.as_tensor(seg), torch.as_tensor(pos_in)), alpha)
    Tn = torch.cumprod(1 - A, 1)
    Tb = torch.cat([torch.ones_like(Tn[:, :1]), Tn[:, :-1]], 1)
    wT = alpha * Tb[torch.as_tensor(seg), torch.as_tensor(pos_in)]
    contrib = wT[:, None] * feat[pid_t]
    out = torch.zeros((P, C), dtype=DT).index_add(0, torch.as_tensor(key), contrib)
    return out


def decode(pyramid, periph, crops_i, L, widths, levels_w, head):
    """Foveal images, packed [crop][3][S][S] flattened: one gated 3x3 conv
    per level (coarse to fine), bilinear x2 upsample with half-pixel centres
    and edge clamp, periphery crop injected at level 0, 1x1 RGB head."""
    crops_i = np.asarray(crops_i, np.int32).reshape(-1, 4)
    base, _ = _layer_table(crops_i, L)
    nd = len(widths)
    outs = []
    for k, (v, x0, y0, S) in enumerate(crops_i):
        h = None
        for l in range(nd - 1, -1, -1):
            o, s = base[(k, l)]
            X = pyramid[o:o + s * s].reshape(s, s, -1).permute(2, 0, 1)[None]
            parts = [X]
            if h is not None:
                parts.append(Fnn.interpolate(h, scale_factor=2, mode="bilinear", align_corners=False))
            if l == 0:
                parts.append(periph[v, :, y0:y0 + S, x0:x0 + S][None])
            x = torch.cat(parts, 1)
            w, b = levels_w[l]
            y = Fnn.conv2d(x, w.permute(0, 3, 1, 2), b, padding=1)
            K = widths[l]
            h = Fnn.elu(y[:, :K]) * torch.sigmoid(y[:, K:])
        hw, hb = head
        F = torch.einsum("ck,bkyx->bcyx", hw, h) + hb[None, :, None, None]
        outs.append(F[0].reshape(-1))
    return torch.cat(outs)


def unpack_decoder(packed, widths, in_ch=4, rgb_ch=3):
    """Views into a packed float64 weight tensor (same layout as the
    library's): [(W_l [2K][3][3][Cin], b_l [2K])...], (W_o [3][K0], b_o [3])."""
    nd = len(widths)
    levels, o = [], 0
    for l in range(nd):
        cin = in_ch + (widths[l + 1] if l + 1 < nd else 0) + (rgb_ch if l == 0 else 0)
        nw = 2 * widths[l] * 9 * cin
        w = packed[o:o + nw].reshape(2 * widths[l], 3, 3, cin)
        o += nw
        b = packed[o:o + 2 * widths[l]]
        o += 2 * widths[l]
        levels.append((w, b))
    hw = packed[o:o + rgb_ch * widths[0]].reshape(rgb_ch, widths[0])
    o += rgb_ch * widths[0]
    return levels, (hw, packed[o:o + rgb_ch])


def composite(P, F, crops_i, gaze, mode=0, ring=64.0, m=0.75, gamma=0.2):
    """Combination (Sec. 3.4, Eqs. 2-5) of P [V][3][H][W] and packed F."""
    crops_i = np.asarray(crops_i, np.int32).reshape(-1, 4)
    gaze = np.asarray(gaze, np.float32).reshape(-1, 2).astype(np.float64)
    out = [P[v] for v in range(P.shape[0])]
    fb = 0
    sob_x = torch.tensor([[-1.0, 0, 1], [-2, 0, 2], [-1, 0, 1]], dtype=DT)
    for k, (v, x0, y0, S) in enumerate(crops_i):
        Fk = F[fb:fb + 3 * S * S].reshape(3, S, S)
        fb += 3 * S * S
        ys = torch.arange(S, dtype=DT)[:, None] + y0 + 0.5 - gaze[k, 1]
        xs = torch.arange(S, dtype=DT)[None, :] + x0 + 0.5 - gaze[k, 0]
        r = torch.sqrt(xs * xs + ys * ys)
        df = 0.5 * S
        if mode == 0:
            c = torch.clamp((df - r) / ring, 0, 1)
        else:
            fp = (torch.clamp(r / df, 0, 1) - m) / (1 - m)
            g = Fk.mean(0)[None, None]
            gp = Fnn.pad(g, (1, 1, 1, 1), mode="replicate")
            gx = Fnn.conv2d(gp, sob_x[None, None])[0, 0]
            gy = Fnn.conv2d(gp, sob_x.T.contiguous()[None, None])[0, 0]
            fe = torch.sqrt(gx * gx + gy * gy + 1e-300) / 4
            u = torch.clamp(fp + gamma * fe, 0, 1)
            c = 1 - (6 * u ** 5 - 15 * u ** 4 + 10 * u ** 3)
        region = out[v][:, y0:y0 + S, x0:x0 + S]
        new = (1 - c)[None] * region + c[None] * Fk
        ov = out[v].clone()
        ov[:, y0:y0 + S, x0:x0 + S] = new
        out[v] = ov
    return torch.stack(out)


def l1(pred, target):
    return (pred - target).abs().mean()


# ------------------------------------------------- tone mapping and losses
def tonemap(img, params, principal):
    """oracle.post.tonemap as differentiable torch ops: the segment and the
    clamp are decided as there (single precision, post._decide32), the
    values in float64.  img [V][3][H][W], params [V][7 + n]."""
    from .post import PARAMS_FIXED, _decide32, vignette_r2
    V, _, H, W = img.shape
    n = params.shape[1] - PARAMS_FIXED
    outs = []
    for v in range(V):
        ev, k, lut = params[v, 0], params[v, 4:7], params[v, 7:]
        r2 = torch.tensor(vignette_r2(W, H, *principal[v]), dtype=DT)
        vig = 1.0 + k[0] * r2 + k[1] * r2 ** 2 + k[2] * r2 ** 3
        ch = []
        for c in range(3):
            t = img[v, c] * torch.pow(torch.tensor(2.0, dtype=DT), -ev) * params[v, 1 + c] * vig
            i, inside = _decide32(img[v, c].detach().numpy(), float(ev.detach()),
                                  float(params[v, 1 + c].detach()), k.detach().numpy(), n, W, H,
                                  *principal[v])
            i = torch.tensor(i)
            tc = torch.where(torch.tensor(inside), t, torch.clamp(t, 0.0, 1.0).detach())
            f = tc * (n - 1) - i
            ch.append((1.0 - f) * lut[i] + f * lut[i + 1])
        outs.append(torch.stack(ch))
    return torch.stack(outs)


def _blur(a):
    from .post import SSIM_WINDOW, ssim_window
    g = torch.tensor(ssim_window(), dtype=DT)
    h = SSIM_WINDOW // 2
    x = a.reshape(-1, 1, *a.shape[-2:])
    x = Fnn.conv2d(x, g.reshape(1, 1, 1, -1), padding=(0, h))
    x = Fnn.conv2d(x, g.reshape(1, 1, -1, 1), padding=(h, 0))
    return x.reshape(a.shape)


def dssim(x, y):
    """oracle.post.dssim as differentiable torch ops."""
    from .post import SSIM_C1, SSIM_C2
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    s = ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2) /
         ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2)))
    return 1.0 - s.mean()


def regulariser(F, P, crops_i):
    """oracle.post.regulariser for packed F [sum 3 S^2] and P [V][3][H][W]."""
    crops_i = np.asarray(crops_i, np.int32).reshape(-1, 4)
    cnt = int(sum(3 * int(s) * int(s) for (_, _, _, s) in crops_i))
    ps = sum(P[v, :, y0:y0 + s, x0:x0 + s].sum() for (v, x0, y0, s) in crops_i)
    return torch.abs((F.sum() - ps) / cnt)
