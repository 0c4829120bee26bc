"""FP64 reference of the stages after the combination and of the training
objective -- test infrastructure, like the rest of ``oracle``: only tests,
the smoke check and the benchmark's CPU leg use it.

Tone mapping (Sec. 3.4, last paragraph: the combined image is mapped to a
displayable range by a differentiable camera model following ADOP).  The
paper does not restate the model; this module fixes the reading used
throughout (per view, planar RGB):

    t = x * 2^-ev * wb[c] * V(r)        V(r) = 1 + k1 r^2 + k2 r^4 + k3 r^6
    y = R(clamp(t, 0, 1))

with ev the exposure value, wb a per-channel white balance, r the distance
of the pixel centre from the principal point divided by the half diagonal
of the image, and R a response curve, piecewise linear through n samples
at s_i = i / (n - 1).  Parameters per view: [ev, wb_r, wb_g, wb_b, k1, k2,
k3, R_0 .. R_{n-1}].  On the segment [s_i, s_{i+1}] (i = min(floor(t (n-1)),
n - 2)) R(t) = (1 - f) R_i + f R_{i+1}, f = t (n - 1) - i; the clamp has zero
derivative outside (0, 1).  The segment and the clamp are integer decisions:
they are taken on t evaluated in single precision in a fixed order (see
_decide32), the values in double precision.

Training objective (Sec. 3.5, Eqs. 6-7): D-SSIM as in 3DGS (1 - SSIM,
11 x 11 Gaussian window with sigma 1.5 normalised to sum 1, zero padding,
C1 = 0.01^2, C2 = 0.03^2, averaged over every pixel and channel), the
regulariser R = |mean F - mean crop(P)| over all crop pixels and channels,
and the Adam step (Kingma and Ba, bias-corrected moments).

Pins (tests/test_oracle_post.py): closed forms (identity model, exposure
and white balance as input scaling, vignetting at the principal point and at
the half diagonal, a gamma response within the linear-interpolation error
bound, SSIM of constant images, first Adam step, constant-gradient Adam),
SSIM against explicit windowed sums at sampled pixels, symmetry, and every
gradient against FP64 central differences.
"""
from __future__ import annotations

import numpy as np

SSIM_WINDOW = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2
PARAMS_FIXED = 7     # ev, wb (3), k (3)


# ------------------------------------------------------------ tone mapping
def vignette_r2(W, H, cx, cy):
    """Squared normalised radius r^2 [H][W] (pixel centres, principal point
    (cx, cy), half diagonal of the W x H image)."""
    x = np.arange(W, dtype=np.float64) + 0.5 - cx
    y = np.arange(H, dtype=np.float64) + 0.5 - cy
    d2 = (W / 2.0) ** 2 + (H / 2.0) ** 2
    return (y[:, None] ** 2 + x[None, :] ** 2) / d2


def _decide32(x, ev, wb_c, k, n, W, H, cx, cy):
    """Segment index and inside-(0, 1) flag of every pixel of one channel,
    from t in single precision: dx = (x + 0.5) - cx, r2 = (dx dx + dy dy)
    inv_d2 with inv_d2 the rounded 1 / half-diagonal^2, vig = ((k3 r2 + k2)
    r2 + k1) r2 + 1, e the rounded 2^-ev, t = ((x e) wb) vig; then
    s = clamp(t, 0, 1) (n - 1), i = min(floor(s), n - 2)."""
    f32 = np.float32
    inv_d2 = f32(1.0 / ((W / 2.0) ** 2 + (H / 2.0) ** 2))
    dx = (np.arange(W, dtype=f32) + f32(0.5)) - f32(cx)
    dy = (np.arange(H, dtype=f32) + f32(0.5)) - f32(cy)
    r2 = (dy[:, None] * dy[:, None] + dx[None, :] * dx[None, :]) * inv_d2
    k = np.asarray(k, f32)
    vig = ((k[2] * r2 + k[1]) * r2 + k[0]) * r2 + f32(1.0)
    e = f32(2.0 ** (-float(ev)))
    t = ((np.asarray(x, f32) * e) * f32(wb_c)) * vig
    inside = (t > 0) & (t < 1)
    s = np.clip(t, f32(0), f32(1)) * f32(n - 1)
    i = np.minimum(np.floor(s), n - 2).astype(np.int64)
    return i, inside


def tonemap(img, params, principal):
    """img [V][3][H][W], params [V][7 + n], principal [V][2] (cx, cy) ->
    (out [V][3][H][W], t) in float64."""
    img = np.asarray(img, np.float64)
    params = np.asarray(params, np.float64)
    V, _, H, W = img.shape
    n = params.shape[1] - PARAMS_FIXED
    out = np.empty_like(img)
    ts = np.empty_like(img)
    for v in range(V):
        ev, wb, k, lut = params[v, 0], params[v, 1:4], params[v, 4:7], params[v, 7:]
        r2 = vignette_r2(W, H, *principal[v])
        vig = 1.0 + k[0] * r2 + k[1] * r2 ** 2 + k[2] * r2 ** 3
        for c in range(3):
            t = img[v, c] * 2.0 ** (-ev) * wb[c] * vig
            i, _ = _decide32(img[v, c], ev, wb[c], k, n, W, H, *principal[v])
            f = np.clip(t, 0.0, 1.0) * (n - 1) - i
            out[v, c] = (1.0 - f) * lut[i] + f * lut[i + 1]
            ts[v, c] = t
    return out, ts


def tonemap_backward(img, params, principal, d_out):
    """Gradients of sum(d_out * tonemap(img)): (d_img, d_params)."""
    img = np.asarray(img, np.float64)
    params = np.asarray(params, np.float64)
    d_out = np.asarray(d_out, np.float64)
    V, _, H, W = img.shape
    n = params.shape[1] - PARAMS_FIXED
    d_img = np.zeros_like(img)
    d_par = np.zeros_like(params)
    for v in range(V):
        ev, wb, k, lut = params[v, 0], params[v, 1:4], params[v, 4:7], params[v, 7:]
        r2 = vignette_r2(W, H, *principal[v])
        vig = 1.0 + k[0] * r2 + k[1] * r2 ** 2 + k[2] * r2 ** 3
        e = 2.0 ** (-ev)
        for c in range(3):
            x = img[v, c]
            t = x * e * wb[c] * vig
            i, inside = _decide32(x, ev, wb[c], k, n, W, H, *principal[v])
            f = np.clip(t, 0.0, 1.0) * (n - 1) - i
            g = d_out[v, c]
            # response samples
            np.add.at(d_par[v, 7:], i, g * (1.0 - f))
            np.add.at(d_par[v, 7:], i + 1, g * f)
            # through the clamp: slope of the segment inside (0, 1)
            dt = np.where(inside, g * (lut[i + 1] - lut[i]) * (n - 1), 0.0)
            d_img[v, c] = dt * e * wb[c] * vig
            d_par[v, 0] += np.sum(dt * t) * -np.log(2.0)
            d_par[v, 1 + c] += np.sum(dt * x * e * vig)
            base = dt * x * e * wb[c]
            d_par[v, 4] += np.sum(base * r2)
            d_par[v, 5] += np.sum(base * r2 ** 2)
            d_par[v, 6] += np.sum(base * r2 ** 3)
    return d_img, d_par


def gamma_params(n_views, n=32, gamma=1.0 / 2.2, ev=0.0):
    """Neutral model with a gamma response (an initialisation)."""
    p = np.zeros((n_views, PARAMS_FIXED + n))
    p[:, 0] = ev
    p[:, 1:4] = 1.0
    p[:, 7:] = np.linspace(0.0, 1.0, n) ** gamma
    return p


# ------------------------------------------------------------------- SSIM
def ssim_window():
    """The 11-tap Gaussian (sigma 1.5) normalised to sum 1; the 2-D window
    is its outer product."""
    x = np.arange(SSIM_WINDOW, dtype=np.float64) - SSIM_WINDOW // 2
    g = np.exp(-x * x / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def blur(a):
    """Zero-padded 'same' correlation of every [..][H][W] plane with the 2-D
    window, as two 1-D passes."""
    g = ssim_window()
    h = SSIM_WINDOW // 2
    a = np.asarray(a, np.float64)
    H, W = a.shape[-2:]
    p = np.zeros(a.shape[:-2] + (H, W + 2 * h))
    p[..., h:h + W] = a
    r = sum(g[j] * p[..., j:j + W] for j in range(SSIM_WINDOW))
    q = np.zeros(a.shape[:-2] + (H + 2 * h, W))
    q[..., h:h + H, :] = r
    return sum(g[j] * q[..., j:j + H, :] for j in range(SSIM_WINDOW))


def ssim_map(x, y):
    """Per-pixel SSIM of x against y (any [..][H][W])."""
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    num = (2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)
    den = (mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2)
    return num / den


def dssim(x, y):
    """D-SSIM = 1 - mean SSIM over every element."""
    return 1.0 - float(np.mean(ssim_map(x, y)))


def dssim_backward(x, y):
    """Gradient of dssim(x, y) with respect to x.  With the map a function
    of (mu_x, mu_y, E[x^2], E[y^2], E[xy]) per pixel, the blur's adjoint is
    the same zero-padded correlation (the window is symmetric)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    a1 = 2 * mx * my + SSIM_C1
    a2 = 2 * sxy + SSIM_C2
    b1 = mx * mx + my * my + SSIM_C1
    b2 = sxx + syy + SSIM_C2
    s = a1 * a2 / (b1 * b2)
    # partials of s in (mu_x, sigma_xx, sigma_xy)
    d_mx = 2 * my * a2 / (b1 * b2) - s * 2 * mx / b1
    d_sxx = -s / b2
    d_sxy = 2 * a1 / (b1 * b2)
    # to (mu_x, E[x^2], E[xy]): sigma_xx = E[x^2] - mu_x^2, sigma_xy = E[xy] - mu_x mu_y
    A = d_mx - 2 * mx * d_sxx - my * d_sxy
    B = d_sxx
    C = d_sxy
    N = x.size
    return -(blur(A) + 2 * x * blur(B) + y * blur(C)) / N


# -------------------------------------------------------------- regulariser
def regulariser(F, P, crops):
    """R = |mean F - mean crop(P)| (Eq. 7): F [n][3][S_i][S_i] (a list, one
    entry per crop), P [V][3][H][W], crops rows (view, x0, y0, size); the
    means run over every pixel and channel of all crops."""
    fs = sum(float(np.sum(np.asarray(f, np.float64))) for f in F)
    ps = 0.0
    cnt = 0
    for (v, x0, y0, s) in crops:
        ps += float(np.sum(np.asarray(P[v, :, y0:y0 + s, x0:x0 + s], np.float64)))
        cnt += 3 * s * s
    return abs(fs / cnt - ps / cnt), fs / cnt - ps / cnt


def regulariser_backward(F, P, crops, d_r=1.0):
    """Gradients of d_r * R: (list of dF, dP); sign(0) = 0."""
    _, diff = regulariser(F, P, crops)
    cnt = sum(3 * s * s for (_, _, _, s) in crops)
    g = d_r * np.sign(diff) / cnt
    dF = [np.full(np.shape(f), g) for f in F]
    dP = np.zeros(np.shape(P))
    for (v, x0, y0, s) in crops:
        dP[v, :, y0:y0 + s, x0:x0 + s] -= g
    return dF, dP


# --------------------------------------------------------------------- Adam
def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (step counts from 1): returns (p, m, v) updated."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
