"""Pins of the FP64 reference for tone mapping (Sec. 3.4, the ADOP camera
model as read in oracle/post.py) and the training objective (Sec. 3.5,
Eqs. 6-7: D-SSIM, the regulariser R, Adam): closed forms, explicit windowed
sums, and central differences."""
import numpy as np
import pytest

from oracle import post


def _img(rng, V=2, H=12, W=16, lo=0.0, hi=1.2):
    return rng.uniform(lo, hi, (V, 3, H, W))


def _params(rng, V=2, n=16):
    p = post.gamma_params(V, n)
    p[:, 0] = rng.uniform(-0.5, 0.5, V)
    p[:, 1:4] = rng.uniform(0.7, 1.3, (V, 3))
    p[:, 4:7] = rng.uniform(-0.3, 0.3, (V, 3))
    p[:, 7:] = np.sort(rng.uniform(0, 1, (V, n)), axis=1)
    return p


PRINC = np.array([[8.0, 6.0], [7.5, 6.5]])


# ------------------------------------------------------------ tone mapping
def test_identity_model_is_a_clamp():
    rng = np.random.default_rng(1)
    x = _img(rng, lo=-0.3, hi=1.4)
    p = post.gamma_params(2, 9, gamma=1.0)
    out, _ = post.tonemap(x, p, PRINC)
    assert np.abs(out - np.clip(x, 0, 1)).max() < 1e-15


def test_exposure_and_white_balance_scale_the_input():
    rng = np.random.default_rng(2)
    x = _img(rng)
    p = _params(rng)
    a, _ = post.tonemap(x, p, PRINC)
    q = p.copy()
    q[:, 0] -= 1.0           # one stop brighter = twice the input
    b, _ = post.tonemap(x / 2.0, q, PRINC)
    assert np.abs(a - b).max() < 1e-15
    q = p.copy()
    q[:, 1:4] = 1.0
    xs = x * p[:, 1:4, None, None]
    c, _ = post.tonemap(xs, q, PRINC)
    assert np.abs(a - c).max() < 1e-14


def test_vignetting_at_the_principal_point_and_half_diagonal():
    """An 8 x 6 image has half diagonal 5.  With the principal point at
    (4.5, 3.5), pixel (4, 3)'s centre is at r = 0 and pixel (0, 0)'s centre
    is (-4, -3) away, at r = 1."""
    k = np.array([0.1, -0.2, 0.05])
    p = post.gamma_params(1, 5, gamma=1.0)
    p[0, 4:7] = k
    x = np.full((1, 3, 6, 8), 0.25)
    out, _ = post.tonemap(x, p, np.array([[4.5, 3.5]]))
    assert abs(out[0, 0, 3, 4] - 0.25) < 1e-15                    # r = 0
    # principal point (4.5, 3.5): pixel (0, 0)'s centre is (-4, -3) away
    assert abs(out[0, 1, 0, 0] - 0.25 * (1 + k.sum())) < 1e-15    # r = 1


def test_gamma_response_within_interpolation_bound():
    """Piecewise-linear samples of x^(1/2.2): on [0.25, 1] the error is at
    most h^2/8 max|f''| over the segments used."""
    n = 33
    g = 1.0 / 2.2
    p = post.gamma_params(1, n, gamma=g)
    rng = np.random.default_rng(3)
    x = rng.uniform(0.25, 1.0, (1, 3, 20, 20))
    out, _ = post.tonemap(x, p, np.array([[10.0, 10.0]]))
    h = 1.0 / (n - 1)
    lo = 0.25 - h
    fpp = abs(g * (g - 1.0)) * lo ** (g - 2.0)
    err = np.abs(out - x ** g).max()
    assert err <= h * h / 8 * fpp
    assert err > 0.01 * h * h / 8 * fpp      # the bound is not vacuous


def test_monotone_response_gives_monotone_output():
    rng = np.random.default_rng(4)
    p = _params(rng, V=1)
    p[:, 4:7] = 0.0          # no vignetting: every pixel maps alike
    x = np.sort(rng.uniform(-0.2, 1.5, 200))
    img = np.broadcast_to(x, (1, 3, 1, 200)).copy()
    out, _ = post.tonemap(img, p, np.array([[100.0, 0.5]]))
    assert np.all(np.diff(out[0, 0, 0]) >= -1e-15)


def _fd(f, theta, h):
    return (f(theta + h) - f(theta - h)) / (2 * h)


def test_tonemap_gradients_against_central_differences():
    rng = np.random.default_rng(5)
    x = _img(rng, lo=0.05, hi=1.3)
    p = _params(rng)
    d = rng.normal(0, 1, x.shape)
    n = p.shape[1] - 7
    d_img, d_par = post.tonemap_backward(x, p, PRINC, d)

    def loss(xx, pp):
        return float(np.sum(d * post.tonemap(xx, pp, PRINC)[0]))

    h = 1e-6
    _, t = post.tonemap(x, p, PRINC)
    s = np.clip(t, 0, 1) * (n - 1)
    near = (np.abs(s - np.round(s)) < 1e-4) | (np.abs(t) < 1e-4) | (np.abs(t - 1) < 1e-4)
    checked = 0
    for idx in zip(*[a[:40] for a in np.nonzero(~near)]):
        e = np.zeros_like(x)
        e[idx] = h
        fd = (loss(x + e, p) - loss(x - e, p)) / (2 * h)
        assert abs(fd - d_img[idx]) < 1e-6 * max(1, abs(fd))
        checked += 1
    assert checked == 40
    # parameters: skip none, but require no t within h-reach of a kink
    for v in range(2):
        for j in range(p.shape[1]):
            e = np.zeros_like(p)
            e[v, j] = h
            fd = (loss(x, p + e) - loss(x, p - e)) / (2 * h)
            assert abs(fd - d_par[v, j]) < 2e-5 * max(1, abs(fd)), (v, j, fd, d_par[v, j])


# ------------------------------------------------------------------- SSIM
def test_window_is_a_normalised_gaussian():
    g = post.ssim_window()
    assert len(g) == 11 and abs(g.sum() - 1) < 1e-15
    assert abs(g[6] / g[5] - np.exp(-1 / (2 * 1.5 ** 2))) < 1e-15


def test_ssim_of_identical_images_is_one():
    rng = np.random.default_rng(6)
    x = rng.uniform(0, 1, (3, 24, 30))
    assert np.abs(post.ssim_map(x, x) - 1).max() < 1e-12
    assert abs(post.dssim(x, x)) < 1e-12
    assert np.abs(post.dssim_backward(x, x)).max() < 1e-12


def test_ssim_of_constant_images():
    a, b = 0.3, 0.7
    x = np.full((1, 30, 30), a)
    y = np.full((1, 30, 30), b)
    m = post.ssim_map(x, y)
    want = (2 * a * b + post.SSIM_C1) / (a * a + b * b + post.SSIM_C1)
    # (the variances come from E[x^2] - mu^2: cancellation of ~1e-16 over C2)
    assert np.abs(m[0, 5:-5, 5:-5] - want).max() < 1e-12


def test_ssim_against_explicit_windowed_sums():
    """At sampled pixels, the weighted moments summed over the 11 x 11
    neighbourhood directly (zero outside the image)."""
    rng = np.random.default_rng(7)
    x = rng.uniform(0, 1, (2, 19, 23))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    m = post.ssim_map(x, y)
    g = post.ssim_window()
    for (c, i, j) in [(0, 0, 0), (1, 9, 11), (0, 18, 22), (1, 3, 20), (0, 12, 4)]:
        sx = sy = sxx = syy = sxy = 0.0
        for di in range(-5, 6):
            for dj in range(-5, 6):
                ii, jj = i + di, j + dj
                if 0 <= ii < 19 and 0 <= jj < 23:
                    w = g[di + 5] * g[dj + 5]
                    a, b = x[c, ii, jj], y[c, ii, jj]
                    sx += w * a
                    sy += w * b
                    sxx += w * a * a
                    syy += w * b * b
                    sxy += w * a * b
        vx, vy, cxy = sxx - sx * sx, syy - sy * sy, sxy - sx * sy
        s = ((2 * sx * sy + post.SSIM_C1) * (2 * cxy + post.SSIM_C2) /
             ((sx * sx + sy * sy + post.SSIM_C1) * (vx + vy + post.SSIM_C2)))
        assert abs(s - m[c, i, j]) < 1e-13


def test_ssim_is_symmetric():
    rng = np.random.default_rng(8)
    x, y = rng.uniform(0, 1, (2, 3, 17, 21))
    assert np.abs(post.ssim_map(x, y) - post.ssim_map(y, x)).max() < 1e-14


def test_dssim_gradient_against_central_differences():
    rng = np.random.default_rng(9)
    x = rng.uniform(0, 1, (2, 14, 17))
    y = np.clip(x + rng.normal(0, 0.2, x.shape), 0, 1)
    d = post.dssim_backward(x, y)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 7, 8), (0, 13, 16), (1, 2, 15), (0, 10, 1), (1, 13, 0)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (post.dssim(x + e, y) - post.dssim(x - e, y)) / (2 * h)
        assert abs(fd - d[idx]) < 1e-9 + 1e-6 * abs(fd)


# -------------------------------------------------------------- regulariser
def test_regulariser_closed_forms_and_gradient():
    rng = np.random.default_rng(10)
    P = rng.uniform(0, 1, (2, 3, 20, 24))
    crops = [(0, 2, 3, 8), (1, 10, 4, 12)]
    F = [P[v, :, y0:y0 + s, x0:x0 + s].copy() for (v, x0, y0, s) in crops]
    assert post.regulariser(F, P, crops)[0] < 1e-15
    Fc = [np.full((3, s, s), 0.8) for (_, _, _, s) in crops]
    Pc = np.full_like(P, 0.3)
    assert abs(post.regulariser(Fc, Pc, crops)[0] - 0.5) < 1e-15
    F = [f + rng.normal(0, 0.1, f.shape) for f in F]
    dF, dP = post.regulariser_backward(F, P, crops, d_r=1.7)
    h = 1e-7
    for k, idx in [(0, (1, 2, 3)), (1, (2, 11, 0))]:
        F2 = [f.copy() for f in F]
        F2[k][idx] += h
        F3 = [f.copy() for f in F]
        F3[k][idx] -= h
        fd = 1.7 * (post.regulariser(F2, P, crops)[0] - post.regulariser(F3, P, crops)[0]) / (2 * h)
        assert abs(fd - dF[k][idx]) < 1e-7
    for idx in [(0, 1, 5, 4), (1, 2, 10, 15), (0, 0, 0, 0)]:
        P2, P3 = P.copy(), P.copy()
        P2[idx] += h
        P3[idx] -= h
        fd = 1.7 * (post.regulariser(F, P2, crops)[0] - post.regulariser(F, P3, crops)[0]) / (2 * h)
        assert abs(fd - dP[idx]) < 1e-7


# --------------------------------------------------------------------- Adam
def test_adam_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(11)
    p = rng.normal(0, 1, 100)
    g = rng.normal(0, 1, 100)
    z = np.zeros(100)
    q, m, v = post.adam(p, g, z, z, 1, lr=0.01, eps=0.0)
    assert np.abs(q - (p - 0.01 * np.sign(g))).max() < 1e-15
    assert np.abs(m - 0.1 * g).max() < 1e-16 and np.abs(v - 0.001 * g * g).max() < 1e-16


def test_adam_constant_gradient_moves_uniformly():
    g = np.array([0.5, -2.0, 3e-3])
    p = np.zeros(3)
    m = v = np.zeros(3)
    for t in range(1, 8):
        p, m, v = post.adam(p, g, m, v, t, lr=0.1, eps=0.0)
    assert np.abs(p - (-0.7 * np.sign(g))).max() < 1e-12


def test_adam_zero_gradient_leaves_parameters():
    p = np.array([1.0, -2.0])
    q, _, _ = post.adam(p, np.zeros(2), np.zeros(2), np.zeros(2), 1, lr=0.1)
    assert np.array_equal(p, q)


# ------------------------------------- the differentiable forms (oracle.diff)
def test_diff_forms_equal_the_reference_and_its_gradients():
    import torch
    from oracle import diff
    rng = np.random.default_rng(12)
    x = _img(rng, lo=0.05, hi=1.3)
    p = _params(rng)
    d = rng.normal(0, 1, x.shape)
    xt = torch.tensor(x, requires_grad=True)
    pt = torch.tensor(p, requires_grad=True)
    out = diff.tonemap(xt, pt, PRINC)
    want, _ = post.tonemap(x, p, PRINC)
    assert np.abs(out.detach().numpy() - want).max() < 1e-14
    (out * torch.tensor(d)).sum().backward()
    d_img, d_par = post.tonemap_backward(x, p, PRINC, d)
    assert np.abs(xt.grad.numpy() - d_img).max() < 1e-12
    assert np.abs(pt.grad.numpy() - d_par).max() < 1e-9 * max(1, np.abs(d_par).max())
    a = rng.uniform(0, 1, (2, 3, 20, 24))
    b = np.clip(a + rng.normal(0, 0.2, a.shape), 0, 1)
    at = torch.tensor(a, requires_grad=True)
    s = diff.dssim(at, torch.tensor(b))
    assert abs(float(s) - post.dssim(a, b)) < 1e-13
    s.backward()
    assert np.abs(at.grad.numpy() - post.dssim_backward(a, b)).max() < 1e-15
    crops = [(0, 2, 3, 8), (1, 10, 4, 12)]
    F = [rng.uniform(0, 1, (3, s_, s_)) for (_, _, _, s_) in crops]
    Fp = torch.tensor(np.concatenate([f.ravel() for f in F]), requires_grad=True)
    Pt = torch.tensor(a, requires_grad=True)
    r = diff.regulariser(Fp, Pt, crops)
    assert abs(float(r) - post.regulariser(F, a, crops)[0]) < 1e-15
    r.backward()
    dF, dP = post.regulariser_backward(F, a, crops)
    assert np.abs(Fp.grad.numpy() - np.concatenate([f.ravel() for f in dF])).max() < 1e-16
    assert np.abs(Pt.grad.numpy() - dP).max() < 1e-16
