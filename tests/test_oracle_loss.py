"""Pins of the oracle's photometric loss (Eq. 8: (1 - lambda) L1 + lambda
(1 - SSIM), Gaussian 11 x 11 window of standard deviation 1.5, C1 = 0.01^2,
C2 = 0.03^2, zero padding).

* SSIM(X, X) = 1 at every pixel, and the loss and its SSIM gradient vanish;
* constant images: the closed form in the window mass w(p) inside the image
  (a product of two one-dimensional partial sums of the window);
* the SSIM map equals one built from scipy.ndimage.correlate moments, and for
  Y = s X + t it takes the affine closed form in X's local mean and variance;
* the gradient equals central differences of the loss, and torch float64
  autograd through an independent conv2d formulation;
* views are normalised separately.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

import gesr_inputs as gi
import oracle

LS = oracle.LossSettings()


def _window2d():
    x = np.arange(-5, 6)
    g = np.exp(-x * x / (2 * 1.5 ** 2))
    g /= g.sum()
    return np.outer(g, g), g


def _ssim_scipy(X, Y, ls=LS):
    w2, _ = _window2d()
    mom = lambda a: ndi.correlate(a, w2, mode="constant", cval=0.0)  # noqa: E731
    mx, my = mom(X), mom(Y)
    sxx, syy, sxy = mom(X * X) - mx * mx, mom(Y * Y) - my * my, mom(X * Y) - mx * my
    return ((2 * mx * my + ls.c1) * (2 * sxy + ls.c2)) / ((mx * mx + my * my + ls.c1) * (sxx + syy + ls.c2))


def test_window_is_the_normalised_gaussian():
    g = oracle.gaussian_window(5, 1.5)
    assert g.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(g / g[5], np.exp(-np.arange(-5, 6) ** 2 / 4.5), rtol=1e-14)


def test_ssim_of_an_image_with_itself_is_one():
    rng = np.random.default_rng(0)
    X = rng.uniform(0, 1, (23, 31))
    S = oracle.ssim_terms(X, X, LS)[0]
    np.testing.assert_allclose(S, 1.0, rtol=0, atol=1e-14)
    cam = gi.look_at((0, 0, -4), width=31, height=23)
    img = rng.uniform(0, 1, 3 * 23 * 31)
    loss, grad = oracle.photometric_loss(img, img, [cam])
    assert abs(loss[0]) < 1e-15 and np.abs(grad).max() < 1e-15


@pytest.mark.parametrize("alpha,beta", [(0.3, 0.8), (0.5, 0.5), (1.0, 0.0)])
def test_constant_images_closed_form(alpha, beta):
    H, W = 17, 26
    _, g = _window2d()

    def mass(n):  # window weight inside [0, n) around each position
        return np.array([sum(g[k + 5] for k in range(-5, 6) if 0 <= i + k < n) for i in range(n)])
    w = np.outer(mass(H), mass(W))
    X, Y = np.full((H, W), alpha), np.full((H, W), beta)
    c1, c2 = LS.c1, LS.c2
    ab, aa = alpha * beta, alpha * alpha + beta * beta
    expect = (2 * ab * w * w + c1) * (2 * ab * (w - w * w) + c2) / ((aa * w * w + c1) * (aa * (w - w * w) + c2))
    np.testing.assert_allclose(oracle.ssim_terms(X, Y, LS)[0], expect, rtol=1e-12, atol=1e-12)
    # interior: w = 1
    assert oracle.ssim_terms(X, Y, LS)[0][8, 13] == pytest.approx((2 * ab + c1) / (aa + c1), rel=1e-12)


def test_ssim_map_equals_scipy_moments_and_the_affine_closed_form():
    rng = np.random.default_rng(1)
    X = rng.uniform(0, 1, (29, 37))
    Y = np.clip(X + rng.normal(0, 0.1, X.shape), 0, 1)
    np.testing.assert_allclose(oracle.ssim_terms(X, Y, LS)[0], _ssim_scipy(X, Y), rtol=1e-11, atol=1e-12)
    s, t = 0.6, 0.25
    w2, _ = _window2d()
    mu = ndi.correlate(X, w2, mode="constant")
    var = ndi.correlate(X * X, w2, mode="constant") - mu * mu
    my = s * mu + t
    expect = ((2 * mu * my + LS.c1) * (2 * s * var + LS.c2)) / ((mu * mu + my * my + LS.c1) * ((1 + s * s) * var + LS.c2))
    S = oracle.ssim_terms(X, s * X + t, LS)[0]
    np.testing.assert_allclose(S[5:-5, 5:-5], expect[5:-5, 5:-5], rtol=1e-10)


def test_gradient_matches_finite_differences_and_torch_autograd():
    import torch
    import torch.nn.functional as F
    rng = np.random.default_rng(2)
    H, W = 13, 11
    cam = gi.look_at((0, 0, -4), width=W, height=H)
    X = rng.uniform(0, 1, 3 * H * W)
    Y = rng.uniform(0, 1, 3 * H * W)
    loss, grad = oracle.photometric_loss(X, Y, [cam])
    for k in rng.choice(X.size, 40, replace=False):
        h = 1e-6
        Xp, Xm = X.copy(), X.copy()
        Xp[k] += h
        Xm[k] -= h
        fd = (oracle.photometric_loss(Xp, Y, [cam])[0][0] - oracle.photometric_loss(Xm, Y, [cam])[0][0]) / (2 * h)
        assert abs(grad[k] - fd) <= 1e-7 * max(abs(fd), 1e-3 * np.abs(grad).max()), (k, grad[k], fd)
    w2, _ = _window2d()
    win = torch.tensor(w2, dtype=torch.float64)[None, None].repeat(3, 1, 1, 1)
    x = torch.tensor(X.reshape(1, 3, H, W), requires_grad=True)
    y = torch.tensor(Y.reshape(1, 3, H, W))
    mom = lambda a: F.conv2d(a, win, padding=5, groups=3)  # noqa: E731
    mx, my = mom(x), mom(y)
    sxx, syy, sxy = mom(x * x) - mx * mx, mom(y * y) - my * my, mom(x * y) - mx * my
    ssim = ((2 * mx * my + LS.c1) * (2 * sxy + LS.c2)) / ((mx * mx + my * my + LS.c1) * (sxx + syy + LS.c2))
    L = (1 - LS.lam) * (x - y).abs().mean() + LS.lam * (1 - ssim.mean())
    L.backward()
    assert float(L.detach()) == pytest.approx(loss[0], rel=1e-13)
    np.testing.assert_allclose(grad, x.grad.numpy().reshape(-1), rtol=0, atol=1e-13 * np.abs(grad).max())


def test_views_are_normalised_separately():
    rng = np.random.default_rng(3)
    cams = [gi.look_at((0, 0, -4), width=w, height=h) for w, h in ((9, 7), (1, 13), (20, 16))]
    n = [3 * c.width * c.height for c in cams]
    X, Y = rng.uniform(0, 1, sum(n)), rng.uniform(0, 1, sum(n))
    loss, grad = oracle.photometric_loss(X, Y, cams)
    off = 0
    for v, c in enumerate(cams):
        lv, gv = oracle.photometric_loss(X[off:off + n[v]], Y[off:off + n[v]], [c])
        assert loss[v] == lv[0]
        np.testing.assert_array_equal(grad[off:off + n[v]], gv)
        off += n[v]
