"""GPU parity of the photometric loss of Eq. 8 ((1 - lambda) L1 + lambda
(1 - SSIM), 11 x 11 Gaussian window, zero padding) against the FP64 oracle.

Same float32 images on both sides.  Bars: each view's loss within 1e-5
(absolute; the loss is a mean of values in [0, 2]); the image gradient within
1e-3 of the reference's inf-norm and 2-norm (the gradient bar of the
rasterizer); bitwise reproducible; ragged and batched views, and the
rendered-versus-target case of the 100k-splat sphere workload at 1008 x 756."""
import numpy as np
import pytest

import gesr_inputs as gi
import oracle
from tests.gpu_util import f32, log, norm_errors, raster_settings, run_gpu

pytestmark = pytest.mark.gpu


def _views(kind):
    if kind == "ragged":
        return [gi.look_at((0, 0, -4), width=w, height=h) for w, h in ((1, 1), (1, 37), (23, 1), (17, 33), (129, 65))]
    if kind == "drt-small":
        sc = gi.make_workload(3, n_override=1000)
        return sc.cameras[:4]
    raise KeyError(kind)


def _gpu_loss(cams, X, Y, lam=0.2):
    import torch
    from paper_2411_09156_amd import Rasterizer
    rast = Rasterizer(cams, raster_settings(oracle.Settings()))
    g, loss = rast.loss_eq8(torch.as_tensor(X, device="cuda"), torch.as_tensor(Y, device="cuda"), lam)
    torch.cuda.synchronize()
    return f32(g), f32(loss)


def _check(cams, X, Y, label, lam=0.2):
    ls = oracle.LossSettings(lam=float(np.float32(lam)))
    loss_o, grad_o = oracle.photometric_loss(X, Y, cams, ls)
    grad, loss = _gpu_loss(cams, X, Y, lam)
    grad2, loss2 = _gpu_loss(cams, X, Y, lam)
    np.testing.assert_array_equal(grad, grad2)
    np.testing.assert_array_equal(loss, loss2)
    assert np.abs(loss - loss_o).max() <= 1e-5, (loss, loss_o)
    einf, e2 = norm_errors(grad, grad_o)
    assert einf <= 1e-3 and e2 <= 1e-3, (einf, e2)
    log(f"[gpu] loss {label}: loss err {np.abs(loss - loss_o).max():.2e}; grad inf/2-norm err {einf:.2e}/{e2:.2e}")


@pytest.mark.parametrize("kind", ["ragged", "drt-small"])
@pytest.mark.parametrize("lam", [0.2, 1.0, 0.0])
def test_loss_random_images(kind, lam):
    cams = _views(kind)
    P = sum(3 * c.width * c.height for c in cams)
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 1, P).astype(np.float32)
    Y = np.clip(X + rng.normal(0, 0.2, P), 0, 1).astype(np.float32)
    Y[::11] = X[::11]  # exact ties: sign(0) = 0
    _check(cams, X, Y, f"{kind} lambda {lam}", lam)


def test_loss_of_a_rendered_image():
    """The 100k-splat sphere workload at 1008 x 756 rendered on the GPU against
    its seeded target image (the loss the benchmark leg of that workload uses)."""
    scene = gi.make_workload(2)
    st = oracle.Settings(sh_degree=3)
    g = run_gpu(scene, st, counts=False)
    X = g["image"].astype(np.float32)
    Y = oracle.flat_images(gi.target_images(scene, 2)).astype(np.float32)
    _check(scene.cameras, X, Y, "spheres-100k rendered")


def test_loss_argument_errors():
    import torch
    from paper_2411_09156_amd import Rasterizer
    from paper_2411_09156_amd._lib import GESR_ERR_INVALID, GesrError
    cams = _views("ragged")
    rast = Rasterizer(cams, raster_settings(oracle.Settings()))
    P = sum(3 * c.width * c.height for c in cams)
    x = torch.zeros(P, device="cuda")
    for lam in (-0.1, 1.5, float("nan")):
        with pytest.raises(GesrError) as ei:
            rast.loss_eq8(x, x.clone(), lam)
        assert ei.value.status == GESR_ERR_INVALID
