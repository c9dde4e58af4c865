"""GPU parity of the extended channels (the depth maps of the mesh-extraction
passage, Sec. 3.3, and the accumulated opacity) against the FP64 oracle.

Same-inputs comparisons, as for the colour stages: the oracle composites its
own tile lists of the GPU's records (their last field is the splat depth),
along the decision path that the GPU's colour result matches.  Bars as for
the colour image and its gradients: depth and alpha within 1e-4 of the
oracle's max |value| per view on every pixel except the masked ones;
screen-space and parameter gradients within 1e-3 (inf- and 2-norm) for seeded
upstream gradients of colour, depth and alpha, zeroed at masked pixels.  The alpha
map is exactly 1 - final_T, and asking for the channels leaves the colour
outputs bitwise unchanged.
"""
import functools

import numpy as np
import pytest

import gesr_inputs as gi
import oracle
from tests.gpu_util import (conic_grads_to_factor, f32, factor_grads_to_conic, log, mask_upstream, norm_errors,
                            raster_settings, run_gpu, same_input_reference)
from tests.test_gpu_parity import _case

pytestmark = pytest.mark.gpu

CASES = ["tiny-d3-2v-bg", "ragged-5v", "plain-2k", "drt-50k-8v"]
PARAMS = ("means", "scales", "quats", "opacities", "betas", "sh")


def _grads(scene, st, g):
    N = scene.n
    K = (st.sh_degree + 1) ** 2
    V = scene.n_views
    return dict(grad2d=f32(g["grad2d"])[:N * V * 12].reshape(N * V, 12),
                means=f32(g["mean"]).reshape(3, N).T, scales=f32(g["scale"]).reshape(3, N).T,
                quats=f32(g["quat"]).reshape(4, N).T, opacities=f32(g["opacity"]), betas=f32(g["beta"]),
                sh=f32(g["sh"]).reshape(K * 3, N).T.reshape(N, K, 3))


@functools.lru_cache(maxsize=1)
def _run(name):
    import torch
    scene, st = _case(name)
    log(f"[gpu] channels case {name}: n={scene.n} views={scene.n_views} px={scene.n_pixels}")
    g = run_gpu(scene, st)
    rast, sp, out = g["torch"]
    ext = rast.render_fwd(out["proj"], out["bins"], scene.n, channels=True)
    torch.cuda.synchronize()
    P = scene.n_pixels
    g["ext"] = {k: f32(ext[k])[:P * (3 if k == "image" else 1)] for k in ("image", "final_T", "depth", "alpha")}
    g["ext"]["n_contrib"] = ext["n_contrib"].cpu().numpy()[:P]
    depth = g["rec"][:, 11].astype(np.float64)
    ref = same_input_reference(scene, st, g, depth=depth)
    return scene, st, g, ref, depth, ref["fwd"]


def _per_view_errors(gpu, ref, amb, cameras, tol=1e-4):
    off = 0
    for c in cameras:
        P = c.width * c.height
        a = np.asarray(gpu[off:off + P], np.float64)
        b = ref[off:off + P]
        ok = ~amb[off:off + P]
        bound = tol * max(np.abs(b).max(), 1.0)
        err = np.abs(a - b)
        assert not (err[ok] > bound).any(), (c.width, c.height, float(err[ok].max()), bound)
        off += P


@pytest.mark.parametrize("name", CASES)
def test_channels_forward_same_inputs(name):
    scene, st, g, ref, depth, fo = _run(name)
    e = g["ext"]
    # the colour outputs do not depend on asking for the channels
    np.testing.assert_array_equal(e["image"], g["image"])
    np.testing.assert_array_equal(e["final_T"], g["final_T"])
    np.testing.assert_array_equal(e["n_contrib"], g["n_contrib"].view(np.int32))
    # alpha is 1 - final_T in float32, bit for bit
    np.testing.assert_array_equal(e["alpha"], (np.float32(1.0) - g["final_T"]).astype(np.float32))
    amb = ref["masked"]
    _per_view_errors(e["depth"], fo["depth"], amb, scene.cameras)
    _per_view_errors(e["alpha"], fo["alpha"], amb, scene.cameras)
    log(f"[gpu] {name}: channels fwd ok; masked px {int(amb.sum())}/{amb.size}")


@pytest.mark.parametrize("name", CASES)
def test_channels_backward_same_inputs(name):
    """Screen-space gradients (eleven terms, dz included) and the parameter
    gradients for seeded upstream gradients of colour, depth and alpha."""
    import torch
    scene, st, g, ref, depth, fo = _run(name)
    rast, sp, out = g["torch"]
    amb = ref["masked"]
    rng = np.random.default_rng(5)
    P = scene.n_pixels
    dL = mask_upstream(oracle.flat_images(gi.upstream_grads(scene, 7)), amb, scene.cameras)
    gD = np.where(amb, 0.0, rng.standard_normal(P)).astype(np.float32).astype(np.float64)
    gA = np.where(amb, 0.0, rng.standard_normal(P)).astype(np.float32).astype(np.float64)
    tz = lambda x: torch.as_tensor(np.asarray(x, np.float32), device="cuda")  # noqa: E731
    gb = rast.render_bwd(sp, out["proj"], out["bins"], out["final_T"], out["n_contrib"], tz(dL), want_grad2d=True,
                         dL_ddepth=tz(gD), dL_dalpha=tz(gA))
    torch.cuda.synchronize()
    got = _grads(scene, st, gb)
    assert (got["grad2d"][:, 11] == 0).all()
    g2 = oracle.render_bwd(scene.n, scene.cameras, ref["rec"], ref["vals"], ref["ranges"], dL, st, depth=depth,
                           dL_ddepth=gD, dL_dalpha=gA, paths=ref["paths"])
    refg = conic_grads_to_factor(g2, g["rec"])
    labels = ["du", "dv", "dL00", "dL10", "dL11", "dop", "dbeta", "dr", "dg", "db", "dz"]
    worst = 0.0
    for k, lab in enumerate(labels):
        einf, e2 = norm_errors(got["grad2d"][:, k], refg[:, k])
        worst = max(worst, einf, e2)
        assert einf <= 1e-3 and e2 <= 1e-3, (lab, einf, e2)
    assert np.abs(refg[:, 10]).max() > 0
    pref = oracle.project_bwd(scene, factor_grads_to_conic(got["grad2d"][:, :11], g["rec"]), st)
    for k in PARAMS:
        einf, e2 = norm_errors(got[k], pref[k])
        worst = max(worst, einf, e2)
        assert einf <= 1e-3 and e2 <= 1e-3, (k, einf, e2)
    log(f"[gpu] {name}: channels bwd ok; worst {worst:.2e}")


@pytest.mark.parametrize("name", ["tiny-d3-2v-bg", "ragged-5v"])
def test_zero_channel_gradients_match_plain_backward(name):
    """The channel kernels with zero depth and alpha gradients reproduce the
    plain backward bit for bit (the added terms are exact zeros)."""
    import torch
    scene, st, g, ref, depth, fo = _run(name)
    rast, sp, out = g["torch"]
    dL = torch.as_tensor(oracle.flat_images(gi.upstream_grads(scene, 3)).astype(np.float32), device="cuda")
    zero = torch.zeros(scene.n_pixels, dtype=torch.float32, device="cuda")
    plain = rast.render_bwd(sp, out["proj"], out["bins"], out["final_T"], out["n_contrib"], dL, want_grad2d=True)
    ext = rast.render_bwd(sp, out["proj"], out["bins"], out["final_T"], out["n_contrib"], dL, want_grad2d=True,
                          dL_ddepth=zero, dL_dalpha=zero)
    torch.cuda.synchronize()
    a, b = _grads(scene, st, plain), _grads(scene, st, ext)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_channels_need_the_one_wave_renderer():
    """Other tile shapes or the four-wave variant reject the channels
    (GESR_ERR_UNSUPPORTED) instead of silently dropping them."""
    from paper_2411_09156_amd import Rasterizer
    from paper_2411_09156_amd._lib import GESR_ERR_UNSUPPORTED, GesrError
    scene, st = _case("tiny-d1")
    for kw in (dict(variant=1), dict(tile_w=8, tile_h=8)):
        rast = Rasterizer(scene.cameras, raster_settings(st, **kw))
        from tests.gpu_util import splats_of
        out = rast.forward(splats_of(scene))
        with pytest.raises(GesrError) as ei:
            rast.render_fwd(out["proj"], out["bins"], scene.n, channels=True)
        assert ei.value.status == GESR_ERR_UNSUPPORTED
