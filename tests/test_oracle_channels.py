"""Pins of the oracle's extended channels: the depth map of the mesh-extraction
passage (DyGASR, arXiv 2411.09156, Sec. 3.3) and the accumulated opacity, both
composited like a colour channel over a zero background:

    D = sum_k alpha_k T_k z_k,     A = sum_k alpha_k T_k,

with z_k the camera-space depth of splat k's centre.  Fixed by a closed form
(three stacked splats, depths from the camera matrix, not from the oracle's
projection), by the telescoping identity A = 1 - T_final, by bounds that any
weighted depth average obeys, and by central differences of the FP64 forward
for the adjoint (dL/dD and dL/dA into every splat parameter, the depth term
reaching the means through the camera transform).
"""
import copy

import numpy as np
import pytest

import gesr_inputs as gi
import oracle
from tests.oracle_util import stacked_scene, with_params

PARAMS = ("means", "scales", "quats", "opacities", "betas", "sh")


def _camera_depth(cam, means):
    """Camera-space z of each mean: third row of [R | t] applied to it."""
    vm = np.asarray(cam.viewmat, np.float64)
    return np.asarray(means, np.float64) @ vm[2, :3] + vm[2, 3]


def test_three_stacked_splats_depth_and_alpha_closed_form():
    """Front-to-back blending of depth and unit opacity: D = a1 z1 + (1-a1) a2 z2
    + (1-a1)(1-a2) a3 z3 and A = a1 + (1-a1) a2 + (1-a1)(1-a2) a3, in the depth
    order of the centres; the colour image is unchanged by asking for them."""
    st = oracle.Settings(bg=(0.05, 0.1, 0.15))
    rgbs = [(0.9, 0.1, 0.1), (0.1, 0.8, 0.2), (0.2, 0.3, 0.9)]
    betas = [1.3, 2.0, 3.1]
    ops = [0.6, 0.5, 0.7]
    for zs in ([-0.5, 0.0, 0.5], [0.5, 0.0, -0.5]):
        means = [(0.0, 0.0, z) for z in zs]
        sc = stacked_scene(means, [(0.08, 0.08, 0.08)] * 3, [(1, 0, 0, 0)] * 3, ops, betas, rgbs, width=32, height=32)
        f = oracle.forward(sc, st, channels=True)
        plain = oracle.forward(sc, st)
        np.testing.assert_array_equal(f["image"], plain["image"])
        pr = f["proj"]
        z = _camera_depth(sc.cameras[0], sc.means)
        order = np.argsort(z)
        ys, xs = np.mgrid[0:32, 0:32]
        D = np.zeros((32, 32))
        A = np.zeros((32, 32))
        T = np.ones((32, 32))
        for i in order:
            a = pr["sigma2d"][i, 0]
            u, v = pr["rec"][i, :2]
            r2 = (xs + 0.5 - u) ** 2 + (ys + 0.5 - v) ** 2
            al = np.minimum(0.99, float(sc.opacities[i]) * np.exp(-0.5 * (r2 / a) ** (float(sc.betas[i]) / 2)))
            al = np.where(al >= float(np.float32(1 / 255)), al, 0.0)
            D += al * T * z[i]
            A += al * T
            T = T * (1 - al)
        assert T.min() > 1e-4  # no termination in this configuration
        np.testing.assert_allclose(f["depth"].reshape(32, 32), D, rtol=0, atol=1e-13)
        np.testing.assert_allclose(f["alpha"].reshape(32, 32), A, rtol=0, atol=1e-14)


def test_alpha_is_one_minus_T_and_depth_is_a_weighted_average():
    """On the 2,000-splat workload with termination: A = 1 - T_final (the
    alpha-blending weights telescope), and D / A lies between the nearest and
    farthest depth of the composited splats (a convex combination)."""
    st = oracle.Settings()
    sc = gi.make_workload(1)
    f = oracle.forward(sc, st, channels=True)
    np.testing.assert_allclose(f["alpha"], 1.0 - f["final_T"], rtol=0, atol=1e-12)
    z = f["proj"]["depth"][f["proj"]["cull"] == 0]
    A, D = f["alpha"], f["depth"]
    assert (A > 0.5).sum() > 1000
    nz = A > 1e-9
    assert (D[nz] >= z.min() * A[nz] - 1e-12).all() and (D[nz] <= z.max() * A[nz] + 1e-12).all()
    assert (D[~nz] == 0).all()


def test_channels_terminate_with_the_colour():
    """A pixel that terminates composites nothing further into D and A: stacking
    more opaque splats behind the terminating one leaves both unchanged."""
    st = oracle.Settings()
    n = 5
    mk = lambda k: stacked_scene([(0.0, 0.0, -0.3 + 0.15 * j) for j in range(k)], [(1.0, 1.0, 1.0)] * k,  # noqa
                                 [(1, 0, 0, 0)] * k, [0.95] * k, [2.0] * k, [(0.5, 0.5, 0.5)] * k, width=16, height=16)
    f4 = oracle.forward(mk(4), st, channels=True)
    f5 = oracle.forward(mk(n), st, channels=True)
    c = 8 * 16 + 8
    assert f5["n_contrib"][c] == 3
    assert f4["depth"][c] == f5["depth"][c] and f4["alpha"][c] == f5["alpha"][c]


def _loss(scene, st, g_img, g_d, g_a):
    pr = oracle.project(scene, st)
    win = np.array([[0, 0, c.width - 1, c.height - 1] for c in scene.cameras], np.int32)
    loss, _, dec = oracle.window_fwdbwd(scene.n, scene.cameras, pr["rec"], pr["zbits"], pr["cull"], pr["pix_rect"],
                                        win, g_img, [], st, depth=pr["depth"], dL_ddepth=g_d, dL_dalpha=g_a)
    return loss, dec


def _perturbed(scene, name, idx, val):
    s = copy.copy(scene)
    arr = np.array(getattr(scene, name), dtype=np.float64, copy=True)
    arr.reshape(-1)[idx] = val
    setattr(s, name, arr)
    return s


def fd_check_channels(scene, st, seed, colour=True, rel=2e-6):
    """Central differences of L = g.C + gD.D + gA.A against the adjoint, with
    every discrete decision held fixed (a step that changes one is halved, up to
    three times, and otherwise skipped)."""
    rng = np.random.default_rng(seed)
    P = scene.n_pixels
    g_img = rng.standard_normal(3 * P) if colour else np.zeros(3 * P)
    g_d = rng.standard_normal(P)
    g_a = rng.standard_normal(P)
    f = oracle.forward(scene, st, channels=True)
    grads = oracle.backward(scene, st, f, g_img, dL_ddepth=g_d, dL_dalpha=g_a)
    base_loss, base_dec = _loss(scene, st, g_img, g_d, g_a)
    expect = float(np.dot(g_img, f["image"]) + np.dot(g_d, f["depth"]) + np.dot(g_a, f["alpha"]))
    assert base_loss == pytest.approx(expect, rel=1e-13)
    assert np.abs(grads["grad2d"][:, 10]).max() > 0
    gmax = max(np.abs(grads[p]).max() for p in PARAMS)
    checked = skipped = 0
    for name in PARAMS:
        base = np.asarray(getattr(scene, name), dtype=np.float64).reshape(-1)
        an = grads[name].reshape(-1)
        for k in range(base.size):
            h = 1e-6 * max(abs(base[k]), 1e-2)
            ok = False
            for _ in range(4):
                lp, dp = _loss(_perturbed(scene, name, k, base[k] + h), st, g_img, g_d, g_a)
                lm, dm = _loss(_perturbed(scene, name, k, base[k] - h), st, g_img, g_d, g_a)
                if dp == base_dec and dm == base_dec:
                    ok = True
                    break
                h *= 0.5
            if not ok:
                skipped += 1
                continue
            fd = (lp - lm) / (2 * h)
            tol = rel * max(abs(fd), 1e-3 * gmax) + 1e-9 * abs(base_loss) / h
            assert abs(an[k] - fd) <= tol, (name, k, an[k], fd)
            checked += 1
    assert checked > 0 and skipped <= max(2, checked // 50)
    return checked, skipped


@pytest.mark.parametrize("seed,deg,views,colour", [(0, 0, 1, False), (1, 1, 2, True), (2, 2, 1, True)])
def test_fd_channel_gradients(seed, deg, views, colour):
    """The adjoint of the depth and opacity channels (alone, and together with
    the colour loss) equals central differences of the forward."""
    st = oracle.Settings(sh_degree=deg, tile_w=8, tile_h=8)
    sc = gi.tiny_scene(30 + seed, n=10, deg=deg, n_views=views)
    fd_check_channels(sc, st, seed, colour=colour)


def test_fd_channel_gradients_with_cap_and_termination():
    """Opaque splats: alpha reaches the cap and pixels terminate early."""
    st = oracle.Settings(sh_degree=0)
    sc = gi.tiny_scene(41, n=12, deg=0, log_scale=(-1.9, -1.2))
    sc = with_params(sc, opacities=np.linspace(0.9, 0.9999, sc.n).astype(np.float32))
    f = oracle.forward(sc, st)
    assert (f["final_T"] < 1e-3).any()
    fd_check_channels(sc, st, 41)
