"""Finite-difference pins of the oracle's adjoint.

The backward (explicit-list render adjoint + dual-number projection Jacobian)
must equal central differences of the FP64 forward, with every discrete
decision (skips, termination, alpha cap, culls) held fixed: the loss is
L = sum(g * image) for a fixed seeded g, so dL/dtheta is what the backward
returns for upstream gradient g.  A step whose decision set differs from the
unperturbed one is halved (up to three times) and otherwise skipped.
"""
import copy

import numpy as np
import pytest

import gesr_inputs as gi
import oracle

PARAMS = ("means", "scales", "quats", "opacities", "betas", "sh")


def _loss(scene, st, g_img):
    pr = oracle.project(scene, st)
    win = np.array([[0, 0, c.width - 1, c.height - 1] for c in scene.cameras], np.int32)
    loss, _, dec = oracle.window_fwdbwd(scene.n, scene.cameras, pr["rec"], pr["zbits"], pr["cull"], pr["pix_rect"],
                                        win, g_img, [], st)
    return loss, dec


def _perturbed(scene, name, idx, val):
    s = copy.copy(scene)
    arr = np.array(getattr(scene, name), dtype=np.float64, copy=True)
    arr.reshape(-1)[idx] = val
    setattr(s, name, arr)
    return s


def fd_check(scene, st, seed, max_params=None, rel=2e-6):
    g_img = oracle.flat_images([np.random.default_rng(seed).standard_normal((3, c.height, c.width))
                                for c in scene.cameras])
    f = oracle.forward(scene, st)
    grads = oracle.backward(scene, st, f, g_img)
    base_loss, base_dec = _loss(scene, st, g_img)
    # the window brute force and the tiled forward agree exactly
    assert base_loss == pytest.approx(float(np.dot(g_img, f["image"])), rel=1e-13)
    gmax = max(np.abs(grads[p]).max() for p in PARAMS)
    checked = skipped = 0
    rng = np.random.default_rng(seed)
    for name in PARAMS:
        base = np.asarray(getattr(scene, name), dtype=np.float64).reshape(-1)
        an = grads[name].reshape(-1)
        idxs = np.arange(base.size)
        if max_params is not None and base.size > max_params:
            idxs = rng.choice(base.size, max_params, replace=False)
        for k in idxs:
            h = 1e-6 * max(abs(base[k]), 1e-2)
            ok = False
            for _ in range(4):
                lp, dp = _loss(_perturbed(scene, name, k, base[k] + h), st, g_img)
                lm, dm = _loss(_perturbed(scene, name, k, base[k] - h), st, g_img)
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


@pytest.mark.parametrize("seed,deg,views,kappa,bg", [
    (0, 0, 1, 0.5, (0.0, 0.0, 0.0)),
    (1, 1, 1, 0.5, (0.2, 0.5, 0.1)),
    (2, 3, 2, 0.5, (0.0, 0.0, 0.0)),
    (3, 2, 1, 1.0, (0.3, 0.3, 0.3)),
])
def test_fd_tiny_scenes(seed, deg, views, kappa, bg):
    st = oracle.Settings(sh_degree=deg, kappa=kappa, bg=bg, tile_w=8, tile_h=8)
    sc = gi.tiny_scene(seed, n=10, deg=deg, n_views=views)
    fd_check(sc, st, seed)


def test_fd_opaque_stack_with_cap_and_termination():
    """High opacity: alpha hits the 0.99 cap and pixels terminate early."""
    st = oracle.Settings(sh_degree=1)
    sc = gi.tiny_scene(11, n=14, deg=1, log_scale=(-1.9, -1.2))
    sc = copy.copy(sc)
    sc.opacities = np.linspace(0.9, 0.9999, sc.n).astype(np.float32)
    f = oracle.forward(sc, st)
    assert (f["final_T"] < 1e-3).any()
    assert any(o > 0.99 for o in sc.opacities)
    fd_check(sc, st, 11)


def test_fd_sharp_and_flat_shapes():
    """beta below 1 (cusp at the centre) and above 2, and near-2D disks whose
    smallest scale is e^-13 (the flattened splats of surface alignment)."""
    st = oracle.Settings(sh_degree=0)
    sc = gi.tiny_scene(12, n=10, deg=0, beta=(0.6, 4.5))
    sc = copy.copy(sc)
    sc.scales = np.array(sc.scales, np.float64)
    sc.scales[::2, 2] = np.exp(-13.0)
    fd_check(sc, st, 12)


def test_fd_frustum_clamped_splats():
    """Centres outside the clamped field of view still project a footprint."""
    st = oracle.Settings(sh_degree=1)
    sc = gi.tiny_scene(13, n=8, deg=1, spread=0.3)
    sc = copy.copy(sc)
    m = np.array(sc.means, np.float64)
    m[:4, 0] = [2.6, -2.7, 2.9, -2.8]
    sc.means = m
    sc.scales = np.array(sc.scales, np.float64) * 4.0
    pr = oracle.project(sc, st)
    cam = sc.cameras[0]
    lim = float(np.float32(1.3)) * cam.width / (2 * cam.fx)
    p = m[:4] @ cam.viewmat[:, :3].T.astype(np.float64) + cam.viewmat[:, 3]
    clamped = np.abs(p[:, 0] / p[:, 2]) > lim
    assert clamped.any() and (pr["cull"][:4][clamped] == 0).any()
    fd_check(sc, st, 13)


def test_fd_sampled_plain_workload():
    """64 sampled parameters of the 2,000-splat workload."""
    st = oracle.Settings(sh_degree=0)
    sc = gi.make_workload(1)
    fd_check(sc, st, 21, max_params=11)
