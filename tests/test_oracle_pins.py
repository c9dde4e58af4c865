"""Pins of the FP64 oracle against things other than itself.

Each test names the passage it pins (DyGASR, arXiv 2411.09156) and what fixes
the expected value: a closed form, a library routine (scipy), brute force, or
an invariant of alpha compositing.
"""
import numpy as np
import pytest
import scipy.special as sps
import scipy.stats as ss
from scipy.spatial.transform import Rotation

import gesr_inputs as gi
import oracle
from tests.oracle_util import single_splat_scene, stacked_scene, subset_views, with_params


def _camera_T(cam, p):
    """2x3 Jacobian of the pinhole map (x,y,z) -> (fx x/z + cx, fy y/z + cy), by
    central differences, composed with the view rotation."""
    def pin(q):
        return np.array([cam.fx * q[0] / q[2] + cam.cx, cam.fy * q[1] / q[2] + cam.cy])
    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-6 * max(1.0, abs(p[k]))
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (pin(p + e) - pin(p - e)) / (2 * h)
    return J @ cam.viewmat[:, :3].astype(np.float64)


# ---------------------------------------------------------------- projection
def test_on_axis_isotropic_closed_form():
    """Sec. 3.2 (Eq. 4 and the Sigma' = J W Sigma W^T J^T passage): an on-axis
    isotropic splat at depth z has Sigma' = ((f phi s / z)^2 + blur) I exactly and
    projects to the principal point."""
    st = oracle.Settings()
    for beta in (1.0, 2.0, 3.5):
        sc = single_splat_scene(scale=(0.07, 0.07, 0.01), beta=beta, width=128, height=128)
        pr = oracle.project(sc, st)
        cam = sc.cameras[0]
        phi = 2.0 / (1.0 + np.exp(-float(np.float32(st.rho)) * (float(np.float32(beta)) - 2.0)))
        s = float(np.float32(0.07))
        expect = (cam.fx * phi * s / 4.0) ** 2 + float(np.float32(st.blur))
        a, b, c = pr["sigma2d"][0]
        assert a == pytest.approx(expect, rel=1e-12)
        assert c == pytest.approx(expect, rel=1e-12)
        assert abs(b) < 1e-12 * expect
        u, v, A, B, C = pr["rec"][0, :5]
        assert (u, v) == (pytest.approx(64.0, abs=1e-12), pytest.approx(64.0, abs=1e-12))
        assert A == pytest.approx(1.0 / expect, rel=1e-12) and C == pytest.approx(1.0 / expect, rel=1e-12)


def test_sigma2d_matches_scipy_rotation_and_fd_jacobian():
    """Eq. (4) Sigma = R S S^T R^T with R from scipy's quaternion routine, and the
    EWA screen covariance with the pinhole Jacobian taken by finite differences
    (rho = 0 so phi = 1, blur = 0)."""
    st = oracle.Settings(rho=0.0, blur=0.0)
    sc = gi.tiny_scene(3, n=40, deg=0)
    pr = oracle.project(sc, st)
    cam = sc.cameras[0]
    checked = 0
    for i in range(sc.n):
        if pr["cull"][i] != 0:
            continue
        q = sc.quats[i].astype(np.float64)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        S = np.diag(sc.scales[i].astype(np.float64))
        Sig = R @ S @ S.T @ R.T
        p = cam.viewmat[:, :3].astype(np.float64) @ sc.means[i].astype(np.float64) + cam.viewmat[:, 3]
        T = _camera_T(cam, p)
        Sp = T @ Sig @ T.T
        np.testing.assert_allclose(pr["sigma2d"][i], [Sp[0, 0], Sp[0, 1], Sp[1, 1]], rtol=2e-7,
                                   atol=1e-9 * np.abs(Sp).max())
        checked += 1
    assert checked > 20


def test_frustum_clamp_uses_jacobian_at_clamped_point():
    """Off-frustum centre: the Jacobian is taken at the centre clamped to
    clip_fac times the half field of view (reading of the unstated clamp)."""
    st = oracle.Settings(rho=0.0, blur=0.0)
    sc = single_splat_scene(mean=(3.5, 0.2, 0.0), scale=(0.3, 0.2, 0.25), quat=(0.9, 0.1, -0.3, 0.2))
    pr = oracle.project(sc, st)
    cam = sc.cameras[0]
    p = cam.viewmat[:, :3].astype(np.float64) @ sc.means[0].astype(np.float64) + cam.viewmat[:, 3]
    lim = float(np.float32(st.clip_fac)) * cam.width / (2 * cam.fx)
    assert abs(p[0] / p[2]) > lim
    pc = p.copy()
    pc[0] = np.sign(p[0]) * lim * p[2]
    T = _camera_T(cam, pc)
    q = sc.quats[0].astype(np.float64)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    Sig = R @ np.diag(sc.scales[0].astype(np.float64) ** 2) @ R.T
    Sp = T @ Sig @ T.T
    np.testing.assert_allclose(pr["sigma2d"][0], [Sp[0, 0], Sp[0, 1], Sp[1, 1]], rtol=2e-7)


def test_phi_special_cases():
    """Eq. (6)-(7) as read (phi = 2 / (1 + exp(-rho (beta - 2)))): phi(2) = 1 for
    any rho, rho = 0 gives phi = 1 for any beta, and with blur = 0 the screen
    covariance scales by phi^2, increasing in beta for rho > 0."""
    base = dict(mean=(0.1, -0.2, 0.3), scale=(0.05, 0.08, 0.03), quat=(0.8, 0.3, 0.1, -0.4))
    st0 = oracle.Settings(blur=0.0)
    s_ref = oracle.project(single_splat_scene(beta=2.0, **base), oracle.Settings(blur=0.0, rho=0.7))["sigma2d"][0]
    for rho in (0.0, 0.1, 0.7):
        s2 = oracle.project(single_splat_scene(beta=2.0, **base), oracle.Settings(blur=0.0, rho=rho))["sigma2d"][0]
        np.testing.assert_allclose(s2, s_ref, rtol=1e-14)
    for beta in (0.5, 1.0, 3.0, 4.0):
        s_b = oracle.project(single_splat_scene(beta=beta, **base), oracle.Settings(blur=0.0, rho=0.0))["sigma2d"][0]
        np.testing.assert_allclose(s_b, s_ref, rtol=1e-14)
    ratios = []
    for beta in (1.0, 1.5, 2.0, 3.0, 4.0):
        s_b = oracle.project(single_splat_scene(beta=beta, **base), st0)["sigma2d"][0]
        ratios.append(s_b[0] / s_ref[0])
        np.testing.assert_allclose(s_b / s_ref, ratios[-1], rtol=1e-12)
    assert all(np.diff(ratios) > 0)
    assert ratios[2] == pytest.approx(1.0, rel=1e-14)


def test_sh_basis_matches_scipy():
    """Real SH with the Condon-Shortley phase (colour model of the splats): the
    oracle's polynomial basis equals sqrt(2) Re/Im of scipy's complex Y_l^m."""
    rng = np.random.default_rng(0)
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = oracle.sh_basis(3, d)
    th = np.arccos(np.clip(d[:, 2], -1, 1))
    ph = np.arctan2(d[:, 1], d[:, 0])
    for l in range(4):
        for m in range(-l, l + 1):
            c = sps.sph_harm_y(l, abs(m), th, ph)
            ref = c.real if m == 0 else (np.sqrt(2) * c.real if m > 0 else np.sqrt(2) * c.imag)
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-13)


def test_sh_orthonormal_by_quadrature():
    """The degree-3 basis is orthonormal on the sphere: Gauss-Legendre in cos(theta)
    times a uniform rule in phi integrates products of degree <= 6 exactly."""
    x, w = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phis = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(x, phis, indexing="ij")
    st_ = np.sqrt(1 - ct ** 2)
    d = np.stack([st_ * np.cos(ph), st_ * np.sin(ph), ct], -1).reshape(-1, 3)
    wt = (np.repeat(w, nphi) * (2 * np.pi / nphi))
    Y = oracle.sh_basis(3, d)
    G = (Y * wt[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)
    assert Y[0, 0] == pytest.approx(1 / (2 * np.sqrt(np.pi)), rel=1e-15)


def test_colour_is_requested_rgb_plus_offset():
    """Colour reading (real SH plus 1/2): splats whose only coefficient is
    (rgb - 1/2) / Y00, with Y00 = 1 / (2 sqrt(pi)) (scipy's degree-0 harmonic),
    project to exactly that rgb; all-zero coefficients give 1/2 in every
    channel."""
    Y00 = float(np.real(sps.sph_harm_y(0, 0, 0.3, 1.1)))
    assert Y00 == pytest.approx(0.5 / np.sqrt(np.pi), rel=1e-15)
    rgbs = [(0.9, 0.1, 0.1), (0.1, 0.8, 0.2), (0.2, 0.3, 0.9), (0.0, 1.0, 0.5)]
    sc = stacked_scene([(0.0, 0.0, z) for z in (-0.5, 0.0, 0.5, 0.2)], [(0.08, 0.08, 0.08)] * 4, [(1, 0, 0, 0)] * 4,
                       [0.6] * 4, [2.0] * 4, rgbs, width=32, height=32, sh_dtype=np.float64)
    sc.sh[:, 0, :] = (np.asarray(rgbs) - 0.5) / Y00
    pr = oracle.project(sc, oracle.Settings())
    np.testing.assert_allclose(pr["rec"][:, 8:11], rgbs, rtol=0, atol=1e-12)
    zero = with_params(sc, sh=np.zeros_like(sc.sh))
    np.testing.assert_array_equal(oracle.project(zero, oracle.Settings())["rec"][:, 8:11], 0.5)


def test_negative_colour_clamps_to_zero_with_zero_gradient():
    """A channel whose SH sum plus 1/2 is negative is clamped to 0: the splat
    adds nothing to that channel (image = (1 - alpha) bg there), and that
    channel's coefficients and the view-direction term it would feed get no
    gradient -- the oracle's adjoint equals central differences of its forward
    for every parameter, and its gradient of the clamped channel's
    coefficients is exactly zero."""
    st = oracle.Settings(sh_degree=1, bg=(0.2, 0.4, 0.6))
    sc = single_splat_scene(mean=(0.3, -0.25, 0.2), scale=(0.07, 0.05, 0.06), quat=(0.9, 0.1, -0.2, 0.3),
                            opacity=0.8, beta=1.7, rgb=(0.7, 0.5, 0.3), width=40, height=32)
    sh = np.zeros((1, 4, 3))
    sh[0, 0] = [0.8, -2.5, 0.4]          # green: -2.5 Y00 + 1/2 < 0 before the degree-1 terms
    sh[0, 1:, :] = [[0.3, 0.2, -0.1], [0.1, -0.3, 0.2], [-0.2, 0.1, 0.3]]
    sc = with_params(sc, sh=sh, sh_degree=1)
    f = oracle.forward(sc, st)
    pr = f["proj"]
    assert pr["clamp"][0] == 2 and pr["rec"][0, 9] == 0.0 and pr["rec"][0, 8] > 0 and pr["rec"][0, 10] > 0
    alpha = 1.0 - f["final_T"]
    bg = float(np.float32(0.4))
    np.testing.assert_allclose(f["image"][40 * 32:2 * 40 * 32], (1.0 - alpha) * bg, rtol=0, atol=1e-15)
    g_img = oracle.flat_images([np.random.default_rng(4).standard_normal((3, 32, 40))])
    g = oracle.backward(sc, st, f, g_img)
    assert (g["sh"][0, :, 1] == 0.0).all() and np.abs(g["sh"][0, :, 0]).min() > 0
    from tests.test_oracle_fd import _loss, _perturbed
    base, dec = _loss(sc, st, g_img)
    for name in ("means", "sh"):
        arr = np.asarray(getattr(sc, name), np.float64).reshape(-1)
        for k in range(arr.size):
            h = 1e-6 * max(abs(arr[k]), 1.0)
            lp, dp = _loss(_perturbed(sc, name, k, arr[k] + h), st, g_img)
            lm, dm = _loss(_perturbed(sc, name, k, arr[k] - h), st, g_img)
            assert dp == dec and dm == dec
            fd = (lp - lm) / (2 * h)
            assert abs(g[name].reshape(-1)[k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g[name]).max()), (name, k)


# ------------------------------------------------------------------- falloff
def _lone_expected(sc, st, pr):
    """Closed-form image of a lone isotropic splat: alpha = min(amax, o exp(-kappa
    (r^2 / s2)^(beta/2))) where >= amin, image = alpha rgb + (1 - alpha) bg."""
    cam = sc.cameras[0]
    a = pr["sigma2d"][0, 0]
    u, v = pr["rec"][0, :2]
    o = float(sc.opacities[0])
    beta = float(sc.betas[0])
    rgb = pr["rec"][0, 8:11]
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    r2 = (xs + 0.5 - u) ** 2 + (ys + 0.5 - v) ** 2
    G = np.exp(-f32(st.kappa) * (r2 / a) ** (beta / 2))
    alpha = np.minimum(f32(st.alpha_max), o * G)
    alpha = np.where(alpha >= f32(st.alpha_min), alpha, 0.0)
    bg = np.array([f32(b) for b in st.bg])
    img = alpha[None] * rgb[:, None, None] + (1 - alpha[None]) * bg[:, None, None]
    return img, 1 - alpha


@pytest.mark.parametrize("beta,kappa", [(2.0, 0.5), (1.0, 0.5), (3.3, 0.5), (1.6, 1.0)])
def test_lone_splat_profile(beta, kappa):
    """Eq. (1)-(3) in screen space: a lone on-axis isotropic splat renders the
    generalized-exponential profile, cut at alpha_min and capped at alpha_max."""
    st = oracle.Settings(kappa=kappa, bg=(0.2, 0.1, 0.3))
    sc = single_splat_scene(scale=(0.06, 0.06, 0.06), beta=beta, opacity=0.995, width=48, height=40)
    f = oracle.forward(sc, st)
    img, T = _lone_expected(sc, st, f["proj"])
    np.testing.assert_allclose(f["image"].reshape(3, 40, 48), img, rtol=0, atol=1e-14)
    np.testing.assert_allclose(f["final_T"].reshape(40, 48), T, rtol=0, atol=1e-14)


def test_beta2_is_textbook_gaussian():
    """Eq. (2): at beta = 2 and kappa = 1/2 the falloff of an anisotropic splat is
    the Gaussian exp(-d^T Sigma'^-1 d / 2), i.e. scipy's normal pdf divided by
    its peak, with Sigma' the oracle's screen covariance."""
    st = oracle.Settings(alpha_min=1e-30, alpha_max=0.999999)
    sc = single_splat_scene(mean=(0.2, -0.1, 0.3), scale=(0.12, 0.05, 0.02), quat=(0.7, 0.2, -0.5, 0.3),
                            beta=2.0, opacity=0.9, rgb=(1.0, 1.0, 1.0), width=48, height=40)
    f = oracle.forward(sc, st)
    pr = f["proj"]
    a, b, c = pr["sigma2d"][0]
    u, v = pr["rec"][0, :2]
    mvn = ss.multivariate_normal(mean=[u, v], cov=[[a, b], [b, c]])
    ys, xs = np.mgrid[0:40, 0:48]
    pts = np.stack([xs + 0.5, ys + 0.5], -1).reshape(-1, 2)
    G = mvn.pdf(pts) / mvn.pdf([u, v])
    # bg = 0 -> red channel = alpha * r = o G r wherever alpha >= alpha_min (no cap reached here)
    expect = float(np.float32(0.9)) * G
    keep = expect >= float(np.float32(1e-30))
    assert keep.sum() > 100
    np.testing.assert_allclose(f["image"][:40 * 48][keep], expect[keep] * pr["rec"][0, 8], rtol=1e-12)
    assert (f["image"][:40 * 48][~keep] == 0).all()


def test_general_beta_uses_mahalanobis_power():
    """Eq. (3) for beta != 2: G = exp(-kappa * m^beta) with m the Mahalanobis
    distance under Sigma' (scipy.spatial.distance.mahalanobis)."""
    from scipy.spatial.distance import mahalanobis
    st = oracle.Settings(alpha_min=1e-30, alpha_max=0.999999)
    sc = single_splat_scene(mean=(0.2, -0.1, 0.3), scale=(0.12, 0.05, 0.02), quat=(0.7, 0.2, -0.5, 0.3),
                            beta=1.37, opacity=0.9, rgb=(1.0, 1.0, 1.0), width=24, height=20)
    f = oracle.forward(sc, st)
    a, b, c = f["proj"]["sigma2d"][0]
    u, v = f["proj"]["rec"][0, :2]
    VI = np.linalg.inv(np.array([[a, b], [b, c]]))
    beta = float(np.float32(1.37))
    for y in range(0, 20, 3):
        for x in range(0, 24, 3):
            m = mahalanobis([x + 0.5, y + 0.5], [u, v], VI)
            expect = float(np.float32(0.9)) * np.exp(-0.5 * m ** beta) * f["proj"]["rec"][0, 8]
            assert f["image"][y * 24 + x] == pytest.approx(expect, rel=1e-11)


# ---------------------------------------------------------------- compositing
def test_three_stacked_splats_closed_form():
    """Eq. (5) as front-to-back alpha blending: three co-axial splats at different
    depths give C = a1 c1 + (1-a1) a2 c2 + (1-a1)(1-a2) a3 c3 + prod(1-a) bg, and
    reversing their depths reverses the order of the terms."""
    st = oracle.Settings(bg=(0.05, 0.1, 0.15))
    rgbs = [(0.9, 0.1, 0.1), (0.1, 0.8, 0.2), (0.2, 0.3, 0.9)]
    betas = [1.3, 2.0, 3.1]
    ops = [0.6, 0.5, 0.7]
    for zs in ([-0.5, 0.0, 0.5], [0.5, 0.0, -0.5]):
        sc = stacked_scene([(0.0, 0.0, z) for z in zs], [(0.08, 0.08, 0.08)] * 3, [(1, 0, 0, 0)] * 3, ops, betas,
                           rgbs, width=32, height=32)
        f = oracle.forward(sc, st)
        pr = f["proj"]
        order = np.argsort(pr["depth"][:3])
        ys, xs = np.mgrid[0:32, 0:32]
        bg = np.array([float(np.float32(b)) for b in st.bg])
        C = np.zeros((3, 32, 32))
        T = np.ones((32, 32))
        for i in order:
            a = pr["sigma2d"][i, 0]
            u, v = pr["rec"][i, :2]
            r2 = (xs + 0.5 - u) ** 2 + (ys + 0.5 - v) ** 2
            al = np.minimum(0.99, float(sc.opacities[i]) * np.exp(-0.5 * (r2 / a) ** (float(sc.betas[i]) / 2)))
            al = np.where(al >= float(np.float32(1 / 255)), al, 0.0)
            C += al[None] * T[None] * pr["rec"][i, 8:11, None, None]
            T = T * (1 - al)
        C += T[None] * bg[:, None, None]
        assert T.min() > 1e-4  # no termination in this configuration
        np.testing.assert_allclose(f["image"].reshape(3, 32, 32), C, atol=1e-14)


def test_termination_semantics():
    """Front-to-back blending stops before a fragment that would take T below
    t_min; that fragment is not composited (reading of the unstated cutoff)."""
    st = oracle.Settings()
    n = 5
    sc = stacked_scene([(0.0, 0.0, -0.3 + 0.15 * k) for k in range(n)], [(1.0, 1.0, 1.0)] * n,
                       [(1, 0, 0, 0)] * n, [0.95] * n, [2.0] * n, [(0.5, 0.5, 0.5)] * n, width=16, height=16)
    f = oracle.forward(sc, st)
    # at the central pixels alpha ~ 0.93, so T ~ 0.07^k: ~3e-4 after 3, ~2e-5 after 4
    c = 8 * 16 + 8
    assert f["n_contrib"][c] == 3
    assert 1e-4 <= f["final_T"][c] < 1e-3
    assert f["n_listed"][c] == 4 and f["n_hit"][c] == 4


def test_compositing_invariants_on_plain_workload():
    """Invariants of alpha blending on the 2,000-splat workload: t_min <= T <= 1,
    colour inside the convex hull of splat colours and background, and
    opacity below alpha_min leaves the background untouched."""
    st = oracle.Settings(bg=(0.3, 0.6, 0.9))
    sc = gi.make_workload(1)
    f = oracle.forward(sc, st)
    T = f["final_T"]
    assert T.min() >= float(np.float32(st.t_min)) and T.max() <= 1.0
    img = f["image"].reshape(3, -1)
    rec = f["proj"]["rec"]
    for c in range(3):
        lo = min(rec[:, 8 + c].min(), st.bg[c]) - 1e-12
        hi = max(rec[:, 8 + c].max(), st.bg[c]) + 1e-12
        assert img[c].min() >= lo and img[c].max() <= hi
    dim = with_params(sc, opacities=np.full(sc.n, 0.5 / 255, np.float32))
    f2 = oracle.forward(dim, st)
    bg = np.array([float(np.float32(b)) for b in st.bg])
    np.testing.assert_array_equal(f2["image"].reshape(3, -1), np.repeat(bg[:, None], 128 * 128, 1))
    assert (f2["proj"]["cull"] == 3).all()


# ------------------------------------------------------------------- binning
def test_binning_brute_force():
    """Tile binning (tile | depth keys, stable order): tiles_touched equals the
    number of tiles meeting each pixel rectangle; the lists hold, per pair, a
    subset of its rectangle's tiles that contains every tile with a pixel
    centre inside the footprint (q <= qmax, brute force in float64 over all
    pixels) and drops some of the others; they are sorted by (tile, z32,
    view*N + splat) and the ranges partition them."""
    st = oracle.Settings(tile_w=8, tile_h=8)
    sc = gi.tiny_scene(5, n=30, width=50, height=37, n_views=2)
    pr = oracle.project(sc, st)
    grid, T = oracle.tile_grid(sc.cameras, 8, 8)
    N = sc.n
    rect_total = 0
    need = set()
    for v, cam in enumerate(sc.cameras):
        tx_n, ty_n, base = grid[v]
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        for i in range(N):
            o = v * N + i
            cnt = 0
            if pr["cull"][o] == 0:
                x0, y0, x1, y1 = pr["pix_rect"][o]
                for ty in range(ty_n):
                    for tx in range(tx_n):
                        if tx * 8 <= x1 and tx * 8 + 7 >= x0 and ty * 8 <= y1 and ty * 8 + 7 >= y0:
                            cnt += 1
                u, vv, A, B, C = pr["rec"][o, :5]
                dx, dy = xs + 0.5 - u, ys + 0.5 - vv
                q = A * dx * dx + 2 * B * dx * dy + C * dy * dy
                for y, x in zip(*np.nonzero(q <= pr["rec"][o, 7])):
                    need.add((base + (y // 8) * tx_n + x // 8, o))
            assert pr["tiles_touched"][o] == cnt
            rect_total += cnt
    keys, vals, ranges = oracle.bin_instances(N, sc.cameras, pr["tile_rect"], pr["tiles_touched"], pr["zbits"], st,
                                              pr["rec"])
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    listed = set(zip(tiles.tolist(), vals.tolist()))
    assert len(listed) == len(vals) > 100
    assert need <= listed
    assert len(vals) < rect_total
    for t, o in listed:  # inside the pair's rectangle
        v = o // N
        tx_n, ty_n, base = grid[v]
        tx, ty = (t - base) % tx_n, (t - base) // tx_n
        r = pr["tile_rect"][o]
        assert r[0] <= tx <= r[2] and r[1] <= ty <= r[3]
    inst = sorted((int(t), int(pr["zbits"][o]), int(o)) for t, o in listed)
    np.testing.assert_array_equal(vals, [e[2] for e in inst])
    np.testing.assert_array_equal(tiles, [e[0] for e in inst])
    np.testing.assert_array_equal(keys & np.uint64(0xFFFFFFFF), [e[1] for e in inst])
    lens = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    assert lens.sum() == len(vals)
    for t in range(T):
        s0, s1 = ranges[t]
        assert all(k >> 32 == t for k in keys[s0:s1])


def _scipy_box_min_q(A, B, C, box):
    """Minimum of q = A dx^2 + 2 B dx dy + C dy^2 over the box of offsets
    (dx0, dx1, dy0, dy1), as the bounded linear least-squares problem
    min |F d|^2 with F^T F = [[A, B], [B, C]] (numpy's Cholesky factor),
    solved by scipy's active-set BVLS method."""
    from scipy.optimize import lsq_linear
    dx0, dx1, dy0, dy1 = box
    F = np.linalg.cholesky(np.array([[A, B], [B, C]])).T
    res = lsq_linear(F, np.zeros(2), bounds=([dx0, dy0], [dx1, dy1]), method="bvls", tol=1e-15)
    return float(res.x @ np.array([[A, B], [B, C]]) @ res.x)


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (32, 16)])
def test_tile_lists_are_the_tiles_the_widened_ellipse_meets(tile):
    """Tile coverage: within its rectangle a pair is listed in exactly the
    tiles whose square [tx tw, (tx+1) tw] x [ty th, (ty+1) th] meets the ellipse
    q <= Q, Q = qmax (1 + 2^-8), checked against scipy's minimum of q over each
    square (bounded least squares; except where that minimum lies within 1e-9
    of Q)."""
    tw, th = tile
    st = oracle.Settings(tile_w=tw, tile_h=th)
    sc = gi.tiny_scene(11, n=300, width=97, height=75, n_views=2)
    pr = oracle.project(sc, st)
    rec = pr["rec"]
    grid, _ = oracle.tile_grid(sc.cameras, tw, th)
    keys, vals, _ = oracle.bin_instances(sc.n, sc.cameras, pr["tile_rect"], pr["tiles_touched"], pr["zbits"], st, rec)
    listed = set(zip((keys >> np.uint64(32)).astype(np.int64).tolist(), vals.tolist()))
    checked = near = dropped = 0
    for o in range(len(sc.cameras) * sc.n):
        if pr["tiles_touched"][o] == 0:
            continue
        tx_n, _, base = grid[o // sc.n]
        u, v, A, B, C = (float(x) for x in rec[o, :5])
        Q = float(rec[o, 7]) * (1.0 + 2.0 ** -8)
        tx0, ty0, tx1, ty1 = (int(x) for x in pr["tile_rect"][o])
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                m = _scipy_box_min_q(A, B, C, (tx * tw - u, (tx + 1) * tw - u, ty * th - v, (ty + 1) * th - v))
                if abs(m - Q) <= 1e-9 * Q:
                    near += 1
                    continue
                checked += 1
                is_listed = (base + ty * tx_n + tx, o) in listed
                assert is_listed == (m < Q), (o, tx, ty, m, Q)
                dropped += not is_listed
    assert checked > 500 and dropped >= 30 and near < 0.01 * checked


def test_tile_band_holds_the_float32_reading():
    """The band of the tile rule (orc_bin_band) contains every decision that a
    float32 reading of the rule can take the other way: re-deciding each tile
    of every rectangle from float32 copies of the record (u, v, the conic and
    qmax rounded to float32, box edges and Q formed in float32, the minimum of
    q by scipy on those values) differs from the FP64 rule only at band
    decisions."""
    st = oracle.Settings()
    sc = gi.make_workload(1)
    pr = oracle.project(sc, st)
    rec = pr["rec"]
    keys, vals, _ = oracle.bin_instances(sc.n, sc.cameras, pr["tile_rect"], pr["tiles_touched"], pr["zbits"], st, rec)
    band = oracle.bin_band(sc.n, sc.cameras, pr["tile_rect"], pr["tiles_touched"], rec, st)
    in_band = set(zip(band["tile"].tolist(), band["pair"].tolist()))
    listed = set(zip((keys >> np.uint64(32)).astype(np.int64).tolist(), vals.tolist()))
    n_in, n_band = oracle.bin_pair_counts(sc.n, sc.cameras, pr["tile_rect"], pr["tiles_touched"], rec, st)
    assert int(n_band.sum()) == len(in_band)
    assert int(n_in.sum()) + sum(1 for t, p in in_band if (t, p) in listed) == len(listed)
    f32 = np.float32
    grid, _ = oracle.tile_grid(sc.cameras, 16, 16)
    rng = np.random.default_rng(3)
    pairs = np.nonzero(pr["tiles_touched"])[0]
    differ = 0
    for o in rng.choice(pairs, 300, replace=False):
        tx_n, _, base = grid[o // sc.n]
        u, v, A, B, C, qmax = (float(f32(x)) for x in rec[o, [0, 1, 2, 3, 4, 7]])
        Q = float(f32(f32(qmax) + f32(qmax) * f32(2.0 ** -8)))
        tx0, ty0, tx1, ty1 = (int(x) for x in pr["tile_rect"][o])
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                box = (float(f32(tx * 16) - f32(u)), float(f32((tx + 1) * 16) - f32(u)),
                       float(f32(ty * 16) - f32(v)), float(f32((ty + 1) * 16) - f32(v)))
                m = _scipy_box_min_q(A, B, C, box)
                t = base + ty * tx_n + tx
                if (m <= Q) != ((t, int(o)) in listed):
                    differ += 1
                    assert (t, int(o)) in in_band, (o, tx, ty, m, Q)
    assert differ <= 3


def test_depth_key_is_float32_rounding_of_depth():
    st = oracle.Settings()
    sc = gi.tiny_scene(1, n=50)
    pr = oracle.project(sc, st)
    np.testing.assert_array_equal(pr["z32"], pr["depth"].astype(np.float32))


# -------------------------------------------------------- tiled == brute force
@pytest.mark.parametrize("seed,views", [(0, 1), (1, 1), (2, 3)])
def test_tiled_equals_brute_force_bitwise(seed, views):
    """Tiling and sorting only reorganise the work: compositing every splat of the
    view in depth order at every pixel (no rectangles, no tiles) gives the same
    image and transmittance bit for bit, because the padded footprint contains
    every fragment with alpha >= alpha_min."""
    st = oracle.Settings(tile_w=8, tile_h=8, sh_degree=1, bg=(0.1, 0.2, 0.3))
    sc = gi.tiny_scene(seed, n=25, n_views=views)
    f = oracle.forward(sc, st)
    pr = f["proj"]
    b = oracle.brute_fwd(sc.n, sc.cameras, pr["rec"], pr["zbits"], pr["cull"], st)
    np.testing.assert_array_equal(b["image"], f["image"])
    np.testing.assert_array_equal(b["final_T"], f["final_T"])
    np.testing.assert_array_equal(b["n_hit"], f["n_hit"])


def test_plain_workload_tiled_equals_brute_force():
    st = oracle.Settings()
    sc = gi.make_workload(1)
    f = oracle.forward(sc, st)
    pr = f["proj"]
    b = oracle.brute_fwd(sc.n, sc.cameras, pr["rec"], pr["zbits"], pr["cull"], st)
    np.testing.assert_array_equal(b["image"], f["image"])
    np.testing.assert_array_equal(b["final_T"], f["final_T"])


def test_tile_size_invariance_bitwise():
    sc = gi.tiny_scene(4, n=40, width=61, height=45, deg=1)
    ref = None
    for tw, th in ((16, 16), (8, 8), (32, 16), (4, 12)):
        f = oracle.forward(sc, oracle.Settings(tile_w=tw, tile_h=th, sh_degree=1))
        if ref is None:
            ref = f
        np.testing.assert_array_equal(f["image"], ref["image"])
        np.testing.assert_array_equal(f["final_T"], ref["final_T"])


def test_batched_equals_per_view_bitwise():
    st = oracle.Settings(sh_degree=1)
    sc = gi.tiny_scene(6, n=30, n_views=3)
    fb = oracle.forward(sc, st)
    off = 0
    for v in range(3):
        fv = oracle.forward(subset_views(sc, [v]), st)
        P = sc.cameras[v].width * sc.cameras[v].height
        np.testing.assert_array_equal(fv["image"], fb["image"][3 * off:3 * (off + P)])
        np.testing.assert_array_equal(fv["final_T"], fb["final_T"][off:off + P])
        np.testing.assert_array_equal(fv["n_contrib"], fb["n_contrib"][off:off + P])
        off += P


def test_rect_filter_does_not_change_brute_force():
    """Every fragment outside a splat's padded pixel rectangle has alpha < alpha_min."""
    st = oracle.Settings(sh_degree=1)
    sc = gi.tiny_scene(7, n=30, beta=(0.8, 1.5))
    pr = oracle.project(sc, st)
    a = oracle.brute_fwd(sc.n, sc.cameras, pr["rec"], pr["zbits"], pr["cull"], st)
    b = oracle.brute_fwd(sc.n, sc.cameras, pr["rec"], pr["zbits"], pr["cull"], st, pix_rect=pr["pix_rect"])
    np.testing.assert_array_equal(a["image"], b["image"])
