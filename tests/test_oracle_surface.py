"""Pins of the oracle's level-set surface points (DyGASR, arXiv 2411.09156,
Sec. 3.3, mesh extraction): rays from the depth map, density of Eq. 9 sampled
over +-3 sigma_g(w) of the dominating distribution, the first upward crossing
of the level by linear interpolation, normals from the density gradient.

Fixed by closed forms that do not use the oracle's arithmetic: along a ray
x(t) = c + t w a splat's Mahalanobis distance is |a + t b| with a, b from the
inverse of M = R(q) diag(phi s) (rotation from scipy), so a lone splat's
crossing solves a quadratic and its normal is Sigma^-1 (x - mu) normalised; two
splats' crossing is a scipy root of the summed density.  Linear interpolation
between K samples converges to these as K grows.
"""
import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.spatial.transform import Rotation

import oracle
from tests.oracle_util import stacked_scene

LEVEL, SPAN = 0.3, 3.0


def _phi(beta, rho):
    return 2.0 / (1.0 + np.exp(-rho * (beta - 2.0)))


def _Minv(scale, quat, beta, rho):
    """Inverse of M = R diag(phi s), R from scipy (quat given w, x, y, z)."""
    q = np.asarray(quat, np.float64)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    d = _phi(float(beta), rho) * np.asarray(scale, np.float64)
    return np.diag(1.0 / d) @ R.T, R @ np.diag(d)


def _ray(cam, px, py):
    R = np.asarray(cam.viewmat, np.float64)[:, :3]
    dc = np.array([(px + 0.5 - cam.cx) / cam.fx, (py + 0.5 - cam.cy) / cam.fy, 1.0])
    nd = np.linalg.norm(dc)
    return np.asarray(cam.campos, np.float64), R.T @ dc / nd, nd


def _run(sc, st, pixels, depth, alpha, K):
    pr = oracle.project(sc, st)
    keys, vals, ranges = oracle.bin_instances(sc.n, sc.cameras, pr["tile_rect"], pr["tiles_touched"], pr["zbits"], st,
                                              pr["rec"])
    return oracle.surface_points(sc, pr["rec"], vals, ranges, depth, alpha, pixels, st, n_samples=K, level=LEVEL,
                                 span=SPAN)


@pytest.mark.parametrize("beta,quat,scale,pix", [
    (2.0, (1, 0, 0, 0), (0.3, 0.3, 0.3), (16, 16)),
    (1.4, (0.9, 0.2, -0.3, 0.1), (0.5, 0.2, 0.35), (16, 16)),
    (3.2, (0.6, -0.4, 0.5, 0.3), (0.45, 0.25, 0.3), (15, 17)),
])
def test_lone_splat_crossing_and_normal_closed_form(beta, quat, scale, pix):
    """One splat: the crossing closest to the camera solves |a + t b| = m* with
    m* = (ln(o/level)/kappa)^(1/beta); the normal is Sigma^-1 (x - mu)
    normalised (the outward density gradient flipped)."""
    st = oracle.Settings()
    o = 0.9
    sc = stacked_scene([(0.0, 0.0, 0.0)], [scale], [quat], [o], [beta], [(0.5, 0.5, 0.5)], width=33, height=33)
    cam = sc.cameras[0]
    P = 33 * 33
    px, py = pix
    c, w, nd = _ray(cam, px, py)
    Minv, M = _Minv(sc.scales[0], sc.quats[0], sc.betas[0], float(np.float32(st.rho)))
    mu = np.asarray(sc.means[0], np.float64)
    # depth-map origin: the point of the ray closest (in Mahalanobis distance) to the centre
    a0, b = Minv @ (c - mu), Minv @ w
    t_c = -a0 @ b / (b @ b)
    z = t_c / nd
    depth = np.zeros(P)
    alpha = np.zeros(P)
    depth[py * 33 + px] = z
    alpha[py * 33 + px] = 1.0
    K = 4001
    out = _run(sc, st, [py * 33 + px], depth, alpha, K)
    assert out["valid"][0] == 1 and out["dominant"][0] == 0
    kappa = float(np.float32(st.kappa))
    mstar = (np.log(float(np.float32(o)) / LEVEL) / kappa) ** (1.0 / float(sc.betas[0]))
    # |a0 + t b|^2 = mstar^2, smaller root
    A2, B2, C2 = b @ b, 2 * a0 @ b, a0 @ a0 - mstar ** 2
    t_star = (-B2 - np.sqrt(B2 * B2 - 4 * A2 * C2)) / (2 * A2)
    sigma = np.linalg.norm(M.T @ w)
    h = 2 * SPAN * sigma / (K - 1)
    assert out["t_star"][0] == pytest.approx(t_star, abs=h * h / sigma)
    x = c + t_star * w
    n = (Minv.T @ Minv) @ (x - mu)
    n /= np.linalg.norm(n)
    np.testing.assert_allclose(out["points"][0], x, atol=h * h / sigma)
    np.testing.assert_allclose(out["normals"][0], n, atol=1e-5)
    assert out["normals"][0] @ w < 0  # facing the camera


def test_two_splats_crossing_is_the_root_of_the_summed_density():
    """Two overlapping splats: t* is the first root of d(c + t w) = level
    (scipy brentq on an independent evaluation of Eq. 9), g is the larger
    term at the depth-map point."""
    st = oracle.Settings()
    means = [(0.05, -0.02, 0.0), (-0.1, 0.08, 0.35)]
    scales = [(0.3, 0.2, 0.25), (0.25, 0.3, 0.2)]
    quats = [(0.9, 0.1, 0.2, -0.1), (0.7, -0.3, 0.1, 0.4)]
    ops, betas = [0.6, 0.8], [1.6, 2.6]
    sc = stacked_scene(means, scales, quats, ops, betas, [(0.5, 0.5, 0.5)] * 2, width=33, height=33)
    cam = sc.cameras[0]
    px = py = 16
    c, w, nd = _ray(cam, px, py)
    rho, kappa = float(np.float32(st.rho)), float(np.float32(st.kappa))
    terms = []
    for i in range(2):
        Minv, _ = _Minv(sc.scales[i], sc.quats[i], sc.betas[i], rho)
        mu = np.asarray(sc.means[i], np.float64)
        o, bt = float(sc.opacities[i]), float(sc.betas[i])
        terms.append(lambda t, Minv=Minv, mu=mu, o=o, bt=bt:
                     o * np.exp(-kappa * (np.sum((Minv @ (c + t * w - mu)) ** 2)) ** (bt / 2)))
    dens = lambda t: terms[0](t) + terms[1](t)  # noqa: E731
    t0 = 4.0 * nd
    depth = np.zeros(33 * 33)
    alpha = np.zeros(33 * 33)
    depth[py * 33 + px], alpha[py * 33 + px] = 4.0, 1.0
    out = _run(sc, st, [py * 33 + px], depth, alpha, 4001)
    assert out["valid"][0] == 1
    g = int(np.argmax([terms[0](t0), terms[1](t0)]))
    assert out["dominant"][0] == g
    _, Mg = _Minv(sc.scales[g], sc.quats[g], sc.betas[g], rho)
    sigma = np.linalg.norm(Mg.T @ w)
    ts = np.linspace(t0 - SPAN * sigma, t0 + SPAN * sigma, 4001)
    d = np.array([dens(t) for t in ts])
    k = int(np.nonzero((d[:-1] < LEVEL) & (d[1:] >= LEVEL))[0][0])
    root = brentq(lambda t: dens(t) - LEVEL, ts[k], ts[k + 1], xtol=1e-15)
    h = ts[1] - ts[0]
    assert out["t_star"][0] == pytest.approx(root, abs=h * h)


def test_rays_without_surface_are_invalid():
    """Alpha below the threshold, or a level above the density anywhere on the
    sampled interval, give no point."""
    st = oracle.Settings()
    sc = stacked_scene([(0.0, 0.0, 0.0)], [(0.3, 0.3, 0.3)], [(1, 0, 0, 0)], [0.25], [2.0], [(0.5, 0.5, 0.5)],
                       width=33, height=33)
    depth = np.full(33 * 33, 4.0)
    alpha = np.zeros(33 * 33)
    alpha[16 * 33 + 16] = 1.0
    alpha[16 * 33 + 15] = 0.4  # below min_alpha = 0.5
    out = _run(sc, st, [16 * 33 + 16, 16 * 33 + 15], depth, alpha, 64)
    # opacity 0.25 < level 0.3: the density never reaches the level
    assert out["valid"].tolist() == [0, 0]
    assert out["dominant"][1] == -1
