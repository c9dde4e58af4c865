"""Seeded synthetic scenes for the GES rasterizer.

This module only *draws inputs*: splat parameters, pinhole cameras, target
images and upstream image gradients.  It holds none of the rasterizer's
arithmetic (no projection, falloff, compositing or adjoint), so the FP64
oracle and the HIP path can both consume its arrays without sharing any of
the method's code.

The paper evaluates on Mip-NeRF360 and Deep Blending captures; those are not
available here, so the five workloads below stand in for them with the
shapes, sizes and value distributions stated for each one.

Seeding: ``numpy.random.default_rng([workload, stream])`` with stream 0 =
scene, 1 = target images, 2 = upstream dL/dimage, 3 = sample choice.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# The degree-0 real spherical harmonic is the constant 1/(2*sqrt(pi)); a DC
# coefficient k gives colour k/(2 sqrt(pi)) + 0.5, so k uniform in
# [-sqrt(pi), sqrt(pi)] makes the view-independent colour uniform in [0, 1].
_DC_HALF_RANGE = math.sqrt(math.pi)


@dataclasses.dataclass
class Camera:
    """Pinhole camera: OpenCV axes (x right, y down, z forward)."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    viewmat: np.ndarray  # (3, 4) float32, world -> camera [R | t]
    campos: np.ndarray   # (3,) float32, camera centre in world coordinates


@dataclasses.dataclass
class Scene:
    """Splat parameters in AoS (row per splat) float32 arrays.

    ``scales`` and ``opacities`` are the activated values the rasterizer
    consumes; ``log_scales`` and ``opacity_logits`` are the leaf parameters
    they were drawn as.
    """
    name: str
    means: np.ndarray          # (N, 3)
    log_scales: np.ndarray     # (N, 3)
    scales: np.ndarray         # (N, 3) = exp(log_scales), rounded to float32
    quats: np.ndarray          # (N, 4) w, x, y, z; not normalised
    opacity_logits: np.ndarray # (N,)
    opacities: np.ndarray      # (N,) = sigmoid(opacity_logits), float32
    betas: np.ndarray          # (N,) shape parameter (epsilon in the paper)
    sh: np.ndarray             # (N, K, 3) real SH coefficients, K=(deg+1)^2
    sh_degree: int
    cameras: List[Camera]
    normals: Optional[np.ndarray] = None  # (N, 3) true surface normal (flattened workload)
    loss: str = "l1"

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_views(self) -> int:
        return len(self.cameras)

    @property
    def n_pixels(self) -> int:
        return int(sum(c.width * c.height for c in self.cameras))


def look_at(position, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), width=128, height=128,
            fov_x_deg=60.0) -> Camera:
    """Camera at ``position`` looking at ``target``; the fov is horizontal, fx = fy,
    principal point at the image centre."""
    pos = np.asarray(position, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - pos
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, dtype=np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    rot = np.stack([right, down, fwd])
    t = -rot @ pos
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    vm = np.concatenate([rot, t[:, None]], axis=1).astype(np.float32)
    return Camera(int(width), int(height), float(np.float32(f)), float(np.float32(f)),
                  float(width / 2.0), float(height / 2.0), vm, pos.astype(np.float32))


def ring_cameras(n_views: int, sizes, radius: float = 4.0) -> List[Camera]:
    """Views on a horizontal ring, C_k = (r sin t_k, 0, -r cos t_k), t_k = 2 pi k / V."""
    cams = []
    for k in range(n_views):
        th = 2.0 * math.pi * k / n_views
        w, h = sizes[k]
        cams.append(look_at((radius * math.sin(th), 0.0, -radius * math.cos(th)), width=w, height=h))
    return cams


def _random_quats(rng, n):
    return rng.standard_normal((n, 4)).astype(np.float32)


def _sh_coeffs(rng, n, degree, rest_std=0.05):
    k = (degree + 1) ** 2
    sh = np.zeros((n, k, 3), dtype=np.float32)
    sh[:, 0, :] = rng.uniform(-_DC_HALF_RANGE, _DC_HALF_RANGE, (n, 3))
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, rest_std, (n, k - 1, 3))
    return sh


def _sphere_points(rng, n, n_spheres, centre_range=1.0):
    centres = rng.uniform(-centre_range, centre_range, (n_spheres, 3))
    radii = rng.uniform(0.2, 1.0, n_spheres)
    which = rng.integers(0, n_spheres, n)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = centres[which] + radii[which, None] * d
    return pts, d


def _finish(name, rng, means, log_scales, quats, betas, sh, deg, cams, normals=None, loss="l1"):
    n = means.shape[0]
    logits = rng.standard_normal(n).astype(np.float32)
    log_scales = log_scales.astype(np.float32)
    return Scene(
        name=name,
        means=means.astype(np.float32),
        log_scales=log_scales,
        scales=np.exp(log_scales.astype(np.float64)).astype(np.float32),
        quats=quats.astype(np.float32),
        opacity_logits=logits,
        opacities=(1.0 / (1.0 + np.exp(-logits.astype(np.float64)))).astype(np.float32),
        betas=betas.astype(np.float32),
        sh=sh.astype(np.float32),
        sh_degree=deg,
        cameras=cams,
        normals=None if normals is None else normals.astype(np.float32),
        loss=loss,
    )


def _uniform_cube_scene(name, rng, n, cams, deg=0, log_scale=(-4.0, -2.0), beta=(1.0, 4.0)):
    means = rng.uniform(-1.0, 1.0, (n, 3))
    log_scales = rng.uniform(log_scale[0], log_scale[1], (n, 3))
    quats = _random_quats(rng, n)
    betas = rng.uniform(beta[0], beta[1], n)
    sh = _sh_coeffs(rng, n, deg)
    return _finish(name, rng, means, log_scales, quats, betas, sh, deg, cams)


DRT_FRACTIONS = (1 / 8, 1 / 4, 1 / 2, 1 / 2, 3 / 4, 3 / 4, 1.0, 1.0)


def drt_view_sizes(full=(1600, 1064), fractions=DRT_FRACTIONS):
    """Per-view (W, H) = round(full * f) for the dynamic-resolution batch."""
    return [(int(round(full[0] * f)), int(round(full[1] * f))) for f in fractions]


def _rotation_from_z_axis(rng, z_axes, tilt_std):
    """Rotation matrices whose third column is ``z_axes`` tilted by N(0, tilt_std) rad
    about a random tangent, with a uniform random twist about the tilted axis."""
    n = z_axes.shape[0]
    a = rng.standard_normal((n, 3))
    t1 = a - (a * z_axes).sum(1, keepdims=True) * z_axes
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(z_axes, t1)
    tilt = rng.normal(0.0, tilt_std, n)[:, None]
    z = np.cos(tilt) * z_axes + np.sin(tilt) * t2   # tilted about t1, so t1 stays orthogonal
    x = t1
    y = np.cross(z, x)
    twist = rng.uniform(0.0, 2.0 * math.pi, n)[:, None]
    x, y = np.cos(twist) * x + np.sin(twist) * y, -np.sin(twist) * x + np.cos(twist) * y
    return np.stack([x, y, z], axis=2)  # columns


def _quat_from_matrix(r):
    """(w, x, y, z) of rotation matrices (n, 3, 3), Shepperd's method."""
    n = r.shape[0]
    q = np.zeros((n, 4))
    tr = r[:, 0, 0] + r[:, 1, 1] + r[:, 2, 2]
    cand = np.stack([tr, r[:, 0, 0], r[:, 1, 1], r[:, 2, 2]], axis=1)
    k = np.argmax(cand, axis=1)
    for i in range(n):
        m = r[i]
        if k[i] == 0:
            s = math.sqrt(1.0 + tr[i]) * 2
            q[i] = [0.25 * s, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
        elif k[i] == 1:
            s = math.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2]) * 2
            q[i] = [(m[2, 1] - m[1, 2]) / s, 0.25 * s, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
        elif k[i] == 2:
            s = math.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2]) * 2
            q[i] = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, 0.25 * s, (m[1, 2] + m[2, 1]) / s]
        else:
            s = math.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1]) * 2
            q[i] = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, 0.25 * s]
    return q


def _quat_from_matrix_fast(r):
    """Vectorised quaternion extraction (w, x, y, z) for well-conditioned traces,
    falling back to Shepperd's branch per row where needed."""
    tr = r[:, 0, 0] + r[:, 1, 1] + r[:, 2, 2]
    good = tr > -0.5
    q = np.zeros((r.shape[0], 4))
    s = np.sqrt(1.0 + tr[good]) * 2
    rg = r[good]
    q[good] = np.stack([0.25 * s, (rg[:, 2, 1] - rg[:, 1, 2]) / s, (rg[:, 0, 2] - rg[:, 2, 0]) / s,
                        (rg[:, 1, 0] - rg[:, 0, 1]) / s], axis=1)
    if (~good).any():
        q[~good] = _quat_from_matrix(r[~good])
    return q


def make_workload(k: int, n_override: Optional[int] = None, views_override: Optional[int] = None) -> Scene:
    """Workloads 1..5 (seeded).  ``n_override``/``views_override`` shrink a workload
    for tests while keeping its distributions."""
    rng = np.random.default_rng([k, 0])
    if k == 1:
        n = n_override or 2000
        cams = [look_at((0.0, 0.0, -4.0), width=128, height=128)]
        return _uniform_cube_scene("plain-2k-1x128", rng, n, cams)
    if k == 2:
        n = n_override or 100_000
        n_s = int(round(0.9 * n))
        pts, _ = _sphere_points(rng, n_s, 20)
        noise = rng.uniform(-2.0, 2.0, (n - n_s, 3))
        means = np.concatenate([pts, noise])
        log_scales = rng.uniform(-4.0, -2.0, (n, 3))
        quats = _random_quats(rng, n)
        betas = rng.uniform(1.0, 4.0, n)
        sh = _sh_coeffs(rng, n, 3)
        cams = [look_at((0.0, 0.0, -4.0), width=1008, height=756)]
        return _finish("spheres-100k-1x1008x756", rng, means, log_scales, quats, betas, sh, 3, cams,
                       loss="l1+dssim")
    if k == 3:
        n = n_override or 500_000
        sizes = drt_view_sizes()
        v = views_override or 8
        cams = ring_cameras(8, sizes)[:v]
        return _uniform_cube_scene("drt-batch-500k-8views", rng, n, cams)
    if k == 4:
        n = n_override or 1_000_000
        n_sph = n // 2
        pts, nrm = _sphere_points(rng, n_sph, 10)
        n_pl = n - n_sph
        pn = rng.standard_normal((10, 3))
        pn /= np.linalg.norm(pn, axis=1, keepdims=True)
        off = rng.uniform(-1.0, 1.0, 10)
        which = rng.integers(0, 10, n_pl)
        # orthonormal in-plane basis per plane
        a = np.where(np.abs(pn[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
        e1 = np.cross(pn, a)
        e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
        e2 = np.cross(pn, e1)
        uv = rng.uniform(-1.0, 1.0, (n_pl, 2))
        ppts = (pn[which] * off[which, None] + e1[which] * uv[:, :1] + e2[which] * uv[:, 1:])
        means = np.concatenate([pts, ppts])
        normals = np.concatenate([nrm, pn[which]])
        rot = _rotation_from_z_axis(rng, normals, 0.1)
        quats = _quat_from_matrix_fast(rot)
        log_scales = np.empty((n, 3))
        log_scales[:, :2] = rng.uniform(-4.0, -2.0, (n, 2))
        log_scales[:, 2] = -13.0
        betas = rng.uniform(1.5, 3.0, n)
        sh = _sh_coeffs(rng, n, 3)
        v = views_override or 4
        cams = ring_cameras(4, [(1957, 1091)] * 4)[:v]
        return _finish("surfels-1m-4x1957x1091", rng, means, log_scales, quats, betas, sh, 3, cams,
                       normals=normals, loss="l1+surface")
    if k == 5:
        n = n_override or 3_000_000
        centres = rng.uniform(-1.0, 1.0, (50, 3))
        which = rng.integers(0, 50, n)
        means = centres[which] + rng.normal(0.0, 0.3, (n, 3))
        log_scales = rng.uniform(-6.0, -4.0, (n, 3))
        quats = _random_quats(rng, n)
        betas = rng.uniform(1.0, 4.0, n)
        sh = _sh_coeffs(rng, n, 3)
        v = views_override or 16
        cams = ring_cameras(16, [(1920, 1080)] * 16)[:v]
        return _finish("blobs-3m-16x1920x1080", rng, means, log_scales, quats, betas, sh, 3, cams)
    raise ValueError(f"unknown workload {k}")


def target_images(scene: Scene, k: int) -> List[np.ndarray]:
    """Seeded U(0,1) targets, one (3, H, W) float32 array per view."""
    rng = np.random.default_rng([k, 1])
    return [rng.uniform(0.0, 1.0, (3, c.height, c.width)).astype(np.float32) for c in scene.cameras]


def upstream_grads(scene: Scene, k: int) -> List[np.ndarray]:
    """Seeded N(0,1) dL/dimage, one (3, H, W) float32 array per view."""
    rng = np.random.default_rng([k, 2])
    return [rng.standard_normal((3, c.height, c.width)).astype(np.float32) for c in scene.cameras]


def sample_rng(k: int) -> np.random.Generator:
    return np.random.default_rng([k, 3])


def tiny_scene(seed: int, n: int = 12, width: int = 40, height: int = 32, deg: int = 1,
               n_views: int = 1, beta=(1.0, 4.0), log_scale=(-2.6, -1.6), spread=0.6) -> Scene:
    """Small random scene for brute force and finite-difference checks."""
    rng = np.random.default_rng([100 + seed, 0])
    means = rng.uniform(-spread, spread, (n, 3))
    log_scales = rng.uniform(log_scale[0], log_scale[1], (n, 3))
    quats = _random_quats(rng, n)
    betas = rng.uniform(beta[0], beta[1], n)
    sh = _sh_coeffs(rng, n, deg, rest_std=0.3)
    cams = ring_cameras(n_views, [(width, height)] * n_views) if n_views > 1 else \
        [look_at((0.0, 0.0, -4.0), width=width, height=height)]
    return _finish(f"tiny-{seed}", rng, means, log_scales, quats, betas, sh, deg, cams)


RAGGED_SIZES = ((1, 1), (1, 37), (23, 1), (17, 33), (129, 65))


def ragged_scene(seed: int, n: int = 200, deg: int = 2) -> Scene:
    """Views of degenerate and ragged sizes (one pixel, one row, one column,
    sizes that are not multiples of any tile) on a ring around a small scene."""
    rng = np.random.default_rng([200 + seed, 0])
    means = rng.uniform(-0.6, 0.6, (n, 3))
    log_scales = rng.uniform(-2.6, -1.6, (n, 3))
    quats = _random_quats(rng, n)
    betas = rng.uniform(1.0, 4.0, n)
    sh = _sh_coeffs(rng, n, deg, rest_std=0.3)
    cams = ring_cameras(len(RAGGED_SIZES), list(RAGGED_SIZES))
    return _finish(f"ragged-{seed}", rng, means, log_scales, quats, betas, sh, deg, cams)


def empty_scene(deg: int = 0, sizes=((1, 1), (37, 19))) -> Scene:
    """No splats at all."""
    rng = np.random.default_rng([300, 0])
    z = np.zeros((0, 3))
    return _finish("empty", rng, z, z, np.zeros((0, 4)), np.zeros(0), np.zeros((0, (deg + 1) ** 2, 3)), deg,
                   ring_cameras(len(sizes), list(sizes)))

