"""Pins of the oracle's surface-alignment regulariser (the flattened-splat
workload's loss): closed forms with scipy rotations and central differences."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle


def _quat_wxyz(rot):
    x, y, z, w = rot.as_quat().T
    return np.stack([w, x, y, z], 1)


def test_aligned_normals_give_zero_and_tilts_give_sin_squared():
    rng = np.random.default_rng(0)
    N = 200
    rots = Rotation.random(N, random_state=1)
    scales = rng.uniform(0.01, 0.2, (N, 3))
    k = rng.integers(0, 3, N)
    scales[np.arange(N), k] = 1e-4  # the flattened axis
    normals = rots.as_matrix()[np.arange(N), :, k]
    Ls, Ln, _ = oracle.surface_alignment(scales, _quat_wxyz(rots), normals, 0.1, 0.1)
    assert Ln == pytest.approx(0.0, abs=1e-15)
    assert Ls == pytest.approx(0.1 * 1e-4, rel=1e-12)
    # tilt each normal by theta about an axis perpendicular to it: 1 - cos^2 = sin^2
    theta = rng.uniform(-1.2, 1.2, N)
    perp = np.cross(normals, rng.standard_normal((N, 3)))
    perp /= np.linalg.norm(perp, axis=1, keepdims=True)
    tilted = (Rotation.from_rotvec(perp * theta[:, None]) * rots)
    _, Ln2, _ = oracle.surface_alignment(scales, _quat_wxyz(tilted), normals, 0.1, 0.1)
    assert Ln2 == pytest.approx(0.1 * np.mean(np.sin(theta) ** 2), rel=1e-12)
    # the normal's sign does not matter
    _, Ln3, _ = oracle.surface_alignment(scales, _quat_wxyz(tilted), -normals, 0.1, 0.1)
    assert Ln3 == pytest.approx(Ln2, rel=1e-14)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(2)
    N = 30
    scales = rng.uniform(0.01, 0.2, (N, 3))
    quats = rng.standard_normal((N, 4)) * rng.uniform(0.5, 2.0, (N, 1))  # unnormalised
    normals = rng.standard_normal((N, 3))
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    _, _, g = oracle.surface_alignment(scales, quats, normals, 0.3, 0.7)

    def loss(s, q):
        a, b, _ = oracle.surface_alignment(s, q, normals, 0.3, 0.7)
        return a + b
    for name, arr in (("scales", scales), ("quats", quats)):
        for i in range(arr.size):
            h = 1e-7
            p, m = arr.copy().reshape(-1), arr.copy().reshape(-1)
            p[i] += h
            m[i] -= h
            args_p = (p.reshape(arr.shape), quats) if name == "scales" else (scales, p.reshape(arr.shape))
            args_m = (m.reshape(arr.shape), quats) if name == "scales" else (scales, m.reshape(arr.shape))
            fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
            assert g[name].reshape(-1)[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), (name, i)
