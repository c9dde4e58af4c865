"""Helpers shared by the oracle tests (scene construction only; no method arithmetic)."""
from __future__ import annotations

import copy

import numpy as np

import gesr_inputs as gi


def single_splat_scene(mean=(0.0, 0.0, 0.0), scale=(0.1, 0.1, 0.1), quat=(1.0, 0.0, 0.0, 0.0), opacity=0.8,
                       beta=2.0, rgb=(0.9, 0.4, 0.2), width=64, height=48, cam_pos=(0.0, 0.0, -4.0)):
    """One splat with degree-0 SH chosen so that its colour is `rgb`."""
    return stacked_scene([mean], [scale], [quat], [opacity], [beta], [rgb], width, height, cam_pos)


def stacked_scene(means, scales, quats, opacities, betas, rgbs, width=64, height=48, cam_pos=(0.0, 0.0, -4.0),
                  sh_dtype=np.float32):
    """Splats with degree-0 SH coefficients (rgb - 1/2) / Y00; sh_dtype float64
    keeps them unrounded."""
    n = len(means)
    c0 = 0.5 / np.sqrt(np.pi)  # the constant degree-0 harmonic 1/(2 sqrt(pi))
    sh = np.zeros((n, 1, 3), sh_dtype)
    sh[:, 0, :] = (np.asarray(rgbs, np.float64) - 0.5) / c0
    scales = np.asarray(scales, np.float32)
    op = np.asarray(opacities, np.float32)
    return gi.Scene(name="synthetic", means=np.asarray(means, np.float32), log_scales=np.log(scales),
                    scales=scales, quats=np.asarray(quats, np.float32),
                    opacity_logits=np.log(op / (1 - op)).astype(np.float32), opacities=op,
                    betas=np.asarray(betas, np.float32), sh=sh, sh_degree=0,
                    cameras=[gi.look_at(cam_pos, width=width, height=height)])


def with_params(scene, **kw):
    s = copy.copy(scene)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def subset_views(scene, idx):
    s = copy.copy(scene)
    s.cameras = [scene.cameras[i] for i in idx]
    return s
