"""Training loop of the schedule (Sec. 3.4 and 4.2) over the library's kernels.

Each iteration renders every view at the dynamic-resolution scale of Eq. 15
(batched in one pass), takes the L1 term of Eq. 8 against the targets
resized to that scale, runs the hand-written adjoint, adds the surface
regulariser's gradients while it is active (Sec. 3.3, Eq. 9-13; neighbour
lists refreshed every `knn_every` iterations), sets the opacity-entropy
weight while that phase lasts, and takes one fused Adam step.  Shape resets
and pruning happen at their iterations.  Every numerical step is a call into
libgesr; this module only schedules the calls and resizes the targets (data
preparation: area averaging by torch).

Schedule defaults follow Sec. 4.2 where it gives numbers: resolution 0.26 -> 1
over 75% of the iterations, shape reset every 1000, entropy regularisation for
1800 iterations after 7000, then the regulariser for 6200 iterations with
16-neighbour lists refreshed every 500, splats with opacity below 0.5 (and,
read as the shape pruning threshold, beta below 0.5) removed when the entropy
phase ends.  The regulariser weights and the entropy weight are not given.
"""
from __future__ import annotations

import dataclasses
from types import SimpleNamespace
from typing import List, Optional, Sequence

import torch

from .drt import drt_resolution, drt_scale
from .gsr import gsr, knn
from .optim import AdamConfig, RawParams, SplatAdam
from .rasterizer import Rasterizer, RasterSettings


@dataclasses.dataclass
class Schedule:
    iterations: int = 15000
    drt_start: float = 0.26
    drt_end: float = 1.0
    drt_fraction: float = 0.75
    entropy_start: int = 7000
    entropy_iters: int = 1800
    entropy_weight: float = 0.1
    gsr_start: int = 8800
    gsr_iters: int = 6200
    w_sdf: float = 0.2  # lambda_1 of Eq. 14 (not given)
    w_nor: float = 0.2  # lambda_2 of Eq. 14 (not given)
    knn_every: int = 500
    shape_reset_every: int = 1000
    shape_reset_value: float = 2.0
    prune_at: Sequence[int] = (8800,)
    min_opacity: float = 0.5
    min_beta: float = 0.5


def scaled_camera(cam, scale: float):
    """The camera with its image (and intrinsics) scaled for a DRT stage."""
    w, h = drt_resolution(int(cam.width), int(cam.height), scale)
    sx, sy = w / float(cam.width), h / float(cam.height)
    return SimpleNamespace(width=w, height=h, fx=cam.fx * sx, fy=cam.fy * sy, cx=cam.cx * sx, cy=cam.cy * sy,
                           viewmat=cam.viewmat, campos=cam.campos)


class Trainer:
    """Optimises one splat set against per-view target images."""

    def __init__(self, cameras, raw: RawParams, targets: List[torch.Tensor], settings: RasterSettings,
                 schedule: Schedule = None, adam: AdamConfig = None, seed: int = 0):
        self.cameras = list(cameras)
        self.targets = [t.contiguous() for t in targets]  # [3, H, W] per view, full resolution
        self.settings = settings
        self.schedule = schedule or Schedule()
        self.opt = SplatAdam(raw, adam or AdamConfig())
        self.gen = torch.Generator(device=raw.mean.device).manual_seed(seed)
        self._rasts = {}
        self._targets = {}
        self._nbrs = None
        self._nbrs_it = -1
        self.it = 0

    # ------------------------------------------------------------- helpers
    def _stage(self, scale: float):
        cams = [scaled_camera(c, scale) for c in self.cameras]
        key = tuple((c.width, c.height) for c in cams)
        if key not in self._rasts:
            self._rasts[key] = Rasterizer(cams, self.settings, store_tile_ids=False)
            resized = [torch.nn.functional.interpolate(t[None], size=(c.height, c.width), mode="area")[0]
                       for t, c in zip(self.targets, cams)]
            self._targets[key] = torch.cat([r.reshape(-1) for r in resized]).contiguous()
        return self._rasts[key], self._targets[key]

    def _active(self, start: int, length: int) -> bool:
        return start <= self.it < start + length

    # ---------------------------------------------------------------- step
    def step(self) -> dict:
        """One iteration; returns the iteration's scale, L1 value and the
        regulariser's losses (None when inactive)."""
        sch = self.schedule
        scale = drt_scale(self.it, sch.iterations, sch.drt_start, sch.drt_end, sch.drt_fraction)
        rast, target = self._stage(scale)
        sp = self.opt.splats
        fwd = rast.forward(sp, sync=True)
        img = fwd["image"][:target.numel()]
        dL = rast.l1_grad(img, target, 1.0 / float(target.numel()))
        grads = rast.render_bwd(sp, fwd["proj"], fwd["bins"], fwd["final_T"], fwd["n_contrib"], dL)
        reg = None
        if self._active(sch.gsr_start, sch.gsr_iters) and sp.n > 0:
            if self._nbrs is None or self.it - self._nbrs_it >= sch.knn_every:
                self._nbrs = knn(sp, 16)
                self._nbrs_it = self.it
            xi = torch.randn((3, sp.n), generator=self.gen, device=sp.mean.device, dtype=torch.float32)
            out = gsr(sp, self.settings, self._nbrs, xi, w_sdf=sch.w_sdf / sp.n, w_nor=sch.w_nor / sp.n,
                      grads=grads)
            reg = out["losses"]
        self.opt.config.entropy_weight = (sch.entropy_weight if self._active(sch.entropy_start, sch.entropy_iters)
                                          else 0.0)
        self.opt.step(grads)
        self.it += 1
        if sch.shape_reset_every > 0 and self.it % sch.shape_reset_every == 0:
            self.opt.shape_reset(sch.shape_reset_value)
        if self.it in tuple(sch.prune_at):
            self.opt.prune(sch.min_opacity, sch.min_beta)
            self._nbrs = None  # indices changed
        l1 = (img - target).abs().mean()  # reporting only
        return dict(iteration=self.it - 1, scale=scale, l1=l1, gsr=reg, n=self.opt.raw.n)

    def run(self, iterations: Optional[int] = None, log_every: int = 0, log=print) -> List[dict]:
        n = self.schedule.iterations if iterations is None else iterations
        hist = []
        for _ in range(n):
            r = self.step()
            hist.append(r)
            if log_every and r["iteration"] % log_every == 0:
                log(f"it {r['iteration']}: scale {r['scale']:.3f} L1 {float(r['l1']):.5f} splats {r['n']}")
        return hist


def raw_from_activated(means, scales, quats, opacities, betas, sh, device="cuda") -> RawParams:
    """Raw parameters (log scale, opacity logit) of activated row-per-splat arrays."""
    import numpy as np
    op = np.clip(np.asarray(opacities, np.float64), 1e-6, 1 - 1e-6)
    return RawParams.from_aos(means, np.log(np.asarray(scales, np.float64)), quats, np.log(op / (1 - op)), betas, sh,
                              device=device)


__all__ = ["Schedule", "Trainer", "scaled_camera", "raw_from_activated"]
