"""Training loop of the schedule (Sec. 3.4 and 4.2) over the library's kernels.

Each iteration renders every view at the dynamic-resolution scale of Eq. 15
(batched in one pass), takes the loss of Eq. 8 ((1 - lambda) L1 + lambda
(1 - SSIM) per view, lambda = 0.2) against the targets resized to that scale,
runs the hand-written adjoint, adds the surface regulariser's gradients while
it is active (Sec. 3.3, Eq. 9-13; neighbour lists refreshed every `knn_every`
iterations), sets the opacity-entropy weight while that phase lasts, and
takes one fused Adam step.  Shape resets and pruning happen at their
iterations.  Every numerical step is a call into libgesr; this module only
schedules the calls and resizes the targets (data preparation: area averaging
by torch).

The render-loss-adjoint part of an iteration is captured once per DRT stage
in a HIP graph (project, bin without synchronisation into a list capacity
from a sizing run with headroom, forward, loss, tile adjoint, projection
adjoint) and replayed; the optimiser step and the regulariser are launched
after it.  No iteration waits for the GPU: the list-overflow flag of each
replay is copied to pinned host memory without blocking and read one
iteration later; an overflow (lists truncated for that iteration) makes the
stage re-size and re-capture.  Pruning changes the splat count and so
re-captures every stage.

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
    lambda_dssim: float = 0.2  # lambda of Eq. 8


def scaled_camera(cam, scale: float):
    """The camera with its image (and intrinsics) scaled for a DRT stage."""
    w, h = drt_resolution(int(cam.width), int(cam.height), scale)
    sx, sy = w / float(cam.width), h / float(cam.height)
    return SimpleNamespace(width=w, height=h, fx=cam.fx * sx, fy=cam.fy * sy, cx=cam.cx * sx, cy=cam.cy * sy,
                           viewmat=cam.viewmat, campos=cam.campos)


class _StageStep:
    """One DRT stage's render, loss and adjoint over fixed buffers, captured in
    a HIP graph (or run eagerly with graph=False)."""

    def __init__(self, rast: Rasterizer, target: torch.Tensor, splats, lam: float, graph: bool):
        self.rast, self.target, self.splats, self.lam = rast, target, splats, lam
        n = splats.n
        m = rast.forward(splats, sync=True)["bins"]["M"]
        self.m_cap = int(m * 1.5) + 4096  # the footprints move while training
        self.loss_ws = rast.alloc_loss_workspace()
        self.graph = None
        if graph:
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                self._body(n)
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                self.out = self._body(n)

    def _body(self, n):
        r, sp = self.rast, self.splats
        proj = r.project(sp)
        bins = r.bin(proj, n, m_cap=self.m_cap, sync=False)
        f = r.render_fwd(proj, bins, n)
        img = f["image"][:self.target.numel()]
        dL, loss = r.loss_eq8(img, self.target, self.lam, workspace=self.loss_ws)
        ws = r.render_bwd_tiles(proj, bins, n, f["final_T"], f["n_contrib"], dL)
        grads = r.project_bwd(sp, proj, bins, ws)
        return dict(image=img, loss=loss, grads=grads, overflow=bins["counters"][1:2])

    def run(self) -> dict:
        if self.graph is None:
            return self._body(self.splats.n)
        self.graph.replay()
        return self.out


class Trainer:
    """Optimises one splat set against per-view target images."""

    def __init__(self, cameras, raw: RawParams, targets: List[torch.Tensor], settings: RasterSettings,
                 schedule: Schedule = None, adam: AdamConfig = None, seed: int = 0, graph: bool = True):
        self.cameras = list(cameras)
        self.targets = [t.contiguous() for t in targets]  # [3, H, W] per view, full resolution
        self.settings = settings
        self.schedule = schedule or Schedule()
        self.opt = SplatAdam(raw, adam or AdamConfig())
        self.gen = torch.Generator(device=raw.mean.device).manual_seed(seed)
        self.use_graph = graph
        self._rasts = {}
        self._targets = {}
        self._steps = {}
        self._nbrs = None
        self._nbrs_it = -1
        self._flag = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        self._flag_event = torch.cuda.Event()
        self._flag_key = None
        self.recaptures = 0
        self.it = 0

    # ------------------------------------------------------------- helpers
    def _stage_key(self, scale: float):
        cams = [scaled_camera(c, scale) for c in self.cameras]
        return tuple((c.width, c.height) for c in cams), cams

    def _stage(self, scale: float):
        key, cams = self._stage_key(scale)
        if key not in self._rasts:
            self._rasts[key] = Rasterizer(cams, self.settings, store_tile_ids=False)
            resized = [torch.nn.functional.interpolate(t[None], size=(c.height, c.width), mode="area")[0]
                       for t, c in zip(self.targets, cams)]
            self._targets[key] = torch.cat([r.reshape(-1) for r in resized]).contiguous()
        return self._rasts[key], self._targets[key]

    def _stage_step(self, scale: float):
        rast, target = self._stage(scale)
        key, _ = self._stage_key(scale)
        st = self._steps.get(key)
        if st is None:
            st = _StageStep(rast, target, self.opt.splats, self.schedule.lambda_dssim, self.use_graph)
            self._steps[key] = st
        return key, st

    def _active(self, start: int, length: int) -> bool:
        return start <= self.it < start + length

    # ---------------------------------------------------------------- step
    def step(self) -> dict:
        """One iteration; returns the iteration's scale, the loss of Eq. 8 summed
        over the views and the L1 term (device scalars: reading them waits for
        the GPU), and the regulariser's losses (None when inactive)."""
        sch = self.schedule
        # the previous replay's overflow flag, once its copy has landed (no wait)
        if self._flag_key is not None and self._flag_event.query():
            if int(self._flag[0]) != 0:
                self._steps.pop(self._flag_key, None)
                self.recaptures += 1
            self._flag_key = None
        scale = drt_scale(self.it, sch.iterations, sch.drt_start, sch.drt_end, sch.drt_fraction)
        key, stage = self._stage_step(scale)
        out = stage.run()
        if self._flag_key is None:
            self._flag.copy_(out["overflow"], non_blocking=True)
            self._flag_event.record()
            self._flag_key = key
        sp = self.opt.splats
        grads = out["grads"]
        reg = None
        if self._active(sch.gsr_start, sch.gsr_iters) and sp.n > 0:
            if self._nbrs is None or self.it - self._nbrs_it >= sch.knn_every:
                self._nbrs = knn(sp, 16)
                self._nbrs_it = self.it
            xi = torch.randn((3, sp.n), generator=self.gen, device=sp.mean.device, dtype=torch.float32)
            res = gsr(sp, self.settings, self._nbrs, xi, w_sdf=sch.w_sdf / sp.n, w_nor=sch.w_nor / sp.n,
                      grads=grads)
            reg = res["losses"]
        self.opt.config.entropy_weight = (sch.entropy_weight if self._active(sch.entropy_start, sch.entropy_iters)
                                          else 0.0)
        self.opt.step(grads)
        self.it += 1
        if sch.shape_reset_every > 0 and self.it % sch.shape_reset_every == 0:
            self.opt.shape_reset(sch.shape_reset_value)
        if self.it in tuple(sch.prune_at):
            self.opt.prune(sch.min_opacity, sch.min_beta)
            self._nbrs = None  # indices changed
            self._steps.clear()  # splat buffers changed: re-capture
            self._flag_key = None
        loss = out["loss"].sum()
        l1 = (out["image"] - stage.target).abs().mean()
        return dict(iteration=self.it - 1, scale=scale, loss=loss, l1=l1, gsr=reg, n=self.opt.raw.n)

    def run(self, iterations: Optional[int] = None, log_every: int = 0, log=print) -> List[dict]:
        n = self.schedule.iterations if iterations is None else iterations
        hist = []
        for _ in range(n):
            r = self.step()
            hist.append(r)
            if log_every and r["iteration"] % log_every == 0:
                log(f"it {r['iteration']}: scale {r['scale']:.3f} loss {float(r['loss']):.5f} "
                    f"L1 {float(r['l1']):.5f} splats {r['n']}")
        return hist


def raw_from_activated(means, scales, quats, opacities, betas, sh, device="cuda") -> RawParams:
    """Raw parameters (log scale, opacity logit) of activated row-per-splat arrays."""
    import numpy as np
    op = np.clip(np.asarray(opacities, np.float64), 1e-6, 1 - 1e-6)
    return RawParams.from_aos(means, np.log(np.asarray(scales, np.float64)), quats, np.log(op / (1 - op)), betas, sh,
                              device=device)


__all__ = ["Schedule", "Trainer", "scaled_camera", "raw_from_activated"]
