"""Python binding of libgesr: buffer allocation (torch) and argument marshalling.

Every step of the rasterizer runs in the HIP library; this module only
allocates device tensors with torch's caching allocator, fills the C structs
of include/gesr.h with their addresses and passes torch's current stream.

Layouts (device, float32 unless noted):
  splats  mean [3, N], scale [3, N], quat [4, N] (w, x, y, z), opacity [N],
          beta [N], sh [K * 3, N] (coefficient k of channel c at row 3k + c)
  image   concatenation over views of [3, H, W] (CHW), flat [3 * P]
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence

import torch

from . import _lib


@dataclasses.dataclass
class RasterSettings:
    """Mirror of gesr_settings (see include/gesr.h for the meaning of each field)."""
    sh_degree: int = 0
    kappa: float = 0.5
    rho: float = 0.1
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    blur: float = 0.3
    znear: float = 0.2
    clip_fac: float = 1.3
    bg: Sequence[float] = (0.0, 0.0, 0.0)
    tile_w: int = 16
    tile_h: int = 16
    batch: int = 0
    radix_bits: int = 8
    variant: int = 0

    def to_c(self) -> _lib.Settings:
        s = _lib.Settings()
        s.sh_degree = self.sh_degree
        s.kappa, s.rho = self.kappa, self.rho
        s.alpha_min, s.alpha_max, s.t_min = self.alpha_min, self.alpha_max, self.t_min
        s.blur, s.znear, s.clip_fac = self.blur, self.znear, self.clip_fac
        for c in range(3):
            s.bg[c] = float(self.bg[c])
        s.tile_w, s.tile_h, s.batch, s.radix_bits = self.tile_w, self.tile_h, self.batch, self.radix_bits
        s.variant = self.variant
        return s


def cameras_to_c(cameras) -> ctypes.Array:
    """Any objects with width, height, fx, fy, cx, cy, viewmat (3x4), campos (3)."""
    arr = (_lib.Camera * len(cameras))()
    for k, c in enumerate(cameras):
        arr[k].width, arr[k].height = int(c.width), int(c.height)
        arr[k].fx, arr[k].fy, arr[k].cx, arr[k].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        vm = [float(x) for row in c.viewmat for x in row]
        for j in range(12):
            arr[k].viewmat[j] = vm[j]
        for j in range(3):
            arr[k].campos[j] = float(c.campos[j])
    return arr


@dataclasses.dataclass
class Splats:
    """SoA device tensors of the rasterizer inputs."""
    mean: torch.Tensor
    scale: torch.Tensor
    quat: torch.Tensor
    opacity: torch.Tensor
    beta: torch.Tensor
    sh: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    def tensors(self):
        return (self.mean, self.scale, self.quat, self.opacity, self.beta, self.sh)

    @staticmethod
    def from_aos(means, scales, quats, opacities, betas, sh, device="cuda") -> "Splats":
        """From row-per-splat arrays ([N,3], [N,3], [N,4], [N], [N], [N,K,3])."""
        def t(x):
            return torch.as_tensor(x, dtype=torch.float32).to(device)
        n = t(opacities).shape[0]
        shc = t(sh)
        width = 1
        for d in shc.shape[1:]:
            width *= int(d)
        return Splats(t(means).reshape(n, 3).t().contiguous(), t(scales).reshape(n, 3).t().contiguous(),
                      t(quats).reshape(n, 4).t().contiguous(), t(opacities).contiguous(), t(betas).contiguous(),
                      shc.reshape(n, width).t().contiguous())

    def to_c(self) -> _lib.Splats:
        s = _lib.Splats()
        s.n = self.n
        s.mean, s.scale, s.quat = self.mean.data_ptr(), self.scale.data_ptr(), self.quat.data_ptr()
        s.opacity, s.beta, s.sh = self.opacity.data_ptr(), self.beta.data_ptr(), self.sh.data_ptr()
        return s


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Rasterizer:
    """One rasterizer per (camera set, settings).  Calls enqueue on torch's
    current stream; outputs are freshly allocated device tensors."""

    def __init__(self, cameras, settings: RasterSettings, device: int = 0, store_tile_ids: bool = True,
                 work_order: bool = True):
        """store_tile_ids=False leaves bins["tile_sorted"] out (the renderers
        read only the ranges and the sorted pair ids).  work_order: the
        rasterizer keeps a per-tile work buffer that every forward fills (the
        list positions each tile evaluated) and, once filled, bins with
        GESR_BIN_WORK_ORDER so the next call starts the longest-running tiles
        first; results are the same either way."""
        self.lib = _lib.load()
        self.store_tile_ids = store_tile_ids
        self.cameras = list(cameras)
        self.V = len(self.cameras)
        self.settings = settings
        self.st_c = settings.to_c()
        self.cams_c = cameras_to_c(self.cameras)
        self.device = torch.device("cuda", device)
        ctx = ctypes.c_void_p()
        self._check(self.lib.gesr_ctx_create(device, ctypes.byref(ctx)), None)
        self.ctx = ctx
        self.m_cap_hint = 0
        self.views = [(int(c.width), int(c.height)) for c in self.cameras]
        self.n_pixels = sum(w * h for w, h in self.views)
        self.work_order = work_order
        self._tile_work = None  # (tile shape, [T] int32 tensor, filled by a forward)
        self._work_filled = False

    def __del__(self):
        lib = getattr(self, "lib", None)
        if lib is not None and getattr(self, "ctx", None):
            lib.gesr_ctx_destroy(self.ctx)
            self.ctx = None

    # ------------------------------------------------------------ helpers
    def _check(self, status: int, ctx) -> None:
        if status != _lib.GESR_OK:
            msg = self.lib.gesr_last_error(ctx).decode() if ctx else self.lib.gesr_status_string(status).decode()
            raise _lib.GesrError(status, msg)

    def sizes(self, n: int, m_cap: int) -> _lib.Sizes:
        out = _lib.Sizes()
        self._check(self.lib.gesr_query_sizes(self.ctx, self.cams_c, self.V, n, ctypes.byref(self.st_c),
                                              max(int(m_cap), 1), ctypes.byref(out)), self.ctx)
        return out

    def _empty(self, n, dtype=torch.float32):
        return torch.empty(max(int(n), 1), dtype=dtype, device=self.device)

    # ---------------------------------------------------------- pipeline
    def project(self, sp: Splats) -> dict:
        vn = self.V * sp.n
        p = dict(rec=self._empty(vn * _lib.REC_FLOATS), tiles_touched=self._empty(vn, torch.int32),
                 rect=self._empty(2 * vn, torch.int32), depth_key=self._empty(vn, torch.int32))
        self._check(self.lib.gesr_project(self.ctx, ctypes.byref(sp.to_c()), self.cams_c, self.V,
                                          ctypes.byref(self.st_c), ctypes.byref(self._proj_c(p)), _stream()),
                    self.ctx)
        return p

    @staticmethod
    def _proj_c(p) -> _lib.Proj:
        c = _lib.Proj()
        c.rec, c.tiles_touched = p["rec"].data_ptr(), p["tiles_touched"].data_ptr()
        c.rect, c.depth_key = p["rect"].data_ptr(), p["depth_key"].data_ptr()
        return c

    def _work_buffer(self, T: int):
        """The per-tile work buffer for the current tile shape (a new shape
        starts an unfilled, zeroed buffer)."""
        shape = (self.settings.tile_w, self.settings.tile_h, T)
        if self._tile_work is None or self._tile_work[0] != shape:
            self._tile_work = (shape, torch.zeros(max(T, 1), dtype=torch.int32, device=self.device))
            self._work_filled = False
        return self._tile_work[1]

    def alloc_bins(self, n: int, m_cap: int, scratch: bool = True) -> dict:
        sz = self.sizes(n, m_cap)
        T = int(sz.total_tiles)
        return dict(m_cap=int(m_cap), tile_sorted=self._empty(m_cap, torch.int32) if self.store_tile_ids else None,
                    val_sorted=self._empty(m_cap, torch.int32), ranges=self._empty(2 * T, torch.int32),
                    worklist=self._empty(T, torch.int32), inst_base=self._empty(self.V * n, torch.int32),
                    counters=self._empty(4, torch.int32),
                    scratch=torch.empty(int(sz.bin_scratch_bytes), dtype=torch.uint8, device=self.device)
                    if scratch else None, scratch_bytes=int(sz.bin_scratch_bytes), total_tiles=T,
                    tile_work=self._work_buffer(T) if self.work_order else None)

    @staticmethod
    def _bins_c(b) -> _lib.Bins:
        c = _lib.Bins()
        c.m_cap = b["m_cap"]
        for k in ("tile_sorted", "val_sorted", "ranges", "worklist", "inst_base", "counters", "scratch"):
            setattr(c, k, b[k].data_ptr() if b[k] is not None else 0)
        c.scratch_bytes = b["scratch"].numel() if b["scratch"] is not None else 0
        tw = b.get("tile_work")
        c.tile_work = tw.data_ptr() if tw is not None else 0
        return c

    def bin(self, proj: dict, n: int, m_cap: Optional[int] = None, sync: bool = True,
            static_scratch: bool = False) -> dict:
        """Bins the projected splats.  With sync (eager) the instance count is read
        back and the buffers regrown if needed; without it the call never
        synchronises and lists beyond m_cap are truncated (counters[1] set).
        static_scratch calls gesr_bin_static (the library's per-GPU static
        scratch instead of a scratch buffer; no scratch is allocated)."""
        if m_cap is None:
            m_cap = self.m_cap_hint or max(4 * self.V * n, 1024)
        fn = self.lib.gesr_bin_static if static_scratch else self.lib.gesr_bin
        while True:
            b = self.alloc_bins(n, m_cap, scratch=not static_scratch)
            flags = _lib.GESR_BIN_SYNC if sync else 0
            if b["tile_work"] is not None and self._work_filled:
                flags |= _lib.GESR_BIN_WORK_ORDER
            m = ctypes.c_uint64(0)
            st = fn(self.ctx, ctypes.byref(self._proj_c(proj)), self.cams_c, self.V, n, ctypes.byref(self.st_c),
                    ctypes.byref(self._bins_c(b)), flags, ctypes.byref(m), _stream())
            if st == _lib.GESR_ERR_CAPACITY and sync and m.value > m_cap:
                m_cap = int(m.value * 1.05) + 1024
                continue
            self._check(st, self.ctx)
            if sync:
                b["M"] = int(m.value)
                self.m_cap_hint = max(self.m_cap_hint, int(m.value * 1.05) + 1024)
            return b

    def render_fwd(self, proj: dict, bins: dict, n: int, counts: bool = False, channels: bool = False) -> dict:
        """Forward compositing; `channels` adds the extended depth (sum alpha T z)
        and alpha (1 - final_T) maps, [P] each."""
        P = self.n_pixels
        out = dict(image=self._empty(3 * P), final_T=self._empty(P), n_contrib=self._empty(P, torch.int32))
        cnt = None
        if counts:
            out["n_listed"] = self._empty(P, torch.int32)
            out["n_hit"] = self._empty(P, torch.int32)
            cnt = _lib.FwdCounts(out["n_listed"].data_ptr(), out["n_hit"].data_ptr())
        chn = None
        if channels:
            out["depth"] = self._empty(P)
            out["alpha"] = self._empty(P)
            chn = _lib.FwdChannels(out["depth"].data_ptr(), out["alpha"].data_ptr())
        self._check(self.lib.gesr_render_fwd_ext(self.ctx, ctypes.byref(self._proj_c(proj)),
                                                 ctypes.byref(self._bins_c(bins)), self.cams_c, self.V, n,
                                                 ctypes.byref(self.st_c), out["image"].data_ptr(),
                                                 out["final_T"].data_ptr(), out["n_contrib"].data_ptr(),
                                                 ctypes.byref(cnt) if cnt is not None else None,
                                                 ctypes.byref(chn) if chn is not None else None, _stream()), self.ctx)
        if bins.get("tile_work") is not None and self._tile_work is not None and bins["tile_work"] is self._tile_work[1]:
            self._work_filled = True  # later binnings on this stream see the figures
        return out

    def alloc_workspace(self, n: int, m_cap: int) -> torch.Tensor:
        """Backward workspace (visited bits, screen-space gradients, partials)."""
        return torch.empty(int(self.sizes(n, m_cap).bwd_workspace_bytes), dtype=torch.uint8, device=self.device)

    def render_bwd(self, sp: Splats, proj: dict, bins: dict, final_T, n_contrib, dL_dimage,
                   want_grad2d: bool = False, dL_ddepth=None, dL_dalpha=None) -> dict:
        ws = self.render_bwd_tiles(proj, bins, sp.n, final_T, n_contrib, dL_dimage, dL_ddepth=dL_ddepth,
                                   dL_dalpha=dL_dalpha)
        return self.project_bwd(sp, proj, bins, ws, want_grad2d=want_grad2d)

    def render_bwd_tiles(self, proj: dict, bins: dict, n: int, final_T, n_contrib, dL_dimage, workspace=None,
                         dL_ddepth=None, dL_dalpha=None):
        """Per-tile render adjoint only (with the extended channels' upstream
        gradients when given): returns the backward workspace."""
        if workspace is None:
            workspace = self.alloc_workspace(n, bins["m_cap"])
        dL = dL_dimage.contiguous()
        gd = dL_ddepth.contiguous() if dL_ddepth is not None else None
        ga = dL_dalpha.contiguous() if dL_dalpha is not None else None
        chn = None
        if gd is not None or ga is not None:
            chn = _lib.BwdChannels(gd.data_ptr() if gd is not None else None,
                                   ga.data_ptr() if ga is not None else None)
        self._check(self.lib.gesr_render_bwd_tiles_ext(self.ctx, ctypes.byref(self._proj_c(proj)),
                                                       ctypes.byref(self._bins_c(bins)), self.cams_c, self.V, n,
                                                       ctypes.byref(self.st_c), final_T.data_ptr(),
                                                       n_contrib.data_ptr(), dL.data_ptr(),
                                                       ctypes.byref(chn) if chn is not None else None,
                                                       workspace.data_ptr(), _stream()), self.ctx)
        return workspace

    def project_bwd(self, sp: Splats, proj: dict, bins: dict, workspace, want_grad2d: bool = False) -> dict:
        """Segmented sum of the visited partials and the projection adjoint."""
        g = dict(mean=torch.empty_like(sp.mean), scale=torch.empty_like(sp.scale), quat=torch.empty_like(sp.quat),
                 opacity=torch.empty_like(sp.opacity), beta=torch.empty_like(sp.beta), sh=torch.empty_like(sp.sh))
        gc = _lib.Grads(*(g[k].data_ptr() for k in ("mean", "scale", "quat", "opacity", "beta", "sh")))
        grad2d = self._empty(self.V * sp.n * _lib.GRAD2D_FLOATS) if want_grad2d else None
        self._check(self.lib.gesr_project_bwd(self.ctx, ctypes.byref(sp.to_c()), ctypes.byref(self._proj_c(proj)),
                                              ctypes.byref(self._bins_c(bins)), self.cams_c, self.V,
                                              ctypes.byref(self.st_c), workspace.data_ptr(),
                                              grad2d.data_ptr() if grad2d is not None else None, ctypes.byref(gc),
                                              _stream()), self.ctx)
        if grad2d is not None:
            g["grad2d"] = grad2d
        return g

    def surface_align(self, sp: Splats, normals, grads: dict, w_scale: float = 0.1, w_normal: float = 0.1,
                      want_losses: bool = True, workspace=None):
        """Surface-alignment regulariser (min-scale + normal terms): its gradient
        is ADDED to grads["scale"] and grads["quat"]; returns the two loss terms
        [2] (or None).  normals: [3][n] float32 device tensor (SoA)."""
        nrm = normals.contiguous()
        gc = _lib.Grads(*(grads[k].data_ptr() if k in grads else None
                          for k in ("mean", "scale", "quat", "opacity", "beta", "sh")))
        losses = torch.empty(2, dtype=torch.float32, device=self.device) if want_losses else None
        if want_losses and workspace is None:
            workspace = torch.empty(int(self.lib.gesr_align_workspace_size(sp.n)), dtype=torch.uint8,
                                    device=self.device)
        self._check(self.lib.gesr_surface_align(self.ctx, ctypes.byref(sp.to_c()), nrm.data_ptr(), float(w_scale),
                                                float(w_normal), ctypes.byref(gc),
                                                losses.data_ptr() if losses is not None else None,
                                                workspace.data_ptr() if workspace is not None else None,
                                                workspace.numel() if workspace is not None else 0, _stream()),
                    self.ctx)
        return losses

    def surface_points(self, sp: Splats, proj: dict, bins: dict, depth, alpha, pixels, n_samples: int = 32,
                       level: float = 0.3, span: float = 3.0, min_alpha: float = 0.5) -> dict:
        """Level-set surface points along the rays of `pixels` (int tensor of
        global pixel ids) from the extended depth and alpha maps: points [R, 4]
        (x, y, z, valid), normals [R, 4] (nx, ny, nz, t*), dominant [R],
        n_candidates [R]."""
        pix = pixels.to(device=self.device, dtype=torch.int32).contiguous()
        R = pix.numel()
        out = dict(points=torch.zeros(max(R, 1), 4, dtype=torch.float32, device=self.device),
                   normals=torch.zeros(max(R, 1), 4, dtype=torch.float32, device=self.device),
                   dominant=torch.zeros(max(R, 1), dtype=torch.int32, device=self.device),
                   n_candidates=torch.zeros(max(R, 1), dtype=torch.int32, device=self.device))
        ss = _lib.SurfaceSettings(int(n_samples), float(level), float(span), float(min_alpha))
        ws = torch.empty(max(sp.n, 1) * _lib.SURFACE_BYTES_PER_SPLAT // 4, dtype=torch.float32, device=self.device)
        self._check(self.lib.gesr_surface_points(self.ctx, ctypes.byref(sp.to_c()), ctypes.byref(self._proj_c(proj)),
                                                 ctypes.byref(self._bins_c(bins)), self.cams_c, self.V,
                                                 ctypes.byref(self.st_c), ctypes.byref(ss), depth.data_ptr(),
                                                 alpha.data_ptr(), pix.data_ptr(), R, out["points"].data_ptr(),
                                                 out["normals"].data_ptr(), out["dominant"].data_ptr(),
                                                 out["n_candidates"].data_ptr(), ws.data_ptr(), _stream()),
                    self.ctx)
        return {k: v[:R] for k, v in out.items()}

    def l1_grad(self, image, target, scale: float):
        grad = torch.empty_like(image)
        self._check(self.lib.gesr_l1_grad(self.ctx, image.data_ptr(), target.data_ptr(), image.numel(),
                                          float(scale), grad.data_ptr(), _stream()), self.ctx)
        return grad

    def loss_eq8(self, image, target, lambda_dssim: float = 0.2, want_loss: bool = True, workspace=None):
        """Eq. 8 per view, (1 - lambda) mean|X - Y| + lambda (1 - mean SSIM):
        returns (dL/dimage for the sum over views, per-view losses [V] or None).
        `workspace` (uint8 tensor of gesr_loss_workspace_size bytes) may be
        passed to keep the call allocation-free (e.g. under graph capture)."""
        ls = _lib.LossSettings()
        self.lib.gesr_default_loss_settings(ctypes.byref(ls))
        ls.lambda_dssim = float(lambda_dssim)
        if workspace is None:
            workspace = self.alloc_loss_workspace()
        grad = torch.empty_like(image)
        loss = torch.empty(self.V, dtype=torch.float32, device=self.device) if want_loss else None
        self._check(self.lib.gesr_loss_eq8(self.ctx, self.cams_c, self.V, ctypes.byref(ls), image.data_ptr(),
                                           target.data_ptr(), grad.data_ptr(),
                                           loss.data_ptr() if loss is not None else None, workspace.data_ptr(),
                                           workspace.numel(), _stream()), self.ctx)
        return grad, loss

    def alloc_loss_workspace(self):
        return torch.empty(int(self.lib.gesr_loss_workspace_size(self.cams_c, self.V)), dtype=torch.uint8,
                           device=self.device)

    def forward(self, sp: Splats, sync: bool = True, m_cap: Optional[int] = None, counts: bool = False,
                channels: bool = False):
        proj = self.project(sp)
        bins = self.bin(proj, sp.n, m_cap=m_cap, sync=sync)
        out = self.render_fwd(proj, bins, sp.n, counts=counts, channels=channels)
        out.update(proj=proj, bins=bins)
        return out

    def autotune(self, sp: Splats, reps: int = 3) -> dict:
        """Times the fwd+bwd pipeline for the library's candidate (tile shape,
        renderer variant, LDS batch) list and then depth-sort digit widths, on
        these splats and cameras, and adopts the fastest.  Returns the chosen
        settings and every trial's milliseconds (-1: could not run)."""
        st = _lib.Settings()
        ctypes.memmove(ctypes.byref(st), ctypes.byref(self.st_c), ctypes.sizeof(st))
        ncand = self.lib.gesr_autotune_candidate(-1, None)
        times = (ctypes.c_float * ncand)()
        ntr = ctypes.c_int(0)
        self._check(self.lib.gesr_autotune(self.ctx, ctypes.byref(sp.to_c()), self.cams_c, self.V, ctypes.byref(st),
                                           int(reps), times, ncand, ctypes.byref(ntr), _stream()), self.ctx)
        trials = []
        for k in range(ntr.value):
            c = _lib.Settings()  # zero tile: a digit-width trial (run with the chosen renderer)
            self.lib.gesr_autotune_candidate(k, c)
            stage = 1 if c.tile_w > 0 else 2
            if stage == 2:
                c.tile_w, c.tile_h, c.variant, c.batch = st.tile_w, st.tile_h, st.variant, st.batch
            trials.append(dict(stage=stage, tile=f"{c.tile_w}x{c.tile_h}", variant=c.variant, batch=c.batch,
                               radix_bits=c.radix_bits, ms=float(times[k])))
        self.settings = dataclasses.replace(self.settings, tile_w=st.tile_w, tile_h=st.tile_h, variant=st.variant,
                                            batch=st.batch, radix_bits=st.radix_bits)
        self.st_c = self.settings.to_c()
        self.m_cap_hint = 0
        return dict(tile=f"{st.tile_w}x{st.tile_h}", variant=st.variant, batch=st.batch, radix_bits=st.radix_bits,
                    trials=trials)

    def split_images(self, flat: torch.Tensor) -> List[torch.Tensor]:
        out, off = [], 0
        for w, h in self.views:
            out.append(flat[off:off + 3 * w * h].view(3, h, w))
            off += 3 * w * h
        return out


class GESRender(torch.autograd.Function):
    """Differentiable GES rendering of all views of `rast` in one batch.

    forward(rast, mean, scale, quat, opacity, beta, sh) -> flat image [3P].
    Saves the projection, the bins, final_T and n_contrib; the backward
    recomputes per-fragment state from them (no per-fragment storage)."""

    @staticmethod
    def forward(ctx, rast: Rasterizer, mean, scale, quat, opacity, beta, sh):
        sp = Splats(mean.detach().contiguous(), scale.detach().contiguous(), quat.detach().contiguous(),
                    opacity.detach().contiguous(), beta.detach().contiguous(), sh.detach().contiguous())
        out = rast.forward(sp)
        ctx.rast = rast
        ctx.sp = sp
        ctx.state = (out["proj"], out["bins"], out["final_T"], out["n_contrib"])
        return out["image"]

    @staticmethod
    def backward(ctx, dL_dimage):
        proj, bins, final_T, n_contrib = ctx.state
        g = ctx.rast.render_bwd(ctx.sp, proj, bins, final_T, n_contrib, dL_dimage)
        return None, g["mean"], g["scale"], g["quat"], g["opacity"], g["beta"], g["sh"]


def render(rast: Rasterizer, mean, scale, quat, opacity, beta, sh) -> torch.Tensor:
    return GESRender.apply(rast, mean, scale, quat, opacity, beta, sh)
