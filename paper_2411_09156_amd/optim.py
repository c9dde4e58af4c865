"""Binding of the fused optimiser step (gesr_adam_step): Adam on the raw splat
parameters with per-group learning rates and the opacity-entropy term of the
training schedule (Sec. 4.2), argument marshalling only.

The optimiser owns the raw parameters (log scales and opacity logits) and the
two moments, SoA device tensors in the layouts of rasterizer.Splats; `splats`
is the activated view the renderer reads: mean, quat, beta and sh share the
raw tensors, scale and opacity are the buffers the step rewrites.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib
from .rasterizer import Splats, _stream

RAW_FIELDS = ("mean", "log_scale", "quat", "opacity_logit", "beta", "sh")


@dataclasses.dataclass
class AdamConfig:
    """Mirror of gesr_adam_settings (without the step counter)."""
    lr_mean: float = 1.6e-4
    lr_scale: float = 5e-3
    lr_quat: float = 1e-3
    lr_opacity: float = 0.05
    lr_beta: float = 1.5e-3
    lr_sh_dc: float = 2.5e-3
    lr_sh_rest: float = 2.5e-3 / 20
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    entropy_weight: float = 0.0

    def to_c(self, step: int) -> _lib.AdamSettings:
        s = _lib.AdamSettings()
        for f in dataclasses.fields(self):
            setattr(s, f.name, float(getattr(self, f.name)))
        s.step = int(step)
        return s


@dataclasses.dataclass
class RawParams:
    """SoA device tensors: mean [3, N], log_scale [3, N], quat [4, N],
    opacity_logit [N], beta [N], sh [K * 3, N]."""
    mean: torch.Tensor
    log_scale: torch.Tensor
    quat: torch.Tensor
    opacity_logit: torch.Tensor
    beta: torch.Tensor
    sh: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.opacity_logit.shape[0])

    @property
    def sh_coeffs(self) -> int:
        return int(self.sh.shape[0]) // 3

    def to_c(self) -> _lib.Params:
        c = _lib.Params()
        c.n, c.sh_coeffs = self.n, self.sh_coeffs
        for k in RAW_FIELDS:
            setattr(c, k, getattr(self, k).data_ptr())
        return c

    def zeros_like(self) -> "RawParams":
        return RawParams(*(torch.zeros_like(getattr(self, k)) for k in RAW_FIELDS))

    @staticmethod
    def from_aos(means, log_scales, quats, opacity_logits, betas, sh, device="cuda") -> "RawParams":
        """From row-per-splat arrays ([N,3], [N,3], [N,4], [N], [N], [N,K,3])."""
        def t(x):
            return torch.as_tensor(x, dtype=torch.float32).to(device)
        n = t(opacity_logits).shape[0]
        shc = t(sh)
        width = 1
        for d in shc.shape[1:]:
            width *= int(d)
        shc = shc.reshape(n, width)
        return RawParams(t(means).reshape(n, 3).t().contiguous(), t(log_scales).reshape(n, 3).t().contiguous(),
                         t(quats).reshape(n, 4).t().contiguous(), t(opacity_logits).contiguous(),
                         t(betas).contiguous(), shc.t().contiguous())


_ctxs = {}


def _ctx(device: int):
    """One library context per device for the free functions below (kept for
    the life of the process)."""
    lib = _lib.load()
    if device not in _ctxs:
        ctx = ctypes.c_void_p()
        st = lib.gesr_ctx_create(device, ctypes.byref(ctx))
        if st != _lib.GESR_OK:
            raise _lib.GesrError(st, lib.gesr_status_string(st).decode())
        _ctxs[device] = ctx
    return lib, _ctxs[device]


def _rows(raw: RawParams):
    return (3, 3, 4, 1, 1, 3 * raw.sh_coeffs)


def prune(raw: RawParams, m: RawParams = None, v: RawParams = None, min_opacity: float = 0.5,
          min_beta: float = 0.5, device: int = 0):
    """Stable compaction of the splats kept by the pruning rule (gesr_prune).
    Returns (raw, m, v, scale, opacity) of the kept splats (m and v None when
    not given; scale and opacity activated).  Synchronises once to read the
    kept count."""
    lib, ctx = _ctx(device)
    n = raw.n

    def alloc_like(src):
        return RawParams(*(torch.empty_like(getattr(src, k)) for k in RAW_FIELDS))
    out_p = alloc_like(raw)
    out_m = alloc_like(m) if m is not None else None
    out_v = alloc_like(v) if v is not None else None
    dev = raw.opacity_logit.device
    scale = torch.empty_like(raw.log_scale)
    opacity = torch.empty_like(raw.opacity_logit)
    n_kept = torch.zeros(4, dtype=torch.int32, device=dev)
    wsb = int(lib.gesr_prune_workspace_size(n))
    ws = torch.empty(max(wsb, 16), dtype=torch.uint8, device=dev)
    ps = _lib.PruneSettings(float(min_opacity), float(min_beta))

    def ref(x):
        return ctypes.byref(x.to_c()) if x is not None else None
    st = lib.gesr_prune(ctx, ref(raw), ref(m), ref(v), ctypes.byref(ps), ref(out_p), ref(out_m), ref(out_v),
                        scale.data_ptr(), opacity.data_ptr(), n_kept.data_ptr(), ws.data_ptr(), wsb, _stream())
    if st != _lib.GESR_OK:
        raise _lib.GesrError(st, lib.gesr_last_error(ctx).decode())
    nk = int(n_kept[0].item())

    def packed(x):
        if x is None:
            return None
        views = []
        for k, r in zip(RAW_FIELDS, _rows(raw)):
            flat = getattr(x, k).reshape(-1)[:r * nk]
            views.append(flat.view(nk) if k in ("opacity_logit", "beta") else flat.view(r, nk))
        return RawParams(*views)
    return (packed(out_p), packed(out_m), packed(out_v), scale.reshape(-1)[:3 * nk].view(3, nk),
            opacity[:nk])


def shape_reset(raw: RawParams, m: RawParams = None, v: RawParams = None, value: float = 2.0,
                device: int = 0) -> None:
    """Sets beta of every splat to `value` and zeroes its moments (gesr_shape_reset)."""
    lib, ctx = _ctx(device)

    def ref(x):
        return ctypes.byref(x.to_c()) if x is not None else None
    st = lib.gesr_shape_reset(ctx, ref(raw), ref(m), ref(v), float(value), _stream())
    if st != _lib.GESR_OK:
        raise _lib.GesrError(st, lib.gesr_last_error(ctx).decode())


class SplatAdam:
    """Adam state for one splat set on one device.  step() enqueues one fused
    kernel on torch's current stream."""

    def __init__(self, raw: RawParams, config: AdamConfig = None, device: int = 0):
        self.lib = _lib.load()
        self.raw = raw
        self.config = config or AdamConfig()
        self.m = raw.zeros_like()
        self.v = raw.zeros_like()
        self.t = 0
        ctx = ctypes.c_void_p()
        st = self.lib.gesr_ctx_create(device, ctypes.byref(ctx))
        if st != _lib.GESR_OK:
            raise _lib.GesrError(st, self.lib.gesr_status_string(st).decode())
        self.ctx = ctx
        # activated buffers: initial values by torch, rewritten by every step
        self.splats = Splats(raw.mean, torch.exp(raw.log_scale), raw.quat, torch.sigmoid(raw.opacity_logit),
                             raw.beta, raw.sh)

    def __del__(self):
        lib = getattr(self, "lib", None)
        if lib is not None and getattr(self, "ctx", None):
            lib.gesr_ctx_destroy(self.ctx)
            self.ctx = None

    def step(self, grads: dict) -> None:
        """grads: the rasterizer's gradients of the activated parameters (keys
        mean, scale, quat, opacity, beta, sh; layouts of Splats)."""
        self.t += 1
        gt = [grads[k].contiguous() for k in ("mean", "scale", "quat", "opacity", "beta", "sh")]
        g = _lib.Grads(*(x.data_ptr() for x in gt))
        st = self.lib.gesr_adam_step(self.ctx, ctypes.byref(self.raw.to_c()), ctypes.byref(self.m.to_c()),
                                     ctypes.byref(self.v.to_c()), ctypes.byref(g),
                                     ctypes.byref(self.config.to_c(self.t)), self.splats.scale.data_ptr(),
                                     self.splats.opacity.data_ptr(), _stream())
        if st != _lib.GESR_OK:
            self.t -= 1
            raise _lib.GesrError(st, self.lib.gesr_last_error(self.ctx).decode())

    def prune(self, min_opacity: float = 0.5, min_beta: float = 0.5) -> int:
        """Removes pruned splats from the parameters, moments and activated
        buffers (new tensors; the step counter continues).  Returns the kept
        count."""
        raw, m, v, scale, opacity = prune(self.raw, self.m, self.v, min_opacity, min_beta)
        self.raw, self.m, self.v = raw, m, v
        self.splats = Splats(raw.mean, scale, raw.quat, opacity, raw.beta, raw.sh)
        return raw.n

    def shape_reset(self, value: float = 2.0) -> None:
        shape_reset(self.raw, self.m, self.v, value)
