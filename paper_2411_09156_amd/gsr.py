"""Binding of the surface regulariser (gesr_knn, gesr_gsr: Sec. 3.3, Eq. 9-13,
with the nearest-neighbour density of Sec. 4.2), argument marshalling only.

Neighbour lists are [N, k] uint32 (as int32 tensors): slot 0 is the splat
itself; `order` is the spatial (cell) order the regulariser runs its samples
in, and the inverse lists refer to positions in it.  The regulariser draws one sample per splat from the caller's
standard-normal xi [3, N]; its gradients are added into a gradient dict of
the rasterizer's layout (keys mean, scale, quat, opacity, beta).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .rasterizer import RasterSettings, Splats, _stream
from .optim import _ctx


def _check(lib, ctx, st):
    if st != _lib.GESR_OK:
        raise _lib.GesrError(st, lib.gesr_last_error(ctx).decode())


def knn(sp: Splats, k: int = 16, device: int = 0) -> dict:
    """Neighbour lists and their inverse (gesr_knn)."""
    lib, ctx = _ctx(device)
    n = sp.n
    dev = sp.mean.device
    out = dict(knn=torch.empty(max(n * k, 1), dtype=torch.int32, device=dev),
               order=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
               inv_offsets=torch.empty(n + 1, dtype=torch.int32, device=dev),
               inv_entries=torch.empty(max(n * k, 1), dtype=torch.int32, device=dev),
               inv_slot=torch.empty(max(n * k, 1), dtype=torch.int32, device=dev), k=k)
    wsb = int(lib.gesr_knn_workspace_size(n, k))
    ws = torch.empty(max(wsb, 16), dtype=torch.uint8, device=dev)
    _check(lib, ctx, lib.gesr_knn(ctx, ctypes.byref(sp.to_c()), int(k), out["knn"].data_ptr(),
                                  out["order"].data_ptr(), out["inv_offsets"].data_ptr(), out["inv_entries"].data_ptr(),
                                  out["inv_slot"].data_ptr(), ws.data_ptr(), wsb, _stream()))
    out["knn"] = out["knn"][:n * k].view(n, k)
    out["inv_entries"] = out["inv_entries"][:n * k]
    out["inv_slot"] = out["inv_slot"][:n * k]
    out["order"] = out["order"][:n]
    return out


def gsr(sp: Splats, settings: RasterSettings, nbrs: dict, xi: torch.Tensor, mask: torch.Tensor = None,
        w_sdf: float = 1.0, w_nor: float = 1.0, grads: dict = None, device: int = 0) -> dict:
    """Regulariser losses on one sample per splat (gesr_gsr).  Returns
    sample_out [N, 4] (l_sdf, l_nor, g* slot, d) and losses [2] (sums); adds
    the gradients into `grads` when given."""
    lib, ctx = _ctx(device)
    n, k = sp.n, int(nbrs["k"])
    dev = sp.mean.device
    xi = xi.contiguous()
    m = mask.contiguous() if mask is not None else None
    sample_out = torch.empty(max(n, 1), 4, dtype=torch.float32, device=dev)
    losses = torch.empty(4, dtype=torch.float32, device=dev)
    gc = None
    if grads is not None:
        gc = _lib.Grads(grads["mean"].data_ptr(), grads["scale"].data_ptr(), grads["quat"].data_ptr(),
                        grads["opacity"].data_ptr(), grads["beta"].data_ptr(), None)
    wsb = int(lib.gesr_gsr_workspace_size(n, k, int(grads is not None)))
    ws = torch.empty(max(wsb, 16), dtype=torch.uint8, device=dev)
    gs = _lib.GsrSettings(float(w_sdf), float(w_nor))
    st_c = settings.to_c()
    _check(lib, ctx, lib.gesr_gsr(ctx, ctypes.byref(sp.to_c()), ctypes.byref(st_c), k, nbrs["knn"].data_ptr(),
                                  nbrs["order"].data_ptr(), nbrs["inv_offsets"].data_ptr(), nbrs["inv_slot"].data_ptr(), xi.data_ptr(),
                                  m.data_ptr() if m is not None else None, ctypes.byref(gs), sample_out.data_ptr(),
                                  losses.data_ptr(), ctypes.byref(gc) if gc is not None else None, ws.data_ptr(),
                                  wsb, _stream()))
    return dict(sample_out=sample_out[:n], losses=losses[:2])
