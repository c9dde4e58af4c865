"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
convert its outputs to the oracle's conventions (all conversions in float64)."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def raster_settings(st: oracle.Settings, **kw):
    from paper_2411_09156_amd import RasterSettings
    return RasterSettings(sh_degree=st.sh_degree, kappa=st.kappa, rho=st.rho, alpha_min=st.alpha_min,
                          alpha_max=st.alpha_max, t_min=st.t_min, blur=st.blur, znear=st.znear,
                          clip_fac=st.clip_fac, bg=tuple(st.bg), tile_w=st.tile_w, tile_h=st.tile_h, **kw)


def u32(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def f32(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.float32)


def splats_of(scene):
    from paper_2411_09156_amd import Splats
    return Splats.from_aos(scene.means, scene.scales, scene.quats, scene.opacities, scene.betas, scene.sh)


def run_gpu(scene, st: oracle.Settings, dL=None, counts=True, rast=None, **kw) -> dict:
    """Full HIP pipeline; returns numpy outputs (plus the torch state under 'torch')."""
    import torch
    from paper_2411_09156_amd import Rasterizer
    if rast is None:
        rast = Rasterizer(scene.cameras, raster_settings(st, **kw))
    sp = splats_of(scene)
    out = rast.forward(sp, counts=counts)
    res = {}
    if dL is not None:
        g = rast.render_bwd(sp, out["proj"], out["bins"], out["final_T"], out["n_contrib"],
                            torch.as_tensor(np.asarray(dL, np.float32), device="cuda"), want_grad2d=True)
    torch.cuda.synchronize()
    N, V = scene.n, scene.n_views
    VN = N * V
    p, b = out["proj"], out["bins"]
    res["rec"] = f32(p["rec"])[:VN * 12].reshape(VN, 12)
    res["tiles_touched"] = u32(p["tiles_touched"])[:VN]
    r = u32(p["rect"])[:2 * VN].reshape(VN, 2)
    res["tile_rect"] = np.stack([r[:, 0] & 0xFFFF, r[:, 0] >> 16, r[:, 1] & 0xFFFF, r[:, 1] >> 16], 1).astype(np.int32)
    res["depth_key"] = u32(p["depth_key"])[:VN]
    cnt = u32(b["counters"])
    res["M"] = int(cnt[0])
    res["overflow"] = int(cnt[1])
    M = min(res["M"], b["m_cap"])
    res["tile_sorted"] = u32(b["tile_sorted"])[:M]
    res["val_sorted"] = u32(b["val_sorted"])[:M]
    T = b["total_tiles"]
    res["ranges"] = u32(b["ranges"])[:2 * T].reshape(T, 2)
    res["worklist"] = u32(b["worklist"])[:T]
    res["inst_base"] = u32(b["inst_base"])[:VN]
    P = scene.n_pixels
    res["image"] = f32(out["image"])[:3 * P]
    res["final_T"] = f32(out["final_T"])[:P]
    res["n_contrib"] = u32(out["n_contrib"])[:P]
    if counts:
        res["n_listed"] = u32(out["n_listed"])[:P]
        res["n_hit"] = u32(out["n_hit"])[:P]
    if dL is not None:
        K = (st.sh_degree + 1) ** 2
        res["grad2d"] = f32(g["grad2d"])[:VN * 10].reshape(VN, 10)
        res["g_means"] = f32(g["mean"]).reshape(3, N).T
        res["g_scales"] = f32(g["scale"]).reshape(3, N).T
        res["g_quats"] = f32(g["quat"]).reshape(4, N).T
        res["g_opacities"] = f32(g["opacity"])
        res["g_betas"] = f32(g["beta"])
        res["g_sh"] = f32(g["sh"]).reshape(K * 3, N).T.reshape(N, K, 3)
    res["torch"] = (rast, sp, out)
    return res


def oracle_rec(gpu_rec: np.ndarray) -> np.ndarray:
    """GPU record (conic factor) -> oracle record (conic A, B, C), in float64."""
    r = gpu_rec.astype(np.float64)
    L00, L10, L11 = r[:, 2], r[:, 3], r[:, 4]
    out = np.zeros((r.shape[0], 11))
    out[:, 0:2] = r[:, 0:2]
    out[:, 2] = L00 * L00
    out[:, 3] = L00 * L10
    out[:, 4] = L10 * L10 + L11 * L11
    out[:, 5:11] = r[:, 5:11]
    return out


def conic_grads_to_factor(g2: np.ndarray, gpu_rec: np.ndarray) -> np.ndarray:
    """Oracle grad2d (dA, dB, dC) -> GPU convention (dL00, dL10, dL11)."""
    r = gpu_rec.astype(np.float64)
    L00, L10, L11 = r[:, 2], r[:, 3], r[:, 4]
    out = g2.copy()
    dA, dB, dC = g2[:, 2], g2[:, 3], g2[:, 4]
    out[:, 2] = 2 * L00 * dA + L10 * dB
    out[:, 3] = L00 * dB + 2 * L10 * dC
    out[:, 4] = 2 * L11 * dC
    return out


def factor_grads_to_conic(g2: np.ndarray, gpu_rec: np.ndarray) -> np.ndarray:
    """GPU grad2d (dL00, dL10, dL11) -> (dA, dB, dC) by inverting the factor map."""
    r = gpu_rec.astype(np.float64)
    L00, L10, L11 = r[:, 2], r[:, 3], r[:, 4]
    out = g2.astype(np.float64).copy()
    with np.errstate(divide="ignore", invalid="ignore"):
        dC = np.where(L11 != 0, out[:, 4] / (2 * L11), 0.0)
        dB = np.where(L00 != 0, (out[:, 3] - 2 * L10 * dC) / L00, 0.0)
        dA = np.where(L00 != 0, (out[:, 2] - L10 * dB) / (2 * L00), 0.0)
    out[:, 2], out[:, 3], out[:, 4] = dA, dB, dC
    return out


def image_errors(gpu_img, or_img, ambiguous, cameras, tol=1e-4):
    """Per view: (#non-ambiguous pixels over tol, max err non-ambiguous, bound, l2 rel err)."""
    out = []
    off_i = off_p = 0
    for c in cameras:
        P = c.width * c.height
        g = np.asarray(gpu_img[off_i:off_i + 3 * P], np.float64).reshape(3, P)
        o = np.asarray(or_img[off_i:off_i + 3 * P], np.float64).reshape(3, P)
        amb = np.asarray(ambiguous[off_p:off_p + P], bool)
        err = np.abs(g - o).max(0)
        bound = tol * max(np.abs(o).max(), 1.0)
        bad = int(((err > bound) & ~amb).sum())
        mx = float(err[~amb].max()) if (~amb).any() else 0.0
        nrm = np.linalg.norm(o)
        l2 = float(np.linalg.norm(g - o) / nrm) if nrm > 0 else float(np.linalg.norm(g - o))
        out.append((bad, mx, bound, l2))
        off_i += 3 * P
        off_p += P
    return out


def norm_errors(a, b):
    """(inf-norm err / inf-norm ref, 2-norm err / 2-norm ref) of arrays a (test) vs b (ref)."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    ninf = np.abs(b).max() if b.size else 0.0
    n2 = np.linalg.norm(b)
    einf = np.abs(a - b).max() if b.size else 0.0
    e2 = np.linalg.norm(a - b)
    return (einf / ninf if ninf > 0 else einf, e2 / n2 if n2 > 0 else e2)


def tile_lists(vals, ranges):
    return [tuple(vals[s0:s1]) for s0, s1 in ranges]


def ambiguous_from_lists(cameras, st, lists_a, lists_b):
    """Pixel mask: True where the pixel's tile list differs between two binnings."""
    grid, T = oracle.tile_grid(cameras, st.tile_w, st.tile_h)
    masks = []
    for v, c in enumerate(cameras):
        tx_n, ty_n, base = grid[v]
        m = np.zeros((c.height, c.width), bool)
        for ty in range(ty_n):
            for tx in range(tx_n):
                t = base + ty * tx_n + tx
                if lists_a[t] != lists_b[t]:
                    m[ty * st.tile_h:(ty + 1) * st.tile_h, tx * st.tile_w:(tx + 1) * st.tile_w] = True
        masks.append(m.reshape(-1))
    return np.concatenate(masks)
