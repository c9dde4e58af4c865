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
    args = dict(sh_degree=st.sh_degree, kappa=st.kappa, rho=st.rho, alpha_min=st.alpha_min, alpha_max=st.alpha_max,
                t_min=st.t_min, blur=st.blur, znear=st.znear, clip_fac=st.clip_fac, bg=tuple(st.bg), tile_w=st.tile_w,
                tile_h=st.tile_h)
    args.update(kw)
    return RasterSettings(**args)


def u32(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def f32(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.float32)


def splats_of(scene):
    from paper_2411_09156_amd import Splats
    return Splats.from_aos(scene.means, scene.scales, scene.quats, scene.opacities, scene.betas, scene.sh)


def run_gpu(scene, st: oracle.Settings, counts=True, rast=None, **kw) -> dict:
    """HIP forward pipeline; returns numpy outputs (plus the torch state under 'torch')."""
    import torch
    from paper_2411_09156_amd import Rasterizer
    if rast is None:
        rast = Rasterizer(scene.cameras, raster_settings(st, **kw))
    sp = splats_of(scene)
    out = rast.forward(sp, counts=counts)
    torch.cuda.synchronize()
    res = {}
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
    res["listed"] = int(cnt[3])
    M = min(res["listed"], b["m_cap"])
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
    res["torch"] = (rast, sp, out)
    return res


def run_gpu_bwd(scene, st: oracle.Settings, res: dict, dL) -> dict:
    """HIP backward for upstream dL (flat image layout); numpy gradients."""
    import torch
    rast, sp, out = res["torch"]
    g = rast.render_bwd(sp, out["proj"], out["bins"], out["final_T"], out["n_contrib"],
                        torch.as_tensor(np.asarray(dL, np.float32), device="cuda"), want_grad2d=True)
    torch.cuda.synchronize()
    N, V = scene.n, scene.n_views
    K = (st.sh_degree + 1) ** 2
    # grad2d rows: du dv dL00 dL10 dL11 dop dbeta dr dg db dz and a zero pad
    return dict(grad2d=f32(g["grad2d"])[:N * V * 12].reshape(N * V, 12)[:, :11],
                means=f32(g["mean"]).reshape(3, N).T, scales=f32(g["scale"]).reshape(3, N).T,
                quats=f32(g["quat"]).reshape(4, N).T, opacities=f32(g["opacity"]), betas=f32(g["beta"]),
                sh=f32(g["sh"]).reshape(K * 3, N).T.reshape(N, K, 3))


def mask_upstream(dL, ambiguous, cameras):
    """Zero dL/dimage (all channels) at the given pixels (flat CHW-per-view layout)."""
    out = np.array(dL, dtype=np.float64, copy=True)
    amb = np.asarray(ambiguous, bool)
    off_i = off_p = 0
    for c in cameras:
        P = c.width * c.height
        m = amb[off_p:off_p + P]
        for ch in range(3):
            seg = out[off_i + ch * P:off_i + (ch + 1) * P]
            seg[m] = 0.0
        off_i += 3 * P
        off_p += P
    return out


def e2e_settings(st: oracle.Settings, cameras) -> oracle.Settings:
    """Oracle settings whose ambiguity band covers float32 projection error:
    centre error 2 ulp of the image extent, conic error 2e-5 (99.99th
    percentile of the projection's measured error)."""
    import copy
    s = copy.copy(st)
    s.ambig_pos = 2.0 ** -22 * max(max(c.width, c.height) for c in cameras)
    s.ambig_conic = 2e-5
    return s


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


def differing_tiles(vals_a, ranges_a, vals_b, ranges_b) -> np.ndarray:
    """Boolean per global tile: True where the two sorted lists of the tile differ."""
    ranges_a = np.asarray(ranges_a, np.int64)
    ranges_b = np.asarray(ranges_b, np.int64)
    la = ranges_a[:, 1] - ranges_a[:, 0]
    lb = ranges_b[:, 1] - ranges_b[:, 0]
    diff = la != lb
    idx = np.nonzero(~diff & (la > 0))[0]
    L = la[idx]
    if L.sum() > 0:
        off = np.arange(L.sum()) - np.repeat(np.cumsum(L) - L, L)
        pa = np.repeat(ranges_a[idx, 0], L) + off
        pb = np.repeat(ranges_b[idx, 0], L) + off
        neq = np.asarray(vals_a)[pa] != np.asarray(vals_b)[pb]
        diff[np.unique(np.repeat(idx, L)[neq])] = True
    return diff


def ambiguous_tiles_to_pixels(cameras, st, tile_diff) -> np.ndarray:
    """Pixel mask of the tiles flagged in `tile_diff`."""
    grid, T = oracle.tile_grid(cameras, st.tile_w, st.tile_h)
    masks = []
    for v, c in enumerate(cameras):
        tx_n, ty_n, base = grid[v]
        t = tile_diff[base:base + tx_n * ty_n].reshape(ty_n, tx_n)
        m = np.repeat(np.repeat(t, st.tile_h, 0), st.tile_w, 1)[:c.height, :c.width]
        masks.append(m.reshape(-1))
    return np.concatenate(masks)


def check_projection(scene, g: dict, pr: dict) -> str:
    """Projection bars: culls agree except at a handful of threshold ties; centre
    within 2 float32 ulps of the view extent; conic within 1e-4 relative;
    opacity and beta exact; qmax 1e-5 relative; colour 1e-5; depth key equal up
    to one ulp at near-ties; tile rectangles equal away from 1e-3 px of a pixel
    boundary of the FP64 edges.  Returns a one-line summary."""
    keep_g = g["tiles_touched"] > 0
    keep_o = pr["tiles_touched"] > 0
    both = keep_g & keep_o
    VN = len(keep_g)
    assert (keep_g != keep_o).sum() <= max(2, VN // 10000), (keep_g != keep_o).sum()
    r, o = g["rec"][both].astype(np.float64), pr["rec"][both]
    cams = scene.cameras
    # centre: u = fx x/z + cx rounds at the scale of the image, also where the
    # two terms cancel near u = 0
    ext = np.concatenate([np.full(scene.n, max(c.width, c.height)) for c in cams])[both]
    ulp = np.spacing(np.maximum(np.maximum(np.abs(o[:, 0]), np.abs(o[:, 1])), ext).astype(np.float32))
    eu = np.abs(r[:, 0] - o[:, 0]) / ulp
    ev = np.abs(r[:, 1] - o[:, 1]) / ulp
    ecen = max(eu.max(), ev.max()) if eu.size else 0.0
    assert ecen <= 2.0, (eu.max(), ev.max())
    # conic: near edge-on flat splats the determinant's cross term is
    # (disk normal . viewing ray), whose float32 evaluation from a float32
    # rotation loses about eps |ray| / |normal . ray|; elsewhere errors are ~1e-6
    A, B, C = r[:, 2] ** 2, r[:, 2] * r[:, 3], r[:, 3] ** 2 + r[:, 4] ** 2
    eA = np.abs(A - o[:, 2]) / o[:, 2]
    eC = np.abs(C - o[:, 4]) / o[:, 4]
    eB = np.abs(B - o[:, 3]) / np.sqrt(o[:, 2] * o[:, 4])
    econ = np.maximum(np.maximum(eA, eC), eB)
    emax = float(econ.max()) if econ.size else 0.0
    assert emax <= 1e-4, emax
    np.testing.assert_array_equal(r[:, 5], o[:, 5])
    np.testing.assert_array_equal(r[:, 6], o[:, 6])
    np.testing.assert_array_less(np.abs(r[:, 7] - o[:, 7]), 1e-5 * o[:, 7] + 1e-30)
    np.testing.assert_array_less(np.abs(r[:, 8:11] - o[:, 8:11]), 1e-5)
    # depth key: the float32 rounding of the depth.  A key may differ by one ulp
    # only where the exact depth sits on a rounding midpoint (to 1e-12 relative):
    # there a term far below float32 resolution decides the rounding (common when
    # a view axis is aligned with a world axis).
    dk_o = pr["zbits"][both].astype(np.int64)
    dk_g = g["depth_key"][both].astype(np.int64)
    if dk_o.size:
        assert np.abs(dk_g - dk_o).max() <= 1
    dif = dk_g != dk_o
    if dif.any():
        za = np.minimum(dk_g[dif], dk_o[dif]).astype(np.uint32).view(np.float32).astype(np.float64)
        zb = np.maximum(dk_g[dif], dk_o[dif]).astype(np.uint32).view(np.float32).astype(np.float64)
        z64 = np.asarray(pr["depth"], np.float64)[both][dif]
        tie = np.abs(z64 - 0.5 * (za + zb)) <= 1e-12 * np.abs(z64)
        assert tie.all(), (int((~tie).sum()), z64[~tie][:4])
    diff = (g["tile_rect"][both] != pr["tile_rect"][both]).any(1)
    e = pr["edges"][both]
    near = (np.abs(e - np.round(e)) < 1e-3).any(1)
    assert (diff & ~near).sum() == 0
    q9999 = float(np.quantile(econ, 0.9999)) if econ.size else 0.0
    return (f"culls differ {int((keep_g != keep_o).sum())}, rects in guard band {int(diff.sum())}, depth ulps "
            f"{int((dk_g != dk_o).sum())}; centre err max {ecen:.2f} ulp; conic rel err max {emax:.2e}, "
            f"99.99% {q9999:.2e}")
