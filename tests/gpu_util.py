"""Helpers for the GPU parity tests: run the HIP path through the C ABI,
convert its outputs to the oracle's conventions (all conversions in float64)
and build the oracle's references.

Parity model.  The oracle decides every threshold in FP64.  A decision whose
threshold lies within the float32 error band derived in the oracle (the skip
and termination decisions of compositing, the footprint rule of binning)
has two correct outcomes.  For binning, the GPU's lists must equal the
oracle's after removing the (pair, tile) decisions within the band.  For
compositing, the oracle enumerates the results of both outcomes at each such
decision (its decision paths) and the GPU's per-pixel result must be one of
them; the comparison then uses that path for the image, transmittance, counts
and the adjoint.  Pixels are masked only where the alpha cap's decision is
within its band (its two outcomes give the same image but different
derivatives) or a pixel has more than 64 paths; their fraction is asserted to
stay below MASKED_MAX.  A GPU result that matches none of the paths fails."""
from __future__ import annotations

import sys

import numpy as np

import oracle

REC = 16  # floats per projected record of the HIP library (the first 12 carry the values)


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
    res["rec"] = f32(p["rec"])[:VN * REC].reshape(VN, REC)[:, :12]
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


MASKED_MAX = 1e-3  # largest fraction of pixels left out of a comparison


def pixel_tiles(cameras, st) -> np.ndarray:
    """Global tile id of every pixel, views concatenated."""
    grid, _ = oracle.tile_grid(cameras, st.tile_w, st.tile_h)
    out = []
    for (tx_n, ty_n, base), c in zip(grid, cameras):
        y, x = np.divmod(np.arange(c.width * c.height, dtype=np.int64), c.width)
        out.append(base + (y // st.tile_h) * tx_n + x // st.tile_w)
    return np.concatenate(out) if out else np.zeros(0, np.int64)


def last_composited(cameras, st, vals, ranges, n_contrib) -> np.ndarray:
    """Record index (view * n + splat) of each pixel's last composited fragment
    (-1 if none), from a renderer's tile lists and n_contrib (a 1-based position
    in the pixel's tile list)."""
    vals = np.asarray(vals, np.int64)
    nc = np.asarray(n_contrib, np.int64)
    pos = np.asarray(ranges, np.int64)[pixel_tiles(cameras, st), 0] + nc - 1
    if vals.size == 0:
        return np.full(nc.size, -1, np.int64)
    return np.where(nc > 0, vals[np.clip(pos, 0, vals.size - 1)], -1)


def compare_lists(g_vals, g_tiles, g_ranges, o_keys, o_vals, o_ranges, band) -> dict:
    """GPU tile lists against the oracle's footprint rule: after removing the
    (pair, tile) decisions within the float32 band (`band`, from
    oracle.bin_band) from both, the sorted lists are identical.  Returns the
    band size, how many band decisions the GPU took the other way than the
    FP64 rule, and the tiles whose lists differ."""
    g_vals = np.asarray(g_vals, np.uint64)
    o_vals = np.asarray(o_vals, np.uint64)
    gid = (np.asarray(g_tiles, np.uint64) << np.uint64(32)) | g_vals
    oid = ((np.asarray(o_keys, np.uint64) >> np.uint64(32)) << np.uint64(32)) | o_vals
    bid = np.sort((band["tile"].astype(np.uint64) << np.uint64(32)) | band["pair"].astype(np.uint64))

    def outside(ids):
        if bid.size == 0:
            return ids
        j = np.minimum(np.searchsorted(bid, ids), bid.size - 1)
        return ids[bid[j] != ids]
    a, b = outside(gid), outside(oid)
    assert a.size == b.size and np.array_equal(a, b), (a.size, b.size)
    g_ranges = np.asarray(g_ranges, np.int64)
    flips = 0
    for t, p_, lo in zip(band["tile"], band["pair"], band["listed"]):
        r0, r1 = g_ranges[t]
        flips += int(bool((g_vals[r0:r1] == p_).any()) != bool(lo))
    diff = differing_tiles(g_vals, g_ranges, o_vals, o_ranges)
    return dict(n_band=int(bid.size), n_flip=flips, tiles_differ=diff)


def check_resolution(status, plain, g_image, g_final_T, last, label) -> np.ndarray:
    """Asserts that every pixel's GPU result is one of the oracle's correct
    results (no status 4) and that at most MASKED_MAX of the pixels are
    masked; returns the masked pixels and logs the counts."""
    status = np.asarray(status)
    bad = np.nonzero(status == 4)[0]
    if bad.size:
        p = int(bad[0])
        raise AssertionError(f"{label}: {bad.size} pixels match no decision path of the oracle; first {p}: "
                             f"T gpu {float(g_final_T[p]):.9g} oracle {plain['final_T'][p]:.9g}, last gpu "
                             f"{int(last[p])} oracle {int(plain['last'][p])}, n_branch {int(plain['n_branch'][p])}")
    masked = (status == 2) | (status == 3)
    frac = float(masked.mean()) if masked.size else 0.0
    log(f"[gpu] {label}: {int((status == 1).sum())} px resolved among decision paths, {int(masked.sum())} masked "
        f"({frac:.1e}; cap band {int((status == 2).sum())}, too many paths {int((status == 3).sum())})")
    assert frac <= MASKED_MAX, (label, frac)
    return masked


def listed_where_same(scene, st, g: dict, tiles_differ):
    """The GPU's per-pixel listed-fragment counts where its tile list equals
    the oracle's, 0xFFFFFFFF (not compared) elsewhere; None without counts."""
    if "n_listed" not in g:
        return None
    px = ambiguous_tiles_to_pixels(scene.cameras, st, tiles_differ)
    return np.where(px, np.uint32(0xFFFFFFFF), np.asarray(g["n_listed"], np.uint32)).astype(np.uint32)


def same_input_reference(scene, st, g: dict, depth=None) -> dict:
    """The oracle fed the GPU's projection records: its own tile lists from
    them (compared with the GPU's outside the band), each pixel's decision path
    resolved to the GPU's forward result, and its forward along those paths."""
    rec = oracle_rec(g["rec"])
    keys, vals, ranges = oracle.bin_instances(scene.n, scene.cameras, g["tile_rect"], g["tiles_touched"],
                                              g["depth_key"], st, rec)
    band = oracle.bin_band(scene.n, scene.cameras, g["tile_rect"], g["tiles_touched"], rec, st)
    lists = compare_lists(g["val_sorted"], g["tile_sorted"], g["ranges"], keys, vals, ranges, band)
    last = last_composited(scene.cameras, st, g["val_sorted"], g["ranges"], g["n_contrib"])
    paths, status, plain = oracle.resolve(scene.n, scene.cameras, rec, vals, ranges, st, g["image"], g["final_T"],
                                          last, g.get("n_hit"),
                                          n_listed=listed_where_same(scene, st, g, lists["tiles_differ"]))
    masked = check_resolution(status, plain, g["image"], g["final_T"], last, "same inputs")
    fwd = oracle.render_fwd(scene.n, scene.cameras, rec, vals, ranges, st, depth=depth, paths=paths)
    return dict(rec=rec, keys=keys, vals=vals, ranges=ranges, band=band, lists=lists, last=last, paths=paths,
                status=status, masked=masked, fwd=fwd)


def end_to_end_reference(scene, st, g: dict, channels: bool = False) -> dict:
    """The oracle run from the splat parameters (its own FP64 records and
    lists), with decision bands widened by the a-priori record error bounds,
    each pixel's decision path resolved to the GPU's forward result."""
    fo = oracle.forward(scene, st, band=True)
    last = last_composited(scene.cameras, st, g["val_sorted"], g["ranges"], g["n_contrib"])
    pr = fo["proj"]
    differ = differing_tiles(g["val_sorted"], g["ranges"], fo["vals"], fo["ranges"])
    paths, status, plain = oracle.resolve(scene.n, scene.cameras, pr["rec"], fo["vals"], fo["ranges"], st,
                                          g["image"], g["final_T"], last, g.get("n_hit"), perr=fo["perr"],
                                          n_listed=listed_where_same(scene, st, g, differ))
    masked = check_resolution(status, plain, g["image"], g["final_T"], last, "end to end")
    fwd = oracle.render_fwd(scene.n, scene.cameras, pr["rec"], fo["vals"], fo["ranges"], st,
                            depth=pr["depth"] if channels else None, perr=fo["perr"], paths=paths)
    fwd.update(proj=pr, keys=fo["keys"], vals=fo["vals"], ranges=fo["ranges"], perr=fo["perr"])
    return dict(fo=fwd, last=last, paths=paths, status=status, masked=masked)


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


def check_projection(scene, g: dict, pr: dict, perr: np.ndarray) -> str:
    """Projection against the FP64 oracle under the a-priori float32 bounds of
    oracle.record_err_bound (perr [V*N, 3]): culls agree except at a handful of
    threshold ties; centre within perr[:, 0] px; the conic's effect on q within
    perr[:, 1] relative in the worst direction (the spectral radius of
    C_or^-1 (C_gpu - C_or)); qmax within perr[:, 2] relative; opacity and beta
    exact; colour within 1e-5; depth key equal up to one ulp at near-ties; tile
    rectangles equal unless an FP64 edge lies within its float32 band of a
    pixel boundary.  Returns a one-line summary."""
    keep_g = g["tiles_touched"] > 0
    keep_o = pr["tiles_touched"] > 0
    both = keep_g & keep_o
    VN = len(keep_g)
    assert (keep_g != keep_o).sum() <= max(2, VN // 10000), (keep_g != keep_o).sum()
    r, o, e = g["rec"][both].astype(np.float64), pr["rec"][both], perr[both]
    ecen = np.maximum(np.abs(r[:, 0] - o[:, 0]), np.abs(r[:, 1] - o[:, 1]))
    rc = float((ecen / e[:, 0]).max()) if ecen.size else 0.0
    assert rc <= 1.0, rc
    A, B, C = r[:, 2] ** 2, r[:, 2] * r[:, 3], r[:, 3] ** 2 + r[:, 4] ** 2
    oA, oB, oC = o[:, 2], o[:, 3], o[:, 4]
    det = oA * oC - oB * oB
    dA, dB, dC = A - oA, B - oB, C - oC
    m00, m01 = (oC * dA - oB * dB) / det, (oC * dB - oB * dC) / det
    m10, m11 = (oA * dB - oB * dA) / det, (oA * dC - oB * dB) / det
    tr, dm = 0.5 * (m00 + m11), m00 * m11 - m01 * m10
    disc = np.sqrt(np.maximum(tr * tr - dm, 0.0))
    econ = np.maximum(np.abs(tr + disc), np.abs(tr - disc))
    rk = float((econ / e[:, 1]).max()) if econ.size else 0.0
    assert rk <= 1.0, rk
    eq = np.abs(r[:, 7] - o[:, 7]) / o[:, 7]
    rq = float((eq / e[:, 2]).max()) if eq.size else 0.0
    assert rq <= 1.0, rq
    np.testing.assert_array_equal(r[:, 5], o[:, 5])
    np.testing.assert_array_equal(r[:, 6], o[:, 6])
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
    # tile rectangles: the pixel edges u -+ rx - 1/2 (rx = sqrt(qmax a)) move by
    # the centre error, rx (qmax + conic errors) / 2 and two roundings
    diff = (g["tile_rect"][both] != pr["tile_rect"][both]).any(1)
    ed = pr["edges"][both]
    sa = np.asarray(pr["sigma2d"], np.float64)[both]
    rx, ry = np.sqrt(o[:, 7] * sa[:, 0]), np.sqrt(o[:, 7] * sa[:, 2])
    u32 = 2.0 ** -24
    w = 0.5 * (e[:, 1] + e[:, 2]) + 2 * u32
    bx = e[:, 0] + rx * w + 2 * u32 * (np.abs(o[:, 0]) + rx + 1)
    by = e[:, 0] + ry * w + 2 * u32 * (np.abs(o[:, 1]) + ry + 1)
    bandw = np.stack([bx, bx, by, by], 1)
    near = (np.abs(ed - np.round(ed)) <= bandw).any(1)
    assert (diff & ~near).sum() == 0, int((diff & ~near).sum())
    return (f"culls differ {int((keep_g != keep_o).sum())}, rects in band {int(near.sum())} (differ {int(diff.sum())}), "
            f"depth ulps {int((dk_g != dk_o).sum())}; worst error / a-priori bound: centre {rc:.2f}, conic {rk:.2f}, "
            f"qmax {rq:.2f}")
