"""FP64 CPU oracle for the GES rasterizer — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and it imports nothing
from the product path.

The arithmetic lives in ``gesr_oracle.cpp`` (double precision, OpenMP); this
module only builds/loads it and marshals numpy arrays.

Settings values are rounded to float32 before they are promoted to double,
so both sides compare against exactly the same thresholds.  Splat parameters
are taken as given (float32 scenes promote exactly; finite-difference checks
pass perturbed float64 values).

Parity status of each function is listed in the header of the C++ source;
every function here is pinned by the CPU tests under ``tests/``
(closed forms, library routines, brute force and finite differences).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gesr_oracle.cpp")
# GESR_ORACLE_LIB selects another build of the same source (the sanitizer test's)
_LIB = os.environ.get("GESR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, OpenMP, strict IEEE double)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        stale = not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
        if stale and "GESR_ORACLE_LIB" not in os.environ:
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.orc_bin_count.restype = ctypes.c_uint64
        _lib.orc_total_tiles.restype = ctypes.c_long
    return _lib


@dataclass
class Settings:
    """Rasterizer constants (values shared with the GPU side, not code)."""
    kappa: float = 0.5
    rho: float = 0.1
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    blur: float = 0.3
    znear: float = 0.2
    clip_fac: float = 1.3
    bg: Sequence[float] = field(default_factory=lambda: (0.0, 0.0, 0.0))
    tile_w: int = 16
    tile_h: int = 16
    sh_degree: int = 0
    # Parity model: multiplier of the derived float32 bands of the skip and
    # termination decisions (1 = the bands derived in frag_band).
    band_scale: float = 1.0

    def array(self) -> np.ndarray:
        f = lambda x: float(np.float32(x))  # noqa: E731
        return np.array([f(self.kappa), f(self.rho), f(self.alpha_min), f(self.alpha_max), f(self.t_min),
                         f(self.blur), f(self.znear), f(self.clip_fac), f(self.bg[0]), f(self.bg[1]),
                         f(self.bg[2]), self.tile_w, self.tile_h, self.sh_degree, self.band_scale, 0, 0, 0],
                        dtype=np.float64)


def views_array(cameras) -> np.ndarray:
    out = np.zeros((len(cameras), 24), dtype=np.float64)
    for k, c in enumerate(cameras):
        out[k, 0] = c.width
        out[k, 1] = c.height
        out[k, 2:6] = [np.float32(c.fx), np.float32(c.fy), np.float32(c.cx), np.float32(c.cy)]
        vm = np.asarray(c.viewmat, dtype=np.float32).astype(np.float64)
        out[k, 6:15] = vm[:, :3].reshape(-1)
        out[k, 15:18] = vm[:, 3]
        out[k, 18:21] = np.asarray(c.campos, dtype=np.float32).astype(np.float64)
    return out


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def tile_grid(cameras, tile_w, tile_h):
    """(tiles_x, tiles_y, tile_base) per view and the total tile count."""
    out, base = [], 0
    for c in cameras:
        tx = (c.width + tile_w - 1) // tile_w
        ty = (c.height + tile_h - 1) // tile_h
        out.append((tx, ty, base))
        base += tx * ty
    return out, base


def project(scene, st: Settings) -> dict:
    """FP64 projection of every (view, splat); arrays indexed [view * N + splat]."""
    N, V = scene.n, scene.n_views
    VN = N * V
    r = dict(
        rec=np.zeros((VN, 11)), depth=np.zeros(VN), z32=np.zeros(VN, np.float32), sigma2d=np.zeros((VN, 3)),
        edges=np.zeros((VN, 4)), pix_rect=np.zeros((VN, 4), np.int32), tile_rect=np.zeros((VN, 4), np.int32),
        tiles_touched=np.zeros(VN, np.uint32), cull=np.zeros(VN, np.uint8), clamp=np.zeros(VN, np.uint8))
    sh = _f64(scene.sh.reshape(N, int(np.prod(scene.sh.shape[1:]))))
    lib().orc_project(N, V, _p(_f64(scene.means)), _p(_f64(scene.scales)), _p(_f64(scene.quats)),
                      _p(_f64(scene.opacities)), _p(_f64(scene.betas)), _p(sh), _p(views_array(scene.cameras)),
                      _p(st.array()), _p(r["rec"]), _p(r["depth"]), _p(r["z32"]), _p(r["sigma2d"]),
                      _p(r["edges"]), _p(r["pix_rect"]), _p(r["tile_rect"]), _p(r["tiles_touched"]),
                      _p(r["cull"]), _p(r["clamp"]))
    r["zbits"] = r["z32"].view(np.uint32)
    return r


def record_err_bound(scene, st: Settings) -> np.ndarray:
    """A-priori bounds [V*N, 3] on how far a float32 projection's record may
    lie from the FP64 one: centre (px, each of u and v), relative error of q
    due to the conic, relative error of qmax (see orc_record_err_bound).
    Culled pairs get zeros."""
    N, V = scene.n, scene.n_views
    out = np.zeros((max(N * V, 1), 3))
    if N > 0:
        lib().orc_record_err_bound(N, V, _p(_f64(scene.means)), _p(_f64(scene.scales)), _p(_f64(scene.quats)),
                                   _p(_f64(scene.opacities)), _p(_f64(scene.betas)), _p(views_array(scene.cameras)),
                                   _p(st.array()), _p(out))
    return out[:N * V]


def _rec11(rec, VN):
    return _f64(np.asarray(rec, np.float64).reshape(-1, 11)) if VN > 0 else np.zeros((1, 11))


def _perr(perr, VN):
    return None if perr is None else _f64(np.asarray(perr, np.float64).reshape(VN, 3))


def bin_instances(N, cameras, tile_rect, tiles_touched, zbits, st: Settings, rec):
    """Stable-sorted (keys, vals, ranges[T, 2]) of the (tile | depth) instances
    under the footprint rule of orc_bin: a tile of a pair's rectangle is listed
    when the minimum of q over its square is <= qmax (1 + 2^-8).  rec:
    [V*N, 11] records (u, v, A, B, C, opacity, beta, qmax, r, g, b)."""
    V = len(cameras)
    tiles_touched = np.ascontiguousarray(tiles_touched, dtype=np.uint32)
    M = int(lib().orc_bin_count(ctypes.c_long(V * N), _p(tiles_touched)))
    _, T = tile_grid(cameras, st.tile_w, st.tile_h)
    keys = np.zeros(max(M, 1), np.uint64)
    vals = np.zeros(max(M, 1), np.uint32)
    ranges = np.zeros((T, 2), np.uint32)
    lib().orc_bin.restype = ctypes.c_long
    L = int(lib().orc_bin(N, V, _p(np.ascontiguousarray(tile_rect, np.int32)), _p(tiles_touched),
                          _p(np.ascontiguousarray(zbits, np.uint32)), _p(views_array(cameras)), st.tile_w, st.tile_h,
                          _p(_rec11(rec, V * N)), _p(keys), _p(vals), _p(ranges)))
    return keys[:L], vals[:L], ranges


def bin_pair_counts(N, cameras, tile_rect, tiles_touched, rec, st: Settings, perr=None):
    """Per pair (n_in, n_band): tiles of its rectangle listed with certainty
    under the footprint rule, and those whose decision lies within the float32
    band (perr [V*N, 3]: end-to-end record error bounds, nullable)."""
    V = len(cameras)
    VN = V * N
    tiles_touched = np.ascontiguousarray(tiles_touched, dtype=np.uint32)
    n_in = np.zeros(max(VN, 1), np.uint32)
    n_band = np.zeros(max(VN, 1), np.uint32)
    if VN:
        lib().orc_bin_pair_counts(N, V, _p(views_array(cameras)), st.tile_w, st.tile_h,
                                  _p(np.ascontiguousarray(tile_rect, np.int32)), _p(tiles_touched),
                                  _p(_rec11(rec, VN)), _p(_perr(perr, VN)), _p(n_in), _p(n_band))
    return n_in[:VN], n_band[:VN]


def bin_band(N, cameras, tile_rect, tiles_touched, rec, st: Settings, perr=None) -> dict:
    """The (pair, global tile) decisions of the footprint rule that lie within
    the float32 band, with the FP64 outcome: dict(pair, tile, listed)."""
    V = len(cameras)
    VN = V * N
    tiles_touched = np.ascontiguousarray(tiles_touched, dtype=np.uint32)
    args = [N, V, _p(views_array(cameras)), st.tile_w, st.tile_h, _p(np.ascontiguousarray(tile_rect, np.int32)),
            _p(tiles_touched), _p(_rec11(rec, VN)), _p(_perr(perr, VN))]
    lib().orc_bin_band.restype = ctypes.c_long
    cap = 1 << 16
    while True:
        pair = np.zeros(cap, np.uint32)
        tile = np.zeros(cap, np.uint32)
        listed = np.zeros(cap, np.uint8)
        n = int(lib().orc_bin_band(*args, ctypes.c_long(cap), _p(pair), _p(tile), _p(listed))) if VN else 0
        if n <= cap:
            return dict(pair=pair[:n], tile=tile[:n], listed=listed[:n].astype(bool))
        cap = n


def instance_status(N, cameras, tile_rect, rec, vals, tiles, st: Settings, perr=None) -> np.ndarray:
    """Per listed instance (pair vals[k], global tile tiles[k]): 0 listed with
    certainty under the footprint rule, 1 within the float32 band, 2 not
    listed with certainty, 3 outside the pair's view or tile rectangle."""
    V = len(cameras)
    vals = np.ascontiguousarray(vals, np.uint32)
    L = vals.size
    out = np.zeros(max(L, 1), np.uint8)
    if L:
        lib().orc_instance_status(N, V, _p(views_array(cameras)), st.tile_w, st.tile_h,
                                  _p(np.ascontiguousarray(tile_rect, np.int32)), _p(_rec11(rec, V * N)),
                                  _p(_perr(perr, V * N)), ctypes.c_long(L), _p(vals),
                                  _p(np.ascontiguousarray(tiles, np.uint32)), _p(out))
    return out[:L]


def fragment_band(rec, px, py, st: Settings, perr=None):
    """(o G, band) of fragments: record rec[k] ([n, 11]) at pixel centre
    (px[k], py[k]); band bounds |d ln(o G)| of a float32 evaluation (see
    frag_band in the C++ source)."""
    rec = _f64(np.asarray(rec, np.float64).reshape(-1, 11))
    n = rec.shape[0]
    oG, band = np.zeros(max(n, 1)), np.zeros(max(n, 1))
    lib().orc_fragment_band(ctypes.c_long(n), _p(rec), _p(_f64(px)), _p(_f64(py)), _p(st.array()),
                            _p(_perr(perr, n)), _p(oG), _p(band))
    return oG[:n], band[:n]


def render_fwd(N, cameras, rec, vals, ranges, st: Settings, depth=None, perr=None, paths=None) -> dict:
    """Tiled forward; with `depth` ([V*N] splat depths) also the extended
    channels "depth" (sum alpha T z) and "alpha" (sum alpha T).  perr: end-to-end
    record error bounds that widen the decision bands (nullable); paths: the
    decision path of each pixel (nullable: the plain FP64 result)."""
    P = sum(c.width * c.height for c in cameras)
    V = len(cameras)
    out = dict(image=np.zeros(3 * P), final_T=np.zeros(P), n_contrib=np.zeros(P, np.uint32),
               n_listed=np.zeros(P, np.uint32), n_hit=np.zeros(P, np.uint32), ambig=np.zeros(P, np.uint8),
               n_branch=np.zeros(P, np.uint8), last=np.zeros(P, np.int64))
    if depth is not None:
        out["depth"], out["alpha"] = np.zeros(P), np.zeros(P)
    vals = np.ascontiguousarray(vals, np.uint32)
    if vals.size == 0:
        vals = np.zeros(1, np.uint32)
    lib().orc_render_fwd(N, V, _p(views_array(cameras)), _p(st.array()), _p(_f64(rec)), _p(vals),
                         _p(np.ascontiguousarray(ranges, np.uint32)), _p(_perr(perr, V * N)),
                         _p(None if paths is None else np.ascontiguousarray(paths, np.uint32)),
                         _p(out["image"]), _p(out["final_T"]),
                         _p(out["n_contrib"]), _p(out["n_listed"]), _p(out["n_hit"]), _p(out["ambig"]),
                         _p(out["n_branch"]), _p(out["last"]), _p(None if depth is None else _f64(depth)),
                         _p(out.get("depth")),
                         _p(out.get("alpha")))
    return out


def resolve(N, cameras, rec, vals, ranges, st: Settings, image, final_T, last, n_hit=None, perr=None,
            tol: float = 1e-4, tol_T: float = 1e-4, max_leaves: int = 64, n_listed=None):
    """Decision paths that reproduce a float32 rasterizer's per-pixel result
    (image, final_T, the record index of the last composited fragment `last`
    (-1 if none), optional n_hit and n_listed (entries 0xFFFFFFFF not compared))
    among the oracle's own correct results (see orc_resolve).  The colour tolerance of view v is
    tol * max(max |C| of the oracle's plain image of v, 1).  Returns (paths,
    status, plain): per pixel the path and its status (0 unique, 1 resolved, 2
    alpha-cap band, 3 too many paths, 4 no match), and the oracle's plain
    (path 0) forward."""
    V = len(cameras)
    P = sum(c.width * c.height for c in cameras)
    plain = render_fwd(N, cameras, rec, vals, ranges, st, perr=perr)
    tv, off = np.zeros(V), 0
    for v, c in enumerate(cameras):
        n = 3 * c.width * c.height
        tv[v] = tol * max(np.abs(plain["image"][off:off + n]).max(initial=0.0), 1.0)
        off += n
    paths = np.zeros(max(P, 1), np.uint32)
    status = np.zeros(max(P, 1), np.uint8)
    vals = np.ascontiguousarray(vals, np.uint32)
    if vals.size == 0:
        vals = np.zeros(1, np.uint32)
    lib().orc_resolve(N, V, _p(views_array(cameras)), _p(st.array()), _p(_f64(rec)), _p(vals),
                      _p(np.ascontiguousarray(ranges, np.uint32)), _p(_perr(perr, V * N)),
                      _p(np.ascontiguousarray(image, np.float32)), _p(np.ascontiguousarray(final_T, np.float32)),
                      _p(np.ascontiguousarray(last, np.int64)),
                      _p(None if n_hit is None else np.ascontiguousarray(n_hit, np.uint32)),
                      _p(None if n_listed is None else np.ascontiguousarray(n_listed, np.uint32)), _p(tv),
                      ctypes.c_double(tol_T), int(max_leaves), _p(paths), _p(status))
    return paths[:P], status[:P], plain


def brute_fwd(N, cameras, rec, zbits, cull, st: Settings, pix_rect=None, window=None) -> dict:
    P = sum(c.width * c.height for c in cameras)
    out = dict(image=np.zeros(3 * P), final_T=np.ones(P), n_hit=np.zeros(P, np.uint32), ambig=np.zeros(P, np.uint8))
    lib().orc_brute_fwd(N, len(cameras), _p(views_array(cameras)), _p(st.array()), _p(_f64(rec)),
                        _p(np.ascontiguousarray(zbits, np.uint32)), _p(np.ascontiguousarray(cull, np.uint8)),
                        _p(None if pix_rect is None else np.ascontiguousarray(pix_rect, np.int32)),
                        _p(None if window is None else np.ascontiguousarray(window, np.int32)),
                        _p(out["image"]), _p(out["final_T"]), _p(out["n_hit"]), _p(out["ambig"]))
    return out


def render_bwd(N, cameras, rec, vals, ranges, dL_dimage, st: Settings, depth=None, dL_ddepth=None,
               dL_dalpha=None, perr=None, paths=None) -> np.ndarray:
    """grad2d [V*N, 11]: du, dv, dA, dB, dC, dopacity, dbeta, dr, dg, db, dz (dz
    only from the extended channels, which need `depth`); each pixel follows
    its decision path (paths nullable, perr as in render_fwd)."""
    V = len(cameras)
    g2 = np.zeros((V * N, 11))
    vals = np.ascontiguousarray(vals, np.uint32)
    if vals.size == 0:
        vals = np.zeros(1, np.uint32)
    lib().orc_render_bwd(N, V, _p(views_array(cameras)), _p(st.array()), _p(_f64(rec)), _p(vals),
                         _p(np.ascontiguousarray(ranges, np.uint32)), _p(_perr(perr, V * N)),
                         _p(None if paths is None else np.ascontiguousarray(paths, np.uint32)), _p(_f64(dL_dimage)),
                         _p(None if depth is None else _f64(depth)),
                         _p(None if dL_ddepth is None else _f64(dL_ddepth)),
                         _p(None if dL_dalpha is None else _f64(dL_dalpha)), _p(g2))
    return g2


def window_fwdbwd(N, cameras, rec, zbits, cull, pix_rect, window, dL_dimage, watch, st: Settings, depth=None,
                  dL_ddepth=None, dL_dalpha=None):
    """(sum_window dL.image [+ dL_ddepth.depth + dL_dalpha.alpha], grad2d rows
    (11 columns) of `watch`, decision hash)."""
    watch = np.ascontiguousarray(watch, dtype=np.int64)
    loss = ctypes.c_double(0.0)
    dec = ctypes.c_uint64(0)
    wg = np.zeros((max(len(watch), 1), 11))
    lib().orc_window_fwdbwd(N, len(cameras), _p(views_array(cameras)), _p(st.array()), _p(_f64(rec)),
                            _p(np.ascontiguousarray(zbits, np.uint32)), _p(np.ascontiguousarray(cull, np.uint8)),
                            _p(np.ascontiguousarray(pix_rect, np.int32)),
                            _p(np.ascontiguousarray(window, np.int32)), _p(_f64(dL_dimage)),
                            _p(None if depth is None else _f64(depth)),
                            _p(None if dL_ddepth is None else _f64(dL_ddepth)),
                            _p(None if dL_dalpha is None else _f64(dL_dalpha)), len(watch),
                            _p(watch), ctypes.byref(loss), _p(wg), ctypes.byref(dec))
    return loss.value, wg[:len(watch)], dec.value


def project_bwd(scene, grad2d, st: Settings) -> dict:
    """grad2d [V*N, 10 or 11] (a missing dz column is zero) -> parameter gradients."""
    N, V = scene.n, scene.n_views
    grad2d = np.asarray(grad2d, np.float64)
    if grad2d.shape[1] == 10:
        grad2d = np.concatenate([grad2d, np.zeros((grad2d.shape[0], 1))], axis=1)
    K = (st.sh_degree + 1) ** 2
    g = dict(means=np.zeros((N, 3)), scales=np.zeros((N, 3)), quats=np.zeros((N, 4)), opacities=np.zeros(N),
             betas=np.zeros(N), sh=np.zeros((N, K, 3)))
    lib().orc_project_bwd(N, V, _p(_f64(scene.means)), _p(_f64(scene.scales)), _p(_f64(scene.quats)),
                          _p(_f64(scene.opacities)), _p(_f64(scene.betas)), _p(_f64(scene.sh.reshape(N, int(np.prod(scene.sh.shape[1:]))))),
                          _p(views_array(scene.cameras)), _p(st.array()), _p(_f64(grad2d)),
                          _p(g["means"]), _p(g["scales"]), _p(g["quats"]), _p(g["opacities"]), _p(g["betas"]),
                          _p(g["sh"]))
    return g


def surface_points(scene, rec, vals, ranges, depth_map, alpha_map, pixels, st: Settings, n_samples: int = 32,
                   level: float = 0.3, span: float = 3.0, min_alpha: float = 0.5) -> dict:
    """Level-set surface points along the rays of `pixels` (global pixel ids):
    points [R, 3], normals [R, 3], valid [R], dominant [R] (pair index of g or
    -1), t_star [R], margins [R, 3] (see orc_surface_points)."""
    N, V = scene.n, scene.n_views
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    R = len(pixels)
    out = dict(points=np.zeros((max(R, 1), 3)), normals=np.zeros((max(R, 1), 3)), valid=np.zeros(max(R, 1), np.int32),
               dominant=np.zeros(max(R, 1), np.int64), t_star=np.zeros(max(R, 1)), margins=np.zeros((max(R, 1), 3)))
    vals = np.ascontiguousarray(vals, np.uint32)
    if vals.size == 0:
        vals = np.zeros(1, np.uint32)
    lib().orc_surface_points(N, V, _p(_f64(scene.means)), _p(_f64(scene.scales)), _p(_f64(scene.quats)),
                             _p(_f64(scene.opacities)), _p(_f64(scene.betas)), _p(views_array(scene.cameras)),
                             _p(st.array()), _p(_f64(rec)), _p(vals), _p(np.ascontiguousarray(ranges, np.uint32)),
                             _p(_f64(depth_map)), _p(_f64(alpha_map)), _p(pixels), ctypes.c_long(R), int(n_samples),
                             ctypes.c_double(level), ctypes.c_double(span), ctypes.c_double(min_alpha),
                             _p(out["points"]), _p(out["normals"]), _p(out["valid"]), _p(out["dominant"]),
                             _p(out["t_star"]), _p(out["margins"]))
    return {k: v[:R] for k, v in out.items()}


def knn(means, K: int = 16) -> np.ndarray:
    """Neighbour lists [N, K] (int32): slot 0 = the splat itself, then its
    K - 1 nearest other centres by (squared distance, index); -1 pads when
    N < K (see orc_knn)."""
    means = _f64(means).reshape(-1, 3)
    N = means.shape[0]
    out = np.zeros((max(N, 1), K), np.int32)
    lib().orc_knn(int(N), _p(means), int(K), _p(out))
    return out[:N]


def gsr(scene, st: Settings, nbrs, xi, mask=None, w_sdf: float = 1.0, w_nor: float = 1.0,
        grads: bool = True) -> dict:
    """Surface regulariser of Sec. 3.3 (Eq. 9-13) on one sample per splat
    (see orc_gsr for the readings).  scene: any object with means, scales,
    quats, opacities, betas (activated, float64-promotable); nbrs [N, K];
    xi [N, 3]; mask [N] (nullable).  Returns per-sample l_sdf, l_nor, gstar
    (slot), margins [N, 7] and, when `grads`, the gradients of
    sum_j mask_j (w_sdf l_sdf + w_nor l_nor) as means/scales/quats/opacities/betas."""
    means = _f64(scene.means).reshape(-1, 3)
    N = means.shape[0]
    nbrs = np.ascontiguousarray(nbrs, np.int32).reshape(N, -1)
    K = nbrs.shape[1]
    out = dict(l_sdf=np.zeros(max(N, 1)), l_nor=np.zeros(max(N, 1)), gstar=np.zeros(max(N, 1), np.int32),
               margins=np.zeros((max(N, 1), 7)))
    g = np.zeros((max(N, 1), 12)) if grads else None
    m = None if mask is None else np.ascontiguousarray(mask, np.uint8)
    lib().orc_gsr(int(N), _p(means), _p(_f64(scene.scales).reshape(-1, 3)), _p(_f64(scene.quats).reshape(-1, 4)),
                  _p(_f64(scene.opacities)), _p(_f64(scene.betas)), _p(st.array()), int(K), _p(nbrs),
                  _p(_f64(xi).reshape(-1, 3)), _p(m), ctypes.c_double(w_sdf), ctypes.c_double(w_nor),
                  _p(out["l_sdf"]), _p(out["l_nor"]), _p(out["gstar"]), _p(out["margins"]), _p(g))
    res = {k: v[:N] for k, v in out.items()}
    if grads:
        g = g[:N]
        res["grads"] = dict(means=g[:, 0:3], scales=g[:, 3:6], quats=g[:, 6:10], opacities=g[:, 10],
                            betas=g[:, 11])
    return res


def sh_basis(degree: int, dirs) -> np.ndarray:
    dirs = _f64(dirs)
    n = dirs.shape[0]
    out = np.zeros((n, (degree + 1) ** 2))
    lib().orc_sh_basis(degree, ctypes.c_long(n), _p(dirs), _p(out))
    return out


def set_threads(n: int):
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------- optimiser
@dataclass
class AdamSettings:
    """Per-group learning rates (3DGS practice, which Sec. 4.2 defers to, and
    the paper's 1.5e-3 for the shape parameter), Adam's constants and the
    weight of the opacity-entropy term (Sec. 4.2: binary opacities)."""
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


RAW_KEYS = ("means", "log_scales", "quats", "opacity_logits", "betas", "sh")


def adam_raw_grads(raw: dict, grads: dict, st: AdamSettings) -> dict:
    """Gradients of the optimised (raw) parameters from those of the activated
    ones: scale = exp(log_scale), opacity = sigmoid(logit), plus the opacity
    entropy term entropy_weight * mean_i H(o_i), H(o) = -o ln o - (1-o) ln(1-o),
    whose derivative in the logit is -logit o (1 - o)."""
    s = np.exp(np.asarray(raw["log_scales"], np.float64))
    lg = np.asarray(raw["opacity_logits"], np.float64)
    o = 1.0 / (1.0 + np.exp(-lg))
    n = max(len(lg), 1)
    g = {"means": np.asarray(grads["means"], np.float64), "quats": np.asarray(grads["quats"], np.float64),
         "betas": np.asarray(grads["betas"], np.float64), "sh": np.asarray(grads["sh"], np.float64)}
    g["log_scales"] = np.asarray(grads["scales"], np.float64) * s
    g["opacity_logits"] = (np.asarray(grads["opacities"], np.float64) * o * (1 - o)
                           + st.entropy_weight / n * (-lg) * o * (1 - o))
    return g


def adam_step(raw: dict, m: dict, v: dict, grads: dict, step: int, st: AdamSettings):
    """One Adam step (bias-corrected, step >= 1) of every raw parameter group
    with its learning rate; returns (raw, m, v, activated) with activated =
    dict(scales=exp(log_scales), opacities=sigmoid(logits))."""
    g = adam_raw_grads(raw, grads, st)
    lrs = {"means": st.lr_mean, "log_scales": st.lr_scale, "quats": st.lr_quat, "opacity_logits": st.lr_opacity,
           "betas": st.lr_beta}
    c1 = 1.0 - st.beta1 ** step
    c2 = 1.0 - st.beta2 ** step
    out_p, out_m, out_v = {}, {}, {}
    for k in RAW_KEYS:
        p = np.asarray(raw[k], np.float64)
        mk = st.beta1 * np.asarray(m[k], np.float64) + (1 - st.beta1) * g[k]
        vk = st.beta2 * np.asarray(v[k], np.float64) + (1 - st.beta2) * g[k] ** 2
        if k == "sh":
            lr = np.full(p.shape, st.lr_sh_rest)
            lr[:, 0, :] = st.lr_sh_dc
        else:
            lr = lrs[k]
        out_p[k] = p - lr * (mk / c1) / (np.sqrt(vk / c2) + st.eps)
        out_m[k], out_v[k] = mk, vk
    act = {"scales": np.exp(out_p["log_scales"]), "opacities": 1.0 / (1.0 + np.exp(-out_p["opacity_logits"]))}
    return out_p, out_m, out_v, act


def prune_keep(raw: dict, min_opacity: float, min_beta: float) -> np.ndarray:
    """Keep mask of the pruning rule (Sec. 4.2: opacity below 0.5 removed; the
    shape threshold read as a lower bound on beta).  The opacity test is
    taken on the float32 logit against the float32 value of
    ln(min_opacity / (1 - min_opacity)), the same comparison the GPU makes;
    a threshold of 0 disables its test."""
    lg = np.asarray(raw["opacity_logits"], np.float32)
    keep = np.ones(lg.shape[0], bool)
    if min_opacity > 0:
        keep &= lg >= np.float32(np.log(np.float64(np.float32(min_opacity)) / (1.0 - np.float64(np.float32(min_opacity)))))
    if min_beta > 0:
        keep &= np.asarray(raw["betas"], np.float32) >= np.float32(min_beta)
    return keep


def prune(raw: dict, m: dict, v: dict, min_opacity: float, min_beta: float):
    """The kept splats of raw (and of the moments m, v when given), in order."""
    keep = prune_keep(raw, min_opacity, min_beta)
    sel = lambda d: None if d is None else {k: np.asarray(d[k])[keep] for k in RAW_KEYS}  # noqa: E731
    return sel(raw), sel(m), sel(v), keep


def shape_reset(raw: dict, m: dict, v: dict, value: float):
    """Shape reset (Sec. 4.2, every 1000 iterations), read as beta := value for
    every splat with beta's moments zeroed."""
    out = [None if d is None else {k: np.array(d[k], copy=True) for k in RAW_KEYS} for d in (raw, m, v)]
    out[0]["betas"][:] = value
    for d in out[1:]:
        if d is not None:
            d["betas"][:] = 0.0
    return tuple(out)


# ------------------------------------------------------- photometric loss (Eq. 8)
@dataclass
class LossSettings:
    """Eq. 8: L = (1 - lambda) L1 + lambda L_SSIM with L_SSIM = 1 - SSIM (Sec. 3.2;
    lambda = 0.2).  SSIM's window and constants are not given in the paper;
    the reading is the usual one: an 11 x 11 Gaussian window of standard
    deviation 1.5, C1 = 0.01^2, C2 = 0.03^2 (images in [0, 1]), zero padding,
    the map averaged over channels and pixels."""
    lam: float = 0.2
    c1: float = 0.01 ** 2
    c2: float = 0.03 ** 2
    sigma: float = 1.5
    radius: int = 5


def gaussian_window(radius: int, sigma: float) -> np.ndarray:
    """Normalised 1-D Gaussian weights at offsets -radius..radius."""
    x = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    return g / g.sum()


def window_sum(a, g1) -> np.ndarray:
    """sum_{i,j} g1[i] g1[j] a[y + i - r, x + j - r] over the window, with
    zero outside the image (r = radius); the window is symmetric, so this is
    also its own adjoint."""
    a = np.asarray(a, np.float64)
    r = (len(g1) - 1) // 2
    H, W = a.shape
    p = np.zeros((H + 2 * r, W + 2 * r))
    p[r:r + H, r:r + W] = a
    out = np.zeros((H, W))
    for i in range(2 * r + 1):
        for j in range(2 * r + 1):
            out += (g1[i] * g1[j]) * p[i:i + H, j:j + W]
    return out


def ssim_terms(X, Y, ls: LossSettings):
    """Per-pixel SSIM map of two single-channel images and its partial
    derivatives with respect to the window moments mu_x = G*X, m2x = G*X^2,
    mxy = G*(X Y): S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)
    (s_x^2 + s_y^2 + C2)) with s_x^2 = m2x - mu_x^2, s_xy = mxy - mu_x mu_y."""
    g1 = gaussian_window(ls.radius, ls.sigma)
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    mx, my = window_sum(X, g1), window_sum(Y, g1)
    sxx = window_sum(X * X, g1) - mx * mx
    syy = window_sum(Y * Y, g1) - my * my
    sxy = window_sum(X * Y, g1) - mx * my
    N1, N2 = 2 * mx * my + ls.c1, 2 * sxy + ls.c2
    D1, D2 = mx * mx + my * my + ls.c1, sxx + syy + ls.c2
    S = N1 * N2 / (D1 * D2)
    # dS/dmu_x (through mu_x, s_x^2 and s_xy), dS/dm2x, dS/dmxy
    d_m1 = 2 * my * N2 / (D1 * D2) - 2 * mx * S / D1 + 2 * mx * S / D2 - 2 * my * N1 / (D1 * D2)
    d_m2 = -S / D2
    d_mxy = 2 * N1 / (D1 * D2)
    return S, d_m1, d_m2, d_mxy, g1


def photometric_loss(image, target, cameras, ls: LossSettings = LossSettings()):
    """Eq. 8 per view, images in the flat CHW-per-view layout: returns
    (loss [V], dL/dimage) with L = sum_v L_v, L_v = (1 - lambda) mean|X - Y| +
    lambda (1 - mean SSIM) over the view's 3 H W values (sign(0) = 0)."""
    image = np.asarray(image, np.float64)
    target = np.asarray(target, np.float64)
    loss = np.zeros(len(cameras))
    grad = np.zeros_like(image)
    off = 0
    for v, c in enumerate(cameras):
        n = 3 * c.width * c.height
        X = image[off:off + n].reshape(3, c.height, c.width)
        Y = target[off:off + n].reshape(3, c.height, c.width)
        G = np.zeros_like(X)
        ssim_sum = 0.0
        for ch in range(3):
            S, a, b, cc, g1 = ssim_terms(X[ch], Y[ch], ls)
            ssim_sum += S.sum()
            # L_SSIM = 1 - mean S: the moments' adjoint, each a window sum
            dS = window_sum(a, g1) + 2 * X[ch] * window_sum(b, g1) + Y[ch] * window_sum(cc, g1)
            G[ch] = (1 - ls.lam) * np.sign(X[ch] - Y[ch]) / n - ls.lam * dS / n
        loss[v] = (1 - ls.lam) * np.abs(X - Y).sum() / n + ls.lam * (1.0 - ssim_sum / n)
        grad[off:off + n] = G.reshape(-1)
        off += n
    return loss, grad


# ------------------------------------------------ surface-alignment regulariser
def rotation_columns(quats):
    """Rotation matrices [N, 3, 3] of quaternions (w, x, y, z), normalised."""
    q = np.asarray(quats, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
                     np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
                     np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)], 1)


def surface_alignment(scales, quats, normals, w_scale: float = 0.1, w_normal: float = 0.1):
    """Surface-alignment regulariser of the flattened-splat workload (the paper
    flattens its splats toward the surface, Sec. 3.3, without giving this loss;
    reading): L = w_scale mean_i min_k s_ik + w_normal mean_i (1 - <n_i, m_i>^2)
    with n_i = R(q_i) e_k*, k* = the axis of the smallest scale (lowest index on
    ties) and m_i the splat's true surface normal (sign-free).  Returns
    (L_scale, L_normal, dict(scales, quats) of dL/d(scales, raw quats)), the
    discrete choice k* held fixed."""
    s = np.asarray(scales, np.float64)
    q = np.asarray(quats, np.float64)
    m = np.asarray(normals, np.float64)
    N = s.shape[0]
    k = np.argmin(s, axis=1)
    idx = np.arange(N)
    R = rotation_columns(q)
    n = R[idx, :, k]
    d = np.einsum("ij,ij->i", n, m)
    L_s = w_scale * s[idx, k].sum() / max(N, 1)
    L_n = w_normal * (1.0 - d * d).sum() / max(N, 1)
    gs = np.zeros_like(s)
    gs[idx, k] = w_scale / max(N, 1)
    gn = (-2.0 * w_normal / max(N, 1)) * d[:, None] * m  # dL/dn
    # column k of R as a function of the normalised quaternion (w, x, y, z)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = qn.T
    zero = np.zeros(N)
    J = np.empty((N, 3, 4))  # d column / d (w, x, y, z)
    J0 = np.stack([np.stack([zero, zero, -4 * y, -4 * z], 1), np.stack([2 * z, 2 * y, 2 * x, 2 * w], 1),
                   np.stack([-2 * y, 2 * z, -2 * w, 2 * x], 1)], 1)
    J1 = np.stack([np.stack([-2 * z, 2 * y, 2 * x, -2 * w], 1), np.stack([zero, -4 * x, zero, -4 * z], 1),
                   np.stack([2 * x, 2 * w, 2 * z, 2 * y], 1)], 1)
    J2 = np.stack([np.stack([2 * y, 2 * z, 2 * w, 2 * x], 1), np.stack([-2 * x, -2 * w, 2 * z, 2 * y], 1),
                   np.stack([zero, -4 * x, -4 * y, zero], 1)], 1)
    for kk, Jk in enumerate((J0, J1, J2)):
        J[k == kk] = Jk[k == kk]
    g_qn = np.einsum("ij,ijk->ik", gn, J)
    # through the normalisation q -> q / |q|
    nq = np.linalg.norm(q, axis=1, keepdims=True)
    g_q = (g_qn - np.einsum("ij,ij->i", g_qn, qn)[:, None] * qn) / nq
    return L_s, L_n, dict(scales=gs, quats=g_q)


# ------------------------------------------------------------------ pipeline
def forward(scene, st: Settings, channels: bool = False, band: bool = False, paths=None) -> dict:
    """Full FP64 pipeline: project -> bin -> tiled render (with the extended
    depth and alpha channels when `channels`).  With `band`, the decision bands
    also cover the a-priori error of a float32 projection's records
    (record_err_bound, kept as "perr") for comparisons with a float32 pipeline
    run from the same parameters.  paths: per-pixel decision paths (nullable)."""
    pr = project(scene, st)
    keys, vals, ranges = bin_instances(scene.n, scene.cameras, pr["tile_rect"], pr["tiles_touched"], pr["zbits"], st,
                                       pr["rec"])
    perr = record_err_bound(scene, st) if band else None
    out = render_fwd(scene.n, scene.cameras, pr["rec"], vals, ranges, st, depth=pr["depth"] if channels else None,
                     perr=perr, paths=paths)
    out.update(proj=pr, keys=keys, vals=vals, ranges=ranges, perr=perr)
    return out


def backward(scene, st: Settings, fwd: dict, dL_dimage, dL_ddepth=None, dL_dalpha=None, paths=None) -> dict:
    """Adjoint of `forward` (each pixel follows its decision path; paths nullable)."""
    ext = dL_ddepth is not None or dL_dalpha is not None
    g2 = render_bwd(scene.n, scene.cameras, fwd["proj"]["rec"], fwd["vals"], fwd["ranges"], dL_dimage, st,
                    depth=fwd["proj"]["depth"] if ext else None, dL_ddepth=dL_ddepth, dL_dalpha=dL_dalpha,
                    perr=fwd.get("perr"), paths=paths)
    g = project_bwd(scene, g2, st)
    g["grad2d"] = g2
    return g


def flat_images(images) -> np.ndarray:
    """Concatenate per-view (3, H, W) arrays in the oracle's view-major CHW layout."""
    return np.concatenate([np.asarray(im, dtype=np.float64).reshape(-1) for im in images])


def split_images(flat, cameras):
    out, off = [], 0
    for c in cameras:
        n = 3 * c.width * c.height
        out.append(np.asarray(flat[off:off + n]).reshape(3, c.height, c.width))
        off += n
    return out
