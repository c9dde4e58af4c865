"""GPU parity of every hot-path stage against the FP64 oracle.

Stage tests feed the oracle the GPU's own inputs for that stage (so a
disagreement is the stage's own), then an end-to-end test compares the whole
GPU pipeline with the oracle run from the splat parameters.

Bars (derived in the design notes):
  * binning: bit-exact keys, values, ranges, instance count and instance bases;
  * images / final_T: max error <= 1e-4 * max(max|C|, 1) on pixels that are not
    ambiguous, and relative L2 <= 1e-4 over all pixels; n_contrib and the
    fragment counts exact on non-ambiguous pixels.  A pixel is ambiguous when
    one of its fragments lies within the float32 error band of alpha_min,
    alpha_max or t_min (1e-5 relative when both sides share the GPU's records;
    end to end the band adds the first-order effect of float32 centre and
    conic error), or, end to end, when compositing the GPU's tile list instead
    of the oracle's changes the oracle's own result at that pixel;
  * gradients: per tensor, inf-norm and 2-norm of the error <= 1e-3 of the
    reference's norms, for the same seeded upstream dL/dimage on both sides,
    zeroed at ambiguous pixels (a threshold flip there is a legitimate
    difference, not an error).
"""
import functools

import numpy as np
import pytest

import gesr_inputs as gi
import oracle
from tests.gpu_util import (check_projection, conic_grads_to_factor, e2e_settings, factor_grads_to_conic,
                            image_errors, log, mask_upstream, norm_errors, oracle_rec, run_gpu, run_gpu_bwd)

pytestmark = pytest.mark.gpu


def _case(name):
    """(scene, oracle settings) of a named parity case; the suffix "-v1" selects the
    four-waves-per-tile renderers instead of the one-wave-per-tile ones."""
    if name.endswith("-v1"):
        return _case(name[:-3])
    if name == "tiny-d1":
        return gi.tiny_scene(0, n=12, deg=1), oracle.Settings(sh_degree=1)
    if name == "tiny-d3-2v-bg":
        return gi.tiny_scene(2, n=30, deg=3, n_views=2), oracle.Settings(sh_degree=3, bg=(0.2, 0.5, 0.1))
    if name == "tiny-kappa1":
        return gi.tiny_scene(3, n=20, deg=2, beta=(0.7, 4.5)), oracle.Settings(sh_degree=2, kappa=1.0)
    if name == "plain-2k":
        return gi.make_workload(1), oracle.Settings()
    if name == "plain-2k-t8":
        return gi.make_workload(1), oracle.Settings(tile_w=8, tile_h=8)
    if name == "plain-2k-t32x16":
        return gi.make_workload(1), oracle.Settings(tile_w=32, tile_h=16)
    if name == "plain-2k-t32":
        return gi.make_workload(1), oracle.Settings(tile_w=32, tile_h=32)
    if name == "spheres-100k":
        return gi.make_workload(2), oracle.Settings(sh_degree=3)
    if name == "drt-50k-8v":
        return gi.make_workload(3, n_override=50_000), oracle.Settings()
    if name == "surfels-40k-2v":
        return gi.make_workload(4, n_override=40_000, views_override=2), oracle.Settings(sh_degree=3)
    if name == "wide-2200x2100":  # > 16k tiles in one view: global counting-grid path
        return gi.tiny_scene(8, n=300, deg=1, width=2200, height=2100, log_scale=(-3.5, -2.5)), \
            oracle.Settings(sh_degree=1)
    if name == "ragged-5v":  # 1x1, 1x37, 23x1, 17x33 and 129x65 views
        return gi.ragged_scene(0), oracle.Settings(sh_degree=2)
    if name == "ragged-5v-t8":
        return gi.ragged_scene(0), oracle.Settings(sh_degree=2, tile_w=8, tile_h=8)
    if name == "blobs-100k-2v":
        return gi.make_workload(5, n_override=100_000, views_override=2), oracle.Settings(sh_degree=3)
    raise KeyError(name)


CASES = ["tiny-d1", "tiny-d3-2v-bg", "tiny-kappa1", "ragged-5v", "ragged-5v-t8", "plain-2k", "plain-2k-v1",
         "plain-2k-t8", "plain-2k-t32x16", "plain-2k-t32", "spheres-100k", "drt-50k-8v", "drt-50k-8v-v1",
         "surfels-40k-2v", "blobs-100k-2v", "wide-2200x2100"]


@functools.lru_cache(maxsize=1)
def _run(name):
    scene, st = _case(name)
    log(f"[gpu] case {name}: n={scene.n} views={scene.n_views} px={scene.n_pixels}")
    g = run_gpu(scene, st, variant=1 if name.endswith("-v1") else 0)
    log(f"[gpu] case {name}: forward done, M={g['M']}")
    return scene, st, g


@functools.lru_cache(maxsize=1)
def _same_inputs(name):
    """Oracle fed the GPU's records and lists; gradients for an upstream dL that
    is zero at pixels whose decisions are ambiguous (identical on both sides)."""
    scene, st, g = _run(name)
    rec = oracle_rec(g["rec"])
    fwd = oracle.render_fwd(scene.n, scene.cameras, rec, g["val_sorted"], g["ranges"], st)
    dL = mask_upstream(oracle.flat_images(gi.upstream_grads(scene, 7)), fwd["ambig"] > 0, scene.cameras)
    log(f"[gpu] case {name}: backward (same inputs)")
    gb = run_gpu_bwd(scene, st, g, dL)
    g2 = oracle.render_bwd(scene.n, scene.cameras, rec, g["val_sorted"], g["ranges"], dL, st)
    return rec, fwd, dL, gb, g2


@functools.lru_cache(maxsize=1)
def _end_to_end(name):
    """Oracle run from the parameters.  Ambiguous pixels: a fragment inside the
    float32 band of a threshold, or a pixel whose oracle result changes when
    the oracle composites the GPU's tile lists instead of its own (the lists
    differ only at guard bands of the rectangles and depth keys)."""
    scene, st, g = _run(name)
    se = e2e_settings(st, scene.cameras)
    fo = oracle.forward(scene, se)
    fl = oracle.render_fwd(scene.n, scene.cameras, fo["proj"]["rec"], g["val_sorted"], g["ranges"], se)
    P = scene.n_pixels
    changed = (fl["image"] != fo["image"]).reshape(-1)
    list_amb = np.zeros(P, bool)
    off_i = off_p = 0
    for c in scene.cameras:
        n = c.width * c.height
        list_amb[off_p:off_p + n] = changed[off_i:off_i + 3 * n].reshape(3, n).any(0)
        off_i += 3 * n
        off_p += n
    list_amb |= fl["final_T"] != fo["final_T"]
    amb = (fo["ambig"] > 0) | (fl["ambig"] > 0) | list_amb
    dL = mask_upstream(oracle.flat_images(gi.upstream_grads(scene, 7)), amb, scene.cameras)
    log(f"[gpu] case {name}: backward (end to end); pixels changed by the GPU lists {int(list_amb.sum())}")
    gb = run_gpu_bwd(scene, st, g, dL)
    go = oracle.backward(scene, se, fo, dL)
    return fo, amb, dL, gb, go


@pytest.mark.parametrize("name", CASES)
def test_project(name):
    scene, st, g = _run(name)
    stats = check_projection(scene, g, oracle.project(scene, st))
    log(f"[gpu] {name}: project ok; {stats}")


@pytest.mark.parametrize("name", CASES)
def test_bin_bit_exact(name):
    """Oracle binning of the GPU's own per-splat results (record, rect, depth
    key) equals the GPU's sorted instance list, ranges, counts and instance
    bases exactly (each rectangle row's columns decided in float32 from the
    record on both sides)."""
    scene, st, g = _run(name)
    keys, vals, ranges = oracle.bin_instances(scene.n, scene.cameras, g["tile_rect"], g["tiles_touched"],
                                              g["depth_key"], st, g["rec"])
    assert g["overflow"] == 0
    assert g["M"] == int(g["tiles_touched"].astype(np.int64).sum()) >= g["listed"]
    assert g["listed"] == len(vals)
    np.testing.assert_array_equal(g["val_sorted"], vals)
    np.testing.assert_array_equal(g["tile_sorted"].astype(np.uint64), keys >> np.uint64(32))
    np.testing.assert_array_equal(g["depth_key"][g["val_sorted"]].astype(np.uint64), keys & np.uint64(0xFFFFFFFF))
    np.testing.assert_array_equal(g["ranges"], ranges)
    # worklist: every tile once, by decreasing list length, ties by tile id
    lens = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    expect = np.lexsort((np.arange(len(lens)), -np.minimum(lens, 0xFFFF)))
    np.testing.assert_array_equal(g["worklist"], expect)
    # instance slots: exclusive scan of tiles_touched in pair order
    base = np.concatenate([[0], np.cumsum(g["tiles_touched"].astype(np.int64))[:-1]])
    np.testing.assert_array_equal(g["inst_base"], base)


@pytest.mark.parametrize("name", CASES)
def test_render_fwd_same_inputs(name):
    scene, st, g = _run(name)
    rec, fwd, dL, gb, g2 = _same_inputs(name)
    amb = fwd["ambig"] > 0
    errs = image_errors(g["image"], fwd["image"], amb, scene.cameras)
    for bad, mx, bound, l2 in errs:
        assert bad == 0 and l2 <= 1e-4, errs
    ok = ~amb
    assert np.abs(g["final_T"][ok] - fwd["final_T"][ok]).max() <= 1e-4
    np.testing.assert_array_equal(g["n_contrib"][ok], fwd["n_contrib"][ok])
    np.testing.assert_array_equal(g["n_listed"][ok], fwd["n_listed"][ok])
    np.testing.assert_array_equal(g["n_hit"][ok], fwd["n_hit"][ok])
    log(f"[gpu] {name}: fwd ok; ambiguous px {int(amb.sum())}/{amb.size}; max err "
        f"{max(e[1] for e in errs):.2e}; listed/px {fwd['n_listed'].mean():.1f} hit/px {fwd['n_hit'].mean():.1f}")


@pytest.mark.parametrize("name", CASES)
def test_render_bwd_same_inputs(name):
    """Screen-space gradients per (view, splat) after the tile partials and the
    segmented sum, against the oracle's explicit-list adjoint."""
    scene, st, g = _run(name)
    rec, fwd, dL, gb, g2 = _same_inputs(name)
    ref = conic_grads_to_factor(g2, g["rec"])
    labels = ["du", "dv", "dL00", "dL10", "dL11", "dop", "dbeta", "dr", "dg", "db"]
    worst = 0.0
    for k, lab in enumerate(labels):
        einf, e2 = norm_errors(gb["grad2d"][:, k], ref[:, k])
        worst = max(worst, einf, e2)
        assert einf <= 1e-3 and e2 <= 1e-3, (lab, einf, e2)
    log(f"[gpu] {name}: bwd ok; worst {worst:.2e}")


@pytest.mark.parametrize("name", CASES)
def test_project_bwd_same_inputs(name):
    """Projection adjoint fed the GPU's own screen-space gradients: the oracle's
    dual-number Jacobian gives the reference parameter gradients."""
    scene, st, g = _run(name)
    rec, fwd, dL, gb, g2 = _same_inputs(name)
    ref = oracle.project_bwd(scene, factor_grads_to_conic(gb["grad2d"], g["rec"]), st)
    for k in ("means", "scales", "quats", "opacities", "betas", "sh"):
        einf, e2 = norm_errors(gb[k], ref[k])
        assert einf <= 1e-3 and e2 <= 1e-3, (k, einf, e2)


@pytest.mark.parametrize("name", CASES)
def test_end_to_end(name):
    """Whole GPU pipeline vs the oracle run from the splat parameters."""
    scene, st, g = _run(name)
    fo, amb, dL, gb, go = _end_to_end(name)
    errs = image_errors(g["image"], fo["image"], amb, scene.cameras)
    for bad, mx, bound, l2 in errs:
        assert bad == 0 and l2 <= 1e-4, errs
    ok = ~amb
    assert np.abs(g["final_T"][ok] - fo["final_T"][ok]).max() <= 1e-4
    worst = 0.0
    for k in ("means", "scales", "quats", "opacities", "betas", "sh"):
        einf, e2 = norm_errors(gb[k], go[k])
        worst = max(worst, einf, e2)
        assert einf <= 1e-3 and e2 <= 1e-3, (k, einf, e2)
    log(f"[gpu] {name}: end-to-end ok; ambiguous px {int(amb.sum())}/{amb.size}; image max err "
        f"{max(e[1] for e in errs):.2e}; grad worst {worst:.2e}")


def _needle_scene(seed=21, n=600):
    """Thin rotated ellipses: long axis exp(U(-2.5, -0.3)), the other two
    shorter by exp(U(3, 9)) and exp(U(0, 2)), random rotations, centres spread
    past the image borders of two views."""
    rng = np.random.default_rng(seed)
    f32 = np.float32
    means = np.column_stack([rng.uniform(-2.6, 2.6, n), rng.uniform(-2.0, 2.0, n), rng.uniform(-0.5, 0.5, n)])
    long = rng.uniform(-2.5, -0.3, n)
    log_scales = np.column_stack([long, long - rng.uniform(3.0, 9.0, n), long - rng.uniform(0.0, 2.0, n)]).astype(f32)
    logits = np.log(1.0 / rng.uniform(0.1, 0.95, n) - 1.0).astype(f32) * f32(-1.0)
    sh = np.zeros((n, 1, 3), f32)
    sh[:, 0, :] = rng.uniform(-1.0, 1.0, (n, 3))
    cams = [gi.look_at((0.0, 0.0, -4.0), width=160, height=120),
            gi.look_at((2.4, 0.9, -3.1), width=131, height=97)]
    return gi.Scene(name="needles", means=means.astype(f32), log_scales=log_scales,
                    scales=np.exp(log_scales.astype(np.float64)).astype(f32), quats=rng.standard_normal((n, 4)).astype(f32),
                    opacity_logits=logits, opacities=(1.0 / (1.0 + np.exp(-logits.astype(np.float64)))).astype(f32),
                    betas=rng.uniform(0.8, 3.5, n).astype(f32), sh=sh, sh_degree=0, cameras=cams)


def _rectangle_lists(scene, st, g):
    """Every tile of every pair's rectangle, in (tile, depth key, pair) order."""
    grid, T = oracle.tile_grid(scene.cameras, st.tile_w, st.tile_h)
    inst = []
    for o in np.nonzero(g["tiles_touched"])[0]:
        tx_n, _, base = grid[o // scene.n]
        tx0, ty0, tx1, ty1 = (int(x) for x in g["tile_rect"][o])
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                inst.append((base + ty * tx_n + tx, int(g["depth_key"][o]), int(o)))
    inst.sort()
    vals = np.array([e[2] for e in inst], np.uint32)
    tiles = np.array([e[0] for e in inst], np.int64)
    ranges = np.zeros((T, 2), np.uint32)
    for t in np.unique(tiles):
        idx = np.nonzero(tiles == t)[0]
        ranges[t] = (idx[0], idx[-1] + 1)
    return vals, ranges


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_needles_tight_lists(tile):
    """Needle-shaped footprints at every angle, many cut by the image border:
    binning equals the oracle's bit for bit, drops part of the rectangles'
    tiles, and loses nothing: the oracle composites the GPU's lists and the
    full rectangles into identical images, hit counts and final T (with fewer
    listed fragments), and the GPU's image agrees with them."""
    scene = _needle_scene()
    st = oracle.Settings(tile_w=tile[0], tile_h=tile[1])
    g = run_gpu(scene, st)
    keys, vals, ranges = oracle.bin_instances(scene.n, scene.cameras, g["tile_rect"], g["tiles_touched"],
                                              g["depth_key"], st, g["rec"])
    assert g["overflow"] == 0 and g["listed"] == len(vals) < 0.9 * g["M"]
    np.testing.assert_array_equal(g["val_sorted"], vals)
    np.testing.assert_array_equal(g["tile_sorted"].astype(np.uint64), keys >> np.uint64(32))
    np.testing.assert_array_equal(g["ranges"], ranges)
    rec = oracle_rec(g["rec"])
    tight = oracle.render_fwd(scene.n, scene.cameras, rec, g["val_sorted"], g["ranges"], st)
    rv, rr = _rectangle_lists(scene, st, g)
    assert len(rv) == g["M"]
    full = oracle.render_fwd(scene.n, scene.cameras, rec, rv, rr, st)
    for k in ("image", "final_T", "n_hit"):  # (n_contrib is a position in the list)
        np.testing.assert_array_equal(tight[k], full[k], err_msg=k)
    assert tight["n_listed"].sum() < full["n_listed"].sum()
    amb = tight["ambig"] > 0
    errs = image_errors(g["image"], tight["image"], amb, scene.cameras)
    for bad, mx, bound, l2 in errs:
        assert bad == 0 and l2 <= 1e-4, errs
    np.testing.assert_array_equal(g["n_hit"][~amb], tight["n_hit"][~amb])
    log(f"[gpu] needles {tile}: listed {g['listed']} of {g['M']} rectangle tiles; ambiguous px {int(amb.sum())}")
