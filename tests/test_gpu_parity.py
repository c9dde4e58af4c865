"""GPU parity of every hot-path stage against the FP64 oracle.

Stage tests feed the oracle the GPU's projection records (so a disagreement
downstream is the stage's own), then an end-to-end test compares the whole GPU
pipeline with the oracle run from the splat parameters.  The parity model
(decision bands, decision paths, masking) is described in tests/gpu_util.py.

Bars:
  * projection: within the a-priori float32 bounds of the oracle's
    record_err_bound (centre, conic, qmax), colour 1e-5, opacity and beta exact;
  * binning: the GPU's sorted lists equal the oracle's footprint rule (FP64)
    after removing the decisions within the rule's float32 band (whose count
    is logged); ranges, worklist and instance bases exact;
  * images / final_T: max error <= 1e-4 * max(max|C|, 1) per view and relative
    L2 <= 1e-4, against the oracle along the decision path that the GPU's
    result matches (every pixel except the masked ones, at most 1e-3 of them);
    the last composited splat and the hit count exact there; n_contrib and the
    listed count exact in tiles whose two lists are identical;
  * gradients: per tensor, inf-norm and 2-norm of the error <= 1e-3 of the
    reference's norms, for the same seeded upstream dL/dimage on both sides,
    zeroed only at masked pixels.
"""
import functools

import numpy as np
import pytest

import gesr_inputs as gi
import oracle
from tests.gpu_util import (ambiguous_tiles_to_pixels, check_projection, compare_lists, conic_grads_to_factor,
                            differing_tiles, end_to_end_reference, factor_grads_to_conic, image_errors, log,
                            mask_upstream, norm_errors, oracle_rec, run_gpu, run_gpu_bwd, same_input_reference)

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
    if name == "giant-640x480":  # splats of more than 512 tiles: the segmented sum's whole-wave pairs
        return gi.tiny_scene(9, n=24, deg=1, width=640, height=480, log_scale=(-0.6, -0.1), spread=0.3), \
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
         "surfels-40k-2v", "blobs-100k-2v", "wide-2200x2100", "giant-640x480"]


@functools.lru_cache(maxsize=1)
def _run(name):
    scene, st = _case(name)
    log(f"[gpu] case {name}: n={scene.n} views={scene.n_views} px={scene.n_pixels}")
    g = run_gpu(scene, st, variant=1 if name.endswith("-v1") else 0)
    log(f"[gpu] case {name}: forward done, M={g['M']}")
    return scene, st, g


@functools.lru_cache(maxsize=1)
def _same_inputs(name):
    """Oracle fed the GPU's records; gradients for an upstream dL that is zero
    at masked pixels only (identical on both sides)."""
    scene, st, g = _run(name)
    ref = same_input_reference(scene, st, g)
    dL = mask_upstream(oracle.flat_images(gi.upstream_grads(scene, 7)), ref["masked"], scene.cameras)
    log(f"[gpu] case {name}: backward (same inputs)")
    gb = run_gpu_bwd(scene, st, g, dL)
    g2 = oracle.render_bwd(scene.n, scene.cameras, ref["rec"], ref["vals"], ref["ranges"], dL, st, paths=ref["paths"])
    return ref, dL, gb, g2


@functools.lru_cache(maxsize=1)
def _end_to_end(name):
    """Oracle run from the parameters, decision paths resolved to the GPU's result."""
    scene, st, g = _run(name)
    ref = end_to_end_reference(scene, st, g)
    dL = mask_upstream(oracle.flat_images(gi.upstream_grads(scene, 7)), ref["masked"], scene.cameras)
    log(f"[gpu] case {name}: backward (end to end)")
    gb = run_gpu_bwd(scene, st, g, dL)
    go = oracle.backward(scene, st, ref["fo"], dL, paths=ref["paths"])
    return ref, dL, gb, go


def _check_forward(scene, g, o, masked, tiles_same, name, label):
    """Image, final T and counts of the GPU against the oracle's forward `o`
    (already along the matched decision paths)."""
    errs = image_errors(g["image"], o["image"], masked, scene.cameras)
    for bad, mx, bound, l2 in errs:
        assert bad == 0 and l2 <= 1e-4, errs
    ok = ~masked
    assert np.abs(g["final_T"][ok] - o["final_T"][ok]).max() <= 1e-4
    np.testing.assert_array_equal(g["last"][ok], o["last"][ok])
    np.testing.assert_array_equal(g["n_hit"][ok], o["n_hit"][ok])
    same = ok & tiles_same
    np.testing.assert_array_equal(g["n_contrib"][same], o["n_contrib"][same])
    np.testing.assert_array_equal(g["n_listed"][same], o["n_listed"][same])
    log(f"[gpu] {name}: {label} fwd ok; masked px {int(masked.sum())}/{masked.size}; max err "
        f"{max(e[1] for e in errs):.2e}; listed/px {o['n_listed'].mean():.1f} hit/px {o['n_hit'].mean():.1f}")


@pytest.mark.parametrize("name", CASES)
def test_project(name):
    scene, st, g = _run(name)
    stats = check_projection(scene, g, oracle.project(scene, st), oracle.record_err_bound(scene, st))
    log(f"[gpu] {name}: project ok; {stats}")


@pytest.mark.parametrize("name", CASES)
def test_bin_lists(name):
    """The GPU's sorted instance lists equal the oracle's footprint rule (FP64,
    on the GPU's own records, rectangles and depth keys) outside the rule's
    float32 band; ranges are those of the lists; worklist, counts and instance
    bases exact."""
    scene, st, g = _run(name)
    rec = oracle_rec(g["rec"])
    keys, vals, ranges = oracle.bin_instances(scene.n, scene.cameras, g["tile_rect"], g["tiles_touched"],
                                              g["depth_key"], st, rec)
    band = oracle.bin_band(scene.n, scene.cameras, g["tile_rect"], g["tiles_touched"], rec, st)
    assert g["overflow"] == 0
    assert g["M"] == int(g["tiles_touched"].astype(np.int64).sum()) >= g["listed"]
    assert g["listed"] == len(g["val_sorted"])
    cmp = compare_lists(g["val_sorted"], g["tile_sorted"], g["ranges"], keys, vals, ranges, band)
    # the GPU's keys: (tile, depth key) of each entry, sorted, ties by pair
    t = g["tile_sorted"].astype(np.int64)
    k = g["depth_key"][g["val_sorted"]].astype(np.int64)
    v = g["val_sorted"].astype(np.int64)
    same_t = t[1:] == t[:-1]
    assert (t[1:] >= t[:-1]).all()
    assert (((k[1:] > k[:-1]) | ((k[1:] == k[:-1]) & (v[1:] > v[:-1]))) | ~same_t).all()
    counts = np.bincount(t, minlength=len(g["ranges"]))
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    np.testing.assert_array_equal(g["ranges"][:, 0], np.where(counts > 0, starts, 0))
    np.testing.assert_array_equal(g["ranges"][:, 1], np.where(counts > 0, starts + counts, 0))
    # worklist: every tile once, by decreasing list length, ties by tile id
    lens = g["ranges"][:, 1].astype(np.int64) - g["ranges"][:, 0]
    expect = np.lexsort((np.arange(len(lens)), -np.minimum(lens, 0xFFFF)))
    np.testing.assert_array_equal(g["worklist"], expect)
    # instance slots: exclusive scan of tiles_touched in pair order
    base = np.concatenate([[0], np.cumsum(g["tiles_touched"].astype(np.int64))[:-1]])
    np.testing.assert_array_equal(g["inst_base"], base)
    log(f"[gpu] {name}: lists ok; {len(vals)} instances; {cmp['n_band']} decisions within the float32 band, "
        f"{cmp['n_flip']} of them taken the other way")


@pytest.mark.parametrize("name", CASES)
def test_render_fwd_same_inputs(name):
    scene, st, g = _run(name)
    ref, dL, gb, g2 = _same_inputs(name)
    same = ~ambiguous_tiles_to_pixels(scene.cameras, st, ref["lists"]["tiles_differ"])
    _check_forward(scene, dict(g, last=ref["last"]), ref["fwd"], ref["masked"], same, name, "same inputs")


@pytest.mark.parametrize("name", CASES)
def test_render_bwd_same_inputs(name):
    """Screen-space gradients per (view, splat) after the tile partials and the
    segmented sum, against the oracle's explicit-list adjoint."""
    scene, st, g = _run(name)
    ref, dL, gb, g2 = _same_inputs(name)
    refg = conic_grads_to_factor(g2, g["rec"])
    labels = ["du", "dv", "dL00", "dL10", "dL11", "dop", "dbeta", "dr", "dg", "db"]
    worst = 0.0
    for k, lab in enumerate(labels):
        einf, e2 = norm_errors(gb["grad2d"][:, k], refg[:, k])
        worst = max(worst, einf, e2)
        assert einf <= 1e-3 and e2 <= 1e-3, (lab, einf, e2)
    log(f"[gpu] {name}: bwd ok; worst {worst:.2e}")


@pytest.mark.parametrize("name", CASES)
def test_project_bwd_same_inputs(name):
    """Projection adjoint fed the GPU's own screen-space gradients: the oracle's
    dual-number Jacobian gives the reference parameter gradients."""
    scene, st, g = _run(name)
    ref, dL, gb, g2 = _same_inputs(name)
    pref = oracle.project_bwd(scene, factor_grads_to_conic(gb["grad2d"], g["rec"]), st)
    for k in ("means", "scales", "quats", "opacities", "betas", "sh"):
        einf, e2 = norm_errors(gb[k], pref[k])
        assert einf <= 1e-3 and e2 <= 1e-3, (k, einf, e2)


@pytest.mark.parametrize("name", CASES)
def test_end_to_end(name):
    """Whole GPU pipeline vs the oracle run from the splat parameters."""
    scene, st, g = _run(name)
    ref, dL, gb, go = _end_to_end(name)
    fo = ref["fo"]
    same = ~ambiguous_tiles_to_pixels(scene.cameras, st, differing_tiles(g["val_sorted"], g["ranges"], fo["vals"],
                                                                          fo["ranges"]))
    _check_forward(scene, dict(g, last=ref["last"]), fo, ref["masked"], same, name, "end to end")
    worst = 0.0
    for k in ("means", "scales", "quats", "opacities", "betas", "sh"):
        einf, e2 = norm_errors(gb[k], go[k])
        worst = max(worst, einf, e2)
        assert einf <= 1e-3 and e2 <= 1e-3, (k, einf, e2)
    log(f"[gpu] {name}: end-to-end gradients ok; worst {worst:.2e}")


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
    the lists equal the oracle's footprint rule outside its float32 band and
    drop part of the rectangles' tiles, and lose nothing: the oracle composites
    the GPU's lists and the full rectangles into identical images, hit counts
    and final T (with fewer listed fragments), and the GPU's image is one of
    the oracle's correct results at every pixel."""
    scene = _needle_scene()
    st = oracle.Settings(tile_w=tile[0], tile_h=tile[1])
    g = run_gpu(scene, st)
    rec = oracle_rec(g["rec"])
    keys, vals, ranges = oracle.bin_instances(scene.n, scene.cameras, g["tile_rect"], g["tiles_touched"],
                                              g["depth_key"], st, rec)
    band = oracle.bin_band(scene.n, scene.cameras, g["tile_rect"], g["tiles_touched"], rec, st)
    assert g["overflow"] == 0 and g["listed"] == len(g["val_sorted"]) < 0.9 * g["M"]
    cmp = compare_lists(g["val_sorted"], g["tile_sorted"], g["ranges"], keys, vals, ranges, band)
    tight = oracle.render_fwd(scene.n, scene.cameras, rec, g["val_sorted"], g["ranges"], st)
    rv, rr = _rectangle_lists(scene, st, g)
    assert len(rv) == g["M"]
    full = oracle.render_fwd(scene.n, scene.cameras, rec, rv, rr, st)
    for k in ("image", "final_T", "n_hit", "last"):  # (n_contrib is a position in the list)
        np.testing.assert_array_equal(tight[k], full[k], err_msg=k)
    assert tight["n_listed"].sum() < full["n_listed"].sum()
    ref = same_input_reference(scene, st, g)
    _check_forward(scene, dict(g, last=ref["last"]), ref["fwd"], ref["masked"],
                   ~ambiguous_tiles_to_pixels(scene.cameras, st, cmp["tiles_differ"]), "needles", str(tile))
    log(f"[gpu] needles {tile}: listed {g['listed']} of {g['M']} rectangle tiles; {cmp['n_band']} decisions within "
        f"the band, {cmp['n_flip']} taken the other way")


def test_giant_case_reaches_whole_wave_pairs():
    """The giant-splat case holds pairs of more than 512 instance slots, which the
    segmented sum hands to a whole wave (the parity tests above cover them)."""
    scene, st, g = _run("giant-640x480")
    big = int((g["tiles_touched"] > 512).sum())
    log(f"[gpu] giant case: {big} pairs of more than 512 slots, largest {int(g['tiles_touched'].max())}")
    assert big > 0
