"""CPU checks of the parity model the GPU tests rely on (see tests/gpu_util.py).

* The float32 band of a fragment's alpha (the oracle's frag_band) holds for a
  float32 evaluation of the renderer's steps (numpy float32 arithmetic, fused
  multiply-adds by exact float64 products, float32 log2 and exp2).
* The resolver finds the decision path along which a result was produced,
  and reports a result that no path produces.
* Decision paths change results only at decisions inside their band.
"""
import numpy as np
import pytest

import gesr_inputs as gi
import oracle

f32 = np.float32


def _factor(rec):
    """Float32 conic factor (L00, L10, L11) of float64 conics (A, B, C)."""
    A, B, C = rec[:, 2], rec[:, 3], rec[:, 4]
    L00 = np.sqrt(A)
    L10 = B / L00
    L11 = np.sqrt(C - L10 * L10)
    return L00.astype(f32), L10.astype(f32), L11.astype(f32)


def _fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


@pytest.mark.parametrize("kappa", [0.5, 1.0])
def test_alpha_band_covers_a_float32_evaluation(kappa):
    st = oracle.Settings(kappa=kappa)
    sc = gi.make_workload(1)
    pr = oracle.project(sc, st)
    keep = pr["tiles_touched"] > 0
    rec = pr["rec"][keep]
    L00, L10, L11 = _factor(rec)
    u, v = rec[:, 0].astype(f32), rec[:, 1].astype(f32)
    o, beta = rec[:, 5].astype(f32), rec[:, 6].astype(f32)
    # the oracle's record of exactly these float32 values
    r64 = rec.copy()
    r64[:, 0], r64[:, 1] = u, v
    l00, l10, l11 = L00.astype(np.float64), L10.astype(np.float64), L11.astype(np.float64)
    r64[:, 2], r64[:, 3], r64[:, 4] = l00 * l00, l00 * l10, l10 * l10 + l11 * l11
    r64[:, 5], r64[:, 6] = o, beta
    rng = np.random.default_rng(1)
    n, per = len(rec), 40
    idx = np.repeat(np.arange(n), per)
    # pixel centres over the footprint, denser near its edge
    ang = rng.uniform(0, 2 * np.pi, idx.size)
    rad = np.sqrt(rec[idx, 7]) * rng.uniform(0.0, 1.05, idx.size) ** 0.3
    # a point at Mahalanobis radius `rad` in direction `ang`: solve L d = (cos, sin) rad
    wy = rad * np.sin(ang) / l11[idx]
    wx = (rad * np.cos(ang) - l10[idx] * wy) / l00[idx]
    px = np.floor(u[idx] + wx) + 0.5
    py = np.floor(v[idx] + wy) + 0.5
    oG64, band = oracle.fragment_band(r64[idx], px, py, st)
    # float32 evaluation, the renderer's order of operations
    dx = (px.astype(f32) - u[idx]).astype(f32)
    dy = (py.astype(f32) - v[idx]).astype(f32)
    t = _fma32(L10[idx], dy, (L00[idx] * dx).astype(f32))
    w = (L11[idx] * dy).astype(f32)
    q = _fma32(t, t, (w * w).astype(f32))
    with np.errstate(divide="ignore"):
        l2q = np.log2(q).astype(f32)
    P = np.exp2((beta[idx] * f32(0.5) * l2q).astype(f32)).astype(f32)
    G = np.exp2((f32(-kappa * np.log2(np.e)) * P).astype(f32)).astype(f32)
    oG32 = (o[idx] * G).astype(f32).astype(np.float64)
    live = (oG64 > 1e-30) & (oG32 > 0)
    err = np.abs(np.log(oG32[live] / oG64[live]))
    ratio = err / band[live]
    assert live.sum() > 50000
    assert ratio.max() <= 1.0, (ratio.max(), np.argmax(ratio))
    # the band is a bound, not an estimate: typical errors are well inside it
    assert np.median(ratio) < 0.2


def test_resolver_finds_the_path_and_rejects_other_results():
    """Results rendered along a non-zero decision path (bands widened 10^4
    times so that many pixels have several paths) resolve to a path that
    reproduces them (to the float32 rounding the resolver applies to a
    result); a result perturbed by 1e-3 matches no path."""
    st = oracle.Settings(band_scale=1e4)
    sc = gi.make_workload(1)
    f = oracle.forward(sc, st)
    nb = f["n_branch"].astype(np.int64)
    multi = nb >= 1
    assert multi.sum() > 200
    rng = np.random.default_rng(2)
    paths = np.where(multi, rng.integers(0, 1 << 30, nb.size) & ((1 << np.minimum(nb, 30)) - 1), 0).astype(np.uint32)
    target = oracle.render_fwd(sc.n, sc.cameras, f["proj"]["rec"], f["vals"], f["ranges"], st, paths=paths)
    changed = (target["last"] != f["last"]) | (target["n_hit"] != f["n_hit"])
    assert changed.sum() > 50
    got, status, plain = oracle.resolve(sc.n, sc.cameras, f["proj"]["rec"], f["vals"], f["ranges"], st,
                                        target["image"], target["final_T"], target["last"], target["n_hit"],
                                        tol=1e-6, tol_T=1e-6)
    assert set(np.unique(status)) <= {0, 1, 3}
    ok = status != 3
    assert ok.mean() > 0.99
    again = oracle.render_fwd(sc.n, sc.cameras, f["proj"]["rec"], f["vals"], f["ranges"], st, paths=got)
    np.testing.assert_array_equal(again["last"][ok], target["last"][ok])
    np.testing.assert_array_equal(again["n_hit"][ok], target["n_hit"][ok])
    P = sc.n_pixels
    np.testing.assert_allclose(again["image"].reshape(3, P)[:, ok], target["image"].reshape(3, P)[:, ok],
                               rtol=0, atol=1e-6)
    bad_img = np.array(target["image"], copy=True)
    bad_img.reshape(3, P)[0] += 1e-3
    _, status2, _ = oracle.resolve(sc.n, sc.cameras, f["proj"]["rec"], f["vals"], f["ranges"], st, bad_img,
                                   target["final_T"], target["last"], target["n_hit"], tol=1e-6, tol_T=1e-6)
    assert (status2[multi & ok] == 4).all()


def test_paths_only_flip_decisions_inside_their_band():
    """With the derived bands, path 1 (the first in-band decision taken the
    other way) changes a pixel's result only where the pixel has such a
    decision; elsewhere any path gives the plain result bit for bit."""
    st = oracle.Settings()
    sc = gi.make_workload(3, n_override=20_000)
    f = oracle.forward(sc, st, band=True)
    ones = np.ones(sc.n_pixels, np.uint32)
    g = oracle.render_fwd(sc.n, sc.cameras, f["proj"]["rec"], f["vals"], f["ranges"], st, perr=f["perr"], paths=ones)
    none = f["n_branch"] == 0
    assert none.mean() > 0.99 and (~none).sum() > 0
    for k in ("final_T", "n_hit", "last", "n_contrib"):
        np.testing.assert_array_equal(g[k][none], f[k][none])
    assert (g["last"][~none] != f["last"][~none]).any() or (g["n_hit"][~none] != f["n_hit"][~none]).any()
