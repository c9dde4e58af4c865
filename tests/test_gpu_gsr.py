"""GPU parity of the surface regulariser (Sec. 3.3, Eq. 9-13) and its
neighbour lists (Sec. 4.2) against the FP64 oracle.

Neighbour lists: the GPU ranks by float32 squared distance, the oracle by
float64; a row may differ only where the neighbours it swaps lie within the
float32 error band of each other's distance (relative 1e-5), and the lists
must agree as sets of float64 distances within that band.  The inverse lists
are checked exactly against a stable sort of the GPU's own lists taken in its
cell order (a permutation of the splats), and the entry-to-record map as their
inverse.

Losses and gradients: the oracle gets the GPU's lists and the same xi.
Samples whose oracle decision margins lie inside the float32 band are masked
out on both sides: g* gap 1e-4; |h| / |x - mu_g*| 1e-3 (the relative
conditioning of h); the kink of |fbar - f| 1e-3; |ln d| 1e-4; the gap of the
two smallest scales 1e-4; |grad d| / sum |grad T_i| 1e-3 (cancellation in the
normal term's direction); the 1e-30 floors of d and |grad d| 1e-3 in log.
Per-sample l_sdf: inf- and 2-norm errors <= 1e-4 of the reference's norms;
l_nor <= 1e-3: its direction carries the float32 error of each flat
neighbour's normal offset, about 6e-8 |x - mu| / s_min times s_max / s_min
(2e-4 on the flat-splat sphere, whose splats are 55 times thinner than wide);
g* exact; gradients <= 1e-3 (the gradient bar of the render path).
"""
import functools

import numpy as np
import pytest

import oracle
from tests.gpu_util import log, norm_errors

pytestmark = pytest.mark.gpu


class _Scene:
    def __init__(self, means, scales, quats, opac, betas):
        n = len(opac)
        self.n = n
        self.means = np.asarray(means, np.float32).reshape(n, 3)
        self.scales = np.asarray(scales, np.float32).reshape(n, 3)
        self.quats = np.asarray(quats, np.float32).reshape(n, 4)
        self.opacities = np.asarray(opac, np.float32)
        self.betas = np.asarray(betas, np.float32)


def _scene(kind, n, seed):
    """Seeded stand-ins for the workload shapes: a uniform cube, flat splats on
    a sphere (the regularised end state), Gaussian clusters."""
    rng = np.random.default_rng([seed, n])
    q = rng.standard_normal((n, 4))
    op = rng.uniform(0.3, 0.95, n)
    be = rng.uniform(1.0, 4.0, n)
    if kind == "cube":
        mu = rng.uniform(-1, 1, (n, 3))
        ls = rng.uniform(-3.2, -2.4, (n, 3)) + np.log(2000.0 / n) / 3
    elif kind == "sphere":
        d = rng.standard_normal((n, 3))
        mu = d / np.linalg.norm(d, axis=1, keepdims=True)
        ls = np.stack([rng.uniform(-3.5, -2.8, n), rng.uniform(-3.5, -2.8, n), rng.uniform(-7, -6, n)], 1)
        ls += np.log(3000.0 / n) / 2
    else:  # clusters
        c = rng.uniform(-1, 1, (12, 3))
        mu = c[rng.integers(0, 12, n)] + 0.12 * rng.standard_normal((n, 3))
        ls = rng.uniform(-4.0, -3.2, (n, 3))
    return _Scene(mu, np.exp(ls), q, op, be)


def _splats(sc):
    import torch
    from paper_2411_09156_amd import Splats
    return Splats.from_aos(sc.means, sc.scales, sc.quats, sc.opacities, sc.betas, np.zeros((sc.n, 1, 3), np.float32),
                           device="cuda" if torch.cuda.is_available() else "cpu")


def _check_knn(means, got, want, k):
    """Row-wise agreement up to float32 distance ties (module docstring)."""
    P = np.asarray(means, np.float64)
    n = P.shape[0]
    differ = 0
    for j in range(n):
        g, w = got[j], want[j]
        assert g[0] == j
        if np.array_equal(g, w):
            continue
        differ += 1
        gv, wv = g[g >= 0], w[w >= 0]
        assert len(gv) == len(wv) and len(set(gv.tolist())) == len(gv), j
        dg = np.sort(((P[gv[1:]] - P[j]) ** 2).sum(1))
        dw = np.sort(((P[wv[1:]] - P[j]) ** 2).sum(1))
        np.testing.assert_allclose(dg, dw, rtol=1e-5, atol=1e-12, err_msg=f"row {j}")
    return differ


@pytest.mark.parametrize("kind,n,k", [("cube", 3000, 16), ("sphere", 4000, 16), ("clusters", 3000, 16),
                                      ("cube", 20000, 16), ("cube", 2000, 5), ("cube", 17, 16), ("cube", 16, 16),
                                      ("cube", 9, 16), ("cube", 1, 16), ("cube", 500, 1)])
def test_knn_matches_oracle(kind, n, k):
    import torch
    from paper_2411_09156_amd.gsr import knn
    log(f"[gpu] knn {kind} n={n} k={k}")
    sc = _scene(kind, n, 1)
    nb = knn(_splats(sc), k)
    torch.cuda.synchronize()
    got = nb["knn"].cpu().numpy().astype(np.int64)  # padding 0xFFFFFFFF reads as -1
    want = oracle.knn(sc.means.astype(np.float64), k).astype(np.int64)
    differ = _check_knn(sc.means, got, want, k)
    # inverse lists: a stable sort of the GPU's own entries, in cell order, by neighbour
    order_g = nb["order"].cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(np.sort(order_g), np.arange(n))
    flat = got[order_g].reshape(-1)
    valid = flat >= 0
    order = np.argsort(np.where(valid, flat, n), kind="stable")[:int(valid.sum())]
    offs = nb["inv_offsets"].cpu().numpy().astype(np.int64)
    ent = nb["inv_entries"].cpu().numpy().astype(np.int64)[:int(valid.sum())]
    np.testing.assert_array_equal(ent, order)
    np.testing.assert_array_equal(offs, np.searchsorted(flat[order], np.arange(n + 1), side="left"))
    slot = nb["inv_slot"].cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(slot[ent], np.arange(ent.size))
    log(f"[gpu] knn {kind} n={n}: {differ} rows differ within the float32 band")


def _clear(m):
    """Samples whose decisions are outside the float32 band (module docstring)."""
    return ((m[:, 0] > 1e-4) & (m[:, 1] > 1e-3) & (m[:, 2] > 1e-3) & (m[:, 3] > 1e-4) & (m[:, 4] > 1e-4)
            & (m[:, 5] > 1e-3) & (m[:, 6] > 1e-3))


@functools.lru_cache(maxsize=4)
def _gsr_case(kind, n, seed=3):
    import torch
    from paper_2411_09156_amd import RasterSettings
    from paper_2411_09156_amd.gsr import gsr, knn
    sc = _scene(kind, n, seed)
    sp = _splats(sc)
    nb = knn(sp, 16)
    torch.cuda.synchronize()
    nbrs = nb["knn"].cpu().numpy().astype(np.int64)
    nbrs = np.where(nbrs < 0, -1, nbrs).astype(np.int32)
    xi = np.random.default_rng([seed, 9]).standard_normal((n, 3)).astype(np.float32)
    st = oracle.Settings()
    first = oracle.gsr(sc, st, nbrs, xi, grads=False)
    m = first["margins"]
    mask = _clear(m)
    ws, wn = 0.8, 0.3
    ref = oracle.gsr(sc, st, nbrs, xi, mask=mask.astype(np.uint8), w_sdf=ws, w_nor=wn)
    grads = {k: torch.zeros_like(getattr(sp, k)) for k in ("mean", "scale", "quat", "opacity", "beta")}
    out = gsr(sp, RasterSettings(), nb, torch.as_tensor(xi.T.copy(), device="cuda"),
              mask=torch.as_tensor(mask.astype(np.uint8), device="cuda"), w_sdf=ws, w_nor=wn, grads=grads)
    torch.cuda.synchronize()
    return sc, sp, nb, xi, mask, ref, out, grads


@pytest.mark.parametrize("kind,n", [("cube", 2000), ("sphere", 3000), ("clusters", 2500)])
def test_gsr_losses_and_gradients_match_oracle(kind, n):
    log(f"[gpu] gsr {kind} n={n}")
    sc, sp, nb, xi, mask, ref, out, grads = _gsr_case(kind, n)
    so = out["sample_out"].cpu().numpy().astype(np.float64)
    assert mask.mean() > 0.9, mask.mean()
    np.testing.assert_array_equal(so[mask, 2].astype(np.int64), ref["gstar"][mask])
    assert (so[~mask, 2] == -1).all() and (so[~mask, :2] == 0).all()
    for c, key, bar in ((0, "l_sdf", 1e-4), (1, "l_nor", 1e-3)):
        einf, e2 = norm_errors(so[:, c], ref[key])
        if not (einf <= bar and e2 <= bar):
            err = np.abs(so[:, c] - ref[key])
            for r in np.argsort(-err)[:6]:
                log(f"[gpu]   {key} sample {r}: gpu {so[r, c]:.6g} ref {ref[key][r]:.6g} d {so[r, 3]:.4g} "
                    f"margins {np.array2string(ref['margins'][r], precision=3)}")
        assert einf <= bar and e2 <= bar, (key, einf, e2)
    tot = out["losses"].cpu().numpy().astype(np.float64)
    log(f"[gpu] {kind}: sums gpu {tot[0]:.7g} {tot[1]:.7g} ref {ref['l_sdf'].sum():.7g} {ref['l_nor'].sum():.7g}")
    assert tot[0] == pytest.approx(ref["l_sdf"].sum(), rel=1e-4)
    assert tot[1] == pytest.approx(ref["l_nor"].sum(), rel=1e-3)
    worst = 0.0
    for gk, rk, w in (("mean", "means", 3), ("scale", "scales", 3), ("quat", "quats", 4), ("opacity", "opacities", 1),
                      ("beta", "betas", 1)):
        g = grads[gk].cpu().numpy().astype(np.float64).reshape(w, -1).T
        einf, e2 = norm_errors(g, ref["grads"][rk].reshape(-1, w))
        worst = max(worst, einf, e2)
        assert einf <= 1e-3 and e2 <= 1e-3, (gk, einf, e2)
    log(f"[gpu] gsr {kind} n={n}: {int(mask.sum())} samples, worst gradient error {worst:.2e}, "
        f"L_sdf {tot[0]:.4g} L_nor {tot[1]:.4g}")


def test_gsr_adds_into_gradients_and_needs_no_gradients():
    """Gradients accumulate (two calls double them); without a gradient dict
    the losses are the same and nothing is written."""
    import torch
    from paper_2411_09156_amd import RasterSettings
    from paper_2411_09156_amd.gsr import gsr
    sc, sp, nb, xi, mask, ref, out, grads = _gsr_case("cube", 2000)
    g2 = {k: v.clone() for k, v in grads.items()}
    xt = torch.as_tensor(xi.T.copy(), device="cuda")
    mt = torch.as_tensor(mask.astype(np.uint8), device="cuda")
    gsr(sp, RasterSettings(), nb, xt, mask=mt, w_sdf=0.8, w_nor=0.3, grads=g2)
    o2 = gsr(sp, RasterSettings(), nb, xt, mask=mt, w_sdf=0.8, w_nor=0.3)
    torch.cuda.synchronize()
    for k in grads:
        np.testing.assert_array_equal(g2[k].cpu().numpy(), 2 * grads[k].cpu().numpy())
    np.testing.assert_array_equal(o2["sample_out"].cpu().numpy(), out["sample_out"].cpu().numpy())


def test_gsr_full_size_sampled():
    """The benchmark's 500k-splat cube: neighbour rows and per-sample losses on
    sampled splats against the oracle (brute-force rows, masked oracle run)."""
    import torch

    import gesr_inputs as gi
    from paper_2411_09156_amd import RasterSettings, Splats
    from paper_2411_09156_amd.gsr import gsr, knn
    scene = gi.make_workload(3)
    log(f"[gpu] gsr full size n={scene.n}")
    sp = Splats.from_aos(scene.means, scene.scales, scene.quats, scene.opacities, scene.betas, scene.sh)
    nb = knn(sp, 16)
    xi = np.random.default_rng(21).standard_normal((scene.n, 3)).astype(np.float32)
    out = gsr(sp, RasterSettings(sh_degree=scene.sh_degree), nb, torch.as_tensor(xi.T.copy(), device="cuda"),
              w_sdf=1.0, w_nor=1.0, grads={k: torch.zeros_like(getattr(sp, k))
                                          for k in ("mean", "scale", "quat", "opacity", "beta")})
    torch.cuda.synchronize()
    got = nb["knn"].cpu().numpy().astype(np.int64)
    P = np.asarray(scene.means, np.float64)
    rows = np.random.default_rng(22).choice(scene.n, 150, replace=False)
    for j in rows:
        d = ((P - P[j]) ** 2).sum(1)
        d[j] = -1
        want = np.lexsort((np.arange(scene.n), d))[:16]
        dg = np.sort(((P[got[j][1:]] - P[j]) ** 2).sum(1))
        np.testing.assert_allclose(dg, np.sort(d[want[1:]]), rtol=1e-5)
        assert got[j][0] == j
    so = out["sample_out"].cpu().numpy().astype(np.float64)
    assert np.isfinite(so).all() and np.isfinite(out["losses"].cpu().numpy()).all()
    mask = np.zeros(scene.n, np.uint8)
    mask[rows] = 1
    sc = _Scene(scene.means, scene.scales, scene.quats, scene.opacities, scene.betas)
    ref = oracle.gsr(sc, oracle.Settings(), got.astype(np.int32), xi, mask=mask, grads=False)
    m = ref["margins"][rows]
    ok = _clear(m)
    assert ok.mean() > 0.9
    r = rows[ok]
    np.testing.assert_array_equal(so[r, 2].astype(np.int64), ref["gstar"][r])
    np.testing.assert_allclose(so[r, 0], ref["l_sdf"][r], rtol=2e-3, atol=1e-6 * np.abs(ref["l_sdf"][r]).max())
    np.testing.assert_allclose(so[r, 1], ref["l_nor"][r], rtol=1e-3, atol=1e-5)
    log(f"[gpu] gsr full size: {len(r)} sampled samples agree")


@pytest.mark.parametrize("n,k", [(9, 16), (1, 16), (300, 5), (200, 1), (64, 16)])
def test_gsr_small_and_padded_lists(n, k):
    """Lists shorter than k (n < k pads them), other list lengths, a lone
    splat, and a mask that drops every other sample: same bars as above."""
    import torch
    from paper_2411_09156_amd import RasterSettings
    from paper_2411_09156_amd.gsr import gsr, knn
    log(f"[gpu] gsr small n={n} k={k}")
    sc = _scene("cube", n, 4)
    sc.scales = (sc.scales * (2000.0 / max(n, 1)) ** (1.0 / 3.0)).astype(np.float32)
    sp = _splats(sc)
    nb = knn(sp, k)
    torch.cuda.synchronize()
    nbrs = nb["knn"].cpu().numpy().astype(np.int64).astype(np.int32)
    xi = np.random.default_rng([n, k]).standard_normal((n, 3)).astype(np.float32)
    st = oracle.Settings()
    first = oracle.gsr(sc, st, nbrs, xi, grads=False)
    mask = _clear(first["margins"]) & (np.arange(n) % 2 == 0)
    ref = oracle.gsr(sc, st, nbrs, xi, mask=mask.astype(np.uint8), w_sdf=0.6, w_nor=0.4)
    grads = {g: torch.zeros_like(getattr(sp, g)) for g in ("mean", "scale", "quat", "opacity", "beta")}
    out = gsr(sp, RasterSettings(), nb, torch.as_tensor(xi.T.copy(), device="cuda"),
              mask=torch.as_tensor(mask.astype(np.uint8), device="cuda"), w_sdf=0.6, w_nor=0.4, grads=grads)
    torch.cuda.synchronize()
    so = out["sample_out"].cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(so[mask, 2].astype(np.int64), ref["gstar"][mask])
    assert (so[~mask, 2] == -1).all()
    for c, key, bar in ((0, "l_sdf", 1e-4), (1, "l_nor", 1e-3)):
        einf, e2 = norm_errors(so[:, c], ref[key])
        assert einf <= bar and e2 <= bar, (key, einf, e2)
    groups = (("mean", "means", 3), ("scale", "scales", 3), ("quat", "quats", 4), ("opacity", "opacities", 1),
              ("beta", "betas", 1))
    # a group whose reference vanishes (k = 1: a lone splat's losses do not
    # depend on its rotation) is held to 1e-3 of the largest group's norm
    scale = max(np.abs(ref["grads"][rk]).max(initial=0.0) for _, rk, _ in groups)
    for gk, rk, w in groups:
        g = grads[gk].cpu().numpy().astype(np.float64).reshape(w, -1).T
        r = ref["grads"][rk].reshape(-1, w)
        if np.abs(r).max(initial=0.0) < 1e-6 * scale:
            assert np.abs(g - r).max(initial=0.0) <= 1e-3 * scale, gk
            continue
        einf, e2 = norm_errors(g, r)
        assert einf <= 1e-3 and e2 <= 1e-3, (gk, einf, e2)
