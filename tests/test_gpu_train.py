"""GPU checks of the training loop (Sec. 3.4, 4.2) on a small synthetic scene
with the schedule compressed to 40 iterations: its first iteration equals the
entry points called by hand (bit for bit), the shape reset, entropy phase,
neighbour-list refreshes and pruning happen at their iterations with their
effects, and, with those phases off, the loss falls while fitting targets
rendered from a ground-truth scene whose colours and opacities were
perturbed."""
import numpy as np
import pytest

from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _setup(seed=5):
    import torch

    import gesr_inputs as gi
    from paper_2411_09156_amd import Rasterizer, RasterSettings, Splats
    from paper_2411_09156_amd.train import Schedule, raw_from_activated
    sc = gi.tiny_scene(seed, n=1500, width=96, height=80, deg=1, n_views=3, spread=0.7)
    rs = RasterSettings(sh_degree=1)
    gt = Splats.from_aos(sc.means, sc.scales, sc.quats, np.clip(sc.opacities, 0.6, 0.95), sc.betas, sc.sh)
    full = Rasterizer(sc.cameras, rs)
    img = full.forward(gt)["image"]
    targets, off = [], 0
    for c in sc.cameras:
        npx = 3 * c.width * c.height
        targets.append(img[off:off + npx].view(3, c.height, c.width).clone())
        off += npx
    rng = np.random.default_rng(seed)
    sh = np.array(sc.sh, np.float64)
    sh[:, 0, :] += 0.3 * rng.standard_normal((sc.n, 3))
    op = np.clip(np.clip(sc.opacities, 0.6, 0.95) + 0.2 * rng.standard_normal(sc.n), 0.05, 0.97)
    raw = raw_from_activated(sc.means, sc.scales, sc.quats, op, sc.betas, sh)
    sch = Schedule(iterations=40, drt_fraction=0.5, entropy_start=10, entropy_iters=10, gsr_start=20,
                   gsr_iters=20, knn_every=5, shape_reset_every=15, prune_at=(20,))
    torch.cuda.synchronize()
    return sc, rs, raw, targets, sch, full


def _clone(raw):
    from paper_2411_09156_amd.optim import RAW_FIELDS, RawParams
    return RawParams(*(getattr(raw, k).clone() for k in RAW_FIELDS))


def test_first_iteration_equals_the_entry_points():
    import torch
    from paper_2411_09156_amd.optim import RAW_FIELDS, SplatAdam
    from paper_2411_09156_amd.train import Trainer
    sc, rs, raw, targets, sch, _ = _setup()
    manual = SplatAdam(_clone(raw))
    tr = Trainer(sc.cameras, _clone(raw), targets, rs, sch)
    tr.step()
    rast, target = tr._stage(sch.drt_start)
    sp = manual.splats
    f = rast.forward(sp, sync=True)
    img = f["image"][:target.numel()]
    dL, _ = rast.loss_eq8(img, target, sch.lambda_dssim)
    g = rast.render_bwd(sp, f["proj"], f["bins"], f["final_T"], f["n_contrib"], dL)
    manual.step(g)
    torch.cuda.synchronize()
    for k in RAW_FIELDS:
        assert torch.equal(getattr(tr.opt.raw, k), getattr(manual.raw, k)), k
        assert torch.equal(getattr(tr.opt.m, k), getattr(manual.m, k)), k


def test_graph_replays_equal_eager_iterations():
    """Ten iterations (two DRT stages, a shape reset) through the captured
    graphs equal the same iterations run eagerly, bit for bit, and no
    iteration overflowed its list capacity."""
    import torch
    from paper_2411_09156_amd.optim import RAW_FIELDS
    from paper_2411_09156_amd.train import Schedule, Trainer
    sc, rs, raw, targets, _, _ = _setup()
    sch = Schedule(iterations=10, drt_fraction=0.5, entropy_start=3, entropy_iters=4, gsr_start=10 ** 9,
                   shape_reset_every=6, prune_at=())
    a = Trainer(sc.cameras, _clone(raw), targets, rs, sch, graph=True)
    b = Trainer(sc.cameras, _clone(raw), targets, rs, sch, graph=False)
    la = [a.step()["loss"] for _ in range(10)]
    lb = [b.step()["loss"] for _ in range(10)]
    torch.cuda.synchronize()
    for k in RAW_FIELDS:
        assert torch.equal(getattr(a.opt.raw, k), getattr(b.opt.raw, k)), k
    assert [float(x) for x in la] == [float(x) for x in lb]
    assert a.recaptures == 0 and len(a._steps) >= 2


def test_schedule_events():
    import torch
    from paper_2411_09156_amd.train import Trainer
    sc, rs, raw, targets, sch, full = _setup()
    tr = Trainer(sc.cameras, raw, targets, rs, sch)

    def full_l1():
        img = full.forward(tr.opt.splats)["image"]
        tgt = torch.cat([t.reshape(-1) for t in targets])
        return float((img - tgt).abs().mean())
    l1_0 = full_l1()
    sizes, refreshed = [], []
    for it in range(sch.iterations):
        r = tr.step()
        sizes.append(r["n"])
        assert np.isfinite(float(r["l1"])) and np.isfinite(float(r["loss"])), it
        if sch.entropy_start <= it < sch.entropy_start + sch.entropy_iters:
            assert tr.opt.config.entropy_weight == sch.entropy_weight
        else:
            assert tr.opt.config.entropy_weight == 0.0
        if sch.gsr_start <= it < sch.gsr_start + sch.gsr_iters:
            assert r["gsr"] is not None and torch.isfinite(r["gsr"]).all()
            if tr._nbrs_it == it:
                refreshed.append(it)
        else:
            assert r["gsr"] is None
        if (it + 1) % sch.shape_reset_every == 0:
            assert bool((tr.opt.raw.beta == sch.shape_reset_value).all())
            assert bool((tr.opt.m.beta == 0).all() and (tr.opt.v.beta == 0).all())
        if it + 1 == 20:
            assert sizes[-1] < sizes[0]
            assert bool((tr.opt.raw.opacity_logit >= 0).all()) and bool((tr.opt.raw.beta >= 0.5).all())
            assert tr.opt.m.n == tr.opt.raw.n == tr.opt.splats.n
    assert refreshed == [20, 25, 30, 35]
    assert tr._rasts, "no DRT stage"
    scales = {k for k in tr._rasts}
    assert len(scales) > 3  # the resolution changed along the schedule
    l1_1 = full_l1()
    # the compressed schedule resets every shape twice and prunes: no fit expected here
    log(f"[gpu] training: splats {sizes[0]} -> {sizes[-1]}, full-resolution L1 {l1_0:.5f} -> {l1_1:.5f}")


def test_fitting_phase_reduces_the_loss():
    """Before the regularisation phases (no resets, pruning, entropy or
    regulariser), the loop fits the perturbed colours and opacities."""
    import torch
    from paper_2411_09156_amd.train import Schedule, Trainer
    sc, rs, raw, targets, _, full = _setup()
    sch = Schedule(iterations=30, drt_start=0.5, drt_fraction=0.5, entropy_start=10 ** 9, gsr_start=10 ** 9,
                   shape_reset_every=0, prune_at=())
    tr = Trainer(sc.cameras, raw, targets, rs, sch)
    tgt = torch.cat([t.reshape(-1) for t in targets])
    l1_0 = float((full.forward(tr.opt.splats)["image"] - tgt).abs().mean())
    tr.run()
    l1_1 = float((full.forward(tr.opt.splats)["image"] - tgt).abs().mean())
    log(f"[gpu] fitting: full-resolution L1 {l1_0:.5f} -> {l1_1:.5f} in {sch.iterations} iterations")
    assert l1_1 < 0.9 * l1_0
