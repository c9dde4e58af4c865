"""Pins of the oracle's optimiser step (the training schedule of Sec. 4.2:
Adam with per-group learning rates, the paper's 1.5e-3 for the shape
parameter, and the opacity-entropy regularisation that drives opacities to a
binary state).

Fixed by Adam's closed forms (the first step moves every parameter by
lr g / (|g| + eps); under a constant gradient the bias-corrected moments are
exactly g and g^2 at every step) and by central differences of the loss the
raw-parameter gradients belong to: L = sum(c . activated(raw)) +
w mean_i H(sigmoid(logit_i)), with H the binary entropy written out here.
"""
import numpy as np
import pytest

import oracle


def _raw(rng, n, K):
    return {"means": rng.standard_normal((n, 3)), "log_scales": rng.uniform(-4, -1, (n, 3)),
            "quats": rng.standard_normal((n, 4)), "opacity_logits": rng.standard_normal(n),
            "betas": rng.uniform(1, 4, n), "sh": rng.standard_normal((n, K, 3)) * 0.1}


def _grads(rng, n, K):
    return {"means": rng.standard_normal((n, 3)), "scales": rng.standard_normal((n, 3)),
            "quats": rng.standard_normal((n, 4)), "opacities": rng.standard_normal(n),
            "betas": rng.standard_normal(n), "sh": rng.standard_normal((n, K, 3))}


def _zeros(raw):
    return {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in raw.items()}


def test_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(0)
    n, K = 50, 4
    raw, gr = _raw(rng, n, K), _grads(rng, n, K)
    st = oracle.AdamSettings(eps=1e-8)
    p, m, v, act = oracle.adam_step(raw, _zeros(raw), _zeros(raw), gr, 1, st)
    g = oracle.adam_raw_grads(raw, gr, st)
    lrs = {"means": st.lr_mean, "log_scales": st.lr_scale, "quats": st.lr_quat, "opacity_logits": st.lr_opacity,
           "betas": st.lr_beta}
    for k, lr in lrs.items():
        np.testing.assert_allclose(p[k], raw[k] - lr * g[k] / (np.abs(g[k]) + 1e-8), rtol=0, atol=1e-15)
    lr_sh = np.full((n, K, 3), st.lr_sh_rest)
    lr_sh[:, 0] = st.lr_sh_dc
    np.testing.assert_allclose(p["sh"], raw["sh"] - lr_sh * g["sh"] / (np.abs(g["sh"]) + 1e-8), atol=1e-15)
    np.testing.assert_allclose(act["scales"], np.exp(p["log_scales"]), rtol=1e-15)
    np.testing.assert_allclose(act["opacities"], 1 / (1 + np.exp(-p["opacity_logits"])), rtol=1e-15)


def test_constant_gradient_walks_linearly():
    """Bias correction makes the moments exactly g and g^2 under a constant raw
    gradient, so t steps move by t lr g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    n = 20
    st = oracle.AdamSettings(eps=1e-8)
    raw = {"means": rng.standard_normal((n, 3)), "log_scales": np.zeros((n, 3)), "quats": np.zeros((n, 4)),
           "opacity_logits": np.zeros(n), "betas": np.zeros(n), "sh": np.zeros((n, 1, 3))}
    gm = rng.standard_normal((n, 3))
    gr = {"means": gm, "scales": np.zeros((n, 3)), "quats": np.zeros((n, 4)), "opacities": np.zeros(n),
          "betas": np.zeros(n), "sh": np.zeros((n, 1, 3))}
    p, m, v = raw, _zeros(raw), _zeros(raw)
    T = 25
    for t in range(1, T + 1):
        p, m, v, _ = oracle.adam_step(p, m, v, gr, t, st)
    np.testing.assert_allclose(p["means"], raw["means"] - T * st.lr_mean * gm / (np.abs(gm) + 1e-8), atol=1e-13)


@pytest.mark.parametrize("w", [0.0, 0.7])
def test_raw_gradients_match_central_differences(w):
    """Chain rule through exp and sigmoid, and the entropy term."""
    rng = np.random.default_rng(2)
    n, K = 6, 4
    raw, c = _raw(rng, n, K), _grads(rng, n, K)
    st = oracle.AdamSettings(entropy_weight=w)

    def loss(r):
        s = np.exp(r["log_scales"])
        o = 1 / (1 + np.exp(-r["opacity_logits"]))
        H = -o * np.log(o) - (1 - o) * np.log(1 - o)
        return (np.sum(c["means"] * r["means"]) + np.sum(c["scales"] * s) + np.sum(c["quats"] * r["quats"])
                + np.sum(c["opacities"] * o) + np.sum(c["betas"] * r["betas"]) + np.sum(c["sh"] * r["sh"])
                + w * H.mean())

    g = oracle.adam_raw_grads(raw, c, st)
    for k in oracle.RAW_KEYS:
        flat = np.asarray(raw[k], np.float64).reshape(-1)
        for j in range(flat.size):
            h = 1e-6
            rp = {kk: np.array(vv, np.float64, copy=True) for kk, vv in raw.items()}
            rm = {kk: np.array(vv, np.float64, copy=True) for kk, vv in raw.items()}
            rp[k].reshape(-1)[j] += h
            rm[k].reshape(-1)[j] -= h
            fd = (loss(rp) - loss(rm)) / (2 * h)
            assert g[k].reshape(-1)[j] == pytest.approx(fd, rel=1e-7, abs=1e-9), (k, j)


def test_prune_hand_example():
    """Opacity 0.5 and beta 0.5 thresholds: logit 0 is kept (opacity exactly
    0.5), -1e-7 is not; beta 0.5 is kept, 0.4 is not; order and moments follow."""
    lg = np.array([-1.0, 0.0, 0.3, -1e-7, 2.0, -0.0])
    be = np.array([1.0, 0.4, 0.6, 3.0, 0.5, 2.0])
    n = 6
    raw = {"means": np.arange(18.0).reshape(n, 3), "log_scales": np.zeros((n, 3)), "quats": np.zeros((n, 4)),
           "opacity_logits": lg, "betas": be, "sh": np.arange(n * 3.0).reshape(n, 1, 3)}
    m = {k: v + 100 for k, v in raw.items()}
    p, pm, pv, keep = oracle.prune(raw, m, None, 0.5, 0.5)
    assert keep.tolist() == [False, False, True, False, True, True]
    assert p["means"][:, 0].tolist() == [6.0, 12.0, 15.0]
    assert pm["betas"].tolist() == [100.6, 100.5, 102.0]
    assert pv is None
    # thresholds of 0 keep everything
    assert oracle.prune_keep(raw, 0.0, 0.0).all()


def test_prune_opacity_rule_matches_sigmoid_away_from_the_threshold():
    """keep == (sigmoid(logit) >= min_opacity) wherever the opacity is not
    within 1e-6 of the threshold."""
    rng = np.random.default_rng(3)
    lg = rng.uniform(-8, 8, 20000).astype(np.float32).astype(np.float64)
    raw = {"opacity_logits": lg, "betas": np.ones_like(lg)}
    for mo in (0.005, 0.3, 0.5, 0.9):
        keep = oracle.prune_keep(raw, mo, 0.0)
        o = 1 / (1 + np.exp(-lg))
        far = np.abs(o - mo) > 1e-6
        np.testing.assert_array_equal(keep[far], (o >= mo)[far])
        assert 0 < keep.sum() < keep.size


def test_shape_reset():
    rng = np.random.default_rng(4)
    n, K = 7, 4
    raw, m = _raw(rng, n, K), _raw(rng, n, K)
    p2, m2, v2 = oracle.shape_reset(raw, m, None, 2.0)
    assert (p2["betas"] == 2.0).all() and (m2["betas"] == 0.0).all() and v2 is None
    np.testing.assert_array_equal(p2["means"], raw["means"])
    assert not (raw["betas"] == 2.0).any()  # inputs untouched
