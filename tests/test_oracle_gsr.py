"""Pins of the oracle's surface regulariser (DyGASR, arXiv 2411.09156, Sec. 3.3,
Eq. 9-13, with the 16-nearest-neighbour density of Sec. 4.2).

Fixed by what does not use the oracle's arithmetic: neighbour lists against a
numpy brute force; a lone splat, where x - mu = M xi makes the Mahalanobis
vector exactly xi, so d = o exp(-kappa |xi|^beta), h = s_min xi_k* and the
normal term reduces to the rotation-free |sign(xi_k*) D^-1 xi / |D^-1 xi| - e_k*|^2
(D = diag(phi s)); two splats through scipy's rotations and an independent
numpy evaluation of Eq. 9; and central differences of the loss for every
parameter of every neighbour (the sample point moves with its splat).
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle


class _Scene:
    def __init__(self, means, scales, quats, opac, betas):
        self.means = np.asarray(means, np.float64).reshape(-1, 3)
        self.scales = np.asarray(scales, np.float64).reshape(-1, 3)
        self.quats = np.asarray(quats, np.float64).reshape(-1, 4)
        self.opacities = np.asarray(opac, np.float64).reshape(-1)
        self.betas = np.asarray(betas, np.float64).reshape(-1)


def _phi(beta, rho):
    return 2.0 / (1.0 + np.exp(-rho * (beta - 2.0)))


def _rot(q):
    q = np.asarray(q, np.float64)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def _random(rng, n, spread=1.0):
    return _Scene(rng.uniform(-spread, spread, (n, 3)), np.exp(rng.uniform(-3.0, -1.5, (n, 3))),
                  rng.standard_normal((n, 4)), rng.uniform(0.3, 0.95, n), rng.uniform(1.0, 4.0, n))


def test_knn_matches_brute_force():
    rng = np.random.default_rng(0)
    for n, K in ((300, 16), (40, 16), (9, 16), (1, 1), (2, 4)):
        P = rng.uniform(-1, 1, (n, 3))
        got = oracle.knn(P, K)
        D = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
        for j in range(n):
            others = [i for i in range(n) if i != j]
            order = sorted(others, key=lambda i: (D[j, i], i))[:K - 1]
            want = [j] + order + [-1] * (K - 1 - len(order))
            assert got[j].tolist() == want, (n, j)


@pytest.mark.parametrize("beta,o,kappa", [(2.0, 1.0, 0.5), (3.3, 1.0, 0.5), (1.4, 0.7, 0.5), (2.6, 0.9, 1.0)])
def test_lone_splat_closed_form(beta, o, kappa):
    rng = np.random.default_rng(int(beta * 10))
    st = oracle.Settings(kappa=kappa)
    rho, kp = float(np.float32(st.rho)), float(np.float32(kappa))
    sc = _Scene([[0.3, -0.2, 0.5]], [[0.4, 0.05, 0.2]], [[0.8, 0.3, -0.4, 0.2]], [o], [beta])
    sigma = _phi(beta, rho) * sc.scales[0]
    ks = int(np.argmin(sigma))
    smin = sigma[ks]
    for _ in range(6):
        xi = rng.standard_normal(3)
        r = oracle.gsr(sc, st, np.zeros((1, 1), np.int32), xi[None], grads=False)
        B = np.sqrt(max(np.linalg.norm(xi) ** beta - np.log(o) / kp, 0.0))
        A = abs(xi[ks]) ** (beta / 2)
        assert r["l_sdf"][0] == pytest.approx(smin * abs(A - B), rel=1e-12, abs=1e-15)
        v = xi / sigma
        sg = 1.0 if xi[ks] >= 0 else -1.0
        e = np.zeros(3)
        e[ks] = 1.0
        assert r["l_nor"][0] == pytest.approx(np.sum((sg * v / np.linalg.norm(v) - e) ** 2), rel=1e-12, abs=1e-14)
        assert r["gstar"][0] == 0


def test_flat_gaussian_on_its_normal_has_zero_sdf_loss():
    """beta = 2, opacity 1, x on the normal line: d equals the ideal density of
    Eq. 10, so f = fbar (the signed distance) and the normal term vanishes."""
    st = oracle.Settings()
    sc = _Scene([[0.0, 0.0, 0.0]], [[0.3, 0.2, 0.01]], [[1.0, 0.0, 0.0, 0.0]], [1.0], [2.0])
    for t in (-2.0, -0.3, 0.7, 2.5):
        r = oracle.gsr(sc, st, np.zeros((1, 1), np.int32), np.array([[0.0, 0.0, t]]), grads=False)
        assert r["l_sdf"][0] == pytest.approx(0.0, abs=1e-15)
        assert r["l_nor"][0] == pytest.approx(0.0, abs=1e-15)


def test_two_splats_match_an_independent_evaluation():
    rng = np.random.default_rng(5)
    st = oracle.Settings()
    rho, kp = float(np.float32(st.rho)), float(np.float32(st.kappa))
    for trial in range(8):
        sc = _random(rng, 2, spread=0.15)
        xi = rng.standard_normal(3)
        nb = np.array([[0, 1], [1, 0]], np.int32)
        r = oracle.gsr(sc, st, nb, np.stack([xi, np.zeros(3)]), mask=[1, 0], grads=False)
        R = [_rot(q) for q in sc.quats]
        sig = [_phi(b, rho) * s for b, s in zip(sc.betas, sc.scales)]
        x = sc.means[0] + R[0] @ (sig[0] * xi)
        T, G = [], []
        for i in range(2):
            y = (R[i].T @ (x - sc.means[i])) / sig[i]
            q = y @ y
            Ti = sc.opacities[i] * np.exp(-kp * q ** (sc.betas[i] / 2))
            T.append(Ti)
            G.append(-kp * sc.betas[i] * q ** (sc.betas[i] / 2 - 1) * Ti * (R[i] @ (y / sig[i])))
        d, gd = sum(T), sum(G)
        g = int(np.argmax(T))
        ks = int(np.argmin(sig[g]))
        n = R[g][:, ks]
        smin = sig[g][ks]
        h = (x - sc.means[g]) @ n
        sg = 1.0 if h >= 0 else -1.0
        fbar = smin * (abs(h) / smin) ** (sc.betas[g] / 2)
        f = smin * np.sqrt(max(-np.log(d), 0.0) / kp)
        assert r["gstar"][0] == g
        assert r["l_sdf"][0] == pytest.approx(abs(fbar - f), rel=1e-10, abs=1e-14)
        assert r["l_nor"][0] == pytest.approx(np.sum((-sg * gd / np.linalg.norm(gd) - n) ** 2), rel=1e-10, abs=1e-13)
        assert r["l_sdf"][1] == 0.0 and r["l_nor"][1] == 0.0 and r["gstar"][1] == -1  # masked


@pytest.mark.parametrize("w_sdf,w_nor", [(1.0, 0.0), (0.0, 1.0), (0.7, 0.3)])
def test_gradients_match_central_differences(w_sdf, w_nor):
    rng = np.random.default_rng(11)
    st = oracle.Settings()
    n, K = 24, 16
    sc = _random(rng, n, spread=0.25)
    nb = oracle.knn(sc.means, K)
    xi = rng.standard_normal((n, 3))
    base = oracle.gsr(sc, st, nb, xi, w_sdf=w_sdf, w_nor=w_nor)
    # keep samples whose discrete choices are far from their thresholds
    m = base["margins"]
    mask = ((m[:, 0] > 1e-2) & (m[:, 1] > 1e-3) & (m[:, 2] > 1e-3) & (m[:, 3] > 1e-3) & (m[:, 4] > 1e-2) & (m[:, 6] > 1e-3))
    assert mask.sum() >= 12
    res = oracle.gsr(sc, st, nb, xi, mask=mask.astype(np.uint8), w_sdf=w_sdf, w_nor=w_nor)

    def loss(s):
        r = oracle.gsr(s, st, nb, xi, mask=mask.astype(np.uint8), grads=False)
        return float(w_sdf * r["l_sdf"].sum() + w_nor * r["l_nor"].sum())
    fields = (("means", 3), ("scales", 3), ("quats", 4), ("opacities", 1), ("betas", 1))
    worst = 0.0
    for name, width in fields:
        g = res["grads"][name].reshape(n, width)
        for i in rng.choice(n, 10, replace=False):
            for a in range(width):
                h = 1e-6 * max(1.0, abs(getattr(sc, name).reshape(n, width)[i, a]))
                plus, minus = _copy(sc), _copy(sc)
                getattr(plus, name).reshape(n, width)[i, a] += h
                getattr(minus, name).reshape(n, width)[i, a] -= h
                fd = (loss(plus) - loss(minus)) / (2 * h)
                err = abs(g[i, a] - fd) / max(abs(fd), 1e-2)
                worst = max(worst, err)
                assert err < 2e-5, (name, i, a, g[i, a], fd)


def _copy(s):
    return _Scene(s.means.copy(), s.scales.copy(), s.quats.copy(), s.opacities.copy(), s.betas.copy())
