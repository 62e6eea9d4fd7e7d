"""Pins of the learned-start oracle: finite differences of the MLP loss,
a one-step Adam closed form, feature special values."""
import numpy as np

import synth
from oracle import mlp as M
from oracle import ri as R


def test_loss_gradient_against_finite_differences():
    rng = np.random.default_rng(1)
    p = M.init_params(seed=2, nfeat=5, width=7)
    x = rng.standard_normal((11, 5))
    t = rng.standard_normal(11)
    loss, g = M.loss_and_grad(p, x, t)
    h = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for k in range(min(flat.size, 6)):
            q = {n: v.copy() for n, v in p.items()}
            q[name].reshape(-1)[k] += h
            lp = M.loss_and_grad(q, x, t)[0]
            q[name].reshape(-1)[k] -= 2 * h
            lm = M.loss_and_grad(q, x, t)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[k]) < 1e-7 * max(1.0, abs(fd)), (name, k)


def test_linear_limit_matches_least_squares_gradient():
    # silu'(0) = 1/2, silu(0) = 0: with zero first-layer weights the network is
    # y = silu(b2-ish) constant; check the bias gradient equals 2 mean(y - t).
    p = M.init_params(seed=3, nfeat=3, width=4)
    p["W1"][:] = 0.0
    x = np.random.default_rng(4).standard_normal((9, 3))
    t = np.random.default_rng(5).standard_normal(9)
    y, _ = M.forward(p, x)
    assert np.allclose(y, y[0])
    loss, g = M.loss_and_grad(p, x, t)
    assert abs(g["b3"][0] - 2 * np.mean(y - t)) < 1e-14


def test_adam_first_step_is_signed_lr():
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    q = M.adam_step(p, g, m, v, 1, lr=0.01, eps=0.0)
    assert np.allclose(q["w"], p["w"] - 0.01 * np.sign(g["w"]))


def test_feature_special_values():
    s = synth.config_system("tiny")
    mu, nu = R.screen_pairs(s)
    f = M.pair_features(s, mu, nu)
    same = s.fn_centre[mu] == s.fn_centre[nu]
    assert np.all(f[same, 0] == 0) and np.all(f[same, 3] == 1) and np.all(f[same, 4] == 1)
    assert np.all(f[~same, 3] == 0) and np.all(f[:, 1] >= f[:, 2])
    # symmetric in (mu, nu)
    g = M.pair_features(s, nu, mu)
    assert np.allclose(f, g, rtol=1e-15, atol=1e-15)
    # single centre: coordination 0, midpoint density 1 (only itself)
    s1 = synth.make_system(np.zeros((1, 3)), [0.5, 2.0], [1.0])
    m1, n1 = R.screen_pairs(s1)
    f1 = M.pair_features(s1, m1, n1)
    assert np.allclose(f1[:, 5], 0) and np.allclose(f1[:, 7], 1)


def test_delta_features_pins():
    """Change features: zero changes for an unchanged geometry; invariant under
    a rigid translation of both geometries; g1 equals the distance change of a
    known displacement of one centre; g0 reads D' at (mu, nu)."""
    s = synth.config_system("tiny")
    mu, nu = R.screen_pairs(s)
    rng = np.random.default_rng(3)
    Dp = rng.standard_normal((s.N, s.N))
    g = M.delta_features(s, s.xyz, mu, nu, Dp)
    assert np.all(g[:, [1, 2, 6, 7]] == 0.0)
    assert np.array_equal(g[:, 0], Dp[mu, nu])
    f = M.pair_features(s, mu, nu)
    assert np.array_equal(g[:, 3:6], f[:, 1:4])
    moved = s.xyz.copy()
    moved[2] += np.array([0.3, -0.1, 0.2])
    g1 = M.delta_features(s.with_xyz(moved), s.xyz, mu, nu, Dp)
    t = np.array([1.5, -2.0, 0.7])
    g2 = M.delta_features(s.with_xyz(moved + t), s.xyz + t, mu, nu, Dp)
    assert np.allclose(g1, g2, rtol=1e-12, atol=1e-12)
    A, B = s.fn_centre[mu], s.fn_centre[nu]
    d_new = np.linalg.norm(moved[A] - moved[B], axis=1)
    d_old = np.linalg.norm(s.xyz[A] - s.xyz[B], axis=1)
    assert np.allclose(g1[:, 1], d_new - d_old, atol=1e-14)
    untouched = (A != 2) & (B != 2)
    assert np.all(g1[untouched, 1] == 0.0) and np.all(g1[untouched, 2] == 0.0)
