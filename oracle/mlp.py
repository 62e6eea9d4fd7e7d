"""Learned SCF start (project extension): oracle of the pair features and of
the 3-layer MLP with its gradient and Adam step.  TEST INFRASTRUCTURE ONLY.

Not from the paper: the paper re-uses the previous geometry's orbitals as
the start of each SCF (AIMD section); this extension predicts the density
instead.  Definitions (shared with the HIP kernels only through this text):

Pair features of (mu, nu), A, B their centres, a = fn_exp[mu], b = fn_exp[nu]:
  f0 = |A - B|
  f1 = ln max(a, b),  f2 = ln min(a, b)
  f3 = 1 if A and B are the same centre else 0
  f4 = exp(-(ab/(a+b)) |A-B|^2)
  f5 = max(c_A, c_B), f6 = min(c_A, c_B), c_X = sum_{C != X} exp(-|R_X - R_C|^2 / 8)
  f7 = sum_C exp(-|P - R_C|^2 / 4),  P = (aA + bB)/(a + b)
Change features of (mu, nu) between a previous geometry R' (converged
density D') and a new one R, same basis and pair list (start along a
geometry sequence: D' plus the predicted change):
  g0 = D'[mu][nu],  g1 = f0(R) - f0(R'),  g2 = f4(R) - f4(R'),
  g3 = f1, g4 = f2, g5 = f3,
  g6 = (c_A + c_B)(R) - (c_A + c_B)(R'),  g7 = f7(R) - f7(R')
Network: x = (f - mu) / sigma;  h1 = silu(x W1 + b1);  h2 = silu(h1 W2 + b2);
  y = h2 w3 + b3,  silu(z) = z / (1 + exp(-z)).  Loss: mean (y - t)^2.
Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
  p -= lr * (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps).
Pins: finite differences of the loss (tests/test_oracle_mlp.py), a one-step
Adam closed form, feature symmetry / special values, and for the change
features the unchanged geometry (all changes zero), a rigid translation of
both geometries (features unchanged) and the distance change of a known
displacement.
"""
from __future__ import annotations

import numpy as np

NFEAT = 8
WIDTH = 256


def pair_features(sys, mu, nu):
    A = sys.xyz[sys.fn_centre[mu]]
    B = sys.xyz[sys.fn_centre[nu]]
    a = sys.fn_exp[mu]
    b = sys.fn_exp[nu]
    R = sys.xyz
    d2 = ((R[:, None, :] - R[None, :, :]) ** 2).sum(-1)
    c = np.exp(-d2 / 8.0).sum(1) - 1.0            # exclude the self term
    cA = c[sys.fn_centre[mu]]
    cB = c[sys.fn_centre[nu]]
    r2 = ((A - B) ** 2).sum(-1)
    P = (a[:, None] * A + b[:, None] * B) / (a + b)[:, None]
    f = np.empty((mu.size, NFEAT))
    f[:, 0] = np.sqrt(r2)
    f[:, 1] = np.log(np.maximum(a, b))
    f[:, 2] = np.log(np.minimum(a, b))
    f[:, 3] = (sys.fn_centre[mu] == sys.fn_centre[nu]).astype(float)
    f[:, 4] = np.exp(-(a * b / (a + b)) * r2)
    f[:, 5] = np.maximum(cA, cB)
    f[:, 6] = np.minimum(cA, cB)
    f[:, 7] = np.exp(-((P[:, None, :] - R[None, :, :]) ** 2).sum(-1) / 4.0).sum(1)
    return f


def delta_features(sys, xyz_prev, mu, nu, D_prev):
    """Change features of each pair between geometry xyz_prev and sys.xyz."""
    new = pair_features(sys, mu, nu)
    old = pair_features(sys.with_xyz(xyz_prev), mu, nu)
    g = np.empty((mu.size, NFEAT))
    g[:, 0] = D_prev[mu, nu]
    g[:, 1] = new[:, 0] - old[:, 0]
    g[:, 2] = new[:, 4] - old[:, 4]
    g[:, 3] = new[:, 1]
    g[:, 4] = new[:, 2]
    g[:, 5] = new[:, 3]
    g[:, 6] = (new[:, 5] + new[:, 6]) - (old[:, 5] + old[:, 6])
    g[:, 7] = new[:, 7] - old[:, 7]
    return g


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed=0, nfeat=NFEAT, width=WIDTH):
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((nfeat, width)) * np.sqrt(2.0 / nfeat),
        "b1": np.zeros(width),
        "W2": rng.standard_normal((width, width)) * np.sqrt(2.0 / width),
        "b2": np.zeros(width),
        "w3": rng.standard_normal(width) * np.sqrt(1.0 / width),
        "b3": np.zeros(1),
    }


def forward(p, x):
    z1 = x @ p["W1"] + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = silu(z2)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(p, x, t):
    y, (x, z1, h1, z2, h2) = forward(p, x)
    n = x.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["w3"]) * dsilu(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"].T) * dsilu(z1)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(p, g, m, v, k, lr, b1=0.9, b2=0.999, eps=1e-8):
    out = {}
    for name in p:
        m[name] = b1 * m[name] + (1 - b1) * g[name]
        v[name] = b2 * v[name] + (1 - b2) * g[name] ** 2
        mh = m[name] / (1 - b1 ** k)
        vh = v[name] / (1 - b2 ** k)
        out[name] = p[name] - lr * mh / (np.sqrt(vh) + eps)
    return out
