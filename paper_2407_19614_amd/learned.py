"""Learned SCF start along a geometry sequence (project extension).

Orchestration only: every numerical step (integrals, SCF, features, network
forward/backward/Adam, density scatter/gather, occupied-space projection)
runs in libri's kernels through the C ABI; this module sequences the calls
and moves tensors.

Workflow (the workload of the extension): a 40-centre cluster (N=400,
N_aux=1200, n_occ=40) displaced by a seeded Gaussian random walk; every
geometry's SCF from the core-Hamiltonian guess supplies the training target
(converged D on significant pairs); the network trains on the first part of
the sequence and starts the SCF on the rest.  Plain core-Hamiltonian SCF is
the fallback and the reference for the energy.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as B

# Feature normalisation fixed from the feature definitions (no data statistics):
# distance ~ [0, 25] bohr, log-exponents ~ [-2.6, 4.6], flags and overlaps in
# [0, 1], coordination and midpoint densities ~ [0, 3].
FEAT_SHIFT = np.array([8.0, 1.0, 1.0, 0.5, 0.5, 1.0, 1.0, 1.0], dtype=np.float32)
FEAT_SCALE = np.array([6.0, 2.0, 2.0, 0.5, 0.5, 1.0, 1.0, 1.0], dtype=np.float32)
# Change features (ri_pair_delta_features), from their definitions and the
# sequence's step (displacements of ~0.05 bohr per coordinate): the previous
# density element ~ [-2, 2], changes of distance ~ 0.05 bohr, changes of the
# overlap factor, coordination and midpoint density ~ 0.02-0.05; exponents and
# the same-centre flag as above.  Targets are the density change times
# DELTA_TARGET_SCALE (changes of ~1e-3 become ~1).
DELTA_SHIFT = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 0.5, 0.0, 0.0], dtype=np.float32)
DELTA_SCALE = np.array([0.5, 0.05, 0.02, 2.0, 2.0, 0.5, 0.05, 0.05], dtype=np.float32)
DELTA_TARGET_SCALE = 1000.0


def init_network(seed=0, device="cuda", delta=False):
    """He-style initial weights; the random draws are inputs (numpy PCG64).
    delta: the network of the density change along a sequence (its feature
    normalisation)."""
    rng = np.random.default_rng(seed)
    nf, w = B.NFEAT, B.WIDTH
    p = {"W1": rng.standard_normal((nf, w)) * np.sqrt(2.0 / nf), "b1": np.zeros(w),
         "W2": rng.standard_normal((w, w)) * np.sqrt(2.0 / w), "b2": np.zeros(w),
         "w3": rng.standard_normal(w) * np.sqrt(1.0 / w), "b3": np.zeros(1)}
    shift, scale = (DELTA_SHIFT, DELTA_SCALE) if delta else (FEAT_SHIFT, FEAT_SCALE)
    return B.MLP(B.pack_params(p), shift, scale, device=device)


def solve(system, guess=None, guess_density=None, tol_E=1e-10, tol_err=1e-8, max_iter=100, gradient=False,
          device="cuda"):
    """One geometry: pairs and 3c integrals, metric factor, SCF (and gradient)."""
    pr = B.RIProblem(system, device=device)
    pr.build_3c()
    pr.metric_factor(B.FP64)
    res, C, F, D = pr.energy(tol_E=tol_E, tol_err=tol_err, max_iter=max_iter, guess=guess,
                             guess_density=guess_density, raise_on_noconv=False)
    g = pr.gradient(C, F) if (gradient and res["converged"]) else None
    return pr, res, C, D, g


def generate(systems, device="cuda", log=None, prev_baseline=True):
    """Reference SCF (core-H start) for each geometry; returns per-geometry
    dicts with features and targets on the device: the density on the pairs
    ("feat", "target") and, from the second geometry on, its change from the
    previous geometry's ("dfeat", "dtarget", targets times
    DELTA_TARGET_SCALE).  With prev_baseline, also records the iterations of
    an SCF started from the previous geometry's orbitals (the paper's
    molecular-dynamics start)."""
    import torch
    out = []
    C_prev = D_prev = xyz_prev = None
    for k, s in enumerate(systems):
        t0 = time.perf_counter()
        pr, res, C, D, _ = solve(s, device=device)
        it_prev = None
        if prev_baseline and C_prev is not None:
            r2 = pr.energy(tol_E=1e-10, tol_err=1e-8, guess=C_prev, raise_on_noconv=False)[0]
            it_prev = r2["n_iter"]
        feat = pr.pair_features().clone()
        targ = pr.density_to_pairs(D).clone()
        rec = {"feat": feat, "target": targ, "E": res["E_total"], "iters_core": res["n_iter"],
               "iters_prev": it_prev, "converged": res["converged"], "n_pairs": pr.n_pairs}
        if D_prev is not None:
            rec["dfeat"] = pr.pair_delta_features(xyz_prev, D_prev).clone()
            rec["dtarget"] = pr.density_change_pairs(D, D_prev, DELTA_TARGET_SCALE).clone()
        out.append(rec)
        D_prev, xyz_prev = D.clone(), pr.xyz.clone()
        C_prev = C.clone()
        torch.cuda.synchronize()
        if log and (k % 50 == 0):
            log(f"geometry {k}: E={res['E_total']:.10f} iters={res['n_iter']} "
                f"{(time.perf_counter() - t0) * 1e3:.1f} ms")
        del pr
    return out


def train(net, data, steps=3000, batch=16384, lr=2e-3, seed=0, log=None, delta=False):
    """Mini-batch Adam on the concatenated training pairs (device-resident);
    delta: on the change records (from the second geometry on)."""
    import torch
    fk, tk = ("dfeat", "dtarget") if delta else ("feat", "target")
    feat = torch.cat([d[fk] for d in data if fk in d])
    targ = torch.cat([d[tk] for d in data if tk in d])
    n = feat.shape[0]
    rng = np.random.default_rng(seed)
    losses = []
    perm = None
    pos = n
    for k in range(steps):
        if pos + batch > n:
            perm = torch.tensor(rng.permutation(n), device=feat.device)
            fs, ts = feat.index_select(0, perm), targ.index_select(0, perm)
            pos = 0
        lr_k = lr * (0.5 * (1 + np.cos(np.pi * k / steps)) * 0.95 + 0.05)
        loss = net.train_step(fs[pos:pos + batch], ts[pos:pos + batch], lr_k)
        pos += batch
        if k % 250 == 0 or k == steps - 1:
            losses.append((k, float(loss.item())))
            if log:
                log(f"train step {k}: loss {losses[-1][1]:.3e}")
    return losses


def predict_density(net, pr, prec=B.MLP_BF16):
    feat = pr.pair_features()
    d = net.forward(feat, prec)
    return pr.density_from_pairs(d)


def delta_start(net_d, pr, xyz_prev, D_prev, prec=B.MLP_BF16):
    """Start for the next geometry of a sequence: the previous geometry's
    converged density D_prev (at positions xyz_prev) plus the change the
    change network predicts on the new geometry's pairs."""
    d = net_d.forward(pr.pair_delta_features(xyz_prev, D_prev), prec)
    return pr.density_add_pairs(d, 1.0 / DELTA_TARGET_SCALE, D_prev)
