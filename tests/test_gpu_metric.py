"""Metric factor and B formation at auxiliary counts that exercise every
branch of the triangular solve: one split with a ragged three-block leaf
(N_aux = 300), two levels of splits with a ragged four-block leaf (690), and
deeper recursion (1200).  Paper: eq. symmetric_ri and eq. biap (A = L L^T,
B = L^{-1} T); Algorithm 1, B formation.

Properties that hold at any size and pin the solve against the factor the
library returned: the residuals of L Bc = T (on a sample of pair columns)
and of L L^{-1} = I, entry by entry against (|L| |X|) for that entry, within
a small multiple of the unit roundoff times the dimension (the backward
error of a triangular solve); L lower triangular with a positive diagonal.
An entry-wise bound, unlike a normwise one, also catches a wrong block of
small entries next to large ones.
The factor itself is pinned against the oracle's metric at the tiny workload
(test_gpu_tiny.py) and through J, K, the energy and the gradient at N=1000.
"""
import numpy as np
import pytest

import synth
from gpu_common import need_gpu, to_np

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.mark.parametrize("n_centres", [10, 23, 40])
def test_solve_and_inverse_residuals(n_centres):
    need_gpu()
    import paper_2407_19614_amd as P
    xyz = synth.ball_cluster(n_centres, 0.01, 2.5, 7)
    s = synth.make_system(xyz, synth.ORB_BIG, synth.AUX_BIG, tau=1e-12)
    print(f"case: metric factor N={s.N} n_aux={s.n_aux}", flush=True)
    pr = P.RIProblem(s, device="cuda", prec=P.FP64)
    pr.build_3c()
    rng = np.random.default_rng(n_centres)
    cols = np.sort(rng.choice(pr.n_pairs, size=min(pr.n_pairs, 384), replace=False))
    cols = np.unique(np.concatenate([cols, [0, pr.n_pairs - 1]]))
    T = to_np(pr.T)[:, cols]                     # (mu nu|P) before the in-place solve
    pr.metric_factor(P.FP64)
    L = to_np(pr.L)
    Linv = to_np(pr.Linv)
    Bc = to_np(pr.T)[:, cols]
    n = s.n_aux
    assert np.all(np.triu(L, 1) == 0.0) and np.all(np.diag(L) > 0.0)
    assert np.all(np.triu(Linv, 1) == 0.0)
    absL = np.abs(L)
    res_b = np.max(np.abs(L @ Bc - T) / (absL @ np.abs(Bc) + 1e-300))
    res_i = np.max(np.abs(L @ Linv - np.eye(n)) / (absL @ np.abs(Linv) + 1e-300))
    print(f"n_aux={n}: entry-wise |L Bc - T| {res_b:.2e}, |L Linv - I| {res_i:.2e} "
          f"(bound {4 * n * EPS:.1e})", flush=True)
    assert res_b < 4 * n * EPS
    assert res_i < 4 * n * EPS
