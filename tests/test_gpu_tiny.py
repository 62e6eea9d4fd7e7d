"""GPU parity at the tiny workload (8 centres, N=32, N_aux=80, n_occ=8,
unscreened): every stage through the C-ABI against the oracle."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import integrals as I
from oracle import ri as R
from oracle import scf as S
from tests.gpu_common import need_gpu, problem, to_np, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    need_gpu()
    s = synth.config_system("tiny")
    ri = R.RIData(s)
    return s, ri


def test_pairs_and_three_centre(tiny):
    s, ri = tiny
    import paper_2407_19614_amd as P
    print("case: tiny build_3c", flush=True)
    pr = P.RIProblem(s)
    n = pr.build_3c()
    # tau = 0 keeps every pair whose (mu nu|mu nu) does not underflow to 0
    assert n == ri.n_pairs
    pairs = to_np(pr.pairs)
    assert np.array_equal(pairs[:, 0], ri.mu) and np.array_equal(pairs[:, 1], ri.nu)
    T = to_np(pr.T)
    assert np.abs(T - ri.T).max() <= 1e-14 * np.abs(ri.T).max() + 0.0


def test_metric_factor_and_B(tiny):
    s, ri = tiny
    print("case: tiny metric_factor", flush=True)
    pr = problem(s)
    L = to_np(pr.L)
    Lref = np.linalg.cholesky(ri.A)
    assert np.abs(L - Lref).max() < 1e-12 * np.abs(Lref).max()
    Linv = to_np(pr.Linv)
    assert np.abs(Linv @ Lref - np.eye(s.n_aux)).max() < 1e-9
    Bc = to_np(pr.T)
    Bref = ri.B_packed_dense()
    # reported, not gated tightly: triangular-solve forward error ~ cond(L) eps
    assert np.abs(Bc - Bref).max() < 1e-9 * np.abs(Bref).max()


def test_fock_jk_random_orbitals(tiny):
    s, ri = tiny
    print("case: tiny fock_jk", flush=True)
    pr = problem(s)
    for seed in (0, 1):
        C = synth.random_coeffs(s.N, s.n_occ, seed=seed)
        J, K, gamma = pr.fock_jk(dev(C))
        Jr, Kr = ri.JK(C)
        J, K = to_np(J), to_np(K)
        assert np.abs(J - Jr).max() < 1e-11, np.abs(J - Jr).max()
        assert np.abs(K - Kr).max() < 1e-11, np.abs(K - Kr).max()
        D = 2 * C @ C.T
        d, c = ri.gamma_fit(D)
        # gamma = L^{-1} d, so |gamma|^2 = d^T A^{-1} d
        g = to_np(gamma)
        assert abs(g @ g - d @ c) < 1e-11 * abs(d @ c)


def test_energy_matches_oracle(tiny):
    s, ri = tiny
    print("case: tiny energy", flush=True)
    ref = S.run_scf(s, ri, tol_E=1e-12, tol_e=1e-9)
    pr = problem(s)
    res, C, F, D = pr.energy(tol_E=1e-12, tol_err=1e-9)
    assert res["converged"]
    assert abs(res["E_total"] - ref.E) < 1e-10, (res["E_total"], ref.E)
    assert abs(res["E_J"] - ref.E_J) < 1e-9 and abs(res["E_K"] - ref.E_K) < 1e-9
    Dg = to_np(D)
    assert np.abs(Dg - ref.D).max() < 1e-7
    C = to_np(C)
    Sm = I.overlap(s)
    assert np.abs(C.T @ Sm @ C - np.eye(s.n_occ)).max() < 1e-12


def test_gradient_matches_oracle_and_fd(tiny):
    s, ri = tiny
    from oracle import gradient as G
    print("case: tiny gradient", flush=True)
    ref = S.run_scf(s, ri, tol_E=1e-12, tol_e=1e-10)
    gref = G.analytic_gradient(s, ref, ri)
    pr = problem(s)
    res, C, F, D = pr.energy(tol_E=1e-12, tol_err=1e-10)
    g = to_np(pr.gradient())
    assert np.abs(g - gref).max() < 1e-8, np.abs(g - gref).max()
    assert np.abs(g.sum(0)).max() < 1e-10
    fd = G.fd_gradient(s, ref, atoms=[2])
    assert np.abs(g[2] - fd[2]).max() < 1e-7
