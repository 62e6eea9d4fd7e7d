"""Pins of the oracle's RI J/K, SCF and gradient (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import integrals as I
from oracle import ri as R
from oracle import scf as S
from oracle import gradient as G


@pytest.fixture(scope="module")
def tiny():
    s = synth.config_system("tiny")
    ri = R.RIData(s)
    res = S.run_scf(s, ri)
    return s, ri, res


def test_product_aux_ri_is_exact():
    # Auxiliary set = products of orbital pairs: the RI tensor equals the
    # exact four-index ERIs (eq. ri_eri becomes an identity).
    s = synth.config_system("tiny")
    sp = R.product_aux_system(s)
    eri_ri = R.ri_tensor_brute(sp)
    eri = I.eri4(s)
    assert np.abs(eri_ri - eri).max() < 1e-11 * np.abs(eri).max()


def test_two_centre_product_set_tight():
    s = synth.make_system(np.array([[0, 0, 0], [1.4, 0, 0]], float), [0.5, 2.0], [1.0])
    sp = R.product_aux_system(s)
    eri = I.eri4(s)
    assert np.abs(R.ri_tensor_brute(sp) - eri).max() < 1e-14 * np.abs(eri).max() * 10


def test_fit_path_matches_brute_force(tiny):
    s, ri, _ = tiny
    C = synth.random_coeffs(s.N, s.n_occ, seed=3)
    D = 2 * C @ C.T
    J, K = ri.JK(C)
    Jb, Kb = R.jk_from_tensor(R.ri_tensor_brute(s), D)
    assert np.abs(J - Jb).max() < 1e-12 * np.abs(Jb).max()
    assert np.abs(K - Kb).max() < 1e-12 * np.abs(Kb).max()


def test_B_convention_reproduces_ri_tensor(tiny):
    s, ri, _ = tiny
    B = ri.B_packed_dense()                      # [N_aux, n_pairs]
    N = s.N
    Bd = np.zeros((s.n_aux, N, N))
    Bd[:, ri.mu, ri.nu] = B
    Bd[:, ri.nu, ri.mu] = B
    eri = np.einsum("pmn,pls->mnls", Bd, Bd)
    ref = R.ri_tensor_brute(s)
    assert np.abs(eri - ref).max() < 1e-11 * np.abs(ref).max()


def test_K_symmetric_psd_and_J_bound(tiny):
    s, ri, res = tiny
    C = synth.random_coeffs(s.N, s.n_occ, seed=11)
    D = 2 * C @ C.T
    J, K = ri.JK(C)
    assert np.abs(K - K.T).max() < 1e-13 * np.abs(K).max()
    assert np.abs(J - J.T).max() < 1e-13 * np.abs(J).max()
    assert np.linalg.eigvalsh(K).min() > -1e-12 * np.abs(K).max()
    # robust fitting: E_J^RI <= E_J^exact for the same density
    Jx, _ = S.exact_jk(s)(C)
    assert 0.5 * np.sum(D * J) <= 0.5 * np.sum(D * Jx) + 1e-12


@pytest.mark.parametrize("a", [0.4, 0.7670, 1.5])
def test_single_helium_closed_form(a):
    s = synth.make_system(np.zeros((1, 3)), [a], [2 * a])
    res = S.run_scf(s)
    E = 3 * a - 4 * 2 * np.sqrt(2 * a / np.pi) + 2 * np.sqrt(a / np.pi)
    assert abs(res.E - E) < 1e-13


def test_single_helium_variational_minimum():
    k = (8 * np.sqrt(2) - 2) / np.sqrt(np.pi)
    a_star = (k / 6) ** 2
    s = synth.make_system(np.zeros((1, 3)), [a_star], [2 * a_star])
    assert abs(S.run_scf(s).E + (8 * np.sqrt(2) - 2) ** 2 / (12 * np.pi)) < 1e-13
    for da in (-1e-3, 1e-3):
        s2 = synth.make_system(np.zeros((1, 3)), [a_star + da], [2 * (a_star + da)])
        assert S.run_scf(s2).E > S.run_scf(s).E


def test_scf_invariants(tiny):
    s, ri, res = tiny
    Sm = I.overlap(s)
    D = res.D
    assert res.converged
    assert abs(np.trace(D @ Sm) - 2 * s.n_occ) < 1e-10
    assert np.abs(D @ Sm @ D - 2 * D).max() < 1e-10
    e = res.F @ D @ Sm - Sm @ D @ res.F
    assert np.abs(e).max() < 1e-8
    assert res.E <= res.E_guess
    # E = tr(Dh) + 1/2 tr(DJ) - 1/2 tr(DK) + Enn
    assert abs(res.E - (res.E_1e + res.E_J + res.E_K + res.E_nuc)) < 1e-12
    # stationarity: a small occupied-virtual rotation raises the energy quadratically
    C = res.C
    n = s.n_occ
    rng = np.random.default_rng(0)
    Kr = np.zeros((s.N, s.N))
    Kr[n:, :n] = rng.normal(size=(s.N - n, n))
    Kr = Kr - Kr.T
    from scipy.linalg import expm
    h = I.core_hamiltonian(s)
    Es = []
    for t in (1e-3, 2e-3):
        Ct = C @ expm(t * Kr)
        Co = Ct[:, :n]
        Dt = 2 * Co @ Co.T
        J, K = ri.JK(Co)
        Es.append(np.sum(Dt * h) + 0.5 * np.sum(Dt * J) - 0.5 * np.sum(Dt * K) + res.E_nuc - res.E)
    assert Es[0] > 0 and Es[1] > 0
    assert abs(Es[1] / Es[0] - 4.0) < 0.05


def test_product_aux_scf_reproduces_exact_hf():
    s = synth.config_system("tiny")
    sp = R.product_aux_system(s)
    E_ri = S.run_scf(sp).E
    E_ex = S.run_scf(s, jk=S.exact_jk(s)).E
    assert abs(E_ri - E_ex) < 1e-9


def test_gradient_against_finite_differences(tiny):
    s, ri, res = tiny
    g = G.analytic_gradient(s, res, ri)
    fd = G.fd_gradient(s, res, atoms=[0, 3, 6])
    assert np.abs(fd[[0, 3, 6]] - g[[0, 3, 6]]).max() < 1e-7


def test_gradient_invariants(tiny):
    s, ri, res = tiny
    g = G.analytic_gradient(s, res, ri)
    assert np.abs(g.sum(0)).max() < 1e-11
    torque = np.cross(s.xyz, g).sum(0)
    assert np.abs(torque).max() < 1e-10


def test_gradient_single_atom_and_dimer():
    s = synth.make_system(np.array([[0.3, -0.2, 0.5]]), [0.3, 1.0, 3.5], [0.2, 0.8, 2.0, 7.0])
    res = S.run_scf(s)
    assert np.abs(G.analytic_gradient(s, res)).max() < 1e-12
    s2 = synth.make_system(np.array([[0, 0, 0], [0, 0, 2.7]], float), [0.3, 1.0, 3.5], [0.2, 0.8, 2.0, 7.0])
    res2 = S.run_scf(s2)
    g = G.analytic_gradient(s2, res2)
    assert np.abs(g[:, :2]).max() < 1e-12
    assert abs(g[0, 2] + g[1, 2]) < 1e-12
    fd = G.fd_gradient(s2, res2, atoms=[1])
    assert abs(fd[1, 2] - g[1, 2]) < 1e-8


def test_planted_factor_mistake_is_caught(tiny, monkeypatch):
    # The paper prints -1/2 in Y and Z (valid for sqrt(2)-scaled orbitals);
    # using it with D = 2 C C^T must fail the finite-difference pin.
    s, ri, res = tiny
    g_ok = G.analytic_gradient(s, res, ri)
    orig = G.sla.cho_solve

    def half(*a, **k):
        return 0.25 * orig(*a, **k)          # turns the factor 2 into 1/2
    calls = {"n": 0}

    def patched(cho, b, **k):
        calls["n"] += 1
        return half(cho, b, **k) if calls["n"] == 1 else orig(cho, b, **k)
    monkeypatch.setattr(G.sla, "cho_solve", patched)
    g_bad = G.analytic_gradient(s, res, ri)
    monkeypatch.undo()
    fd = G.fd_gradient(s, res, atoms=[0])
    assert np.abs(fd[0] - g_ok[0]).max() < 1e-7
    assert np.abs(fd[0] - g_bad[0]).max() > 1e-5
