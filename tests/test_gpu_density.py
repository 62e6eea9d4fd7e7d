"""Fock build from a density matrix alone (no orbitals), and the SCF started
from the Fock matrix of a guess density."""
import numpy as np
import pytest

import synth
from oracle import ri as R
from oracle import scf as S
from tests.gpu_common import need_gpu, problem, to_np, dev

pytestmark = pytest.mark.gpu


def random_density(N, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, N)) * 0.1
    return A + A.T           # symmetric, indefinite, not idempotent


def test_density_jk_matches_brute_force_tiny():
    need_gpu()
    print("case: density J/K tiny vs oracle brute force", flush=True)
    s = synth.config_system("tiny")
    pr = problem(s)
    eri = R.ri_tensor_brute(s)
    for seed in (0, 1):
        D = random_density(s.N, seed)
        J, K = (to_np(t) for t in pr.fock_jk_density(dev(D)))
        Jr, Kr = R.jk_from_tensor(eri, D)
        assert np.abs(J - Jr).max() < 1e-11 * max(1.0, np.abs(Jr).max())
        assert np.abs(K - Kr).max() < 1e-11 * max(1.0, np.abs(Kr).max())
        assert np.array_equal(K, K.T)


def test_density_jk_equals_orbital_jk():
    need_gpu()
    print("case: density J/K vs orbital J/K, tiny and n400 (150 slabs)", flush=True)
    for name in ("tiny", "n400"):
        s = synth.config_system(name)
        pr = problem(s)
        C = synth.random_coeffs(s.N, s.n_occ, seed=11)
        J0, K0, _ = (to_np(t) for t in pr.fock_jk(dev(C)))
        J1, K1 = (to_np(t) for t in pr.fock_jk_density(dev(2.0 * C @ C.T)))
        assert np.abs(J1 - J0).max() < 1e-11 * np.abs(J0).max(), name
        assert np.abs(K1 - K0).max() < 1e-11 * np.abs(K0).max(), name


def test_scf_from_density_fock_start():
    need_gpu()
    print("case: SCF from the Fock matrix of a perturbed density, tiny", flush=True)
    s = synth.config_system("tiny")
    ri = R.RIData(s)
    ref = S.run_scf(s, ri, tol_E=1e-12, tol_e=1e-10)
    pr = problem(s)
    D = ref.D + 0.05 * random_density(s.N, 3)
    r, *_ = pr.energy(tol_E=1e-11, tol_err=1e-9, guess_density=dev(D), density_fock=True)
    assert r["converged"] and abs(r["E_total"] - ref.E) < 1e-10
    r2, *_ = pr.energy(tol_E=1e-11, tol_err=1e-9, guess_density=dev(ref.D), density_fock=True)
    assert r2["converged"] and abs(r2["E_total"] - ref.E) < 1e-10 and r2["n_iter"] <= 3
