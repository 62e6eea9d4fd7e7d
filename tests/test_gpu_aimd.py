"""AIMD wrapper (velocity Verlet, NVE) through the C ABI: trajectory parity
with the oracle's Verlet on its own RI-HF energies and gradients, and the
second-order energy error of the integrator as an end-to-end gradient check."""
import numpy as np
import pytest

import synth
from oracle import md as M
from tests.gpu_common import need_gpu

pytestmark = pytest.mark.gpu


def test_aimd_trajectory_matches_oracle():
    need_gpu()
    from paper_2407_19614_amd.aimd import NVE
    print("case: aimd tiny vs oracle, 5 steps of 100 au", flush=True)
    s = synth.config_system("tiny")
    dt, n = 100.0, 5
    md = NVE(s, dt, tol_E=1e-12, tol_err=1e-10)
    g = md.run(n, keep_xyz=True)
    ref = M.verlet(s.xyz, np.zeros_like(s.xyz), np.full(s.n_centres, M.HE_MASS), M.ri_hf_energy_grad(s), dt, n)
    for k in range(n + 1):
        x, v, E, K = ref[k]
        assert np.abs(g["xyz"][k] - x).max() < 1e-9, k
        assert abs(g["E_pot"][k] - E) < 1e-9, (k, g["E_pot"][k], E)
        assert abs(g["E_kin"][k] - K) < 1e-11 + 1e-7 * K, (k, g["E_kin"][k], K)
    assert g["E_kin"][-1] > 0.0


def test_aimd_energy_error_is_second_order():
    need_gpu()
    from paper_2407_19614_amd.aimd import NVE
    print("case: aimd tiny dt^2 scaling, 2000 au", flush=True)
    s = synth.config_system("tiny")
    exc = []
    for dt, n in ((100.0, 20), (50.0, 40)):
        g = NVE(s, dt, tol_E=1e-12, tol_err=1e-10).run(n)
        Et = np.array(g["E_tot"])
        exc.append(np.abs(Et - Et[0]).max())
        # the previous step's orbitals start each SCF: later steps need fewer iterations
        assert np.mean(g["scf_iters"][1:]) < g["scf_iters"][0]
    assert 3.0 < exc[0] / exc[1] < 5.0, exc
