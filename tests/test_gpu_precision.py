"""Reduced-precision exchange (FP32 B and X/K contractions) at the tiny
workload: errors against the FP64 oracle, to the precision extension's bar
(|dE| <= 1e-6 Eh, gradient <= 1e-5 Eh/bohr)."""
import numpy as np
import pytest

import synth
from oracle import ri as R
from oracle import scf as S
from oracle import gradient as G
from tests.gpu_common import need_gpu, problem, to_np, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ref():
    need_gpu()
    s = synth.config_system("tiny")
    ri = R.RIData(s)
    res = S.run_scf(s, ri, tol_E=1e-12, tol_e=1e-10)
    return s, ri, res, G.analytic_gradient(s, res, ri)


def test_fp32_fock_jk(ref):
    s, ri, *_ = ref
    import paper_2407_19614_amd as P
    print("case: tiny fock_jk fp32", flush=True)
    pr = problem(s, P.FP32)
    C = synth.random_coeffs(s.N, s.n_occ, seed=0)
    J, K, _ = pr.fock_jk(dev(C))
    Jr, Kr = ri.JK(C)
    dJ = np.abs(to_np(J) - Jr).max()
    dK = np.abs(to_np(K) - Kr).max()
    print(f"fp32 max|dJ|={dJ:.2e} max|dK|={dK:.2e}", flush=True)
    assert dJ < 1e-11            # J stays FP64 (compressed B)
    assert dK < 1e-5 * np.abs(Kr).max()


def test_fp32_energy_and_gradient(ref):
    s, ri, res, gref = ref
    import paper_2407_19614_amd as P
    print("case: tiny energy+gradient fp32", flush=True)
    pr = problem(s, P.FP32)
    r, C, F, D = pr.energy(tol_E=1e-10, tol_err=1e-7)
    dE = abs(r["E_total"] - res.E)
    g = to_np(pr.gradient())
    dg = np.abs(g - gref).max()
    print(f"fp32 |dE|={dE:.2e} max|dg|={dg:.2e}", flush=True)
    assert dE <= 1e-6
    assert dg <= 1e-5


def test_fp32_final_fp64_energy(ref):
    """FP32 exchange iterations, then one exchange build in FP64 arithmetic at
    the converged density (RI_FINAL_FP64): the same iterations as plain FP32,
    and an energy within 1e-8 Eh of the oracle at the tiny workload; on a
    40-centre cluster (N = 400) within 1e-7 Eh of the FP64 path."""
    s, ri, res, _ = ref
    import paper_2407_19614_amd as P
    print("case: tiny energy fp32 + final fp64", flush=True)
    pr = problem(s, P.FP32)
    r32, *_ = pr.energy(tol_E=1e-10, tol_err=1e-7)
    rf, *_ = pr.energy(tol_E=1e-10, tol_err=1e-7, final_fp64=True)
    print(f"tiny: fp32 |dE|={abs(r32['E_total'] - res.E):.2e} final |dE|={abs(rf['E_total'] - res.E):.2e}", flush=True)
    assert rf["converged"] and rf["n_iter"] == r32["n_iter"]
    assert abs(rf["E_1e"] - r32["E_1e"]) <= 1e-12 * abs(r32["E_1e"])
    assert abs(rf["E_total"] - res.E) < 1e-8
    print("case: N=400 energy fp32 + final fp64 vs fp64", flush=True)
    xyz = synth.ball_cluster(40, 0.01, 2.5, 7)
    s4 = synth.make_system(xyz, synth.ORB_BIG, synth.AUX_BIG, tau=1e-12)
    r64, *_ = problem(s4, P.FP64).energy(tol_E=1e-10, tol_err=1e-8)
    p4 = problem(s4, P.FP32)
    r32, *_ = p4.energy(tol_E=1e-8, tol_err=1e-6)
    rf, *_ = p4.energy(tol_E=1e-8, tol_err=1e-6, final_fp64=True)
    e32, ef = abs(r32["E_total"] - r64["E_total"]), abs(rf["E_total"] - r64["E_total"])
    print(f"N=400: fp32 |dE|={e32:.2e} final |dE|={ef:.2e}", flush=True)
    assert rf["converged"] and ef < 1e-7


@pytest.mark.parametrize("prec_name,tolK,tolE", [("BF16X3", 5e-4, 1e-4), ("BF16X6", 1e-6, 1e-6)])
def test_bf16_split_fock_and_energy(ref, prec_name, tolK, tolE):
    s, ri, res, _ = ref
    import paper_2407_19614_amd as P
    prec = {"BF16X3": P.BF16X3, "BF16X6": P.BF16X6}[prec_name]
    print(f"case: tiny {prec_name}", flush=True)
    pr = problem(s, prec)
    C = synth.random_coeffs(s.N, s.n_occ, seed=0)
    J, K, _ = pr.fock_jk(dev(C))
    Jr, Kr = ri.JK(C)
    dJ = np.abs(to_np(J) - Jr).max()
    dK = np.abs(to_np(K) - Kr).max() / np.abs(Kr).max()
    r, *_ = pr.energy(tol_E=1e-9, tol_err=1e-6, max_iter=60, raise_on_noconv=False)
    dE = abs(r["E_total"] - res.E)
    print(f"{prec_name} max|dJ|={dJ:.2e} max rel|dK|={dK:.2e} |dE|={dE:.2e} conv={r['converged']}", flush=True)
    assert dJ < 1e-11
    assert dK < tolK
    assert dE < tolE
