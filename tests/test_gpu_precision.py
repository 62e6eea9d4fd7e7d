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


# Relative max|dK| bounds for a random occupied block at the 8-centre workload.
# Two bfloat16 parts hold each operand of X = B C and K = X X^T to 2^-17
# relative, and the three products drop lo x lo (at most 2^-18): a CPU
# emulation with exact accumulation gives 8.2e-6 for BF16X3, so 3e-5 allows
# four such errors.  Three parts leave 2^-25 and FP32 accumulation inside each
# 64-deep chunk dominates; 1e-6 is FP32's own bar on K.
KTOL = {"BF16X3": 3e-5, "BF16X6": 1e-6}


@pytest.mark.parametrize("prec_name", ["BF16X3", "BF16X6"])
def test_bf16_split_fock(ref, prec_name):
    s, ri, res, _ = ref
    import paper_2407_19614_amd as P
    prec = {"BF16X3": P.BF16X3, "BF16X6": P.BF16X6}[prec_name]
    print(f"case: tiny fock_jk {prec_name}", flush=True)
    pr = problem(s, prec)
    C = synth.random_coeffs(s.N, s.n_occ, seed=0)
    J, K, _ = pr.fock_jk(dev(C))
    Jr, Kr = ri.JK(C)
    dJ = np.abs(to_np(J) - Jr).max()
    dK = np.abs(to_np(K) - Kr).max() / np.abs(Kr).max()
    print(f"{prec_name} max|dJ|={dJ:.2e} max rel|dK|={dK:.2e}", flush=True)
    assert dJ < 1e-11
    assert dK < KTOL[prec_name]


@pytest.mark.parametrize("prec_name,final", [("BF16X3", True), ("BF16X6", False), ("BF16X6", True)])
def test_bf16_split_energy_and_gradient(ref, prec_name, final):
    """Split-BF16 SCF at the precision bar: |dE| <= 1e-6 Eh from a converged
    SCF and a gradient within 1e-5 Eh/bohr of the oracle.  BF16X3 runs with the
    final FP64 exchange build (its plain SCF is rejected, see
    test_bf16x3_plain_scf_rejected); the gradient of the split forms is the
    FP64 gradient at the orbitals the split SCF converged to."""
    s, ri, res, gref = ref
    import paper_2407_19614_amd as P
    prec = {"BF16X3": P.BF16X3, "BF16X6": P.BF16X6}[prec_name]
    print(f"case: tiny energy+gradient {prec_name} final={final}", flush=True)
    pr = problem(s, prec)
    # with the final FP64 build the density's error enters the energy only to
    # second order, so the split iterations stop above their noise floor
    # (BF16X3's iteration energies carry ~1e-5 Eh of rounding noise: its energy
    # test sits above that and the commutator test governs)
    tol = ((1e-4 if prec_name == "BF16X3" else 1e-6), 3e-5) if final else (1e-9, 1e-6)
    r, *_ = pr.energy(tol_E=tol[0], tol_err=tol[1], max_iter=60, final_fp64=final)
    assert r["converged"]
    dE = abs(r["E_total"] - res.E)
    g = to_np(pr.gradient())
    dg = np.abs(g - gref).max()
    print(f"{prec_name} final={final} |dE|={dE:.2e} iters={r['n_iter']} max|dg|={dg:.2e}", flush=True)
    assert dE <= 1e-6
    assert dg <= 1e-5


def test_bf16x3_plain_scf_rejected(ref):
    s, *_ = ref
    import paper_2407_19614_amd as P
    print("case: tiny plain BF16X3 SCF is rejected", flush=True)
    pr = problem(s, P.BF16X3)
    with pytest.raises(P.RIError) as e:
        pr.energy(tol_E=1e-9, tol_err=1e-6)
    assert e.value.code == 7


def test_bf16_final_fp64_n400():
    """40-centre cluster (N = 400): the split-BF16 SCF with the final FP64
    build within 1e-7 Eh of the FP64 path, and its gradient within 1e-5."""
    need_gpu()
    import paper_2407_19614_amd as P
    xyz = synth.ball_cluster(40, 0.01, 2.5, 7)
    s4 = synth.make_system(xyz, synth.ORB_BIG, synth.AUX_BIG, tau=1e-12)
    print("case: N=400 energy+gradient fp64 reference", flush=True)
    p64 = problem(s4, P.FP64)
    r64, *_ = p64.energy(tol_E=1e-10, tol_err=1e-8)
    g64 = to_np(p64.gradient())
    for name, prec in (("BF16X3", P.BF16X3), ("BF16X6", P.BF16X6)):
        print(f"case: N=400 {name} + final fp64", flush=True)
        pb = problem(s4, prec)
        rb, *_ = pb.energy(tol_E=1e-4 if name == "BF16X3" else 1e-6, tol_err=3e-5, final_fp64=True)
        dE = abs(rb["E_total"] - r64["E_total"])
        dg = np.abs(to_np(pb.gradient()) - g64).max()
        print(f"N=400 {name}: |dE|={dE:.2e} iters={rb['n_iter']} max|dg|={dg:.2e}", flush=True)
        assert rb["converged"] and dE < 1e-7 and dg < 1e-5
