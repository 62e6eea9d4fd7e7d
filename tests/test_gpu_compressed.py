"""Compressed-B form (B not resident; B_c decompressed per auxiliary slab on
every call): results identical to the resident packed form, and to the
oracle, for the Fock build, the SCF and the gradient."""
import numpy as np
import pytest

import synth
from oracle import ri as R
from tests.gpu_common import need_gpu, to_np, dev

pytestmark = pytest.mark.gpu


def pair(system, prec):
    import paper_2407_19614_amd as P
    out = []
    for comp in (False, True):
        pr = P.RIProblem(system, prec=prec, compressed=comp)
        pr.build_3c()
        pr.metric_factor(prec)
        out.append(pr)
    assert out[0].B is not None and out[1].B is None
    return out


@pytest.mark.parametrize("prec_name", ["FP64", "FP32"])
def test_compressed_fock_identical_tiny(prec_name):
    need_gpu()
    import paper_2407_19614_amd as P
    prec = getattr(P, prec_name)
    print(f"case: compressed tiny {prec_name}", flush=True)
    s = synth.config_system("tiny")
    res, comp = pair(s, prec)
    C = dev(synth.random_coeffs(s.N, s.n_occ, seed=3))
    J0, K0, g0 = (to_np(t) for t in res.fock_jk(C))
    J1, K1, g1 = (to_np(t) for t in comp.fock_jk(C))
    assert np.array_equal(J0, J1) and np.array_equal(K0, K1) and np.array_equal(g0, g1)
    if prec == P.FP64:
        Jr, Kr = R.RIData(s).JK(to_np(C))
        assert np.abs(K1 - Kr).max() < 1e-11 and np.abs(J1 - Jr).max() < 1e-11


def test_compressed_energy_and_gradient_tiny():
    need_gpu()
    import paper_2407_19614_amd as P
    print("case: compressed tiny energy+gradient", flush=True)
    s = synth.config_system("tiny")
    res, comp = pair(s, P.FP64)
    r0, C0, F0, _ = res.energy(tol_E=1e-11, tol_err=1e-9)
    r1, C1, F1, _ = comp.energy(tol_E=1e-11, tol_err=1e-9)
    assert r0["E_total"] == r1["E_total"] and r0["n_iter"] == r1["n_iter"]
    g0 = to_np(res.gradient(C0, F0))
    g1 = to_np(comp.gradient(C1, F1))
    # the per-atom gradient sums use atomic adds: equal up to summation order
    assert np.abs(g0 - g1).max() < 1e-13


def test_compressed_multi_slab_identical():
    """N=400 (1200 auxiliaries: slabs of 256 with a ragged last one)."""
    need_gpu()
    import paper_2407_19614_amd as P
    print("case: compressed n400 fp64, 5 slabs", flush=True)
    s = synth.config_system("n400")
    assert s.n_aux > 4 * P.binding.COMPRESSED_SLAB and s.n_aux % P.binding.COMPRESSED_SLAB != 0
    res, comp = pair(s, P.FP64)
    C = dev(synth.random_coeffs(s.N, s.n_occ, seed=5))
    J0, K0, _ = (to_np(t) for t in res.fock_jk(C))
    J1, K1, _ = (to_np(t) for t in comp.fock_jk(C))
    assert np.array_equal(J0, J1) and np.array_equal(K0, K1)
