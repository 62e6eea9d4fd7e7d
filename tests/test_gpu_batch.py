"""Batched lockstep SCF (many molecules per launch, HIP-graph replay)
against the per-molecule SCF and the oracle."""
import numpy as np
import pytest

import synth
from oracle import ri as R
from oracle import scf as S
from tests.gpu_common import need_gpu

pytestmark = pytest.mark.gpu


def small_batch():
    out = []
    for k, nc in enumerate([3, 7, 5, 12, 9, 4]):
        xyz = synth.ball_cluster(nc, 0.01, 2.5, 300 + k)
        out.append(synth.make_system(xyz, synth.ORB_BIG[::2], synth.AUX_BIG[::3], tau=1e-12))
    return out


@pytest.mark.parametrize("graph", [False, True])
def test_batched_fp64_matches_single_and_oracle(graph):
    need_gpu()
    import paper_2407_19614_amd as P
    from paper_2407_19614_amd.binding import energy_batched
    print(f"case: batched fp64 graph={graph}", flush=True)
    systems = small_batch()
    probs = []
    for s in systems:
        pr = P.RIProblem(s)
        pr.build_3c()
        pr.metric_factor(P.FP64)
        probs.append(pr)
    res, Cs, _ = energy_batched(probs, P.FP64, tol_E=1e-11, tol_err=1e-9, use_graph=graph)
    for k, (s, pr, r) in enumerate(zip(systems, probs, res)):
        single, *_ = pr.energy(tol_E=1e-11, tol_err=1e-9)
        assert r["converged"]
        assert abs(r["E_total"] - single["E_total"]) < 1e-9, (k, r["E_total"], single["E_total"])
        if k < 3:
            ref = S.run_scf(s, R.RIData(s), tol_E=1e-12, tol_e=1e-10)
            assert abs(r["E_total"] - ref.E) < 1e-9


def test_batched_fp32_error():
    need_gpu()
    import paper_2407_19614_amd as P
    from paper_2407_19614_amd.binding import energy_batched
    print("case: batched fp32", flush=True)
    systems = small_batch()
    probs = []
    for s in systems:
        pr = P.RIProblem(s, prec=P.FP32)
        pr.build_3c()
        pr.metric_factor(P.FP32)
        probs.append(pr)
    res, _, _ = energy_batched(probs, P.FP32, tol_E=1e-7, tol_err=1e-5)
    for s, r in zip(systems, res):
        ref = S.run_scf(s, R.RIData(s), tol_E=1e-12, tol_e=1e-10)
        assert r["converged"] and abs(r["E_total"] - ref.E) < 1e-6
