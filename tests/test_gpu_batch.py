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
    res, Cs, _ = energy_batched(probs, P.FP64, tol_E=1e-11, tol_err=1e-9, use_graph=graph, raise_on_noconv=False)
    print(" ".join(f"[N={s.N} conv={r['converged']} it={r['n_iter']} E={r['E_total']:.10f}]"
                   for s, r in zip(systems, res)), flush=True)
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
    res, _, _ = energy_batched(probs, P.FP32, tol_E=1e-7, tol_err=1e-5, raise_on_noconv=False)
    print(" ".join(f"[N={s.N} conv={r['converged']} it={r['n_iter']} E={r['E_total']:.10f}]"
                   for s, r in zip(systems, res)), flush=True)
    for s, r in zip(systems, res):
        ref = S.run_scf(s, R.RIData(s), tol_E=1e-12, tol_e=1e-10)
        assert r["converged"] and abs(r["E_total"] - ref.E) < 1e-6


def test_pack_b_matches_metric_factor():
    """ri_pack_b repacks the fitted tensor into the same bytes that
    ri_metric_factor writes, in FP64, FP32 and the split-BF16 forms."""
    need_gpu()
    import torch
    import paper_2407_19614_amd as P
    print("case: ri_pack_b vs ri_metric_factor", flush=True)
    s = small_batch()[3]
    for prec in (P.FP64, P.FP32, P.BF16X3, P.BF16X6):
        pr = P.RIProblem(s, prec=prec)
        pr.build_3c()
        pr.metric_factor(prec)
        B2 = pr.pack_b(prec)
        torch.cuda.synchronize()
        assert B2.numel() == pr.B.numel() and torch.equal(B2, pr.B), prec


def test_batched_fp32_final_fp64():
    """FP32 exchange through the SCF, then one exchange build in FP64
    arithmetic (from the FP32-stored B) at the converged density.  The energy
    is stationary in the density, so only B's FP32 rounding is left to first
    order: the energy agrees with the FP64 batched SCF and the oracle to
    1e-7 Eh, ten times inside the 1e-6 Eh bar of reduced precision."""
    need_gpu()
    import paper_2407_19614_amd as P
    from paper_2407_19614_amd.binding import energy_batched, prepare_batch
    print("case: batched fp32 + final fp64", flush=True)
    systems = small_batch()
    probs = prepare_batch(systems, P.FP32 | P.FINAL_FP64, workers=2)
    res, _, _ = energy_batched(probs, P.FP32 | P.FINAL_FP64, tol_E=1e-8, tol_err=1e-6)
    res32, _, _ = energy_batched(probs, P.FP32, tol_E=1e-8, tol_err=1e-6)
    p64 = prepare_batch(systems, P.FP64, workers=2)
    res64, _, _ = energy_batched(p64, P.FP64, tol_E=1e-11, tol_err=1e-9)
    for k, (s, r, r32, r64) in enumerate(zip(systems, res, res32, res64)):
        print(k, r["E_total"] - r64["E_total"], r32["E_total"] - r64["E_total"], flush=True)
        assert r["converged"] and r["n_iter"] == r32["n_iter"]
        assert abs(r["E_total"] - r64["E_total"]) < 1e-7, (k, r["E_total"], r64["E_total"])
        # only the exchange energy changes: h, J and D are those of the last FP32 iteration
        assert abs(r["E_1e"] - r32["E_1e"]) < 1e-12 * max(1.0, abs(r32["E_1e"]))
        if k < 2:
            ref = S.run_scf(s, R.RIData(s), tol_E=1e-12, tol_e=1e-10)
            assert abs(r["E_total"] - ref.E) < 1e-7
    # molecules that do not converge keep their FP32 energies
    rn, _, _ = energy_batched(probs, P.FP32 | P.FINAL_FP64, max_iter=2, raise_on_noconv=False)
    rn32, _, _ = energy_batched(probs, P.FP32, max_iter=2, raise_on_noconv=False)
    for r, r32 in zip(rn, rn32):
        assert not r["converged"] and r["E_total"] == r32["E_total"] and r["E_K"] == r32["E_K"]


def test_batched_autotune_and_forced_shapes_agree():
    """Molecules in four size buckets (N = 40, 140, 270, 400): the autotuner's
    choices are valid, and the SCF energies under the default shapes, the
    autotuned ones and two forced extremes (128-tiles with split 8, 64-tiles
    with split 1) agree to 1e-9 Eh."""
    need_gpu()
    import paper_2407_19614_amd as P
    from paper_2407_19614_amd.binding import BatchTuning, batch_autotune, energy_batched
    print("case: batched autotune, 4 buckets", flush=True)
    systems = []
    for k, nc in enumerate([4, 14, 27, 40]):
        xyz = synth.ball_cluster(nc, 0.01, 2.5, 500 + k)
        systems.append(synth.make_system(xyz, synth.ORB_BIG, synth.AUX_BIG[::2], tau=1e-12))
    assert [s.N for s in systems] == [40, 140, 270, 400]
    probs = []
    for s in systems:
        pr = P.RIProblem(s)
        pr.build_3c()
        pr.metric_factor(P.FP64)
        probs.append(pr)
    tune = batch_autotune(probs, P.FP64)
    d = tune.as_dict()
    print("tuning", d, flush=True)
    assert d["n_buckets"] == 4
    for b in range(4):
        assert d["gemm_tile"][b] in (64, 128) and d["syrk_split"][b] in (1, 2, 4, 8, 16)
        assert d["gemm_ms"][b] > 0 and d["syrk_ms"][b] > 0

    def forced(tile, split):
        t = BatchTuning()
        t.n_buckets = 4
        for b in range(4):
            t.gemm_tile[b], t.syrk_split[b] = tile, split
        return t

    kw = dict(tol_E=1e-11, tol_err=1e-9)
    E0 = [r["E_total"] for r in energy_batched(probs, P.FP64, **kw)[0]]
    for t in (tune, forced(128, 16), forced(64, 1)):
        res = energy_batched(probs, P.FP64, tuning=t, **kw)[0]
        for k, r in enumerate(res):
            assert r["converged"]
            assert abs(r["E_total"] - E0[k]) < 1e-9, (k, r["E_total"], E0[k])


def test_prepare_batch_matches_sequential_setup():
    """Setups issued from several host threads on their own streams give the
    same pairs, fitted tensors, factors and packed B as one-by-one setup, and
    the batched SCF on them the same energies."""
    need_gpu()
    import torch
    import paper_2407_19614_amd as P
    from paper_2407_19614_amd.binding import energy_batched, prepare_batch
    print("case: prepare_batch, 6 molecules, 4 workers", flush=True)
    systems = small_batch()
    par = prepare_batch(systems, P.FP64, workers=4)
    for s, pp in zip(systems, par):
        pr = P.RIProblem(s)
        pr.build_3c()
        pr.metric_factor(P.FP64)
        torch.cuda.synchronize()
        assert pp.n_pairs == pr.n_pairs
        for name in ("pairs", "T", "L", "Linv", "B"):
            assert torch.equal(getattr(pp, name), getattr(pr, name)), name
    res, _, _ = energy_batched(par, P.FP64, tol_E=1e-11, tol_err=1e-9)
    for s, r in zip(systems, res):
        ref = S.run_scf(s, R.RIData(s), tol_E=1e-12, tol_e=1e-10)
        assert r["converged"] and abs(r["E_total"] - ref.E) < 1e-9


def test_prepared_batch_beside_a_running_scf():
    """A batch prepared on a host thread while another batch's SCF runs on the
    caller's stream gives bit-identical setups and the same SCF energies as a
    batch prepared alone."""
    need_gpu()
    import torch
    import paper_2407_19614_amd as P
    from paper_2407_19614_amd.binding import PreparedBatch, energy_batched, prepare_batch
    print("case: PreparedBatch beside a running batched SCF", flush=True)
    systems = small_batch()
    first, second = systems[:3], systems[3:]
    p1 = prepare_batch(first, P.FP64, workers=2)
    nxt = PreparedBatch(second, P.FP64, workers=2)
    r1, _, _ = energy_batched(p1, P.FP64, tol_E=1e-11, tol_err=1e-9)
    p2 = nxt.result()
    r2, _, _ = energy_batched(p2, P.FP64, tol_E=1e-11, tol_err=1e-9)
    alone = prepare_batch(second, P.FP64, workers=2)
    torch.cuda.synchronize()
    for a, b in zip(p2, alone):
        for name in ("pairs", "T", "L", "Linv", "B"):
            assert torch.equal(getattr(a, name), getattr(b, name)), name
    ra, _, _ = energy_batched(alone, P.FP64, tol_E=1e-11, tol_err=1e-9)
    for x, y in zip(r2, ra):
        assert x["converged"] and y["converged"] and x["E_total"] == y["E_total"]
    assert all(r["converged"] for r in r1)
