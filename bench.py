"""RI-JK Fock-build throughput on one MI355X at N=1000.

Workload: 100 helium-like centres in a seeded random cluster (0.01 /bohr^3,
minimum separation 2.5 bohr), orbital basis 10 even-tempered s-Gaussians per
centre from 0.08 with ratio 2.2 (N=1000), auxiliary basis 30 per centre from
0.05 with ratio 1.6 (N_aux=3000), n_occ=100, Schwarz threshold 1e-12; B stored
decompressed (packed symmetric tiles) in FP64 in HBM.

A step is one RI Fock build (gamma/J on compressed pairs, X^P = B^P C_occ,
K = sum X X^T) with the converged occupied orbitals.  Before the timed loop the
whole hot path runs once (screening and 3c integrals, metric factor and B,
SCF to convergence, analytic gradient) and its phase times are reported.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--calib]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 MFMA
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 MFMA
COUNTERS = os.path.join(ROOT, "profiles", "x_kernel_n1000_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2407_19614_amd", "csrc", "fock.hip")


def x_kernel_hash():
    """First 16 hex digits of the sha256 of the FP64 X kernel's source text
    (x2_body_f64 through x2_kernel_f64)."""
    import hashlib
    src = open(KERNEL_SRC).read()
    a = src.index("__device__ __forceinline__ void x2_body_f64(")
    b = src.index("void x2_kernel_f64(", a)
    c = src.index("\n}\n", b) + 3
    return hashlib.sha256(src[a:c].encode()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the X kernel from the committed counter
    summary, or None when the kernel's source changed since it was taken."""
    try:
        txt = open(COUNTERS).read()
        val = float(txt.split("traffic_bytes_per_launch:")[1].split()[0])
        sha = txt.split("x_kernel_source_sha256_16:")[1].split()[0]
        cur = x_kernel_hash()
    except (OSError, IndexError, ValueError):
        return None
    return val if cur == sha else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-pipeline", action="store_true", help="skip SCF/gradient phase timings")
    ap.add_argument("--calib", action="store_true", help="also run a plain 2 GiB device copy (counter calibration)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-SCF-start workload (40-centre random walk; on by default)")
    ap.add_argument("--learned-steps", type=int, default=240,
                    help="random-walk steps of that workload (the full sequence has 3000)")
    ap.add_argument("--batched", action="store_true",
                    help="run the batched workload (256 molecules, 10-60 centres); on by default")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workload")
    ap.add_argument("--batched-n", type=int, default=256, help="molecules in the batched workload")
    ap.add_argument("--batched-prec", default="fp32f64", choices=["fp32", "fp64", "fp32f64"],
                    help="exchange precision of the batched workload")
    ap.add_argument("--aimd", action="store_true",
                    help="also run Born-Oppenheimer NVE dynamics of the N=1000 workload (1 fs steps)")
    ap.add_argument("--aimd-steps", type=int, default=10, help="time steps of that run")
    ap.add_argument("--no-batched-overlap", action="store_true",
                    help="batched workload: set each wave up before its SCF instead of beside the previous one")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched workload with the default launch shapes instead of autotuned ones")
    ap.add_argument("--quick", action="store_true",
                    help="profiling mode: seeded random occupied orbitals instead of the converged SCF "
                         "(same shapes and kernels), no pipeline, no CPU baseline")
    ap.add_argument("--only", choices=["pipeline", "batched", "learned"],
                    help="profiling mode: only the N=1000 energy+gradient pipeline (a cold and a warm pass), "
                         "only the batched workload (no single-path or oracle baselines), or only the "
                         "learned-start workload (no oracle baseline); prints its JSON")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2407_19614_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only == "learned":
        print(json.dumps({"learned_start": learned_leg(args.learned_steps, oracle_sample=False)}))
        return
    if args.only == "batched":
        print(json.dumps({"batched": batched_leg(args.batched_n, baseline_n=0, prec_name=args.batched_prec,
                                                 autotune=not args.no_autotune, oracle_sample=False,
                                                 allow_overlap=not args.no_batched_overlap)}))
        return
    s = synth.config_system("n1000")
    pr = P.RIProblem(s, device=dev, prec=P.FP64)
    sync = torch.cuda.synchronize
    phases = {}

    def timed(name, fn):
        sync()
        t = time.perf_counter()
        out = fn()
        sync()
        phases[name] = time.perf_counter() - t
        return out

    # The pipeline twice: the first pass pays one-time costs (device memory
    # taken into torch's caching allocator, first launches of each kernel);
    # the second is the steady state that every step of a dynamics run repeats.
    if args.quick:
        args.no_pipeline = args.no_cpu = True
    cold = {}
    for rep in range(1 if args.no_pipeline else 2):
        phases = {}
        timed("build_3c_s", pr.build_3c)
        timed("metric_factor_s", lambda: pr.metric_factor(P.FP64))
        if args.quick:
            C = torch.tensor(synth.random_coeffs(s.N, s.n_occ, seed=0), dtype=torch.float64, device=dev)
            res = {"E_total": None, "n_iter": 0, "converged": 0}
        else:
            res, C, F, D = timed("scf_s", lambda: pr.energy(tol_E=1e-10, tol_err=1e-8))
        if not args.no_pipeline:
            g = timed("gradient_s", pr.gradient)
        phases = {k: round(v, 4) for k, v in phases.items()}
        if rep == 0:
            cold = phases
    if args.only == "pipeline":
        print(json.dumps({"pipeline_cold_s": cold, "pipeline_s": phases,
                          "scf": {"E_total": res["E_total"], "n_iter": res["n_iter"]}}))
        return

    N, na, no, npairs = s.N, s.n_aux, s.n_occ, pr.n_pairs
    J = torch.empty((N, N), dtype=torch.float64, device=dev)
    K = torch.empty_like(J)
    gam = torch.empty(na, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        pr.fock_jk(C, J, K, gam)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    cur = torch.cuda.current_stream(dev)
    for e4 in ev:
        for e in e4:
            e.record(cur)          # creates the events
    sync()
    t0 = time.perf_counter()
    for e4 in ev:
        pr.fock_jk_timed(C, J, K, gam, e4)
    sync()
    wall = time.perf_counter() - t0
    ms_step = wall / args.steps * 1e3
    ph = np.array([pr.fock_phases(e4) for e4 in ev])  # ms: gamma/J (beside X), X, SYRK
    t_j, t_x, t_k = ph.mean(0)

    # algorithmic work per build (N, not padded sizes)
    fl_x = 2.0 * N * N * no * na
    fl_k = float(N) * (N + 1) * no * na
    by_j = 2.0 * 8 * na * npairs
    achieved = fl_x / (t_x * 1e-3) / 1e12
    out = {
        "metric": "RI-JK Fock builds/s + %MFMA peak at N=1000; batched SCF/s at dE<=1e-6 Eh",
        "value": round(args.steps / wall, 3),
        "unit": "builds/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "n1000: 100 He-like centres, N=1000, N_aux=3000, n_occ=100, tau=1e-12, "
                               "decompressed packed-tile FP64 B",
                   "n_pairs": int(npairs), "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "kernel": "x_kernel_f64 (X^P = B^P C_occ)",
                     "achieved": round(achieved, 2), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": measured_traffic(),
                     "flops_per_launch": fl_x, "avg_launch_ms": round(t_x, 4)},
        "phases_ms": {"gamma_J": round(t_j, 4), "X": round(t_x, 4), "K_syrk": round(t_k, 4)},
        "fock_build_frac_fp64_peak": round((fl_x + fl_k) / (ms_step * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
        "K_syrk_tflops": round(fl_k / (t_k * 1e-3) / 1e12, 2),
        # gamma/J runs beside X on the side stream (128 workgroups at this size): its span
        # is hidden under the exchange, so its rate here is not its bandwidth when alone
        "gamma_J_beside_X": {"ms": round(t_j, 4), "GBs": round(by_j / (t_j * 1e-3) / 1e9, 1)},
        "pipeline_s": phases,
        "pipeline_cold_s": cold,
        "scf": {"E_total": res["E_total"], "n_iter": res["n_iter"], "converged": res["converged"]},
    }
    gold = os.path.join(ROOT, "tests", "golden", "n1000_oracle.json")
    if os.path.exists(gold) and not args.quick:
        ref = json.load(open(gold))
        out["scf"]["abs_dE_vs_oracle"] = abs(res["E_total"] - ref["E_total"])
        if not args.no_pipeline:
            out["gradient_max_abs_diff_vs_oracle"] = float(np.abs(g.cpu().numpy() - np.array(ref["gradient"])).max())
    out["precision"] = precision_leg(s, C, None if args.quick else res, args, P, torch, np, ms_step,
                                     phases.get("scf_s"), K64=K.clone(),
                                     g64=None if args.no_pipeline else g)
    out["compressed"] = compressed_leg(s, C, None if args.quick else res, args, P, torch, np, ms_step)
    out["density_fock"] = density_leg(pr, C, torch, np)
    if args.batched or not args.no_batched:
        # the second half of the headline metric: batched SCF/s at |dE| <= 1e-6 Eh.  The
        # N=1000 legs' blocks go back to the driver first: the batched leg holds two waves
        # at once, and allocating them beside a full cache would make the allocator free
        # and re-map memory (device-wide synchronisations) inside the timed region
        del pr, J, K, gam
        torch.cuda.empty_cache()
        out["batched"] = batched_leg(args.batched_n, prec_name=args.batched_prec, autotune=not args.no_autotune,
                                     oracle_sample=not args.no_cpu, allow_overlap=not args.no_batched_overlap)
    if not args.no_learned and not args.quick:
        out["learned_start"] = learned_leg(args.learned_steps, oracle_sample=not args.no_cpu)
    if args.aimd:
        out["aimd"] = aimd_leg(args.aimd_steps)
    if args.calib:
        # counter calibration: one kernel that writes 2 GiB (fill) and one that reads 2 GiB (sum)
        src = torch.empty(2 ** 28, dtype=torch.float64, device=dev)
        src.fill_(1.0)                      # writes 2 GiB
        sync()
        dst = torch.mul(src, 2.0)           # plain copy kernel: reads 2 GiB, writes 2 GiB
        sync()
        tot = src.sum()                     # reads 2 GiB
        sync()
        out["calib_bytes"] = 2 ** 31
        del src, dst, tot
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(s, C.cpu().numpy())
    print(json.dumps(out), flush=True)


def precision_leg(s, C, res64, args, P, torch, np, ms_fp64, scf_s64=None, K64=None, g64=None):
    """Reduced-precision exchange contractions at the same workload: Fock
    builds/s and speedup over FP64, the exchange matrix's largest difference
    from the FP64 one for the same orbitals, and per SCF form (skipped when
    res64 is None) the converged energy's difference from the FP64 SCF, the
    SCF time against the FP64 SCF (scf_s64) and the largest difference of the
    gradient at its orbitals from the FP64 gradient (g64).  FP32: FP32 MFMA;
    BF16X3 / BF16X6: two- and three-part BF16 splits with 3 and 6 products on
    BF16 MFMA.  gamma and J stay FP64.  "scf_final_fp64" is the SCF followed by
    one exchange build in FP64 arithmetic at the converged density
    (RI_FINAL_FP64); BF16X3 is offered only in that form.  The X roofline
    counts the MFMA work actually issued: full square tiles of the padded size
    times the product count."""
    dev = C.device
    N, na = s.N, s.n_aux
    out = {}
    # (final build?, SCF thresholds): plain forms iterate to just above their
    # energy noise floor (once converged, the iteration energy still moves by
    # up to ~1.5e-7 Eh for FP32 and ~3e-8 Eh for BF16X6 from rounding alone,
    # so a lower energy threshold is met only by chance); with the final FP64
    # build the density's error enters the energy to second order, so
    # 1e-6 / 3e-5 suffices (see batched_leg).  BF16X3's iteration energies
    # move by ~1e-5 Eh, so its energy test sits above that (1e-4) and the
    # commutator test governs.
    forms = (("fp32", P.FP32, ((False, (3e-7, 1e-5)), (True, (1e-6, 3e-5)))),
             ("bf16x3", P.BF16X3, ((True, (1e-4, 3e-5)),)),
             ("bf16x6", P.BF16X6, ((False, (1e-7, 1e-6)), (True, (1e-6, 3e-5)))))
    for name, prec, scfs in forms:
        pr = P.RIProblem(s, device=dev, prec=prec)
        pr.build_3c()
        pr.metric_factor(prec)
        J = torch.empty((N, N), dtype=torch.float64, device=dev)
        K = torch.empty_like(J)
        g = torch.empty(na, dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            pr.fock_jk(C, J, K, g)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        for e4 in ev:
            for e in e4:
                e.record(torch.cuda.current_stream(dev))
        torch.cuda.synchronize()
        t = time.perf_counter()
        for e4 in ev:
            pr.fock_jk_timed(C, J, K, g, e4)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        bf = prec in (P.BF16X3, P.BF16X6)
        ph = np.array([pr.fock_phases(e4, bf16=bf) for e4 in ev]).mean(0)
        out[name] = {"builds_per_s": round(1.0 / dt, 3), "ms_per_build": round(dt * 1e3, 3),
                     "speedup_vs_fp64": round(ms_fp64 / (dt * 1e3), 3),
                     "phases_ms": {"gamma_J_beside_SYRK" if bf else "gamma_J_beside_X": round(float(ph[0]), 3),
                                   "X": round(float(ph[1]), 3), "K_syrk": round(float(ph[2]), 3)}}
        if K64 is not None:
            out[name]["max_abs_dK_vs_fp64"] = float((K - K64).abs().max())
            out[name]["max_abs_K_fp64"] = float(K64.abs().max())
        if prec in (P.BF16X3, P.BF16X6):
            ns, nprod = (2, 3) if prec == P.BF16X3 else (3, 6)
            npad = 64 * ((N + 63) // 64)
            w = 16 * ((s.n_occ + 15) // 16)
            fl = 2.0 * na * npad * npad * w * nprod          # MFMA work issued
            by = 2.0 * ns * na * npad * npad                  # B parts read (full square tiles)
            tx = ph[1] * 1e-3
            out[name]["x_roofline"] = {"mfma_tflops": round(fl / tx / 1e12, 1),
                                       "mfma_frac": round(fl / tx / 1e12 / PEAK_BF16_TFLOPS, 4),
                                       "b_read_GBs": round(by / tx / 1e9, 1),
                                       "hbm_frac": round(by / tx / 1e9 / PEAK_HBM_GBS, 4)}
        if prec == P.BF16X3:
            out[name]["scf"] = "not offered: two-part B and C_occ alone move the energy past 1e-6 Eh"
        if res64 is not None:
            for fin, tol in scfs:
                torch.cuda.synchronize()
                t = time.perf_counter()
                r, *_ = pr.energy(tol_E=tol[0], tol_err=tol[1], max_iter=60, raise_on_noconv=False,
                                  final_fp64=fin)
                torch.cuda.synchronize()
                t_scf = time.perf_counter() - t
                rec = {"E": r["E_total"], "iters": r["n_iter"], "converged": r["converged"],
                       "tol_E": tol[0], "tol_err": tol[1], "scf_s": round(t_scf, 4),
                       "abs_dE_vs_fp64": abs(r["E_total"] - res64["E_total"]),
                       "speedup_vs_fp64_scf": round(scf_s64 / t_scf, 3) if scf_s64 else None}
                if g64 is not None and r["converged"]:
                    gg = pr.gradient()
                    torch.cuda.synchronize()
                    rec["max_abs_dgrad_vs_fp64"] = float((gg - g64).abs().max())
                out[name]["scf_final_fp64" if fin else "scf"] = rec
        del pr, J, K, g   # blocks stay in torch's cache for the next leg (see batched_leg)
    return out


def density_leg(pr, C, torch, np, reps=3):
    """Fock build from the density alone at the same workload (as a density
    start needs): K = 1/2 sum_P B^P D B^P on FP64 MFMA GEMMs, 4 N^3 N_aux
    flops.  Reports its time, rate, and the largest difference of its J and
    K from the orbital build for D = 2 C C^T."""
    N, na = pr.N, pr.n_aux
    D = 2.0 * C @ C.T
    J0, K0, _ = pr.fock_jk(C)
    pr.fock_jk_density(D)                       # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        J1, K1 = pr.fock_jk_density(D)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    fl = 4.0 * N ** 3 * na
    return {"ms_per_build": round(dt * 1e3, 2), "flops": fl, "tflops": round(fl / dt / 1e12, 2),
            "frac_fp64_peak": round(fl / dt / 1e12 / PEAK_FP64_TFLOPS, 4),
            "max_abs_dJ_vs_orbital": float((J1 - J0).abs().max()),
            "max_abs_dK_vs_orbital": float((K1 - K0).abs().max())}


def compressed_leg(s, C, res64, args, P, torch, np, ms_fp64):
    """The compressed-B form at the same workload: B is never resident; every
    Fock build unpacks B_c into packed FP64 tiles 256 auxiliaries at a time in
    the workspace and transforms each slab (the per-iteration decompression
    of Algorithm 1).  Reports builds/s, phase times (the X phase includes the
    unpacking), the device memory the form saves, and the converged SCF
    energy against the resident form's."""
    dev = C.device
    N, na = s.N, s.n_aux
    pr = P.RIProblem(s, device=dev, prec=P.FP64, compressed=True)
    pr.build_3c()
    pr.metric_factor(P.FP64)
    J = torch.empty((N, N), dtype=torch.float64, device=dev)
    K = torch.empty_like(J)
    g = torch.empty(na, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        pr.fock_jk(C, J, K, g)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    for e4 in ev:
        for e in e4:
            e.record(torch.cuda.current_stream(dev))
    torch.cuda.synchronize()
    t = time.perf_counter()
    for e4 in ev:
        pr.fock_jk_timed(C, J, K, g, e4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    ph = np.array([pr.fock_phases(e4) for e4 in ev]).mean(0)
    ws_plain = P.workspace_bytes(P.binding.OP_FOCK, N, na, s.n_occ, pr.n_pairs, P.FP64)
    ws_comp = P.workspace_bytes(P.binding.OP_FOCK, N, na, s.n_occ, pr.n_pairs, P.FP64 | P.COMPRESSED)
    out = {"builds_per_s": round(1.0 / dt, 3), "ms_per_build": round(dt * 1e3, 3),
           "slowdown_vs_resident": round(dt * 1e3 / ms_fp64, 3),
           "phases_ms": {"gamma_J": round(float(ph[0]), 3), "unpack_and_X": round(float(ph[1]), 3),
                         "K_syrk": round(float(ph[2]), 3)},
           "resident_B_GB": round(P.packed_b_bytes(N, na, P.FP64) / 1e9, 2),
           "extra_workspace_GB": round((ws_comp - ws_plain) / 1e9, 2)}
    if res64 is not None:
        r, *_ = pr.energy(tol_E=1e-10, tol_err=1e-8)
        out["scf_E"] = r["E_total"]
        out["abs_dE_vs_resident"] = abs(r["E_total"] - res64["E_total"])
    return out


def batched_leg(n_mol, wave=128, baseline_n=32, prec_name="fp32f64", autotune=True, oracle_sample=True,
                allow_overlap=True):
    """256 independent He-like clusters with n_centres ~ U{10..60} (N = 10 per
    centre, N_aux = 30 per centre, n_occ = n_centres), seeds 4001...: pairs, 3c
    integrals and B per molecule, then one lockstep SCF per wave of molecules
    (HIP-graph replay, FP64 everything but the exchange).  prec_name picks the
    exchange: "fp32f64" FP32 iterations and one final exchange build in FP64
    arithmetic at the converged density, "fp32" FP32 only, "fp64".  SCF/s
    counts the whole job from the first screening to the last convergence.
    The plain FP64 single-molecule path is timed on the first baseline_n
    molecules for comparison; energies are checked against stored oracle
    energies for a seeded subset."""
    import numpy as np
    import torch
    import synth
    import paper_2407_19614_amd as P
    from paper_2407_19614_amd.binding import (PreparedBatch, batch_autotune, batch_workspace_bytes, energy_batched,
                                              prepare_batch)
    systems = synth.batched_systems(n_mol)
    prec = {"fp32": P.FP32, "fp64": P.FP64, "fp32f64": P.FP32 | P.FINAL_FP64}[prec_name]
    # FP32 exchange iterates to its own noise floor.  With the final FP64 build the
    # density's error enters the energy only to second order, so its iterations stop
    # earlier: at these thresholds the error stays that of B's FP32 rounding.
    tol = {"fp32": dict(tol_E=1e-7, tol_err=1e-5), "fp32f64": dict(tol_E=1e-6, tol_err=3e-5),
           "fp64": dict(tol_E=1e-10, tol_err=1e-8)}[prec_name]
    log = lambda m: print(m, file=sys.stderr, flush=True)
    E = np.full(len(systems), np.nan)
    iters = np.zeros(len(systems), dtype=int)
    conv = np.zeros(len(systems), dtype=bool)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_setup = t_scf = t_tune = 0.0
    tune = None
    starts = list(range(0, len(systems), wave))
    nxt = None
    for w, w0 in enumerate(starts):
        ts = time.perf_counter()
        # per-molecule 3c, metric factor and B, four molecules' launches in flight at once;
        # after the first wave, each wave's setup has run beside the previous wave's SCF
        # and only what is left of it is waited for here
        probs = prepare_batch(systems[w0:w0 + wave], prec, workers=4) if nxt is None else nxt.result()
        torch.cuda.synchronize()
        t_setup += time.perf_counter() - ts
        if tune is None and autotune:
            # launch shapes per size bucket, timed on the first wave's molecules and kept for the rest
            ts = time.perf_counter()
            tune = batch_autotune(probs, prec)
            t_tune = time.perf_counter() - ts
        if w == 0:
            # the next wave's setup runs beside this wave's SCF only if both waves' data and
            # the SCF workspace fit in device memory at once (the FP32-stored forms do; two
            # waves of FP64 B do not), with the first wave's footprint standing in for the next
            data0 = torch.cuda.memory_allocated()
            need = 2 * data0 + batch_workspace_bytes(probs, prec) + (8 << 30)
            overlap = allow_overlap and need < torch.cuda.get_device_properties(0).total_memory
            log(f"batched: first wave {data0 / 2**30:.1f} GiB, two waves + workspace {need / 2**30:.1f} GiB: "
                f"{'setup beside SCF' if overlap else 'setup before each wave'}")
        nxt = (PreparedBatch(systems[starts[w + 1]:starts[w + 1] + wave], prec, workers=4)
               if overlap and w + 1 < len(starts) else None)
        ts = time.perf_counter()
        res, _, _ = energy_batched(probs, prec, use_graph=True, raise_on_noconv=False, tuning=tune, **tol)
        torch.cuda.synchronize()
        t_scf += time.perf_counter() - ts
        for k, r in enumerate(res):
            E[w0 + k], iters[w0 + k], conv[w0 + k] = r["E_total"], r["n_iter"], r["converged"]
        log(f"batched wave {w0}: setup waited {t_setup:.2f}s scf {t_scf:.2f}s")
        del probs, res
    wall = time.perf_counter() - t0
    # the single-molecule path on the first molecules, one by one: plain FP64
    # at 1e-10 / 1e-8, and the batched form's own precision and thresholds
    base = {}
    E64 = []
    for label, p1, tl in (("fp64", P.FP64, dict(tol_E=1e-10, tol_err=1e-8)), ("same_form", prec, tol)):
        if baseline_n == 0:
            break
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for s in systems[:baseline_n]:
            pr = P.RIProblem(s, prec=p1 & ~P.FINAL_FP64)
            pr.build_3c()
            pr.metric_factor(p1 & ~P.FINAL_FP64)
            r, *_ = pr.energy(final_fp64=bool(p1 & P.FINAL_FP64), **tl)
            if label == "fp64":
                E64.append(r["E_total"])
            del pr
        torch.cuda.synchronize()
        base[label] = baseline_n / (time.perf_counter() - tb)
    mode = {"fp32": "FP32 exchange", "fp64": "FP64 exchange",
            "fp32f64": "FP32 exchange, then one FP64 exchange build at the converged density"}[prec_name]
    out = {"workload": f"{len(systems)} He-like clusters, 10-60 centres (N 100-600, N_aux 300-1800), {mode}",
           "scf_per_s": round(len(systems) / wall, 3), "wall_s": round(wall, 2),
           "scf_per_s_steady": round(len(systems) / (wall - t_tune), 3),
           "setup_waited_s": round(t_setup, 2), "autotune_s": round(t_tune, 3), "batched_scf_s": round(t_scf, 2),
           "wave": wave, "setup_beside_scf": bool(overlap), "tuning": tune.as_dict() if tune is not None else None,
           "all_converged": bool(conv.all()), "mean_iters": round(float(iters.mean()), 2)}
    if baseline_n > 0:
        out.update({
           "single_path_scf_per_s": {"fp64_1e-10": round(base["fp64"], 3),
                                     "same_form_and_thresholds": round(base["same_form"], 3)},
           "single_path_sample": f"first {baseline_n} molecules, one by one",
           "speedup_vs_single_path": {"fp64_1e-10": round(len(systems) / wall / base["fp64"], 3),
                                      "same_form_and_thresholds": round(len(systems) / wall / base["same_form"], 3)},
           "max_abs_dE_batched_vs_fp64_single": float(np.max(np.abs(E[:baseline_n] - np.array(E64))))})
    gold = os.path.join(ROOT, "tests", "golden", "batch_oracle.json")
    if os.path.exists(gold) and len(systems) == 256:
        ref = json.load(open(gold))
        out["max_abs_dE_vs_oracle_subset"] = float(max(abs(E[m["index"]] - m["E"]) for m in ref["subset"]))
        out["oracle_subset_size"] = len(ref["subset"])
    if oracle_sample:
        out["cpu_baseline"] = batched_oracle_baseline(systems, tol)
    return out


def batched_oracle_baseline(systems, tol, targets=(150, 250, 350)):
    """The oracle's SCF (FP64, core-Hamiltonian start, the batched form's
    thresholds) on this host's cores for three molecules of the batch with N
    near `targets`, a power law t = a N^p fitted to their times, and the
    whole batch's oracle time predicted from it."""
    import numpy as np
    from oracle import ri as R, scf as S
    Ns = np.array([s.N for s in systems])
    picked = [int(np.argmin(np.abs(Ns - t))) for t in targets]
    ts = []
    for i in picked:
        t = time.perf_counter()
        S.run_scf(systems[i], R.RIData(systems[i]), tol_E=tol["tol_E"], tol_e=tol["tol_err"])
        ts.append(time.perf_counter() - t)
    p, loga = np.polyfit(np.log(Ns[picked]), np.log(ts), 1)
    total = float(np.sum(np.exp(loga) * Ns.astype(float) ** p))
    return {"value": round(len(systems) / total, 5), "unit": "SCF/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "sample": f"oracle SCF of molecules {picked} (N = {[int(n) for n in Ns[picked]]}) timed; "
                      f"t = a N^p fitted (p = {p:.2f}) and summed over the {len(systems)} molecules",
            "sample_seconds": [round(x, 2) for x in ts]}


def aimd_leg(n_steps, name="n1000"):
    """Born-Oppenheimer NVE dynamics of the N=1000 workload released at rest
    from its (non-equilibrium) geometry with 1 fs steps.  Each step: Verlet
    kick and drift, 3c build, metric factor and B, SCF started from the
    previous step's orbitals, analytic gradient, closing kick.  Reports
    steady-state steps/s (steps after the first, whose SCF starts from the
    core Hamiltonian), ps of simulation per day, SCF iterations per step and
    the total-energy excursion."""
    import numpy as np
    import synth
    from paper_2407_19614_amd.aimd import FS, NVE
    log = lambda m: print(m, file=sys.stderr, flush=True)
    s = synth.config_system(name)
    md = NVE(s, 1.0 * FS)
    out = md.run(n_steps, log=log)
    st = np.array(out["step_s"][1:])
    Et = np.array(out["E_tot"])
    return {"workload": f"{name}: {s.n_centres} He-like centres (N={s.N}, N_aux={s.n_aux}), at rest, NVE, "
                        f"1 fs steps, previous-step orbitals as the SCF start",
            "steps": n_steps, "steps_per_s": round(1.0 / st.mean(), 3), "step_s_mean": round(float(st.mean()), 4),
            "first_step_s": round(out["step_s"][0], 4), "ps_per_day": round(86400.0 / st.mean() * 1e-3, 1),
            "scf_iters_first": out["scf_iters"][0], "scf_iters_mean_after": round(float(np.mean(out["scf_iters"][1:])), 2),
            "E_tot_excursion_Eh": float(np.abs(Et - Et[0]).max()), "E_kin_final_Eh": out["E_kin"][-1]}


def learned_leg(n_steps, oracle_sample=True):
    """40-centre cluster (N=400, N_aux=1200, n_occ=40) on a seeded Gaussian
    random walk (sigma 0.05 bohr per coordinate per step): reference SCF from
    the core-Hamiltonian guess at every training geometry, MLP trained on the
    first two thirds.  On the last third four starts are timed as whole
    energy+gradient evaluations (3c, metric factor and B, SCF, gradient):
    the core-Hamiltonian guess; the previous geometry's orbitals (the paper's
    molecular-dynamics start); the network's density at the new geometry
    ("learned"); and the previous geometry's converged density plus the
    change a second network predicts from the pair's change features
    (ri_pair_delta_features), trained on consecutive training geometries
    ("learned_delta").
    The sequence starts (previous orbitals, learned_delta) chain from their
    own previous result, as a dynamics run would; means count test geometries
    after the first.  Every start's energy is checked against the core-H SCF,
    and a start that fails or lands higher falls back to core-H.  Beside it,
    the oracle's energy and gradient at one test geometry (SCF from the
    core-Hamiltonian guess, as the core_h start) on this host's cores."""
    import numpy as np
    import torch
    import synth
    import paper_2407_19614_amd as P
    import paper_2407_19614_amd.learned as Lr
    s0 = synth.config_system("n400")
    traj = synth.random_walk(s0.xyz, n_steps, 0.05, 2.0, seed=7)
    systems = [s0.with_xyz(x) for x in traj]
    n_train = (2 * len(systems)) // 3
    log = lambda m: print(m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    data = Lr.generate(systems[:n_train], log=log, prev_baseline=False)
    t_gen = time.perf_counter() - t0
    net = Lr.init_network(seed=0)
    net_d = Lr.init_network(seed=1, delta=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = Lr.train(net, data, steps=4000, batch=16384, lr=2e-3, log=log)
    losses_d = Lr.train(net_d, data, steps=4000, batch=16384, lr=2e-3, log=log, delta=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del data
    kinds = ("core_h", "previous_orbitals", "learned", "learned_delta")
    iters = {k: [] for k in kinds}
    secs = {k: 0.0 for k in kinds}
    dE = {k: 0.0 for k in kinds}
    fallbacks = {k: 0 for k in kinds}
    C_prev = D_prev = xyz_prev = None
    tol = dict(tol_E=1e-10, tol_err=1e-8, raise_on_noconv=False)

    def evaluate(kind, s, start):
        t = time.perf_counter()
        pr = P.RIProblem(s)
        pr.build_3c()
        pr.metric_factor(P.FP64)
        extra = start(pr)
        res, C, F, D = pr.energy(**tol, **extra)
        if kind != "core_h" and (not res["converged"] or res["E_total"] > E_ref + 1e-8):
            fallbacks[kind] += 1
            res, C, F, D = pr.energy(**tol)
        pr.gradient(C, F)
        torch.cuda.synchronize()
        return res, C, D, pr, time.perf_counter() - t

    test = systems[n_train:]
    for k, s in enumerate(test):
        E_ref = None
        res, C0, D0, pr0, dt = evaluate("core_h", s, lambda pr: {})
        E_ref = res["E_total"]
        if k == 0:
            C_prev, D_prev, xyz_prev = C0, D0, pr0.xyz.clone()
            continue
        iters["core_h"].append(res["n_iter"])
        secs["core_h"] += dt
        r, C_new, _, _, dt = evaluate("previous_orbitals", s, lambda pr: {"guess": C_prev})
        iters["previous_orbitals"].append(r["n_iter"])
        secs["previous_orbitals"] += dt
        dE["previous_orbitals"] = max(dE["previous_orbitals"], abs(r["E_total"] - E_ref))
        r, *_, dt = evaluate("learned", s, lambda pr: {"guess_density": Lr.predict_density(net, pr)})
        iters["learned"].append(r["n_iter"])
        secs["learned"] += dt
        dE["learned"] = max(dE["learned"], abs(r["E_total"] - E_ref))
        r, _, D_new, pr_d, dt = evaluate(
            "learned_delta", s, lambda pr: {"guess_density": Lr.delta_start(net_d, pr, xyz_prev, D_prev)})
        iters["learned_delta"].append(r["n_iter"])
        secs["learned_delta"] += dt
        dE["learned_delta"] = max(dE["learned_delta"], abs(r["E_total"] - E_ref))
        C_prev, D_prev, xyz_prev = C_new, D_new, pr_d.xyz.clone()
        if k % 20 == 0:
            log(f"test geometry {k}: iters " + " ".join(f"{q} {iters[q][-1]}" for q in kinds))
    n_eval = len(iters["core_h"])
    out = {"workload": f"n400: 40 He-like centres, N=400, N_aux=1200, n_occ=40; {n_steps}-step walk, "
                       f"train {n_train} / test {len(test)}",
           "mean_iters": {q: round(float(np.mean(iters[q])), 3) for q in kinds},
           "energy_gradient_evals_per_s": {q: round(n_eval / secs[q], 3) for q in kinds},
           "max_abs_dE_vs_core_h": {q: dE[q] for q in kinds if q != "core_h"},
           "fallbacks": {q: fallbacks[q] for q in kinds if q != "core_h"},
           "iterations_saved_vs_previous_orbitals": {
               q: round(float(np.mean(iters["previous_orbitals"]) - np.mean(iters[q])), 3)
               for q in ("learned", "learned_delta")},
           "train_loss_first_last": {"learned": [losses[0][1], losses[-1][1]],
                                     "learned_delta": [losses_d[0][1], losses_d[-1][1]]},
           "generate_s": round(t_gen, 1), "train_s": round(t_train, 2)}
    if oracle_sample:
        # the oracle's energy and gradient at the last test geometry from the core-H guess
        from oracle import ri as R, scf as S, gradient as G
        sl = test[-1]
        t = time.perf_counter()
        ri = R.RIData(sl)
        rr = S.run_scf(sl, ri, tol_E=1e-10, tol_e=1e-8)
        G.analytic_gradient(sl, rr, ri)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(1.0 / dt, 4), "unit": "energy+gradient evaluations/s",
                               "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                               "sample": "one test geometry: 3c integrals, SCF from the core-Hamiltonian guess "
                                         f"({rr.n_iter} iterations), analytic gradient",
                               "seconds": round(dt, 2)}
    return out


def cpu_baseline(s, C):
    """The oracle's RI Fock build (fit path with scipy Cholesky solves) at the
    same workload, one full build, on this host's cores."""
    from oracle import ri as R
    cores = len(os.sched_getaffinity(0))
    ri = R.RIData(s)
    t = time.perf_counter()
    ri.JK(C)
    dt = time.perf_counter() - t
    # beside it: the whole tiny workload (3c, fit, SCF to 1e-10) on the oracle
    import synth
    from oracle import scf as S
    tiny = synth.config_system("tiny")
    t = time.perf_counter()
    S.run_scf(tiny, R.RIData(tiny), tol_E=1e-10, tol_e=1e-8)
    dt_tiny = time.perf_counter() - t
    return {"value": round(1.0 / dt, 5), "unit": "builds/s", "cores": cores, "kind": "oracle",
            "sample": "one full N=1000 oracle Fock build (J and K for the converged orbitals); "
                      "3c-integral setup excluded", "seconds": round(dt, 2),
            "tiny_scf_seconds": round(dt_tiny, 3)}


if __name__ == "__main__":
    main()
