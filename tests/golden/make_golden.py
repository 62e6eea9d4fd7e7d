"""Write oracle reference values for the N=1000 workload (100 He-like
centres, N=1000, N_aux=3000, n_occ=100, tau=1e-12) to n1000_oracle.json,
and the full J and K (lower triangles, row-major, FP64) for the seeded
occupied block to n1000_jk.npz.

Calls only the CPU oracle and the seeded input generators.  Run once:
    python tests/golden/make_golden.py            (everything)
    python tests/golden/make_golden.py --jk-only  (n1000_jk.npz only)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import ri as R, scf as S, gradient as G  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "n1000_oracle.json")
OUT_JK = os.path.join(os.path.dirname(os.path.abspath(__file__)), "n1000_jk.npz")
ROWS = [0, 1, 137, 499, 500, 731, 998, 999]


def main():
    t0 = time.time()
    s = synth.config_system("n1000")
    ri = R.RIData(s)
    print(f"pairs {ri.n_pairs}  T {time.time()-t0:.1f}s", flush=True)
    # J and K for seeded random orbitals, sampled rows
    C = synth.random_coeffs(s.N, s.n_occ, seed=0)
    t = time.time()
    J, K = ri.JK(C)
    tjk = time.time() - t
    print(f"JK {tjk:.1f}s", flush=True)
    lo = np.tril_indices(s.N)
    np.savez_compressed(OUT_JK, seed=np.int64(0), J_lower=J[lo], K_lower=K[lo])
    print("wrote", OUT_JK, flush=True)
    if "--jk-only" in sys.argv:
        return
    res = S.run_scf(s, ri, tol_E=1e-12, tol_e=1e-9)
    print(f"SCF E={res.E:.12f} iters={res.n_iter} conv={res.converged} {time.time()-t0:.1f}s", flush=True)
    g = G.analytic_gradient(s, res, ri)
    print(f"grad done {time.time()-t0:.1f}s", flush=True)
    out = dict(
        workload="n1000", n_pairs=int(ri.n_pairs),
        pair_mu_sum=int(ri.mu.sum()), pair_nu_sum=int(ri.nu.sum()),
        jk_seed=0, rows=ROWS, J_rows=J[ROWS].tolist(), K_rows=K[ROWS].tolist(),
        J_trace=float(np.trace(J)), K_trace=float(np.trace(K)),
        E_total=res.E, E_nuc=res.E_nuc, E_1e=res.E_1e, E_J=res.E_J, E_K=res.E_K,
        n_iter=res.n_iter, converged=bool(res.converged), gradient=g.tolist(),
        oracle_jk_seconds=tjk,
    )
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
