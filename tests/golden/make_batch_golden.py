"""Oracle SCF energies for a seeded subset of the batched workload (256
He-like clusters, 10-60 centres, N = 10 per centre, N_aux = 30 per centre,
tau = 1e-12): the smallest, the largest and 14 seeded random molecules.
Calls only the CPU oracle and the seeded input generators.
    python tests/golden/make_batch_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import ri as R, scf as S  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_oracle.json")


def subset(systems):
    sizes = np.array([s.n_centres for s in systems])
    idx = {int(np.argmin(sizes)), int(np.argmax(sizes))}
    rng = np.random.default_rng(99)
    for k in rng.permutation(len(systems)):
        if len(idx) >= 16:
            break
        idx.add(int(k))
    return sorted(idx)


def main():
    systems = synth.batched_systems()
    out = {"n_mol": len(systems), "sizes": [int(s.n_centres) for s in systems], "subset": []}
    for k in subset(systems):
        s = systems[k]
        t = time.time()
        res = S.run_scf(s, R.RIData(s), tol_E=1e-11, tol_e=1e-9)
        out["subset"].append({"index": k, "n_centres": int(s.n_centres), "E": res.E, "n_iter": res.n_iter,
                              "converged": bool(res.converged)})
        print(f"mol {k} nc={s.n_centres} E={res.E:.10f} it={res.n_iter} {time.time()-t:.1f}s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
