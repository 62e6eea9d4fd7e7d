"""Born-Oppenheimer molecular dynamics driver (the paper's AIMD wrapper).

Orchestration only: each time step runs, through the C ABI, the Verlet
kick-and-drift of the nuclei (ri_md_verlet), the three-centre build and
metric factor at the new geometry, the SCF started from the previous step's
converged orbitals (the paper's AIMD start), the analytic gradient and the
closing kick; positions, velocities and forces stay in device memory.
Ensemble NVE; atomic units (bohr, electron masses, Eh, atomic time).
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import binding as B

AMU = 1822.888486           # electron masses per dalton
HE_MASS = 4.002602 * AMU
FS = 41.341374575751        # atomic units of time per femtosecond


class NVE:
    """Velocity-Verlet dynamics of one system on the current HIP device."""

    def __init__(self, system, dt, mass=None, vel0=None, device="cuda", prec=B.FP64, tol_E=1e-10, tol_err=1e-8,
                 max_iter=100):
        import torch
        self.torch = torch
        self.pr = B.RIProblem(system, device=device, prec=prec)
        self.n = system.n_centres
        self.dt = float(dt)
        self.prec = prec
        f64 = dict(dtype=torch.float64, device=self.pr.device)
        m = np.full(self.n, HE_MASS) if mass is None else np.asarray(mass, dtype=float)
        self.mass = torch.tensor(m, **f64)
        v = np.zeros((self.n, 3)) if vel0 is None else np.asarray(vel0, dtype=float)
        self.vel = torch.tensor(v, **f64)
        self.ekin = torch.zeros(1, **f64)
        self.tol = dict(tol_E=tol_E, tol_err=tol_err, max_iter=max_iter)
        self.C = None
        self.grad = None

    def _stream(self):
        return self.pr.stream()

    def _verlet(self, stage):
        code = B.lib().ri_md_verlet(self.n, self.dt, B._ptr(self.mass), B._ptr(self.grad), B._ptr(self.pr.xyz),
                                    B._ptr(self.vel), stage, self._stream())
        B._check(code, "ri_md_verlet")

    def _kinetic(self):
        code = B.lib().ri_md_kinetic(self.n, B._ptr(self.mass), B._ptr(self.vel), B._ptr(self.ekin), self._stream())
        B._check(code, "ri_md_kinetic")
        return float(self.ekin.item())

    def _forces(self):
        pr = self.pr
        pr.build_3c()
        pr.metric_factor(self.prec)
        r, C, F, _ = pr.energy(guess=self.C, **self.tol)
        self.grad = pr.gradient(C, F)
        self.C = C
        return r

    def run(self, n_steps, log=None, keep_xyz=False):
        """Returns per time (t = 0 .. n_steps): E_pot, E_kin, E_tot, SCF
        iterations, wall seconds of the step; and positions when keep_xyz."""
        torch = self.torch
        out = {"E_pot": [], "E_kin": [], "E_tot": [], "scf_iters": [], "step_s": [], "xyz": []}

        def record(r, t):
            ek = self._kinetic()
            out["E_pot"].append(r["E_total"])
            out["E_kin"].append(ek)
            out["E_tot"].append(r["E_total"] + ek)
            out["scf_iters"].append(r["n_iter"])
            out["step_s"].append(t)
            if keep_xyz:
                out["xyz"].append(self.pr.xyz.cpu().numpy().copy())

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = self._forces()
        torch.cuda.synchronize()
        record(r, time.perf_counter() - t0)
        for k in range(n_steps):
            t0 = time.perf_counter()
            self._verlet(0)
            r = self._forces()
            self._verlet(1)
            torch.cuda.synchronize()
            record(r, time.perf_counter() - t0)
            if log and (k + 1) % max(1, n_steps // 5) == 0:
                log(f"aimd step {k + 1}/{n_steps}: E_tot {out['E_tot'][-1]:.10f} iters {r['n_iter']}")
        return out
