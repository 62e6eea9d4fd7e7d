"""Born-Oppenheimer molecular dynamics of the nuclei, oracle side (the
paper's AIMD wrapper: Verlet integration in the NVE ensemble, Ab Initio
Molecular Dynamics subsection).  TEST INFRASTRUCTURE ONLY.

Velocity Verlet from its definition, with a(x) = -grad E(x) / m:
  v(t + dt/2) = v(t) + dt/2 a(x(t))
  x(t + dt)   = x(t) + dt v(t + dt/2)
  v(t + dt)   = v(t + dt/2) + dt/2 a(x(t + dt))
Pins (tests/test_oracle_md.py): the harmonic oscillator, whose Verlet
positions obey x_{n+1} = 2 x_n - x_{n-1} - (w dt)^2 x_n and so equal
x0 cos(n th) with cos th = 1 - (w dt)^2 / 2; and the second-order energy
error of the method (halving dt divides the energy excursion by ~4) on an
anharmonic pair potential and on RI-HF itself.
"""
from __future__ import annotations

import numpy as np

AMU = 1822.888486           # electron masses per dalton
HE_MASS = 4.002602 * AMU    # helium-4 nucleus + electrons (atomic mass)
FS = 41.341374575751        # atomic units of time per femtosecond


def kinetic(mass, v):
    return 0.5 * float(np.sum(mass[:, None] * v * v))


def verlet(x0, v0, mass, energy_grad, dt, n_steps):
    """Integrate n_steps; returns a list of (x, v, E_pot, E_kin) per time,
    including t = 0.  energy_grad(x) -> (E, dE/dx)."""
    x = np.array(x0, dtype=float)
    v = np.array(v0, dtype=float)
    E, g = energy_grad(x)
    out = [(x.copy(), v.copy(), E, kinetic(mass, v))]
    for _ in range(n_steps):
        v = v - 0.5 * dt * g / mass[:, None]
        x = x + dt * v
        E, g = energy_grad(x)
        v = v - 0.5 * dt * g / mass[:, None]
        out.append((x.copy(), v.copy(), E, kinetic(mass, v)))
    return out


def ri_hf_energy_grad(system, tol_E=1e-12, tol_e=1e-10):
    """energy_grad for the oracle's converged RI-HF energy and analytic
    gradient of `system` moved to positions x."""
    from . import gradient as G
    from . import ri as R
    from . import scf as S

    def f(x):
        s = system.with_xyz(x)
        ri = R.RIData(s)
        res = S.run_scf(s, ri, tol_E=tol_E, tol_e=tol_e)
        return res.E, G.analytic_gradient(s, res, ri)

    return f
