"""Pins of the oracle's velocity-Verlet integrator (AIMD wrapper)."""
import numpy as np

import synth
from oracle import md as M


def test_harmonic_oscillator_discrete_solution():
    # E = 1/2 k |x|^2 in 3D: each coordinate follows x_n = x_0 cos(n th),
    # cos th = 1 - (w dt)^2 / 2, from rest.
    k, m, dt = 0.7, 3.0, 0.3
    w = np.sqrt(k / m)
    x0 = np.array([[0.5, -1.2, 2.0]])
    traj = M.verlet(x0, np.zeros_like(x0), np.array([m]), lambda x: (0.5 * k * np.sum(x * x), k * x), dt, 60)
    th = np.arccos(1.0 - (w * dt) ** 2 / 2.0)
    for n, (x, v, _, _) in enumerate(traj):
        assert np.allclose(x, x0 * np.cos(n * th), atol=1e-12, rtol=0)
    # the half-step velocity of the discrete solution: v_{n+1/2} = (x_{n+1} - x_n) / dt
    x1, x2 = traj[5][0], traj[6][0]
    v_half = traj[5][1] - 0.5 * dt * (k * x1) / m
    assert np.allclose(v_half, (x2 - x1) / dt, atol=1e-13, rtol=0)


def morse_pair(De=0.02, a=1.1, r0=2.0):
    def f(x):
        d = x[0] - x[1]
        r = np.linalg.norm(d)
        e = np.exp(-a * (r - r0))
        E = De * (1 - e) ** 2
        dEdr = 2 * De * (1 - e) * a * e
        g0 = dEdr * d / r
        return E, np.array([g0, -g0])
    return f


def excursion(traj):
    Et = np.array([E + K for _, _, E, K in traj])
    return np.abs(Et - Et[0]).max()


def test_second_order_energy_error_anharmonic():
    x0 = np.array([[0.0, 0.0, 0.0], [2.6, 0.3, 0.0]])
    m = np.array([1800.0, 2500.0])
    f = morse_pair()
    e1 = excursion(M.verlet(x0, np.zeros_like(x0), m, f, 20.0, 100))
    e2 = excursion(M.verlet(x0, np.zeros_like(x0), m, f, 10.0, 200))
    assert 3.5 < e1 / e2 < 4.5
    # a force inconsistent with the energy drifts instead (planted mistake)
    bad = lambda x: (f(x)[0], 1.05 * f(x)[1])
    assert excursion(M.verlet(x0, np.zeros_like(x0), m, bad, 10.0, 200)) > 20 * e2


def test_ri_hf_dimer_dynamics_second_order():
    # He2 pushed together, released from rest; RI-HF energies and analytic
    # gradients from the oracle, product-complete enough for a smooth surface
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 2.2]])
    s = synth.make_system(xyz, [0.3, 1.0, 3.5], [0.2, 0.6, 2.0, 7.0], tau=0.0)
    m = np.full(2, M.HE_MASS)
    f = M.ri_hf_energy_grad(s)
    t1 = M.verlet(xyz, np.zeros_like(xyz), m, f, 80.0, 12)
    t2 = M.verlet(xyz, np.zeros_like(xyz), m, f, 40.0, 24)
    # the pair separates along z only, symmetric about the midpoint
    x = t1[-1][0]
    assert abs(x[0, 0]) < 1e-12 and abs(x[1, 1]) < 1e-12 and abs(x[0, 2] + x[1, 2] - 2.2) < 1e-10
    assert x[1, 2] - x[0, 2] > 2.2
    r = excursion(t1) / excursion(t2)
    assert 3.0 < r < 5.0, r
