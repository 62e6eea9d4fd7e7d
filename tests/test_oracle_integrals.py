"""Pins of the oracle's integrals against quadrature and closed forms."""
import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import integrals as I

RNG = np.random.default_rng(7)


def one_centre(a, Z=2.0):
    return synth.make_system(np.zeros((1, 3)), [a], [a], Zval=Z)


def two_fn_system(a, b, A, B, aux=(0.7,)):
    xyz = np.array([A, B], dtype=float)
    s = synth.make_system(xyz, [1.0], list(aux))
    s.fn_exp = np.array([a, b])
    s.fn_centre = np.array([0, 1], dtype=np.int32)
    return s


@pytest.mark.parametrize("t", [0.0, 1e-9, 1e-4, 0.3, 1.0, 2.5, 17.0, 60.0])
def test_boys_against_quadrature(t):
    f0 = integrate.quad(lambda u: np.exp(-t * u * u), 0, 1, epsabs=1e-15, epsrel=1e-14)[0]
    f1 = integrate.quad(lambda u: u * u * np.exp(-t * u * u), 0, 1, epsabs=1e-15, epsrel=1e-14)[0]
    assert abs(I.boys0(np.array([t]))[0] - f0) < 1e-14
    assert abs(I.boys1(np.array([t]))[0] - f1) < 1e-14


@pytest.mark.parametrize("a", [0.08, 0.77, 12.0, 96.6])
def test_single_function_closed_forms(a):
    s = one_centre(a)
    assert abs(I.overlap(s)[0, 0] - 1.0) < 1e-14
    assert abs(I.kinetic(s)[0, 0] - 1.5 * a) < 1e-12 * a
    assert abs(I.nuclear(s)[0, 0] + 2 * 2.0 * np.sqrt(2 * a / np.pi)) < 1e-12 * np.sqrt(a)
    assert abs(I.eri4(s)[0, 0, 0, 0] - 2 * np.sqrt(a / np.pi)) < 1e-13 * np.sqrt(a)


def test_gaussian_product_pointwise():
    a, b = 0.9, 2.3
    A, B = np.array([0.1, -0.4, 0.3]), np.array([1.2, 0.5, -0.7])
    p = a + b
    P = (a * A + b * B) / p
    K = np.exp(-a * b / p * np.sum((A - B) ** 2))
    for _ in range(5):
        r = RNG.normal(size=3)
        lhs = np.exp(-a * np.sum((r - A) ** 2)) * np.exp(-b * np.sum((r - B) ** 2))
        assert abs(lhs - K * np.exp(-p * np.sum((r - P) ** 2))) < 1e-15


def _g1(a, x0):
    return lambda x: np.exp(-a * (x - x0) ** 2)


def test_overlap_kinetic_quadrature():
    a, b = 0.6, 1.7
    A, B = np.array([0.0, 0.3, -0.2]), np.array([0.9, -0.5, 0.4])
    s = two_fn_system(a, b, A, B)
    Na, Nb = I.norm(a), I.norm(b)
    ov = [integrate.quad(lambda x: _g1(a, A[k])(x) * _g1(b, B[k])(x), -20, 20, epsabs=1e-15)[0] for k in range(3)]
    dd = [integrate.quad(lambda x: (-2 * a * (x - A[k])) * _g1(a, A[k])(x) * (-2 * b * (x - B[k])) * _g1(b, B[k])(x),
                         -20, 20, epsabs=1e-15)[0] for k in range(3)]
    S_ref = Na * Nb * np.prod(ov)
    T_ref = 0.5 * Na * Nb * sum(dd[k] * np.prod([ov[j] for j in range(3) if j != k]) for k in range(3))
    assert abs(I.overlap(s)[0, 1] - S_ref) < 1e-13
    assert abs(I.kinetic(s)[0, 1] - T_ref) < 1e-12


def test_nuclear_attraction_quadrature():
    # 1/|r - C| = 2/sqrt(pi) int_0^inf exp(-u^2 |r-C|^2) du; each u gives a
    # separable 3-D Gaussian integral, done by 1-D quadrature per axis.
    a, b = 0.8, 1.3
    A, B = np.array([0.0, 0.0, 0.0]), np.array([0.7, 0.2, -0.3])
    s = two_fn_system(a, b, A, B)
    s.Z = np.array([1.0, 0.0])
    C = A
    Na, Nb = I.norm(a), I.norm(b)

    def inner(u):
        v = 1.0
        w = 1.0 / np.sqrt(a + b + u * u)
        for k in range(3):
            v *= integrate.quad(lambda x: np.exp(-a * (x - A[k]) ** 2 - b * (x - B[k]) ** 2 - u * u * (x - C[k]) ** 2),
                                C[k] - 12 * w - 2, C[k] + 12 * w + 2, epsabs=0, epsrel=1e-13, points=[C[k]],
                                limit=200)[0]
        return v
    # u = t / (1 - t) maps [0, inf) onto [0, 1)
    f = lambda t: inner(t / (1 - t)) / (1 - t) ** 2
    val = -2 / np.sqrt(np.pi) * Na * Nb * integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-12, limit=400)[0]
    assert abs(I.nuclear(s)[0, 1] - val) < 1e-10


def _gauss_potential(p, charge):
    """Potential of a spherical Gaussian charge by the shell theorem (radial quadrature)."""
    rho = lambda r: charge * (p / np.pi) ** 1.5 * np.exp(-p * r * r)

    def V(R):
        inside = integrate.quad(lambda r: 4 * np.pi * r * r * rho(r), 0, R, epsabs=1e-15)[0] / R
        outside = integrate.quad(lambda r: 4 * np.pi * r * rho(r), R, np.inf, epsabs=1e-15)[0]
        return inside + outside
    return V


def test_four_centre_eri_electrostatics():
    # (ab|cd) = interaction of charge clouds rho_ab and rho_cd; each is a
    # spherical Gaussian of charge S_ab (product theorem, pinned above).
    a, b, c, d = 0.5, 1.1, 0.7, 0.9
    X = [np.array(v, float) for v in ([0, 0, 0], [0.8, 0, 0], [0, 1.5, 0.4], [0.3, 1.0, -0.2])]
    s = synth.make_system(np.array(X), [1.0], [1.0])
    s.fn_exp = np.array([a, b, c, d])
    s.fn_centre = np.arange(4, dtype=np.int32)
    S = I.overlap(s)
    p, q = a + b, c + d
    P = (a * X[0] + b * X[1]) / p
    Q = (c * X[2] + d * X[3]) / q
    R = np.linalg.norm(P - Q)
    V1 = _gauss_potential(p, S[0, 1])
    rho2 = lambda r: S[2, 3] * (q / np.pi) ** 1.5 * np.exp(-q * r * r)
    f = lambda ct, r: 2 * np.pi * r * r * rho2(r) * V1(np.sqrt(max(r * r + R * R - 2 * r * R * ct, 1e-30)))
    val = integrate.dblquad(f, 0, 8.0, -1, 1, epsabs=1e-12, epsrel=1e-11)[0]
    assert abs(I.eri4(s)[0, 1, 2, 3] - val) < 1e-9


def test_eri_symmetry_and_schwarz():
    s = synth.config_system("tiny")
    eri = I.eri4(s)
    assert np.allclose(eri, eri.transpose(1, 0, 2, 3), atol=0, rtol=1e-14)
    assert np.allclose(eri, eri.transpose(2, 3, 0, 1), atol=0, rtol=1e-14)
    T = I.eri3_dense(s)
    assert np.allclose(T, T.transpose(0, 2, 1), atol=0, rtol=1e-14)
    A = I.metric(s)
    assert np.allclose(A, A.T, atol=0, rtol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0
    Q = I.schwarz_diag(s)
    assert np.allclose(Q, np.einsum("mnmn->mn", eri), rtol=1e-13, atol=0)
    bound = np.sqrt(Q)[None] * np.sqrt(np.diag(A))[:, None, None]
    assert np.all(np.abs(T) <= bound * (1 + 1e-12) + 1e-150)
    # four-centre Schwarz
    assert np.all(np.abs(eri) <= np.sqrt(Q)[:, :, None, None] * np.sqrt(Q)[None, None] * (1 + 1e-12) + 1e-150)


def _fd(fun, sys, centre, k, h=1e-4):
    out = []
    for sgn in (-2, -1, 1, 2):
        x = sys.xyz.copy()
        x[centre, k] += sgn * h
        out.append(fun(sys.with_xyz(x)))
    return (out[0] - 8 * out[1] + 8 * out[2] - out[3]) / (12 * h)


def test_derivative_integrals_against_fd():
    s = synth.config_system("tiny")
    s = synth.make_system(s.xyz[:3], [0.3, 1.0, 3.5], [0.2, 0.9, 4.0])
    dS, dT = I.overlap_kinetic_derivs(s)
    vA, vB, vC = I.nuclear_derivs(s)
    mu, nu = np.tril_indices(s.N)
    dA3, dB3 = I.eri3_derivs_pairs(s, mu, nu)
    dM = I.metric_derivs(s)
    fc = s.fn_centre
    for c in range(s.n_centres):
        for k in range(3):
            # analytic derivative of each integral w.r.t. centre c, coordinate k
            on_mu = (fc[:, None] == c).astype(float)
            on_nu = (fc[None, :] == c).astype(float)
            aS = dS[..., k] * on_mu - dS[..., k] * on_nu
            aT = dT[..., k] * on_mu - dT[..., k] * on_nu
            aV = vA[..., k] * on_mu + vB[..., k] * on_nu + vC[c, ..., k]
            assert np.abs(aS - _fd(I.overlap, s, c, k)).max() < 1e-9
            assert np.abs(aT - _fd(I.kinetic, s, c, k)).max() < 1e-8
            assert np.abs(aV - _fd(I.nuclear, s, c, k)).max() < 1e-8
            onP = (s.aux_centre == c).astype(float)
            a3 = dA3[..., k] * (fc[mu] == c) + dB3[..., k] * (fc[nu] == c) - (dA3[..., k] + dB3[..., k]) * onP[:, None]
            f3 = _fd(lambda ss: I.eri3_pairs(ss, mu, nu), s, c, k)
            assert np.abs(a3 - f3).max() < 1e-8
            a2 = dM[..., k] * onP[:, None] - dM[..., k] * onP[None, :]
            assert np.abs(a2 - _fd(I.metric, s, c, k)).max() < 1e-8


def test_translational_invariance_of_derivatives():
    s = synth.config_system("tiny")
    vA, vB, vC = I.nuclear_derivs(s)
    assert np.abs(vA + vB + vC.sum(0)).max() < 1e-12
