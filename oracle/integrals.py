"""Closed-form integrals over normalised primitive s-Gaussians (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

phi_a(r) = N_a exp(-a |r - A|^2),  N_a = (2a/pi)^{3/4}.
Gaussian product: p = a + b, P = (aA + bB)/p, K_ab = exp(-(ab/p)|A-B|^2).

The integrals are those defined in the paper's Notation section (the
four-centre ERI in chemist's notation, the two- and three-centre ERIs); the
closed forms for s functions are the standard ones from the quantum-chemistry
text the paper cites for Hartree-Fock.  The Boys function is
F_m(t) = int_0^1 u^{2m} exp(-t u^2) du.

Pins (tests/test_oracle_integrals.py): quadrature of the Boys definitions,
radial-quadrature nuclear attraction, electrostatics of two Gaussian charges
by 2-D quadrature, self-overlap / kinetic / attraction / self-repulsion closed
forms, symmetry, Schwarz bound and translational invariance of derivatives.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

PI = np.pi


def norm(a):
    return (2.0 * a / PI) ** 0.75


def boys0(t):
    """F_0(t) = (1/2) sqrt(pi/t) erf(sqrt t); Taylor series for t < 1e-3."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    small = t < 1e-3
    ts = t[small]
    # sum_k (-t)^k / (k! (2k+1))
    s = np.zeros_like(ts)
    term = np.ones_like(ts)
    for k in range(8):
        s += term / (2 * k + 1)
        term = term * (-ts) / (k + 1)
    out[small] = s
    tl = t[~small]
    out[~small] = 0.5 * np.sqrt(PI / tl) * erf(np.sqrt(tl))
    return out


def boys1(t):
    """F_1(t) = (F_0(t) - exp(-t)) / (2t); Taylor series for t < 1."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    small = t < 1.0
    ts = t[small]
    # sum_k (-t)^k / (k! (2k+3))
    s = np.zeros_like(ts)
    term = np.ones_like(ts)
    for k in range(30):
        s += term / (2 * k + 3)
        term = term * (-ts) / (k + 1)
    out[small] = s
    tl = t[~small]
    out[~small] = (boys0(tl) - np.exp(-tl)) / (2.0 * tl)
    return out


def _pair_arrays(xyz, fcen, fexp):
    A = xyz[fcen]                        # [N,3]
    a = fexp
    p = a[:, None] + a[None, :]
    P = (a[:, None, None] * A[:, None, :] + a[None, :, None] * A[None, :, :]) / p[..., None]
    AB2 = ((A[:, None, :] - A[None, :, :]) ** 2).sum(-1)
    mu = a[:, None] * a[None, :] / p
    K = np.exp(-mu * AB2)
    nn = norm(a)[:, None] * norm(a)[None, :]
    return A, p, P, AB2, mu, K, nn


def overlap(sys):
    _, p, _, _, _, K, nn = _pair_arrays(sys.xyz, sys.fn_centre, sys.fn_exp)
    return nn * (PI / p) ** 1.5 * K


def kinetic(sys):
    _, p, _, AB2, mu, K, nn = _pair_arrays(sys.xyz, sys.fn_centre, sys.fn_exp)
    S = nn * (PI / p) ** 1.5 * K
    return mu * (3.0 - 2.0 * mu * AB2) * S


def nuclear(sys):
    _, p, P, _, _, K, nn = _pair_arrays(sys.xyz, sys.fn_centre, sys.fn_exp)
    V = np.zeros_like(p)
    for C, Zc in zip(sys.xyz, sys.Z):
        PC2 = ((P - C) ** 2).sum(-1)
        V -= Zc * nn * (2.0 * PI / p) * K * boys0(p * PC2)
    return V


def core_hamiltonian(sys):
    return kinetic(sys) + nuclear(sys)


def nuclear_repulsion(sys):
    e = 0.0
    n = sys.n_centres
    for A in range(n):
        for B in range(A + 1, n):
            if sys.Z[A] * sys.Z[B] != 0.0:       # charge-free fitting centres
                e += sys.Z[A] * sys.Z[B] / np.linalg.norm(sys.xyz[A] - sys.xyz[B])
    return e


def eri4(sys):
    """Dense (mu nu|lam sig) [N,N,N,N]; small systems only."""
    _, p, P, _, _, K, nn = _pair_arrays(sys.xyz, sys.fn_centre, sys.fn_exp)
    N = p.shape[0]
    pf = p.reshape(-1)
    Pf = P.reshape(-1, 3)
    Kf = (K * nn).reshape(-1)
    out = np.empty((N * N, N * N))
    for r in range(N * N):
        q = pf
        PQ2 = ((Pf[r] - Pf) ** 2).sum(-1)
        rho = pf[r] * q / (pf[r] + q)
        out[r] = (2.0 * PI ** 2.5 / (pf[r] * q * np.sqrt(pf[r] + q))) * Kf[r] * Kf * boys0(rho * PQ2)
    return out.reshape(N, N, N, N)


def metric(sys):
    """A_PQ = (P|Q) over the auxiliary basis."""
    R = sys.xyz[sys.aux_centre]
    al = sys.aux_exp
    s = al[:, None] + al[None, :]
    pr = al[:, None] * al[None, :]
    R2 = ((R[:, None, :] - R[None, :, :]) ** 2).sum(-1)
    na = norm(al)
    return na[:, None] * na[None, :] * 2.0 * PI ** 2.5 / (pr * np.sqrt(s)) * boys0(pr / s * R2)


def eri3_pairs(sys, mu_idx, nu_idx):
    """(mu nu|P) for the listed pairs: returns [N_aux, n_pairs]."""
    A = sys.xyz[sys.fn_centre[mu_idx]]
    B = sys.xyz[sys.fn_centre[nu_idx]]
    a = sys.fn_exp[mu_idx]
    b = sys.fn_exp[nu_idx]
    p = a + b
    P = (a[:, None] * A + b[:, None] * B) / p[:, None]
    K = np.exp(-(a * b / p) * ((A - B) ** 2).sum(-1)) * norm(a) * norm(b)
    R = sys.xyz[sys.aux_centre]
    al = sys.aux_exp
    out = np.empty((al.size, p.size))
    for k in range(al.size):
        w = p * al[k] / (p + al[k])
        PR2 = ((P - R[k]) ** 2).sum(-1)
        out[k] = norm(al[k]) * 2.0 * PI ** 2.5 / (p * al[k] * np.sqrt(p + al[k])) * K * boys0(w * PR2)
    return out


def eri3_dense(sys):
    """(mu nu|P) as [N_aux, N, N]."""
    N = sys.N
    mu, nu = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    return eri3_pairs(sys, mu.reshape(-1), nu.reshape(-1)).reshape(sys.n_aux, N, N)


def schwarz_diag(sys):
    """Q_mu_nu = (mu nu|mu nu) for all pairs [N, N]."""
    _, p, _, _, _, K, nn = _pair_arrays(sys.xyz, sys.fn_centre, sys.fn_exp)
    return (nn * K) ** 2 * 2.0 * PI ** 2.5 / (p * p * np.sqrt(2.0 * p))


# ---------------------------------------------------------------- derivatives
# Each returns derivatives with respect to the centres the integral depends on;
# the gradient module scatters them onto atoms.

def overlap_kinetic_derivs(sys):
    """dS/dA and dT/dA for every (mu, nu), A = centre of mu: [N, N, 3].
    The derivative with respect to nu's centre is the negative."""
    A, p, _, AB2, mu, K, nn = _pair_arrays(sys.xyz, sys.fn_centre, sys.fn_exp)
    S = nn * (PI / p) ** 1.5 * K
    T = mu * (3.0 - 2.0 * mu * AB2) * S
    d = A[:, None, :] - A[None, :, :]
    dS = -2.0 * mu[..., None] * d * S[..., None]
    dT = -2.0 * mu[..., None] * d * (2.0 * mu * S + T)[..., None]
    return dS, dT


def nuclear_derivs(sys):
    """For V^C_mu_nu: derivatives w.r.t. A (mu centre), B (nu centre) and C.
    Returns dA, dB [N,N,3] summed over C, and dC [n_centres, N, N, 3]."""
    A, p, P, _, mu, K, nn = _pair_arrays(sys.xyz, sys.fn_centre, sys.fn_exp)
    a = sys.fn_exp
    N = a.size
    dA = np.zeros((N, N, 3))
    dB = np.zeros((N, N, 3))
    dC = np.zeros((sys.n_centres, N, N, 3))
    d = A[:, None, :] - A[None, :, :]
    for c, (C, Zc) in enumerate(zip(sys.xyz, sys.Z)):
        PC = P - C
        x = p * (PC ** 2).sum(-1)
        pre = Zc * nn * (2.0 * PI / p) * K
        V = -pre * boys0(x)
        f1 = boys1(x)
        # dV/dA = V * dlnK/dA - pre * (-F1) * dx/dA ; dx/dA = 2 a (P - C)
        dA += V[..., None] * (-2.0 * mu[..., None] * d) + (pre * f1)[..., None] * 2.0 * a[:, None, None] * PC
        dB += V[..., None] * (2.0 * mu[..., None] * d) + (pre * f1)[..., None] * 2.0 * a[None, :, None] * PC
        dC[c] = -(pre * f1)[..., None] * 2.0 * p[..., None] * PC
    return dA, dB, dC


def eri3_derivs_pairs(sys, mu_idx, nu_idx, aux_idx=None):
    """d(mu nu|P)/dA and /dB for the listed pairs: [n_P, n_pairs, 3] each,
    over the auxiliary functions aux_idx (default: all).
    The derivative w.r.t. the auxiliary centre is -(dA + dB)."""
    A = sys.xyz[sys.fn_centre[mu_idx]]
    B = sys.xyz[sys.fn_centre[nu_idx]]
    a = sys.fn_exp[mu_idx]
    b = sys.fn_exp[nu_idx]
    p = a + b
    P = (a[:, None] * A + b[:, None] * B) / p[:, None]
    m = a * b / p
    K = np.exp(-m * ((A - B) ** 2).sum(-1)) * norm(a) * norm(b)
    aux_idx = np.arange(sys.n_aux) if aux_idx is None else np.asarray(aux_idx)
    R = sys.xyz[sys.aux_centre[aux_idx]]
    al = sys.aux_exp[aux_idx]
    dA = np.empty((al.size, p.size, 3))
    dB = np.empty((al.size, p.size, 3))
    for k in range(al.size):
        w = p * al[k] / (p + al[k])
        PR = P - R[k]
        x = w * (PR ** 2).sum(-1)
        c0 = norm(al[k]) * 2.0 * PI ** 2.5 / (p * al[k] * np.sqrt(p + al[k])) * K
        I = c0 * boys0(x)
        g = c0 * boys1(x) * 2.0 * w          # -dF0/dx * dx/dP factor
        dA[k] = -2.0 * m[:, None] * (A - B) * I[:, None] - (g * a / p)[:, None] * PR
        dB[k] = 2.0 * m[:, None] * (A - B) * I[:, None] - (g * b / p)[:, None] * PR
    return dA, dB


def metric_derivs(sys):
    """d(P|Q)/dR_P as [N_aux, N_aux, 3]; d/dR_Q is the negative."""
    R = sys.xyz[sys.aux_centre]
    al = sys.aux_exp
    s = al[:, None] + al[None, :]
    pr = al[:, None] * al[None, :]
    w = pr / s
    d = R[:, None, :] - R[None, :, :]
    na = norm(al)
    c0 = na[:, None] * na[None, :] * 2.0 * PI ** 2.5 / (pr * np.sqrt(s))
    return -(c0 * boys1(w * (d ** 2).sum(-1)) * 2.0 * w)[..., None] * d


def nuclear_repulsion_grad(sys):
    g = np.zeros_like(sys.xyz)
    n = sys.n_centres
    for A in range(n):
        for B in range(n):
            if A != B and sys.Z[A] * sys.Z[B] != 0.0:
                r = sys.xyz[A] - sys.xyz[B]
                g[A] -= sys.Z[A] * sys.Z[B] * r / np.linalg.norm(r) ** 3
    return g
