"""Analytic RI-HF nuclear gradient and finite differences (oracle).
TEST INFRASTRUCTURE ONLY.

Follows eq. rihf_gradient of the Gradient-formulation section:
  g = sum D h' - sum W S' + sum_{P mu nu} Y^P_mu_nu (mu nu|P)' - 1/2 sum_PQ Z_PQ (P|Q)'
      + E_nn'
in the reading for unscaled occupied coefficients (D = 2 C C^T):
  c        = A^{-1} d,  d_P = sum D_mu_nu (mu nu|P)
  Xi^P_ij  = sum_Q [A^{-1}]_PQ (ij|Q),  (ij|Q) = (C^T T_Q C)_ij
  Y^P      = c_P D - 2 C Xi^P C^T
  Z_PQ     = c_P c_Q - 2 sum_ij Xi^P_ij Xi^Q_ij
  W        = 2 C_occ diag(eps_occ) C_occ^T
The paper prints -1/2 in Y and Z, which holds for sqrt(2)-scaled orbitals
(D = C C^T); the factor 2 here is the same expression for D = 2 C C^T, and the
finite-difference pin decides between the two.  The nuclear-repulsion term
and the operator part of h' are included (the paper's expression is the
electronic gradient).

``fd_gradient`` differentiates the converged RI energy with a 4-point central
stencil, warm-starting every displaced SCF from the reference orbitals.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import integrals as ints
from .ri import RIData
from .scf import run_scf


def _scatter(g, centres, vec):
    np.add.at(g, centres, vec)


def analytic_gradient(sys, res, ri: RIData | None = None, parts=False):
    if ri is None:
        ri = RIData(sys)
    n = sys.n_occ
    Cc = res.C[:, :n]
    eps = res.eps[:n]
    D = res.D
    W = 2.0 * (Cc * eps) @ Cc.T
    fc = sys.fn_centre
    g1 = np.zeros_like(sys.xyz)
    # one-electron part: sum over all (mu, nu)
    dS, dT = ints.overlap_kinetic_derivs(sys)
    vA, vB, vC = ints.nuclear_derivs(sys)
    N = sys.N
    muc = np.repeat(fc, N)
    nuc = np.tile(fc, N)
    hA = (D[..., None] * (dT + vA)).reshape(-1, 3)
    hB = (D[..., None] * (-dT + vB)).reshape(-1, 3)
    _scatter(g1, muc, hA)
    _scatter(g1, nuc, hB)
    g1 += np.einsum("mn,cmnx->cx", D, vC)
    sA = (W[..., None] * dS).reshape(-1, 3)
    _scatter(g1, muc, -sA)
    _scatter(g1, nuc, sA)
    # fitting coefficients
    d, c = ri.gamma_fit(D)
    # t_P,ij = (C^T T_P C)_ij for the density-generating orbitals
    Co = res.C_occ
    na = sys.n_aux
    t = np.empty((na, n, n))
    for p0 in range(0, na, 64):
        p1 = min(na, p0 + 64)
        Tp = ri.dense_T_chunk(p0, p1)
        t[p0:p1] = Co.T @ Tp @ Co          # (C^T T_P C) for each P of the chunk
    Xi = sla.cho_solve(ri.cho, t.reshape(na, n * n)).reshape(na, n, n)
    # three-centre term over significant pairs (both orders -> weight w)
    g3 = np.zeros_like(sys.xyz)
    mu, nu = ri.mu, ri.nu
    Dp = D[mu, nu]
    for P in range(na):
        dA, dB = ints.eri3_derivs_pairs(sys, mu, nu, [P])
        V = Co @ Xi[P] @ Co.T
        Y = (c[P] * Dp - 2.0 * V[mu, nu]) * ri.w
        cA = Y[:, None] * dA[0]
        cB = Y[:, None] * dB[0]
        _scatter(g3, fc[mu], cA)
        _scatter(g3, fc[nu], cB)
        g3[sys.aux_centre[P]] -= cA.sum(0) + cB.sum(0)
    # two-centre term
    Xf = Xi.reshape(na, n * n)
    Z = np.outer(c, c) - 2.0 * Xf @ Xf.T
    dM = ints.metric_derivs(sys)
    g2 = np.zeros_like(sys.xyz)
    contrib = (-0.5 * Z)[..., None] * dM
    _scatter(g2, sys.aux_centre, contrib.sum(1))
    _scatter(g2, sys.aux_centre, -contrib.sum(0))
    gn = ints.nuclear_repulsion_grad(sys)
    g = g1 + g3 + g2 + gn
    if parts:
        return g, dict(one=g1, three=g3, two=g2, nuc=gn, c=c, Xi=Xi, Z=Z, W=W)
    return g


def fd_gradient(sys, res, h=1e-3, atoms=None, tol_E=1e-13):
    """4-point central finite differences of the converged RI energy."""
    g = np.zeros_like(sys.xyz)
    atoms = range(sys.n_centres) if atoms is None else atoms
    for A in atoms:
        for x in range(3):
            E = []
            for s in (-2, -1, 1, 2):
                xyz = sys.xyz.copy()
                xyz[A, x] += s * h
                sd = sys.with_xyz(xyz)
                r = run_scf(sd, tol_E=tol_E, tol_e=1e-9, C_guess=res.C_occ)
                E.append(r.E)
            g[A, x] = (E[0] - 8 * E[1] + 8 * E[2] - E[3]) / (12 * h)
    return g
