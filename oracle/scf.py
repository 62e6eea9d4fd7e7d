"""Closed-shell Roothaan SCF with DIIS (oracle).  TEST INFRASTRUCTURE ONLY.

Follows the paper's Energy formulation: solve F C = S C eps iteratively with
F = h + J - K (library sign of K, see ``ri``), D = 2 C_occ C_occ^T, DIIS
extrapolation and diagonalisation between iterations (Energy section).
Readings where the paper is silent:
* energy E = 1/2 tr[D (h + F)] + E_nn;
* Loewdin orthogonaliser S^{-1/2}; core-Hamiltonian guess; Aufbau filling of
  the n_occ lowest orbitals;
* DIIS(6) on e = F D S - S D F (Pulay), extrapolating once two vectors are
  held; converged when |dE| < tol_E and max|e| < tol_e.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from . import integrals as ints
from .ri import RIData


@dataclasses.dataclass
class SCFResult:
    E: float
    E_nuc: float
    E_1e: float
    E_J: float
    E_K: float
    C_occ: np.ndarray
    eps: np.ndarray
    C: np.ndarray
    D: np.ndarray
    F: np.ndarray
    J: np.ndarray
    K: np.ndarray
    n_iter: int
    converged: bool
    E_guess: float
    history: list


def orthogonaliser(S):
    w, V = np.linalg.eigh(S)
    if w.min() < 1e-10:
        raise ValueError("overlap matrix numerically singular")
    return (V / np.sqrt(w)) @ V.T


def aufbau(F, X, n_occ):
    eps, Cp = np.linalg.eigh(X @ F @ X)
    C = X @ Cp
    return eps, C, C[:, :n_occ]


def run_scf(sys, ri: RIData | None = None, tol_E=1e-12, tol_e=1e-8, max_iter=100,
            diis_n=6, C_guess=None, jk=None):
    """Returns an SCFResult.  ``jk(C_occ) -> (J, K)`` may replace the RI
    fit path (used to run the exact four-index reference)."""
    if ri is None and jk is None:
        ri = RIData(sys)
    if jk is None:
        jk = ri.JK
    S = ints.overlap(sys)
    h = ints.core_hamiltonian(sys)
    Enn = ints.nuclear_repulsion(sys)
    X = orthogonaliser(S)
    n_occ = sys.n_occ
    if C_guess is None:
        eps, C, Cocc = aufbau(h, X, n_occ)
    else:
        Cocc = np.array(C_guess)
        eps = np.zeros(sys.N)
        C = None
    Fs, es = [], []
    E_old = None
    hist = []
    E_guess = None
    converged = False
    for it in range(1, max_iter + 1):
        D = 2.0 * Cocc @ Cocc.T
        J, K = jk(Cocc)
        F = h + J - K
        E1 = float(np.sum(D * h))
        EJ = 0.5 * float(np.sum(D * J))
        EK = -0.5 * float(np.sum(D * K))
        E = E1 + EJ + EK + Enn
        if E_guess is None:
            E_guess = E
        e = F @ D @ S - S @ D @ F
        err = float(np.abs(e).max())
        hist.append((E, err))
        if E_old is not None and abs(E - E_old) < tol_E and err < tol_e:
            converged = True
            break
        E_old = E
        Fs.append(F)
        es.append(e)
        if len(Fs) > diis_n:
            Fs.pop(0)
            es.pop(0)
        Fx = F
        m = len(Fs)
        if m >= 2:
            Bm = np.empty((m + 1, m + 1))
            Bm[-1, :] = -1.0
            Bm[:, -1] = -1.0
            Bm[-1, -1] = 0.0
            for i in range(m):
                for j in range(m):
                    Bm[i, j] = np.sum(es[i] * es[j])
            rhs = np.zeros(m + 1)
            rhs[-1] = -1.0
            c = np.linalg.solve(Bm, rhs)[:m]
            Fx = sum(ci * Fi for ci, Fi in zip(c, Fs))
        eps, C, Cocc = aufbau(Fx, X, n_occ)
    # final canonical orbitals of the converged Fock matrix
    eps, C, Cocc_c = aufbau(F, X, n_occ)
    return SCFResult(E, Enn, E1, EJ, EK, Cocc, eps, C, D, F, J, K, it, converged, E_guess, hist)


def exact_jk(sys):
    """J, K from the exact four-index ERIs (tiny systems)."""
    eri = ints.eri4(sys)

    def jk(Cocc):
        D = 2.0 * Cocc @ Cocc.T
        return (np.einsum("mnls,ls->mn", eri, D), 0.5 * np.einsum("msln,ls->mn", eri, D))
    return jk
