"""RI J/K by the fitting path (oracle).  TEST INFRASTRUCTURE ONLY.

Definitions followed:
* eq. ri_eri: (mu nu|lam sig)_RI = sum_PQ (mu nu|P) [A^{-1}]_PQ (lam sig|Q),
  A_PQ = (P|Q).
* eq. fock_build / eq. j / eq. k with closed-shell D = 2 C_occ C_occ^T:
  J_mu_nu = sum_ls D_ls (mu nu|ls)_RI,
  K_mu_nu = +(1/2) sum_ls D_ls (mu s|l nu)_RI  (the library's sign: the
  paper's exchange term is -K, so F = h + J - K).
* Schwarz screening (Basis-function pair sparsity section): pair (mu nu),
  mu >= nu, is kept iff (mu nu|mu nu) > tau.
* eq. biap under the reading A = L L^T (lower), B = L^{-1} T, so that
  sum_P B^P B^P = T^T A^{-1} T (eq. symmetric_ri).

The fit path never forms B: it solves with the Cholesky factor of A through
scipy (cho_factor / cho_solve), so it is structurally independent of the
GPU path.  ``ri_tensor_brute`` forms the N^4 RI tensor for tiny systems as a
second, brute-force definition.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import integrals as ints


def screen_pairs(sys, tau=None):
    """Significant pairs (mu >= nu) in row-major order of the lower triangle:
    sorted by mu, then nu.  Returns (mu_idx, nu_idx) int arrays."""
    tau = sys.tau if tau is None else tau
    Q = ints.schwarz_diag(sys)
    mu, nu = np.tril_indices(sys.N)
    keep = Q[mu, nu] > tau
    return mu[keep].astype(np.int64), nu[keep].astype(np.int64)


class RIData:
    """Three-centre integrals over significant pairs plus the metric factor."""

    def __init__(self, sys, tau=None):
        self.sys = sys
        self.mu, self.nu = screen_pairs(sys, tau)
        self.T = ints.eri3_pairs(sys, self.mu, self.nu)      # [N_aux, n_pairs]
        self.A = ints.metric(sys)
        self.cho = sla.cho_factor(self.A, lower=True)
        self.w = np.where(self.mu == self.nu, 1.0, 2.0)      # both (mu,nu),(nu,mu)

    @property
    def n_pairs(self):
        return self.mu.size

    def dense_T_chunk(self, p0, p1):
        N = self.sys.N
        out = np.zeros((p1 - p0, N, N))
        out[:, self.mu, self.nu] = self.T[p0:p1]
        out[:, self.nu, self.mu] = self.T[p0:p1]
        return out

    def gamma_fit(self, D):
        """d_P = sum_mu_nu D_mu_nu (mu nu|P); c = A^{-1} d."""
        d = self.T @ (self.w * D[self.mu, self.nu])
        return d, sla.cho_solve(self.cho, d)

    def J(self, D):
        _, c = self.gamma_fit(D)
        jp = c @ self.T
        N = self.sys.N
        J = np.zeros((N, N))
        J[self.mu, self.nu] = jp
        J[self.nu, self.mu] = jp
        return J

    def U(self, C_occ, chunk=64):
        """U^P = T^P C_occ, [N_aux, N, n_occ]."""
        na = self.sys.n_aux
        U = np.empty((na, self.sys.N, C_occ.shape[1]))
        for p0 in range(0, na, chunk):
            p1 = min(na, p0 + chunk)
            U[p0:p1] = self.dense_T_chunk(p0, p1) @ C_occ
        return U

    def K(self, C_occ):
        """K = sum_i sum_PQ U^P_:i [A^{-1}]_PQ (U^Q_:i)^T, via cho_solve."""
        U = self.U(C_occ)
        na, N, no = U.shape
        W = sla.cho_solve(self.cho, U.reshape(na, N * no)).reshape(na, N, no)
        return np.tensordot(U, W, axes=([0, 2], [0, 2]))

    def JK(self, C_occ):
        D = 2.0 * C_occ @ C_occ.T
        return self.J(D), self.K(C_occ)

    def B_packed_dense(self):
        """B = L^{-1} T over pairs (reading of eq. biap), [N_aux, n_pairs]."""
        L = np.tril(self.cho[0])
        return sla.solve_triangular(L, self.T, lower=True)


def ri_tensor_brute(sys):
    """(mu nu|lam sig)_RI as a dense [N,N,N,N] tensor (tiny systems)."""
    T = ints.eri3_dense(sys)
    A = ints.metric(sys)
    N = sys.N
    Tf = T.reshape(sys.n_aux, N * N)
    return (Tf.T @ np.linalg.solve(A, Tf)).reshape(N, N, N, N)


def jk_from_tensor(eri, D):
    """J_mn = sum_ls D_ls (mn|ls);  K_mn = 1/2 sum_ls D_ls (ms|ln)."""
    J = np.einsum("mnls,ls->mn", eri, D)
    K = 0.5 * np.einsum("msln,ls->mn", eri, D)
    return J, K


def product_aux_system(sys, tau=1e-16):
    """Auxiliary set = the distinct Gaussian products of significant orbital
    pairs, each a normalised s function of exponent p at P.  Then the RI
    factorisation is exact for those pairs."""
    import synth
    mu, nu = screen_pairs(sys, tau)
    a = sys.fn_exp[mu]
    b = sys.fn_exp[nu]
    p = a + b
    P = (a[:, None] * sys.xyz[sys.fn_centre[mu]] + b[:, None] * sys.xyz[sys.fn_centre[nu]]) / p[:, None]
    keyset = {}
    for k in range(p.size):
        key = (round(p[k], 12), round(P[k, 0], 10), round(P[k, 1], 10), round(P[k, 2], 10))
        keyset.setdefault(key, (p[k], P[k]))
    exps = np.array([v[0] for v in keyset.values()])
    cen = np.array([v[1] for v in keyset.values()])
    # auxiliary functions sit on "centres" that carry no charge
    xyz = np.concatenate([sys.xyz, cen])
    Z = np.concatenate([sys.Z, np.zeros(cen.shape[0])])
    aux_centre = np.arange(sys.n_centres, sys.n_centres + cen.shape[0], dtype=np.int32)
    return synth.System(xyz, Z, sys.fn_centre.copy(), sys.fn_exp.copy(), aux_centre, exps,
                        sys.n_occ, sys.tau)
