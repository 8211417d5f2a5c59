"""O1: the whole spatial operator as one dense matrix (tiny grids only).

Follows the paper's construction directly:

1. Build A and B per axis as printed (Section 3.1) and the d-dimensional
   Kronecker-sum operator T = A_d^-1 B_d (Sections 3.2-3.3), as the symmetric
   pencil (W B_d, W A_d) from ``matrices.dense_pair``.
2. Diagonalise it with LAPACK (generalised symmetric-definite eigh), so
   T = V diag(lam) V^-1 with V^-1 = V^T (W A_d).
3. Raise to alpha/2 by the eigendecomposition (Lemma, Section 2):
   A_s = kappa_s V diag(lam^(alpha_s/2)) V^-1 (Def. 1 with the matrix transfer
   technique, eq. MTT).
4. Form each coefficient *matrix* of tau*A_s: dense solves of the P13
   polynomials, or matrix exponentials and phi-functions (exponential scheme).
5. Step eq. ETDRK4P13 in physical space with these matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import coefficients, matrices


class DenseOperator:
    def __init__(self, bc, shape, h, alpha, kappa, tau, scheme="p13"):
        self.bc, self.shape, self.h = bc, tuple(shape), tuple(h)
        self.tau = float(tau)
        WB, WA = matrices.dense_pair(bc, self.shape, self.h)
        lam, V = scipy.linalg.eigh(WB, WA)
        lam = np.where(np.abs(lam) < 1e-12 * np.max(np.abs(lam)), 0.0, lam)
        self.lam, self.V, self.Vinv = lam, V, V.T @ WA
        self.weights = matrices.dense_weights(bc, self.shape)
        self.coef = []
        for al, ka in zip(alpha, kappa):
            tA = self.tau * ka * (V * lam ** (al / 2.0)) @ self.Vinv
            self.coef.append(coefficients.matrix(scheme, tA, self.tau))

    def fractional_laplacian(self, x, alpha):
        """T^(alpha/2) x for one field (Def. 1 / eq. MTT)."""
        y = (self.V * self.lam ** (alpha / 2.0)) @ (self.Vinv @ x.ravel())
        return y.reshape(x.shape)

    def apply(self, name, X):
        return np.stack([(self.coef[s][name] @ X[s].ravel()).reshape(self.shape)
                         for s in range(X.shape[0])])

    def step(self, U, t, N):
        """One ETDRK4 step (eq. ETDRK4P13); N(U, t) is the nonlinear term."""
        tau, G = self.tau, self.apply
        Nu = N(U, t)
        a = G("Q", U) + G("phi", Nu)
        Na = N(a, t + tau / 2)
        b = G("Q", U) + G("phi", Na)
        Nb = N(b, t + tau / 2)
        c = G("Q", a) + G("phi", 2.0 * Nb - Nu)
        Nc = N(c, t + tau)
        return G("R", U) + G("phi1", Nu) + G("phi2", Na + Nb) + G("phi3", Nc)

    def integrate(self, U, nsteps, N, t0=0.0):
        U = np.array(U, dtype=np.float64)
        for k in range(nsteps):
            U = self.step(U, t0 + k * self.tau, N)
        return U
