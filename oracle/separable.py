"""O2: per-axis LAPACK eigenbases, usable up to the full benchmark sizes.

The d-dimensional operator is a Kronecker sum of 1D operators
(Sections 3.2-3.3), so it is diagonalised by the tensor product of the 1D
eigenbases. Per axis, LAPACK solves (W B) v = lam (W A) v (``matrices``), so
V^T (W A) V = I and T_1D = V diag(lam) P with P = V^T W A. The d-dim
eigenvalues are sums lam_x + lam_y (+ lam_z) (E16-E18, E22) and every
coefficient operator is applied as

    g(T) x = (V_x (x) V_y ..) [ g(L) * ((P_x (x) P_y ..) x) ],
    L = kappa tau Lambda^(alpha/2)  (Alg. 1 precompute),

with dense per-axis tensordots (no closed-form eigenvalues, no FFT). The step
is eq. ETDRK4P13 in physical space, each operator applied on its own.

With ``periodic_basis="hartley"`` a periodic axis takes the exact eigenbasis
of its circulant operator instead (Section 3.1: A and B are circulant, so the
Fourier modes diagonalise them; real Hartley vectors cas(2 pi jk/n) =
cos + sin span each pair k, n-k of equal eigenvalues): v_k = c_k /
sqrt(c_k^T A c_k), lam_k = (c_k^T B c_k)/(c_k^T A c_k). LAPACK's eigenvectors
of a long periodic axis carry errors of order eps ||A|| / gap in the
clustered top modes; sensitivities weighted by dL/dkappa, which grows with
the mode, show them (about 2e-10 relative on a 1024-point axis).

``step_adjoint`` is the discrete adjoint of that step, written from the chain
rule with explicit transposes g(T)^T = P^T g(L) V^T, the reaction Jacobians
transposed, and parameter sensitivities d g(T)/d theta = V g'(L) dL/dtheta P.
``step_tangent`` is the forward-mode linearisation of the same step.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import coefficients, matrices


def _along(M, x, ax):
    return np.moveaxis(np.tensordot(M, x, axes=([1], [ax])), 0, ax)


def circulant_eig(A, B):
    """Generalised eigenpairs B v = lam A v of symmetric circulant A, B from
    the Hartley vectors, normalised to V^T A V = I (Section 3.1)."""
    n = A.shape[0]
    jk = np.outer(np.arange(n), np.arange(n)) % n
    C = np.cos(2.0 * np.pi * jk / n) + np.sin(2.0 * np.pi * jk / n)
    mu = np.sum(C * (A @ C), axis=0)  # c_k^T A c_k
    nu = np.sum(C * (B @ C), axis=0)
    return nu / mu, C / np.sqrt(mu)


class SeparableOperator:
    def __init__(self, bc, shape, h, periodic_basis="lapack"):
        self.bc, self.shape, self.h = bc, tuple(shape), tuple(h)
        self.d = len(shape)
        self.V, self.P, self.lam, self.w = [], [], [], []
        for n, hh in zip(self.shape, self.h):
            A, B = matrices.ab(bc, n, hh)
            W = np.diag(matrices.weights(bc, n))
            if bc == "periodic" and periodic_basis == "hartley":
                lam, V = circulant_eig(W @ A, W @ B)
            else:
                lam, V = scipy.linalg.eigh(W @ B, W @ A)
            lam = np.where(np.abs(lam) < 1e-12 * np.max(np.abs(lam)), 0.0, lam)
            self.V.append(V)
            self.P.append(V.T @ W @ A)
            self.lam.append(lam)
            self.w.append(matrices.weights(bc, n))
        Lam = np.zeros(self.shape)
        for a, lam in enumerate(self.lam):
            sh = [1] * self.d
            sh[a] = -1
            Lam = Lam + lam.reshape(sh)
        self.Lam = Lam

    # x has the spatial axes last
    def fwd(self, x):
        off = x.ndim - self.d
        for a in range(self.d):
            x = _along(self.P[a], x, off + a)
        return x

    def inv(self, X):
        off = X.ndim - self.d
        for a in range(self.d):
            X = _along(self.V[a], X, off + a)
        return X

    def fwd_T(self, y):
        off = y.ndim - self.d
        for a in range(self.d):
            y = _along(self.P[a].T, y, off + a)
        return y

    def inv_T(self, y):
        off = y.ndim - self.d
        for a in range(self.d):
            y = _along(self.V[a].T, y, off + a)
        return y

    def fractional_laplacian(self, x, alpha):
        return self.inv(self.Lam ** (alpha / 2.0) * self.fwd(x))


class SeparableScheme:
    """ETDRK4 (P13 or exponential) on a separable operator, several species."""

    def __init__(self, bc, shape, h, alpha, kappa, tau, scheme="p13", periodic_basis="lapack"):
        self.op = SeparableOperator(bc, shape, h, periodic_basis)
        self.alpha, self.kappa = tuple(alpha), tuple(kappa)
        self.tau, self.scheme = float(tau), scheme
        self.S = len(alpha)
        self.L = [ka * self.tau * self.op.Lam ** (al / 2.0)
                  for al, ka in zip(self.alpha, self.kappa)]
        self.coef = [coefficients.scalar(scheme, L, self.tau) for L in self.L]
        self._dcoef = None

    @property
    def dcoef(self):
        if self._dcoef is None:
            self._dcoef = [coefficients.scalar(self.scheme, L, self.tau, deriv=True)
                           for L in self.L]
        return self._dcoef

    def dL(self, s, which):
        """dL/dkappa_s or dL/dalpha_s per mode (0 where Lambda = 0)."""
        L = self.L[s]
        if which == "kappa":
            return self.tau * self.op.Lam ** (self.alpha[s] / 2.0)
        lnlam = np.log(np.where(self.op.Lam > 0, self.op.Lam, 1.0))
        return 0.5 * L * lnlam

    # ------------------------------------------------------------ forward
    def apply(self, name, X):
        op = self.op
        return np.stack([op.inv(self.coef[s][name] * op.fwd(X[s])) for s in range(self.S)])

    def step(self, U, t, N, record=None):
        tau, G = self.tau, self.apply
        Nu = N(U, t)
        Qu = G("Q", U)
        a = Qu + G("phi", Nu)
        Na = N(a, t + tau / 2)
        b = Qu + G("phi", Na)
        Nb = N(b, t + tau / 2)
        c = G("Q", a) + G("phi", 2.0 * Nb - Nu)
        Nc = N(c, t + tau)
        Un = G("R", U) + G("phi1", Nu) + G("phi2", Na + Nb) + G("phi3", Nc)
        if record is not None:
            record.append(dict(U=U, a=a, b=b, c=c, Nu=Nu, Na=Na, Nb=Nb, Nc=Nc, t=t))
        return Un

    def integrate(self, U, nsteps, N, t0=0.0, record=None):
        U = np.array(U, dtype=np.float64)
        for k in range(nsteps):
            U = self.step(U, t0 + k * self.tau, N, record)
        return U

    # ------------------------------------------------------------ adjoint
    def apply_T(self, name, Y):
        op = self.op
        return np.stack([op.fwd_T(self.coef[s][name] * op.inv_T(Y[s])) for s in range(self.S)])

    def _sens(self, name, Ybar, X, acc):
        """acc[s] += per-mode  (V^T ybar) * g'(L) * (P x)  for y = g(T) x."""
        op = self.op
        for s in range(self.S):
            acc[s] += op.inv_T(Ybar[s]) * self.dcoef[s][name] * op.fwd(X[s])

    def step_adjoint(self, ubar_next, rec, jacT, dparamsN=None, sens=None, pgrad=None):
        """Cotangent of the step input given the cotangent of its output.

        ``rec`` holds the forward stage values of this step. ``jacT(U, G, t)``
        returns J_N(U)^T G; ``dparamsN(U, G, t)`` the reaction-parameter
        partials. ``sens`` (list of per-species mode arrays) accumulates the
        L-sensitivities for kappa/alpha; ``pgrad`` accumulates reaction-parameter
        gradients.
        """
        tau, AT = self.tau, self.apply_T
        U, a, b, c, t = rec["U"], rec["a"], rec["b"], rec["c"], rec["t"]
        ubar = AT("R", ubar_next)
        gu = AT("phi1", ubar_next)
        ga = AT("phi2", ubar_next)
        gb = AT("phi2", ubar_next)
        gc = AT("phi3", ubar_next)
        cbar = jacT(c, gc, t + tau)
        abar = AT("Q", cbar)
        tmp = AT("phi", cbar)
        gb = gb + 2.0 * tmp
        gu = gu - tmp
        bbar = jacT(b, gb, t + tau / 2)
        ubar = ubar + AT("Q", bbar)
        ga = ga + AT("phi", bbar)
        abar = abar + jacT(a, ga, t + tau / 2)
        ubar = ubar + AT("Q", abar)
        gu = gu + AT("phi", abar)
        ubar = ubar + jacT(U, gu, t)
        if sens is not None:
            Nu, Na, Nb, Nc = rec["Nu"], rec["Na"], rec["Nb"], rec["Nc"]
            self._sens("Q", abar, U, sens)
            self._sens("phi", abar, Nu, sens)
            self._sens("Q", bbar, U, sens)
            self._sens("phi", bbar, Na, sens)
            self._sens("Q", cbar, a, sens)
            self._sens("phi", cbar, 2.0 * Nb - Nu, sens)
            self._sens("R", ubar_next, U, sens)
            self._sens("phi1", ubar_next, Nu, sens)
            self._sens("phi2", ubar_next, Na + Nb, sens)
            self._sens("phi3", ubar_next, Nc, sens)
        if pgrad is not None and dparamsN is not None:
            pgrad += dparamsN(c, gc, t + tau)
            pgrad += dparamsN(b, gb, t + tau / 2)
            pgrad += dparamsN(a, ga, t + tau / 2)
            pgrad += dparamsN(U, gu, t)
        return ubar

    def gradients(self, U0, nsteps, N, jacT, dparamsN, grad_uT, t0=0.0, nparams=0):
        """Reverse sweep over a whole trajectory (records every step)."""
        rec = []
        UT = self.integrate(U0, nsteps, N, t0, rec)
        ubar = np.array(grad_uT, dtype=np.float64)
        sens = [np.zeros(self.op.shape) for _ in range(self.S)]
        pgrad = np.zeros(nparams)
        for k in reversed(range(nsteps)):
            ubar = self.step_adjoint(ubar, rec[k], jacT, dparamsN, sens, pgrad)
        gk = np.array([np.sum(sens[s] * self.dL(s, "kappa")) for s in range(self.S)])
        ga = np.array([np.sum(sens[s] * self.dL(s, "alpha")) for s in range(self.S)])
        return dict(uT=UT, u0=ubar, kappa=gk, alpha=ga, params=pgrad)

    # ------------------------------------------------------------ tangent
    def _dapply(self, name, X, s, dtheta):
        """(d g(T_s)/d theta) x for one species, dtheta = dL per mode."""
        op = self.op
        return op.inv(self.dcoef[s][name] * dtheta * op.fwd(X))

    def step_tangent(self, U, dU, t, N, jac, dN_dp=None, dL=None, dp=None):
        """Forward-mode linearisation of one step.

        dU: field tangent; dL: optional list per species of dL (per mode);
        dp: optional parameter tangent with dN_dp(U, t, dp) its effect on N.
        Returns (U_next, dU_next).
        """
        tau, G = self.tau, self.apply

        def dG(name, X, dX):
            out = G(name, dX)
            if dL is not None:
                out = out + np.stack([self._dapply(name, X[s], s, dL[s]) for s in range(self.S)])
            return out

        def dNf(X, dX, tt):
            out = jac(X, dX, tt)
            if dN_dp is not None and dp is not None:
                out = out + dN_dp(X, tt, dp)
            return out

        Nu = N(U, t)
        dNu = dNf(U, dU, t)
        a = G("Q", U) + G("phi", Nu)
        da = dG("Q", U, dU) + dG("phi", Nu, dNu)
        Na = N(a, t + tau / 2)
        dNa = dNf(a, da, t + tau / 2)
        b = G("Q", U) + G("phi", Na)
        db = dG("Q", U, dU) + dG("phi", Na, dNa)
        Nb = N(b, t + tau / 2)
        dNb = dNf(b, db, t + tau / 2)
        c = G("Q", a) + G("phi", 2.0 * Nb - Nu)
        dc = dG("Q", a, da) + dG("phi", 2.0 * Nb - Nu, 2.0 * dNb - dNu)
        Nc = N(c, t + tau)
        dNc = dNf(c, dc, t + tau)
        Un = G("R", U) + G("phi1", Nu) + G("phi2", Na + Nb) + G("phi3", Nc)
        dUn = (dG("R", U, dU) + dG("phi1", Nu, dNu) + dG("phi2", Na + Nb, dNa + dNb)
               + dG("phi3", Nc, dNc))
        return Un, dUn
