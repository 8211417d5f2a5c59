"""Manufactured-solution problems of Section 5.1 (Examples 1 and 2).

Example 1 (1D fractional Fisher with a source, homogeneous Dirichlet on
[0, 1]): exact u = e^-t sin^3(2 pi x). With sin^3 = (3 sin - sin 3.)/4 and the
Dirichlet eigenfunctions sin(2 pi x), sin(6 pi x) of -Delta, the source that
makes it exact is

    -2 e^-t sin^3(2 pi x) + (kappa/4) e^-t (3 (2pi)^a sin(2 pi x) - (6pi)^a sin(6 pi x))
    + e^-2t sin^6(2 pi x),

to which the reaction u - u^2 is added. (The printed source repeats kappa;
one factor kappa/4 is what makes e^-t sin^3 exact.)

Example 2 (2D fractional Huxley with a source on [0, 1]^2, periodic or
homogeneous Neumann): exact u = t^a C(x) C(y), C = cos^3(2 pi .), u(.,0) = 0,
reaction u(1-u)(u-1) plus the source

    a t^(a-1) CC + t^a Phi - t^a CC (1 - t^a CC)(t^a CC - 1),
    Phi = (kappa/16)(9 (8pi^2)^(a/2) c1x c1y + 3 (40pi^2)^(a/2) (c3x c1y + c1x c3y)
                     + (72pi^2)^(a/2) c3x c3y),

with c1 = cos(2 pi .), c3 = cos(6 pi .): Phi is kappa (-Delta)^(a/2) CC. (The
printed third term reads (40 pi)^(a/2); by symmetry with the second term and
the eigenvalue (6pi)^2 + (2pi)^2 it is (40 pi^2)^(a/2).)

The error is the max-norm against the exact solution at the final time
(Section 5) and the order is log2(E_h / E_{h/2}).
"""
from __future__ import annotations

import numpy as np

from .separable import SeparableScheme


def example1(N: int, alpha: float, kappa: float, tau: float, T: float):
    """Solve Example 1 with N intervals; returns (max error at T, steps)."""
    U, exact, M = example1_fields(N, alpha, kappa, tau, T)
    return float(np.max(np.abs(U - exact))), M


def example1_fields(N: int, alpha: float, kappa: float, tau: float, T: float):
    """Example 1 with N intervals: (computed u at T, exact u at T, steps), on
    the N - 1 interior nodes."""
    h = 1.0 / N
    x = np.arange(1, N) * h
    s1 = np.sin(2 * np.pi * x)
    s3 = np.sin(6 * np.pi * x)

    def Nfun(U, t):
        u = U[0]
        src = (-2 * np.exp(-t) * s1 ** 3
               + kappa / 4 * np.exp(-t) * (3 * (2 * np.pi) ** alpha * s1 - (6 * np.pi) ** alpha * s3)
               + np.exp(-2 * t) * s1 ** 6)
        return (src + u - u * u)[None]

    M = int(round(T / tau))
    sch = SeparableScheme("dirichlet", (N - 1,), (h,), (alpha,), (kappa,), tau)
    U = sch.integrate((s1 ** 3)[None], M, Nfun)
    exact = np.exp(-M * tau) * s1 ** 3
    return U[0], exact, M


def example2(bc: str, inv_h: int, alpha: float, kappa: float = 1.0, T: float = 1.0,
             tau_over_h: float = 0.1):
    """Solve Example 2; returns (max error at T, steps)."""
    U, exact, M = example2_fields(bc, inv_h, alpha, kappa, T, tau_over_h)
    return float(np.max(np.abs(U - exact))), M


def example2_fields(bc: str, inv_h: int, alpha: float, kappa: float = 1.0, T: float = 1.0,
                    tau_over_h: float = 0.1):
    """Example 2: (computed u at T, exact u at T, steps), indexed [y, x] over
    the nodes x_j = j h."""
    h = 1.0 / inv_h
    n = inv_h if bc == "periodic" else inv_h + 1
    x = np.arange(n) * h
    c1, c3 = np.cos(2 * np.pi * x), np.cos(6 * np.pi * x)
    C = c1 ** 3
    CC = np.outer(C, C)
    a2 = alpha / 2.0
    Phi = kappa / 16.0 * (9 * (8 * np.pi ** 2) ** a2 * np.outer(c1, c1)
                          + 3 * (40 * np.pi ** 2) ** a2 * (np.outer(c1, c3) + np.outer(c3, c1))
                          + (72 * np.pi ** 2) ** a2 * np.outer(c3, c3))

    def Nfun(U, t):
        u = U[0]
        ta = t ** alpha
        dta = alpha * t ** (alpha - 1.0) if t > 0 else 0.0
        src = dta * CC + ta * Phi - ta * CC * (1 - ta * CC) * (ta * CC - 1)
        return (u * (1 - u) * (u - 1) + src)[None]

    tau = tau_over_h * h
    M = int(round(T / tau))
    sch = SeparableScheme(bc, (n, n), (h, h), (alpha,), (kappa,), tau)
    U = sch.integrate(np.zeros((1, n, n)), M, Nfun)
    exact = (M * tau) ** alpha * CC
    return U[0], exact, M
