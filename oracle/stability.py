"""Linear stability of the time stepping (Section 4.2.2) — test infrastructure
(only tests/, the smoke check and the benchmark's CPU baseline use the
oracle; the library never does).

Linearising u_t + c u = f(u) about a fixed point gives the test equation
u_t + c u = gamma u. With y = -c tau and x = gamma tau, one step of the
four-stage scheme (eq. ETDRK4P13, the same stages for both coefficient
schemes) multiplies u by the amplification factor r(x, y) (eq. Eq41), a
quartic in x whose coefficients depend on y. The stability boundary for a
fixed real y is the set of complex x with |r(x, y)| = 1: the roots of
r(x, y) = e^{i theta} for theta in [0, 2 pi).

Here r is obtained by running the stages themselves on the scalar equation
(tau = 1, L = c tau = -y, f(u) = x u), with the coefficients of
``coefficients.scalar`` — not from the printed closed forms, which the tests
use as an independent check.
"""
from __future__ import annotations

import numpy as np

from . import coefficients


def _coefs(scheme: str, y: float):
    if not y <= 0.0:
        raise ValueError("y = -c tau must be <= 0")
    co = coefficients.scalar(scheme, np.array([-float(y)]), 1.0)
    return [float(co[k][0]) for k in coefficients.NAMES]


def _step(R, Q, phi, phi1, phi2, phi3, one, f):
    """One step of the four stages from u = one with reaction f (linear)."""
    fu = f(one)
    a = Q * one + phi * fu
    fa = f(a)
    b = Q * one + phi * fa
    fb = f(b)
    c = Q * a + phi * (2 * fb - fu)
    fc = f(c)
    return R * one + phi1 * fu + phi2 * (fa + fb) + phi3 * fc


def amplification(scheme: str, x, y: float):
    """r(x, y) for complex x (scalar or array) at one real y <= 0."""
    x = np.asarray(x, dtype=np.complex128)
    return _step(*_coefs(scheme, y), np.ones_like(x), lambda v: x * v)


def amplification_poly(scheme: str, y: float) -> np.ndarray:
    """c_0..c_4 with r(x, y) = sum_k c_k x^k: the same stages on polynomials in x."""
    P = np.polynomial.Polynomial
    X = P([0.0, 1.0])
    r = _step(*_coefs(scheme, y), P([1.0]), lambda v: X * v)
    out = np.zeros(5)
    out[: len(r.coef)] = r.coef
    return out


def boundary(scheme: str, y: float, ntheta: int) -> np.ndarray:
    """[ntheta, 4] complex: the x with r(x, y) = e^{i theta_k},
    theta_k = 2 pi k / ntheta (roots of the quartic, numpy.roots)."""
    c = amplification_poly(scheme, y)
    out = np.empty((ntheta, 4), dtype=np.complex128)
    for k in range(ntheta):
        rhs = np.exp(2j * np.pi * k / ntheta)
        q = c.astype(np.complex128)
        q[0] -= rhs
        out[k] = np.roots(q[::-1])
    return out
