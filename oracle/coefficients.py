"""Time-stepping coefficients (Section 4).

Two schemes share the same four-stage structure (eq. ETDRK4P13):

    a = Q u + phi f(u, t)
    b = Q u + phi f(a, t + tau/2)
    c = Q a + phi (2 f(b, t + tau/2) - f(u, t))
    u' = R u + phi1 f(u, t) + phi2 (f(a) + f(b)) + phi3 f(c, t + tau)

* ``p13``: the paper's ETDRK4-P13. With L = tau * (linear operator) the six
  coefficients are the rational functions of the Alg. 1 precompute,
  R = R13(L), Q = R13(L/2) (written out as 24(8-L)/(192+72L+12L^2+L^3)),
  phi, phi1, phi2, phi3.
* ``exp``: the exact-exponential ETDRK4 of Cox and Matthews (2002): R = e^-L,
  Q = e^-L/2, phi = tau(1 - e^-L/2)/L and phi1, phi2, phi3 equal to their
  f1, 2 f2, f3 evaluated at z = -L.

Scalar forms take an FP64 numpy array of L >= 0. The exponential scheme is
evaluated from its definition in mpmath at enough digits to absorb the
cancellation near L = 0; matrix forms use dense solves (P13) and scipy's
``expm`` of the augmented block matrix for the phi-functions (EXP).
"""
from __future__ import annotations

import functools

import mpmath
import numpy as np
import scipy.linalg

NAMES = ("R", "Q", "phi", "phi1", "phi2", "phi3")

# ---------------------------------------------------------------- P13 (scalar)
# Each entry: (numerator coefficients in L, denominator coefficients in L,
# power of tau in front). Coefficients are lowest order first, as printed in
# Alg. 1 of Section 4.1.
_D = (24.0, 18.0, 6.0, 1.0)
_DH = (192.0, 72.0, 12.0, 1.0)
P13_RATIONAL = {
    "R": ((24.0, -6.0), _D, 0),
    "Q": ((192.0, -24.0), _DH, 0),
    "phi": ((96.0, 12.0, 1.0), _DH, 1),
    "phi1": ((4.0, -1.0), _D, 1),
    "phi2": ((8.0, 2.0), _D, 1),
    "phi3": ((4.0, 3.0, 1.0), _D, 1),
}


def _poly(c, L):
    out = np.zeros_like(L)
    for k in reversed(range(len(c))):
        out = out * L + c[k]
    return out


def _dpoly(c, L):
    out = np.zeros_like(L)
    for k in reversed(range(1, len(c))):
        out = out * L + k * c[k]
    return out


def p13(L, tau):
    """Dict of the six P13 coefficient arrays at L (FP64)."""
    L = np.asarray(L, dtype=np.float64)
    out = {}
    for name, (num, den, tp) in P13_RATIONAL.items():
        out[name] = tau ** tp * _poly(num, L) / _poly(den, L)
    return out


def p13_dL(L, tau):
    """Derivatives d/dL of the six P13 coefficients (quotient rule)."""
    L = np.asarray(L, dtype=np.float64)
    out = {}
    for name, (num, den, tp) in P13_RATIONAL.items():
        n, dn = _poly(num, L), _dpoly(num, L)
        d, dd = _poly(den, L), _dpoly(den, L)
        out[name] = tau ** tp * (dn * d - n * dd) / (d * d)
    return out


# ---------------------------------------------------------------- EXP (scalar)
def _exp_mp(L, tau):
    """The six exponential-scheme coefficients at one L, from their definitions."""
    L = mpmath.mpf(L)
    tau = mpmath.mpf(tau)
    if L == 0:
        return {"R": mpmath.mpf(1), "Q": mpmath.mpf(1), "phi": tau / 2,
                "phi1": tau / 6, "phi2": tau / 3, "phi3": tau / 6}
    z = -L
    ez = mpmath.exp(z)
    return {
        "R": ez,
        "Q": mpmath.exp(z / 2),
        "phi": tau * (1 - mpmath.exp(z / 2)) / L,
        "phi1": tau * (-4 - z + ez * (4 - 3 * z + z * z)) / z ** 3,
        "phi2": 2 * tau * (2 + z + ez * (z - 2)) / z ** 3,
        "phi3": tau * (-4 - 3 * z - z * z + ez * (4 - z)) / z ** 3,
    }


def _digits_for(L: float) -> int:
    # The z^-3 formulas cancel about 3*log10(1/L) digits for small L.
    if L <= 0:
        return 40
    return 40 + int(max(0.0, -3.0 * np.log10(L))) + 5


@functools.lru_cache(maxsize=1 << 20)
def _exp_cached(L: float, tau: float, deriv: bool):
    with mpmath.workdps(_digits_for(L)):
        if not deriv:
            v = _exp_mp(L, tau)
            return tuple(float(v[k]) for k in NAMES)
        if L == 0.0:
            # Linear Taylor terms at L = 0, from phi_k(z) = sum_j z^j/(j+k)!
            # with z = -L: e^-L -> -1, e^-L/2 -> -1/2, tau(1-e^-L/2)/L -> -tau/8,
            # tau(phi1-3phi2+4phi3) -> -tau/6, 2tau(phi2-2phi3) -> -tau/6,
            # tau(-phi2+4phi3) -> 0.
            return (-1.0, -0.5, -tau / 8.0, -tau / 6.0, -tau / 6.0, 0.0)
        out = []
        for k in NAMES:
            f = (lambda x, k=k: _exp_mp(x, tau)[k])
            out.append(float(mpmath.diff(f, mpmath.mpf(L))))
        return tuple(out)


def exp_scheme(L, tau, deriv=False):
    """Dict of the six exponential-scheme coefficients (or their d/dL)."""
    L = np.asarray(L, dtype=np.float64)
    flat = L.ravel()
    uniq, inv = np.unique(flat, return_inverse=True)
    vals = np.array([_exp_cached(float(x), float(tau), bool(deriv)) for x in uniq])
    return {k: vals[inv, i].reshape(L.shape) for i, k in enumerate(NAMES)}


def scalar(scheme: str, L, tau, deriv=False):
    if scheme == "p13":
        return p13_dL(L, tau) if deriv else p13(L, tau)
    if scheme == "exp":
        return exp_scheme(L, tau, deriv)
    raise ValueError(scheme)


# ---------------------------------------------------------------- matrix forms
def matrix_p13(tA: np.ndarray, tau: float):
    """P13 coefficient matrices of the matrix tA = tau * A (Section 4):
    each is numerator(tA) times denominator(tA)^-1, computed by a dense solve
    (numerator and denominator are polynomials in tA and commute)."""
    n = tA.shape[0]
    I = np.eye(n)
    powers = [I, tA, tA @ tA, tA @ tA @ tA]
    out = {}
    for name, (num, den, tp) in P13_RATIONAL.items():
        N = sum(c * powers[k] for k, c in enumerate(num))
        D = sum(c * powers[k] for k, c in enumerate(den))
        out[name] = tau ** tp * np.linalg.solve(D, N)
    return out


def phi_functions(Z: np.ndarray, kmax: int = 3):
    """phi_1..phi_kmax of the matrix Z from one expm of the augmented block
    matrix [[Z, I, 0..], [0, 0, I, ..], ..] (Saad 1992; Sidje 1998)."""
    n = Z.shape[0]
    big = np.zeros(((kmax + 1) * n, (kmax + 1) * n))
    big[:n, :n] = Z
    for k in range(kmax):
        big[k * n:(k + 1) * n, (k + 1) * n:(k + 2) * n] = np.eye(n)
    E = scipy.linalg.expm(big)
    return [E[:n, :n]] + [E[:n, (k + 1) * n:(k + 2) * n] for k in range(kmax)]


def matrix_exp(tA: np.ndarray, tau: float):
    """Exponential-scheme coefficient matrices of tA = tau * A."""
    Z = -tA
    e, p1, p2, p3 = phi_functions(Z, 3)
    eh, p1h = phi_functions(Z / 2.0, 1)
    return {
        "R": e,
        "Q": eh,
        "phi": 0.5 * tau * p1h,
        "phi1": tau * (p1 - 3.0 * p2 + 4.0 * p3),
        "phi2": 2.0 * tau * (p2 - 2.0 * p3),
        "phi3": tau * (-p2 + 4.0 * p3),
    }


def matrix(scheme: str, tA, tau):
    if scheme == "p13":
        return matrix_p13(tA, tau)
    if scheme == "exp":
        return matrix_exp(tA, tau)
    raise ValueError(scheme)
