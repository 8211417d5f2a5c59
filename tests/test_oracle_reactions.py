"""Pins of the oracle's reaction terms (oracle/reactions.py) against the model
equations of Section 5.2 (FitzHugh-Nagumo, Gierer-Meinhardt eq. GM,
Gray-Scott eq. SG, Schnakenberg eq. SB) and the linear test equation of
Section 4.2.2.

Two kinds of pin, neither of which re-evaluates the oracle's own formula:

* homogeneous steady states, where every reaction term vanishes exactly
  (found by solving f = 0 by hand for each model);
* one point off equilibrium per model with small rational inputs, where the
  value of the printed equation was worked out by hand as an exact fraction
  (the arithmetic is written in the comment next to each value).

Parameters differ from one another at the off-equilibrium points, so that a
swapped, dropped or sign-flipped term (u^2 written as u, F + K written as K,
sigma_u and sigma_v exchanged) changes the result.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import reactions

TOL = 4e-16  # a few roundings of O(1) quantities


def _f(kind, p, u):
    U = np.array([[float(x)] for x in u], dtype=np.float64)
    return reactions.f(kind, [float(x) for x in p], U)[:, 0]


def _close(got, want):
    want = np.array([float(w) for w in want])
    scale = max(1.0, float(np.max(np.abs(want))))
    assert np.max(np.abs(got - want)) <= TOL * scale, (got, want)


# ---------------------------------------------------------------- steady states
def test_fhn_rest_state():
    # u(1-u)(u-mu) - v = 0 and eps(beta u - gamma v - delta) = 0 at (0, 0)
    # when delta = 0 (the paper's constants mu 0.1, eps 0.01, beta 0.5, gamma 1)
    _close(_f("fhn", (0.1, 0.01, 0.5, 1.0, 0.0), (0.0, 0.0)), (0, 0))


def test_fhn_cubic_roots():
    # with v = 0 the cubic u(1-u)(u-mu) vanishes at u = 0, mu and 1
    for u in (0.0, 0.1, 1.0):
        assert abs(_f("fhn", (0.1, 0.01, 0.5, 1.0, 0.0), (u, 0.0))[0]) <= TOL


def test_gray_scott_trivial_state():
    # (u, v) = (1, 0): -u v^2 + F(1 - u) = 0, u v^2 - (F + K) v = 0
    _close(_f("gray_scott", (0.04, 0.06), (1.0, 0.0)), (0, 0))


def test_schnakenberg_steady_state():
    # gamma(a - u + u^2 v) = 0 = gamma(b - u^2 v) gives u = a + b, v = b/(a+b)^2;
    # the 3D configurations' a = 0.1305, b = 0.7695: (0.9, 0.95)
    a, b = 0.1305, 0.7695
    _close(_f("schnakenberg", (1.0, a, b), (0.9, 0.95)), (0, 0))
    # the application of Section 5.2 (a = 0.1, b = 0.9): (1, 0.9)
    _close(_f("schnakenberg", (1.0, 0.1, 0.9), (1.0, 0.9)), (0, 0))


def test_gierer_meinhardt_steady_states():
    # rho - mu_u u + sigma_u u^2/v = 0 = sigma_v u^2 - mu_v v with
    # (0.1, 1, 1, 1, 1): v = u^2 and 0.1 - u + 1 = 0, so (1.1, 1.21)
    _close(_f("gierer_meinhardt", (0.1, 1.0, 1.0, 1.0, 1.0), (1.1, 1.21)), (0, 0))
    # the paper's form u^2/v - u, u^2/(eps mu) - v/mu: v = u and u^2 = eps v,
    # so u = v = eps, the state the solution approaches in Section 5.2
    eps, mu = 0.04, 0.1
    p = (0.0, 1.0, 1.0, 1.0 / (eps * mu), 1.0 / mu)
    _close(_f("gierer_meinhardt", p, (eps, eps)), (0, 0))


# ---------------------------------------------------------------- off equilibrium
def test_fhn_point():
    # mu 1/10, eps 1/100, beta 1/2, gamma 2, delta 1/40 at (u, v) = (1/2, 1/5):
    # f_u = (1/2)(1/2)(2/5) - 1/5 = 1/10 - 1/5 = -1/10
    # f_v = (1/100)(1/4 - 2/5 - 1/40) = (1/100)(-7/40) = -7/4000
    p = (Fr(1, 10), Fr(1, 100), Fr(1, 2), Fr(2), Fr(1, 40))
    _close(_f("fhn", p, (Fr(1, 2), Fr(1, 5))), (Fr(-1, 10), Fr(-7, 4000)))


def test_gray_scott_point():
    # F 1/25, K 3/50 at (1/2, 1/4):
    # f_u = -(1/2)(1/16) + (1/25)(1/2) = -1/32 + 1/50 = -9/800
    # f_v = 1/32 - (1/10)(1/4) = 1/32 - 1/40 = 1/160
    _close(_f("gray_scott", (Fr(1, 25), Fr(3, 50)), (Fr(1, 2), Fr(1, 4))),
           (Fr(-9, 800), Fr(1, 160)))


def test_schnakenberg_point():
    # gamma 2, a 1/10, b 9/10 at (1/2, 3/2), u^2 v = 3/8:
    # f_u = 2(1/10 - 1/2 + 3/8) = 2(-1/40) = -1/20
    # f_v = 2(9/10 - 3/8) = 2(21/40) = 21/20
    _close(_f("schnakenberg", (Fr(2), Fr(1, 10), Fr(9, 10)), (Fr(1, 2), Fr(3, 2))),
           (Fr(-1, 20), Fr(21, 20)))


def test_gierer_meinhardt_point():
    # rho 1/10, mu_u 2, sigma_u 3, sigma_v 5, mu_v 7 at (1/2, 1/3), u^2/v = 3/4:
    # f_u = 1/10 - 1 + 9/4 = 27/20
    # f_v = 5/4 - 7/3 = -13/12
    p = (Fr(1, 10), Fr(2), Fr(3), Fr(5), Fr(7))
    _close(_f("gierer_meinhardt", p, (Fr(1, 2), Fr(1, 3))), (Fr(27, 20), Fr(-13, 12)))


@pytest.mark.parametrize("S", [1, 2, 3, 4])
def test_linear_is_gamma_u(S):
    # the test equation of Section 4.2.2 per species: f_s = g_s u_s
    g = [Fr(3, 2), Fr(-1, 4), Fr(5), Fr(-2, 3)][:S]
    u = [Fr(2, 3), Fr(4), Fr(1, 5), Fr(-3, 2)][:S]
    want = [Fr(1), Fr(-1), Fr(1), Fr(1)][:S]
    _close(_f("linear", g, u), want)


# ---------------------------------------------------------------- planted slips
def _slipped(kind, p, U):
    """Plausible mistakes in the reaction terms, one per model."""
    u, v = U[0], U[1]
    if kind == "fhn":
        mu, eps, beta, gam, dlt = p
        return np.stack([u * (1 - u) * (mu - u) - v, eps * (beta * u - gam * v - dlt)])
    if kind == "gray_scott":
        F, K = p
        return np.stack([-u * v * v + F * (1 - u), u * v * v - K * v])
    if kind == "schnakenberg":
        g, a, b = p
        return np.stack([g * (a - u + u * v), g * (b - u * u * v)])
    rho, mu_u, s_u, s_v, mu_v = p
    return np.stack([rho - mu_u * u + s_v * u * u / v, s_u * u * u - mu_v * v])


@pytest.mark.parametrize("kind,p,u", [
    ("fhn", (0.1, 0.01, 0.5, 2.0, 0.025), (0.5, 0.2)),
    ("gray_scott", (0.04, 0.06), (0.5, 0.25)),
    ("schnakenberg", (2.0, 0.1, 0.9), (0.5, 1.5)),
    ("gierer_meinhardt", (0.1, 2.0, 3.0, 5.0, 7.0), (0.5, 1.0 / 3.0)),
])
def test_planted_slips_are_caught(kind, p, u, monkeypatch):
    # the off-equilibrium pins reject each slipped variant
    pins = {"fhn": test_fhn_point, "gray_scott": test_gray_scott_point,
            "schnakenberg": test_schnakenberg_point,
            "gierer_meinhardt": test_gierer_meinhardt_point}
    monkeypatch.setattr(reactions, "f", lambda k, pp, U, t=0.0: _slipped(k, pp, U))
    with pytest.raises(AssertionError):
        pins[kind]()
