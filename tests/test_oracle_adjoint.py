"""Pins of the oracle's discrete adjoint: dot-product test against the
forward-mode tangent, and central finite differences of the discrete map."""
import numpy as np
import pytest

from oracle import reactions
from oracle.separable import SeparableScheme

CASES = [
    ("periodic", (6, 5), "gray_scott", (0.04, 0.06), (0.6, 0.3)),
    ("dirichlet", (5, 6), "schnakenberg", (1.0, 0.1305, 0.7695), (0.9, 0.9)),
    ("neumann", (5, 5), "gierer_meinhardt", (0.1, 1.0, 1.0, 1.0, 1.0), (1.1, 1.2)),
    ("neumann", (4, 3, 5), "fhn", (0.1, 0.01, 0.5, 1.0, 0.0), (0.5, 0.1)),
]
ALPHA, KAPPA, TAU, M = (1.45, 1.75), (0.03, 0.06), 0.15, 3


def _fns(kind, p):
    N = lambda U, t: reactions.f(kind, p, U, t)
    jacT = lambda U, G, t: reactions.jacT(kind, p, U, G)
    jac = lambda U, dU, t: reactions.jac(kind, p, U, dU)
    dparamsN = lambda U, G, t: reactions.dparams(kind, p, U, G)

    def dN_dp(U, t, dp):
        D = reactions.param_partials(kind, p, U)
        return np.stack([sum(dp[k] * D[k][s] for k in range(len(dp))) for s in range(U.shape[0])])
    return N, jacT, jac, dparamsN, dN_dp


def _setup(case, scheme, seed=0):
    bc, shape, kind, p, mean = case
    rng = np.random.default_rng(seed)
    h = tuple(0.25 + 0.03 * i for i in range(len(shape)))
    U0 = np.stack([m + 0.05 * rng.standard_normal(shape) for m in mean])
    sch = SeparableScheme(bc, shape, h, ALPHA, KAPPA, TAU, scheme)
    return sch, U0, rng, h


def _tangent(sch, U0, dU, fns, dL=None, dp=None):
    N, _, jac, _, dN_dp = fns
    U, d = U0, dU
    for k in range(M):
        U, d = sch.step_tangent(U, d, k * TAU, N, jac, dN_dp, dL, dp)
    return d


@pytest.mark.parametrize("scheme", ["p13", "exp"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{len(c[1])}d-{c[2]}")
def test_adjoint_dot_product_and_tangents(case, scheme):
    sch, U0, rng, h = _setup(case, scheme)
    kind, p = case[2], case[3]
    fns = _fns(kind, p)
    N, jacT, jac, dparamsN, dN_dp = fns
    Wbar = rng.standard_normal(U0.shape)
    g = sch.gradients(U0, M, N, jacT, dparamsN, Wbar, nparams=len(p))

    dU = rng.standard_normal(U0.shape)
    lhs = np.sum(_tangent(sch, U0, dU, fns) * Wbar)
    rhs = np.sum(dU * g["u0"])
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)

    zero = np.zeros_like(U0)
    for s in range(2):
        for which, gref in (("kappa", g["kappa"][s]), ("alpha", g["alpha"][s])):
            dL = [np.zeros(sch.op.shape), np.zeros(sch.op.shape)]
            dL[s] = sch.dL(s, which)
            t = np.sum(_tangent(sch, U0, zero, fns, dL=dL) * Wbar)
            assert abs(t - gref) <= 1e-11 * max(abs(t), 1e-3), (which, s, t, gref)
    for k in range(len(p)):
        dp = np.zeros(len(p))
        dp[k] = 1.0
        t = np.sum(_tangent(sch, U0, zero, fns, dp=dp) * Wbar)
        assert abs(t - g["params"][k]) <= 1e-11 * max(abs(t), 1e-3), (k, t, g["params"][k])


@pytest.mark.parametrize("case", [CASES[0], CASES[2]], ids=lambda c: c[0])
def test_adjoint_against_central_differences(case):
    bc, shape, kind, p, mean = case
    sch, U0, rng, h = _setup(case, "p13", seed=5)
    N, jacT, jac, dparamsN, dN_dp = _fns(kind, p)
    Wbar = rng.standard_normal(U0.shape)
    g = sch.gradients(U0, M, N, jacT, dparamsN, Wbar, nparams=len(p))

    def J(U0_=U0, alpha=ALPHA, kappa=KAPPA, params=p):
        s = SeparableScheme(bc, shape, h, alpha, kappa, TAU, "p13")
        UT = s.integrate(U0_, M, lambda U, t: reactions.f(kind, params, U, t))
        return np.sum(UT * Wbar)

    eps = 1e-4
    d = rng.standard_normal(U0.shape)
    fd = (J(U0 + eps * d) - J(U0 - eps * d)) / (2 * eps)
    assert abs(fd - np.sum(d * g["u0"])) <= 1e-6 * max(abs(fd), 1.0)
    for s in range(2):
        for which in ("kappa", "alpha"):
            base = list(KAPPA if which == "kappa" else ALPHA)
            hi, lo = list(base), list(base)
            e = eps * abs(base[s])          # relative step for scalars
            hi[s] += e
            lo[s] -= e
            if which == "kappa":
                fd = (J(kappa=tuple(hi)) - J(kappa=tuple(lo))) / (2 * e)
            else:
                fd = (J(alpha=tuple(hi)) - J(alpha=tuple(lo))) / (2 * e)
            assert abs(fd - g[which][s]) <= 1e-6 * max(abs(fd), 1e-2), (which, s, fd, g[which][s])
    for k in range(len(p)):
        hi, lo = list(p), list(p)
        e = eps * max(abs(p[k]), 1e-2)
        hi[k] += e
        lo[k] -= e
        fd = (J(params=tuple(hi)) - J(params=tuple(lo))) / (2 * e)
        assert abs(fd - g["params"][k]) <= 1e-6 * max(abs(fd), 1e-2), (k, fd, g["params"][k])
