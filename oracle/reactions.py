"""Reaction terms of the pattern models in Section 5.2, with Jacobians.

Every function takes the species fields ``U`` shaped ``[S, ...]`` (FP64) and
returns arrays of the same shape. ``jacT(kind, p, U, G)`` returns J(U)^T G
point by point (out_r = sum_s G_s d f_s / d u_r) and ``dparams`` returns the
list over parameters of sum_x sum_s G_s d f_s / d p (optionally weighted per
point).

Parameter vectors:

* linear            (g_0, .., g_{S-1})      f_s = g_s u_s (the test equation of
                                            Section 4.2.2 per species)
* fhn               (mu, eps, beta, gamma, delta)
                    f_u = u(1-u)(u-mu) - v,  f_v = eps(beta u - gamma v - delta)
* gray_scott        (F, K)
                    f_u = -u v^2 + F(1-u),   f_v = u v^2 - (F+K) v
* schnakenberg      (gamma, a, b)
                    f_u = gamma(a - u + u^2 v),  f_v = gamma(b - u^2 v)
* gierer_meinhardt  (rho, mu_u, sigma_u, sigma_v, mu_v)
                    f_u = rho - mu_u u + sigma_u u^2/v,  f_v = sigma_v u^2 - mu_v v
                    (the paper's form is rho = 0, mu_u = 1, sigma_u = 1,
                    sigma_v = 1/(eps mu), mu_v = 1/mu)
"""
from __future__ import annotations

import numpy as np

NPARAMS = {"fhn": 5, "gray_scott": 2, "schnakenberg": 3, "gierer_meinhardt": 5}


def nparams(kind: str, nspecies: int) -> int:
    return nspecies if kind == "linear" else NPARAMS[kind]


def f(kind, p, U, t=0.0):
    if kind == "linear":
        return np.stack([p[s] * U[s] for s in range(U.shape[0])])
    u, v = U[0], U[1]
    if kind == "fhn":
        mu, eps, beta, gam, dlt = p
        return np.stack([u * (1 - u) * (u - mu) - v, eps * (beta * u - gam * v - dlt)])
    if kind == "gray_scott":
        F, K = p
        return np.stack([-u * v * v + F * (1 - u), u * v * v - (F + K) * v])
    if kind == "schnakenberg":
        g, a, b = p
        return np.stack([g * (a - u + u * u * v), g * (b - u * u * v)])
    if kind == "gierer_meinhardt":
        rho, mu_u, s_u, s_v, mu_v = p
        return np.stack([rho - mu_u * u + s_u * u * u / v, s_v * u * u - mu_v * v])
    raise ValueError(kind)


def jacobian(kind, p, U):
    """J[s][r] = d f_s / d u_r, each an array shaped like one field."""
    if kind == "linear":
        S = U.shape[0]
        z = np.zeros_like(U[0])
        return [[(p[s] * np.ones_like(U[0]) if r == s else z) for r in range(S)]
                for s in range(S)]
    u, v = U[0], U[1]
    if kind == "fhn":
        mu, eps, beta, gam, dlt = p
        # d/du [u(1-u)(u-mu)] = -3u^2 + 2(1+mu)u - mu
        return [[-3 * u * u + 2 * (1 + mu) * u - mu, -np.ones_like(u)],
                [eps * beta * np.ones_like(u), -eps * gam * np.ones_like(u)]]
    if kind == "gray_scott":
        F, K = p
        return [[-v * v - F, -2 * u * v], [v * v, 2 * u * v - (F + K)]]
    if kind == "schnakenberg":
        g, a, b = p
        return [[g * (-1 + 2 * u * v), g * u * u], [g * (-2 * u * v), g * (-u * u)]]
    if kind == "gierer_meinhardt":
        rho, mu_u, s_u, s_v, mu_v = p
        return [[-mu_u + 2 * s_u * u / v, -s_u * u * u / (v * v)],
                [2 * s_v * u, -mu_v * np.ones_like(u)]]
    raise ValueError(kind)


def jacT(kind, p, U, G):
    J = jacobian(kind, p, U)
    S = U.shape[0]
    return np.stack([sum(G[s] * J[s][r] for s in range(S)) for r in range(S)])


def jac(kind, p, U, dU):
    J = jacobian(kind, p, U)
    S = U.shape[0]
    return np.stack([sum(J[s][r] * dU[r] for r in range(S)) for s in range(S)])


def param_partials(kind, p, U):
    """D[k][s] = d f_s / d p_k, each an array shaped like one field."""
    S = U.shape[0]
    z = np.zeros_like(U[0])
    one = np.ones_like(U[0])
    if kind == "linear":
        return [[U[s] if s == k else z for s in range(S)] for k in range(S)]
    u, v = U[0], U[1]
    if kind == "fhn":
        mu, eps, beta, gam, dlt = p
        return [[-u * (1 - u), z],
                [z, beta * u - gam * v - dlt],
                [z, eps * u],
                [z, -eps * v],
                [z, -eps * one]]
    if kind == "gray_scott":
        # f_u = -u v^2 + F(1-u), f_v = u v^2 - (F+K) v
        return [[1 - u, -v], [z, -v]]
    if kind == "schnakenberg":
        g, a, b = p
        return [[a - u + u * u * v, b - u * u * v], [g * one, z], [z, g * one]]
    if kind == "gierer_meinhardt":
        return [[one, z], [-u, z], [u * u / v, z], [z, u * u], [z, -v]]
    raise ValueError(kind)


def dparams(kind, p, U, G, w=None):
    D = param_partials(kind, p, U)
    out = []
    for Dk in D:
        tot = sum(G[s] * Dk[s] for s in range(U.shape[0]))
        if w is not None:
            tot = tot * w
        out.append(float(np.sum(tot)))
    return np.array(out)
