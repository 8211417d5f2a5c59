"""Pins of the oracle's exact periodic eigenbasis (``periodic_basis="hartley"``).

The periodic compact operator's A and B are circulant (Section 3.1), so
Hartley vectors are exact generalised eigenvectors and the eigenvalues have
the closed form (4/h^2) s^2 / (1 - s^2/3), s = sin(pi k / n). These tests
check the basis against that definition, and the oracle runs on it against
the LAPACK-basis runs where LAPACK is accurate (short axes).
"""
import numpy as np
import pytest

import workloads as W
from oracle import matrices, problem
from oracle.separable import circulant_eig


@pytest.mark.parametrize("n", [8, 12, 33, 1024])
def test_hartley_vectors_are_generalised_eigenvectors(n):
    h = 1.0 / n
    A, B = matrices.ab("periodic", n, h)
    lam, V = circulant_eig(A, B)
    BV, AV = B @ V, A @ V
    assert np.max(np.abs(BV - AV * lam)) <= 1e-13 * np.max(np.abs(BV))
    assert np.max(np.abs(V.T @ AV - np.eye(n))) <= 1e-12


@pytest.mark.parametrize("n", [8, 33, 1024])
def test_hartley_eigenvalues_are_the_closed_form(n):
    h = 2.0 / n
    A, B = matrices.ab("periodic", n, h)
    lam, _ = circulant_eig(A, B)
    s = np.sin(np.pi * np.arange(n) / n)
    closed = 4.0 * s ** 2 / (h ** 2 * (1.0 - s ** 2 / 3.0))
    assert abs(lam[0]) <= 1e-12 * np.max(closed)
    # the Rayleigh quotients of the smallest nonzero eigenvalues carry the
    # rounding of entries of size 1/h^2 (1e-13 relative at n = 1024; LAPACK's
    # generalised solver is off by 9e-12 there)
    assert np.max(np.abs(lam[1:] - closed[1:]) / closed[1:]) <= 5e-13


def test_cosine_vectors_alone_are_not_a_basis():
    # a plausible slip (cos without sin) repeats columns k and n - k
    n = 12
    A, B = matrices.ab("periodic", n, 1.0 / n)
    jk = np.outer(np.arange(n), np.arange(n)) % n
    C = np.cos(2.0 * np.pi * jk / n)
    mu = np.sum(C * (A @ C), axis=0)
    V = C / np.sqrt(mu)
    assert np.max(np.abs(V.T @ A @ V - np.eye(n))) > 0.1


PERIODIC = W.Workload(name="gs2d-per-small", bc="periodic", shape=(10, 12), domain=(-1.0, 1.0),
                      alpha=(1.7, 1.5), kappa=(2e-3, 1e-3), reaction="gray_scott",
                      params=(0.04, 0.06), dt=1.0, nsteps=4, seed=3, init="gs_square")


def test_hartley_and_lapack_bases_agree_on_short_axes():
    u0 = W.initial_fields(PERIODIC)
    a = problem.run(PERIODIC, u0, 4)
    b = problem.run(PERIODIC, u0, 4, periodic_basis="hartley")
    assert problem.rel_err(b, a) <= 1e-13
    wbar = np.random.default_rng(4).standard_normal(u0.shape)
    ga = problem.gradients(PERIODIC, u0, 4, wbar)
    gb = problem.gradients(PERIODIC, u0, 4, wbar, periodic_basis="hartley")
    for key in ("u0", "kappa", "alpha", "params"):
        x, y = np.asarray(gb[key]), np.asarray(ga[key])
        assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(y)), key
