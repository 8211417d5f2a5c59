"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: printed
values (tests/golden), closed forms, textbook special cases, identities
between independently computed objects, or brute force.
"""
import os

import mpmath
import numpy as np
import pytest

from oracle import coefficients as co
from oracle import matrices
from oracle.dense import DenseOperator
from oracle.examples import example1, example2
from oracle.separable import SeparableOperator, SeparableScheme
from oracle import reactions

GOLD = os.path.join(os.path.dirname(__file__), "golden")
BCS = ("periodic", "dirichlet", "neumann")


def _closed_form(bc, n, h):
    """Eigenvalues printed in Section 3.1: 4 s^2 / (h^2 (1 - s^2/3))."""
    if bc == "periodic":
        N = n
        s = np.sin(np.arange(N) * np.pi / N)           # sin(k pi / N), k = 0..N-1
    elif bc == "dirichlet":
        N = n + 1
        s = np.sin(np.arange(1, N) * np.pi / (2 * N))  # k = 1..N-1
    else:
        N = n - 1
        s = np.sin(np.arange(0, N + 1) * np.pi / (2 * N))  # k = 0..N
    return np.sort(4 * s * s / (h * h * (1 - s * s / 3)))


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [2, 3, 8, 17, 64])
def test_eigenvalues_match_closed_form(bc, n):
    h = 0.37 / max(n - 1, 1)
    op = SeparableOperator(bc, (n,), (h,))
    lam = np.sort(op.lam[0])
    ref = _closed_form(bc, n, h)
    assert np.max(np.abs(lam - ref)) <= 1e-12 * np.max(ref)


def test_printed_periodic_index_is_not_the_spectrum():
    # The periodic eigenvalue is printed with sin^2((n-1) pi / 2N); the
    # spectrum of the printed circulant A^-1 B is sin^2(k pi / N).
    n, h = 16, 0.1
    lam = np.sort(SeparableOperator("periodic", (n,), (h,)).lam[0])
    s = np.sin(np.arange(n) * np.pi / (2 * n))
    printed = np.sort(4 * s * s / (h * h * (1 - s * s / 3)))
    assert np.max(np.abs(lam - printed)) > 1e-3 * np.max(lam)


@pytest.mark.parametrize("bc", BCS)
def test_alpha2_is_compact_laplacian_2d(bc):
    # alpha = 2: T^1 x must be A^-1 B applied along each axis and summed
    # (eq. Lap in 2D), computed here by plain dense solves.
    rng = np.random.default_rng(0)
    shape, h = (7, 9), (0.11, 0.13)
    x = rng.standard_normal(shape)
    op = SeparableOperator(bc, shape, h)
    got = op.fractional_laplacian(x, 2.0)
    Ay, By = matrices.ab(bc, shape[0], h[0])
    Ax, Bx = matrices.ab(bc, shape[1], h[1])
    ref = np.linalg.solve(Ay, By @ x) + np.linalg.solve(Ax, (Bx @ x.T)).T
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("alpha", [1.2, 1.7])
def test_dense_and_separable_fractional_operator_agree(bc, alpha):
    rng = np.random.default_rng(1)
    shape, h = (5, 6), (0.2, 0.15)
    x = rng.standard_normal(shape)
    o1 = DenseOperator(bc, shape, h, (alpha,), (1.0,), 0.1)
    o2 = SeparableOperator(bc, shape, h)
    a, b = o1.fractional_laplacian(x, alpha), o2.fractional_laplacian(x, alpha)
    assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(b))


@pytest.mark.parametrize("alpha", [1.3, 2.0])
def test_neumann_and_dirichlet_are_periodic_on_the_extension(alpha):
    # The Neumann operator on n = N+1 nodes equals the periodic operator on
    # the even extension of length 2N; the Dirichlet one on n = N-1 nodes the
    # periodic operator on the odd extension (with zeros at 0 and N).
    rng = np.random.default_rng(2)
    N, h = 10, 0.1
    per = SeparableOperator("periodic", (2 * N, 2 * N), (h, h))
    neu = SeparableOperator("neumann", (N + 1, N + 1), (h, h))
    x = rng.standard_normal((N + 1, N + 1))
    ext = np.zeros((2 * N, 2 * N))
    idx = np.r_[np.arange(N + 1), np.arange(N - 1, 0, -1)]
    ext[:, :] = x[np.ix_(idx, idx)]
    ref = per.fractional_laplacian(ext, alpha)[:N + 1, :N + 1]
    got = neu.fractional_laplacian(x, alpha)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))

    dir_ = SeparableOperator("dirichlet", (N - 1, N - 1), (h, h))
    y = rng.standard_normal((N - 1, N - 1))
    ext = np.zeros((2 * N, 2 * N))
    sgn = np.r_[0, np.ones(N - 1), 0, -np.ones(N - 1)]
    src = np.r_[0, np.arange(N - 1), 0, np.arange(N - 2, -1, -1)]
    for i in range(2 * N):
        for j in range(2 * N):
            if sgn[i] and sgn[j]:
                ext[i, j] = sgn[i] * sgn[j] * y[src[i], src[j]]
    ref = per.fractional_laplacian(ext, alpha)[1:N, 1:N]
    got = dir_.fractional_laplacian(y, alpha)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


# ------------------------------------------------------------------ coefficients
def test_p13_pade_error_term():
    # R13 is the (1,3) Pade approximant: R13(L) - e^-L = -L^5/480 + O(L^6).
    for L in (0.02, 0.05):
        r = co.p13(np.array([L]), 1.0)["R"][0]
        ratio = (r - np.exp(-L)) / (-L ** 5 / 480.0)
        assert abs(ratio - 1.0) < 3 * L


def test_p13_structure():
    tau = 0.37
    L = np.array([0.0, 1e-6, 0.3, 1.0, 4.0, 7.5, 60.0, 1e4])
    c = co.p13(L, tau)
    half = co.p13(L / 2.0, tau)
    assert np.allclose(c["Q"], half["R"], rtol=1e-15, atol=0)
    nz = L > 0
    assert np.allclose(c["phi"][nz], tau * (1.0 - c["Q"][nz]) / L[nz], rtol=1e-9, atol=0)
    z = co.p13(np.array([0.0]), tau)
    for k, v in zip(co.NAMES, (1.0, 1.0, tau / 2, tau / 6, tau / 3, tau / 6)):
        assert abs(z[k][0] - v) <= 1e-15


def test_p13_equals_cox_matthews_with_pade_exponential():
    # ETDRK4-P13 is the Cox-Matthews ETDRK4 with e^-L replaced by R13(L) and
    # e^-L/2 by R13(L/2); evaluate the Cox-Matthews formulas at 50 digits.
    tau = 0.8
    mpmath.mp.dps = 50
    for L in (1e-3, 0.25, 1.0, 3.0, 11.0, 250.0):
        Lm = mpmath.mpf(L)
        R = (24 - 6 * Lm) / (24 + 18 * Lm + 6 * Lm ** 2 + Lm ** 3)
        Rh = (24 - 3 * Lm) / (24 + 9 * Lm + 1.5 * Lm ** 2 + Lm ** 3 / 8)
        z = -Lm
        cm = {"R": R, "Q": Rh, "phi": tau * (1 - Rh) / Lm,
              "phi1": tau * (-4 - z + R * (4 - 3 * z + z * z)) / z ** 3,
              "phi2": 2 * tau * (2 + z + R * (z - 2)) / z ** 3,
              "phi3": tau * (-4 - 3 * z - z * z + R * (4 - z)) / z ** 3}
        got = co.p13(np.array([L]), tau)
        for k in co.NAMES:
            ref = float(cm[k])
            assert abs(got[k][0] - ref) <= 1e-13 * max(abs(ref), 1e-300), (L, k)
    mpmath.mp.dps = 15


@pytest.mark.parametrize("scheme", ["p13", "exp"])
def test_coefficient_derivatives_by_finite_differences(scheme):
    tau = 0.3
    for L in (0.0, 1e-5, 0.4, 2.5, 30.0):
        d = co.scalar(scheme, np.array([L]), tau, deriv=True)
        eps = 1e-6 * max(L, 1.0)
        if L == 0.0:
            p = co.scalar(scheme, np.array([eps]), tau)
            m = co.scalar(scheme, np.array([0.0]), tau)
            fd = {k: (p[k][0] - m[k][0]) / eps for k in co.NAMES}
            tol = 1e-5
        else:
            p = co.scalar(scheme, np.array([L + eps]), tau)
            m = co.scalar(scheme, np.array([L - eps]), tau)
            fd = {k: (p[k][0] - m[k][0]) / (2 * eps) for k in co.NAMES}
            tol = 1e-7
        for k in co.NAMES:
            assert abs(d[k][0] - fd[k]) <= tol * max(1.0, abs(fd[k])), (scheme, L, k)


def test_exponential_coefficients_match_augmented_expm():
    # The mpmath definitions agree with phi-functions from one expm of the
    # augmented block matrix (an independent evaluation route).
    tau = 0.5
    for L in (0.0, 1e-9, 1e-4, 0.1, 1.0, 5.0, 40.0):
        ref = co.matrix_exp(np.array([[tau * (L / tau)]]), tau)
        got = co.exp_scheme(np.array([L]), tau)
        for k in co.NAMES:
            r = ref[k][0, 0]
            assert abs(got[k][0] - r) <= 1e-12 * max(abs(r), 1e-300), (L, k)


def test_exponential_scheme_small_L_limits():
    tau = 1.0
    got = co.exp_scheme(np.array([0.0, 1e-12]), tau)
    for k, v in zip(co.NAMES, (1.0, 1.0, 0.5, 1 / 6, 1 / 3, 1 / 6)):
        assert abs(got[k][0] - v) < 1e-15 and abs(got[k][1] - v) < 1e-11


# ------------------------------------------------------------------ stepping
def _N(kind, p):
    return lambda U, t: reactions.f(kind, p, U, t)


CASES = [
    ("periodic", (5, 6), "gray_scott", (0.04, 0.06), (0.6, 0.3)),
    ("dirichlet", (4, 5), "schnakenberg", (1.0, 0.1305, 0.7695), (0.9, 0.9)),
    ("neumann", (5, 4), "gierer_meinhardt", (0.1, 1.0, 1.0, 1.0, 1.0), (1.1, 1.2)),
    ("neumann", (3, 4, 3), "fhn", (0.1, 0.01, 0.5, 1.0, 0.0), (0.5, 0.1)),
    ("periodic", (4, 3, 4), "schnakenberg", (1.0, 0.1305, 0.7695), (0.9, 0.9)),
    ("dirichlet", (3, 3, 4), "gray_scott", (0.04, 0.06), (0.6, 0.3)),
]


@pytest.mark.parametrize("scheme", ["p13", "exp"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{len(c[1])}d-{c[2]}")
def test_dense_O1_matches_separable_O2(case, scheme):
    bc, shape, kind, p, mean = case
    rng = np.random.default_rng(3)
    h = tuple(0.3 + 0.05 * i for i in range(len(shape)))
    U0 = np.stack([m + 0.05 * rng.standard_normal(shape) for m in mean])
    alpha, kappa, tau = (1.4, 1.8), (0.02, 0.05), 0.2
    o1 = DenseOperator(bc, shape, h, alpha, kappa, tau, scheme)
    o2 = SeparableScheme(bc, shape, h, alpha, kappa, tau, scheme)
    a = o1.integrate(U0, 6, _N(kind, p))
    b = o2.integrate(U0, 6, _N(kind, p))
    assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(b))


def _paper_r(x, y, printed_c1=False):
    """Amplification factor r(x, y) of Section 4.2.2 (eq. 41)."""
    D = 24 - 18 * y + 6 * y ** 2 - y ** 3
    Dh = 192 - 72 * y + 12 * y ** 2 - y ** 3
    c0 = 6 * (4 + y) / D
    num1 = (169869312 - 148635648 * y - 9621504 * y ** 3 + 470016 * y ** 4 + 165888 * y ** 5
            - 46464 * y ** 6 + 6240 * y ** 7 - 600 * y ** 8 + 32 * y ** 9 - y ** 10)
    if not printed_c1:
        num1 = num1 + 55738368 * y ** 2
    c1 = num1 / (Dh ** 3 * D)
    c2 = (442368 - 221184 * y + 34560 * y ** 2 + 11712 * y ** 3 - 2976 * y ** 4 + 404 * y ** 5
          - 25 * y ** 6 + y ** 7) / (Dh ** 2 * D)
    c3 = 2 * (96 - 12 * y + y ** 2) ** 2 * (1536 - 960 * y + 240 * y ** 2 + 8 * y ** 3 + y ** 4) / (Dh ** 3 * D)
    c4 = 2 * (96 - 12 * y + y ** 2) ** 3 * (4 - 3 * y + y ** 2) / (Dh ** 3 * D)
    return c0 + c1 * x + c2 * x ** 2 + c3 * x ** 3 + c4 * x ** 4


def _mode(bc, n, k):
    j = np.arange(n)
    if bc == "periodic":
        return np.cos(2 * np.pi * k * j / n), np.sin(np.pi * k / n)
    if bc == "dirichlet":
        N = n + 1
        return np.sin(np.pi * (j + 1) * k / N), np.sin(np.pi * k / (2 * N))
    N = n - 1
    return np.cos(np.pi * j * k / N), np.sin(np.pi * k / (2 * N))


@pytest.mark.parametrize("bc", BCS)
def test_single_eigenmode_amplification(bc):
    # Linear test equation per mode (Section 4.2.2): one step multiplies an
    # eigenmode by r(gamma tau, -L) with the closed-form c0..c4 (c1 with the
    # y^2 term the printed numerator lacks).
    ny, nx, h, tau, kappa, alpha = 6, 7, 0.08, 0.05, 0.3, 1.6
    for (ky, kx), gam in (((1, 2), 0.7), ((2, 3), -2.0), ((1, 1), 5.0)):
        my, sy = _mode(bc, ny, ky)
        mx, sx = _mode(bc, nx, kx)
        lam = sum(4 * s * s / (h * h * (1 - s * s / 3)) for s in (sy, sx))
        L = kappa * tau * lam ** (alpha / 2)
        mode = np.outer(my, mx)
        sch = SeparableScheme(bc, (ny, nx), (h, h), (alpha,), (kappa,), tau)
        U = sch.step(mode[None], 0.0, lambda U, t: gam * U)
        r = _paper_r(gam * tau, -L)
        assert np.max(np.abs(U[0] - r * mode)) <= 1e-13
        assert abs(_paper_r(gam * tau, -L, printed_c1=True) - r) > 1e-6
        # f = 0: M steps multiply the mode by R13(L)^M.
        V = sch.integrate(mode[None], 5, lambda U, t: 0.0 * U)
        R = (24 - 6 * L) / (24 + 18 * L + 6 * L ** 2 + L ** 3)
        assert np.max(np.abs(V[0] - R ** 5 * mode)) <= 1e-13


def test_amplification_reduces_to_rk4():
    # Remark of Section 4.2.2: r(x, 0) = 1 + x + x^2/2 + x^3/6 + x^4/24.
    for x in (-2.0, -0.3, 0.5, 1.7):
        assert abs(_paper_r(x, 0.0) - (1 + x + x * x / 2 + x ** 3 / 6 + x ** 4 / 24)) < 1e-13


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("scheme", ["p13", "exp"])
def test_uniform_field_steps_like_classical_rk4(bc, scheme):
    # A spatially uniform field sits in the zero mode (L = 0), where every
    # coefficient takes its L -> 0 value: the step is classical RK4 on the
    # reaction ODE system.
    kind, p = "schnakenberg", (1.0, 0.1305, 0.7695)
    tau = 0.07
    u0 = np.array([0.7, 1.3])
    sch = SeparableScheme(bc, (4, 5), (0.1, 0.1), (1.5, 1.5), (0.3, 2.0), tau, scheme)
    U = sch.integrate(u0[:, None, None] * np.ones((2, 4, 5)), 3, _N(kind, p))

    def F(y):
        return reactions.f(kind, p, y.reshape(2, 1))[:, 0]

    y = u0.copy()
    for _ in range(3):
        k1 = F(y)
        k2 = F(y + tau / 2 * k1)
        k3 = F(y + tau / 2 * k2)
        k4 = F(y + tau * k3)
        y = y + tau / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    assert np.max(np.abs(U - y[:, None, None])) <= 1e-13


# ------------------------------------------------------------------ printed tables
def _table2():
    rows = []
    with open(os.path.join(GOLD, "table2_example2.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                a, ih, e_neu, e_per = line.split()
                rows.append((float(a), int(ih), float(e_neu), float(e_per)))
    return rows


@pytest.mark.parametrize("row", [r for r in _table2() if r[1] <= 80],
                         ids=lambda r: f"a{r[0]}-h{r[1]}")
def test_table2_example2_printed_errors(row):
    alpha, inv_h, e_neu, e_per = row
    for bc, ref in (("neumann", e_neu), ("periodic", e_per)):
        err, _ = example2(bc, inv_h, alpha)
        # printed to 5 significant digits
        assert abs(err - ref) <= 0.6e-4 * ref, (bc, err, ref)


@pytest.mark.slow
@pytest.mark.parametrize("alpha,bc", [(2.0, "periodic"), (1.2, "neumann")])
def test_table2_example2_finest_row(alpha, bc):
    row = [r for r in _table2() if r[0] == alpha and r[1] == 160][0]
    ref = row[2] if bc == "neumann" else row[3]
    err, _ = example2(bc, 160, alpha)
    assert abs(err - ref) <= 0.6e-4 * ref


def test_table2_orders_are_four():
    errs = [example2("periodic", ih, 1.4)[0] for ih in (10, 20, 40)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 4.0) < 0.2), orders


def test_table1_example1_printed_errors():
    rows = []
    with open(os.path.join(GOLD, "table1_example1.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                ih, e, _ = line.split()
                rows.append((int(ih), float(e)))
    errs = []
    for inv_h, ref in rows:
        h = 1.0 / inv_h
        err, _ = example1(inv_h, 1.8, 10.0, h / 40.0, 1.0)
        assert abs(err - ref) <= 0.6e-4 * ref, (inv_h, err, ref)
        errs.append(err)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 3.9)


# ------------------------------------------------------------------ stability (Section 4.2.2)
from oracle import stability


@pytest.mark.parametrize("y", [0.0, -0.5, -3.0, -20.0, -250.0])
def test_stability_amplification_matches_printed_quartic(y):
    # The stages run on the test equation give eq. Eq41's quartic (with the
    # y^2 term of c1's numerator that the printed formula lacks).
    xs = np.array([0.3, -2.0 + 1.5j, 4.0 - 7.0j, -11.0 + 0.1j])
    got = stability.amplification("p13", xs, y)
    ref = _paper_r(xs, y)
    assert np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref))) <= 1e-12
    c = stability.amplification_poly("p13", y)
    assert np.max(np.abs(np.polyval(c[::-1], xs) - ref) / np.maximum(1.0, np.abs(ref))) <= 1e-12


@pytest.mark.parametrize("scheme", ["p13", "exp"])
def test_stability_reduces_to_rk4_at_y0(scheme):
    # Remark of Section 4.2.2: at y = 0 the factor is RK4's Taylor polynomial.
    c = stability.amplification_poly(scheme, 0.0)
    assert np.allclose(c, [1, 1, 1 / 2, 1 / 6, 1 / 24], rtol=0, atol=1e-14)
    # RK4's real stability limit: |r(x, 0)| = 1 at x = -2.785293563...
    roots = stability.boundary(scheme, 0.0, 2)[1]      # r = -1 has no real root;
    roots0 = stability.boundary(scheme, 0.0, 1)[0]     # r = +1: x = 0 and x = -2.7853
    real = np.sort(roots0[np.abs(roots0.imag) < 1e-9].real)
    assert np.allclose(real, [-2.785293563405282, 0.0], atol=1e-9)
    assert np.all(np.abs(roots.imag) > 1e-3)


def test_stability_exp_scheme_zero_reaction_is_the_exponential():
    for y in (-0.1, -2.0, -9.0):
        assert abs(stability.amplification("exp", 0.0, y) - np.exp(y)) <= 1e-14
        assert abs(stability.amplification("p13", 0.0, y)
                   - (24 + 6 * y) / (24 - 18 * y + 6 * y * y - y ** 3)) <= 1e-14


@pytest.mark.parametrize("scheme", ["p13", "exp"])
@pytest.mark.parametrize("y", [-1.0, -10.0, -60.0])
def test_stability_boundary_points_have_unit_modulus(scheme, y):
    b = stability.boundary(scheme, y, 16)
    r = stability.amplification(scheme, b.ravel(), y)
    assert np.max(np.abs(np.abs(r) - 1.0)) <= 1e-9
    # the regions grow as y decreases (Section 4.2.2): compare the leftmost
    # real crossing with that of a less negative y
    def left(yy):
        rts = stability.boundary(scheme, yy, 2).ravel()
        return np.min(rts[np.abs(rts.imag) < 1e-7].real)
    assert left(y) < left(y / 2)
