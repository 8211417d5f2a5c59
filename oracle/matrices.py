"""Compact fourth-order Laplacian matrices (Section 3, eq. Lap; Section 3.1).

The compact scheme approximates -Delta by -h^-2 (1 + delta^2/12)^-1 delta^2,
which in matrix form is T = A^-1 B with A = tridiag(1/12, 5/6, 1/12) and
B = h^-2 tridiag(-1, 2, -1), closed differently for each boundary condition:

* periodic  (Section 3.1.1): N x N circulant A and B.
* Dirichlet (Section 3.1.2): (N-1) x (N-1), the boundary values are zero.
* Neumann   (Section 3.1.3): (N+1) x (N+1), boundary rows (5/6, 1/6) in A and
  h^-2 (2, -2) in B.

Here ``n`` is the number of unknowns (the size of the matrix), so N is n for
periodic, n + 1 for Dirichlet and n - 1 for Neumann.

The Neumann A and B are not symmetric (the paper states they are, which only
holds for the other two conditions). With W = diag(1/2, 1, ..., 1, 1/2) both
W A and W B are symmetric, and W A is positive definite; ``weights`` returns
that W (the identity for periodic and Dirichlet).
"""
from __future__ import annotations

import numpy as np


def ab(bc: str, n: int, h: float):
    """Dense FP64 (A, B) of size n x n for one axis, as printed in Section 3.1."""
    if n < 2:
        raise ValueError("need at least 2 unknowns per axis")
    A = np.zeros((n, n))
    B = np.zeros((n, n))
    for i in range(n):
        A[i, i] = 5.0 / 6.0
        B[i, i] = 2.0
        if i > 0:
            A[i, i - 1] = 1.0 / 12.0
            B[i, i - 1] = -1.0
        if i < n - 1:
            A[i, i + 1] = 1.0 / 12.0
            B[i, i + 1] = -1.0
    if bc == "periodic":
        A[0, n - 1] += 1.0 / 12.0
        A[n - 1, 0] += 1.0 / 12.0
        B[0, n - 1] += -1.0
        B[n - 1, 0] += -1.0
    elif bc == "dirichlet":
        pass
    elif bc == "neumann":
        A[0, 1] = 1.0 / 6.0
        A[n - 1, n - 2] = 1.0 / 6.0
        B[0, 1] = -2.0
        B[n - 1, n - 2] = -2.0
    else:
        raise ValueError(bc)
    return A, B / (h * h)


def weights(bc: str, n: int) -> np.ndarray:
    """Diagonal of W that symmetrises A and B (identity except Neumann)."""
    w = np.ones(n)
    if bc == "neumann":
        w[0] = w[-1] = 0.5
    return w


def kron_all(mats):
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(out, m)
    return out


def dense_pair(bc: str, shape, h):
    """The d-dimensional symmetric pair (WB_d, WA_d) whose pencil is the
    Kronecker sum of the 1D operators (Sections 3.2-3.3: the d-dim operator
    acts as T_x on the x index, T_y on the y index, ... and these commute).

    With WA_d = (x)_a (W_a A_a) and WB_d = sum_a (W_a B_a) (x) (W_b A_b, b != a),
    WA_d^-1 WB_d = sum_a I (x) .. (x) T_a (x) .. (x) I.  ``shape`` and ``h`` are
    in numpy order (slowest axis first), matching np.kron's ordering.
    """
    wa, wb = [], []
    for n, hh in zip(shape, h):
        A, B = ab(bc, n, hh)
        W = np.diag(weights(bc, n))
        wa.append(W @ A)
        wb.append(W @ B)
    WA = kron_all(wa)
    WB = np.zeros_like(WA)
    for a in range(len(shape)):
        mats = [wb[b] if b == a else wa[b] for b in range(len(shape))]
        WB += kron_all(mats)
    return WB, WA


def dense_weights(bc: str, shape) -> np.ndarray:
    return kron_all([np.diag(weights(bc, n)) for n in shape]).diagonal().copy()
