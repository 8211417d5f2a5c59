"""FP64 CPU oracle for the fractional ETDRK4 step (TEST INFRASTRUCTURE).

This package is a plain, slow, obviously correct CPU implementation of what
the GPU library computes. It exists to check the library; it is not part of
the product. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it. It shares no code with the HIP
library: it builds the compact matrices of Section 3 as printed, diagonalises
them with LAPACK, and steps the scheme of Section 4 in physical space.

Modules
-------
matrices      1D matrices A and B per boundary condition (Section 3.1) and the
              d-dimensional Kronecker assembly (Sections 3.2-3.3).
coefficients  The six ETDRK4-P13 functions (Section 4, Alg. 1 precompute) and
              the exact-exponential (Cox-Matthews) coefficients, scalar and
              matrix forms, with derivatives.
reactions     Reaction terms of Section 5 and their Jacobians.
dense         O1: tiny grids, the whole operator as one dense matrix.
separable     O2: per-axis LAPACK eigenbases, full benchmark sizes; the
              discrete adjoint of the step.
examples      The manufactured-solution problems of Section 5.1.
"""
