// Eigenvalues and ETDRK4 coefficients, evaluated in FP64 on host and device.
//
// Eigenvalues (Section 3.1): lambda = 4 s^2 / (h^2 (1 - s^2/3)) with
//   periodic  (N = n):     s = sin(pi k / N),        k = 0..N-1
//   Dirichlet (N = n + 1): s = sin(pi k / (2N)),     k = 1..N-1
//   Neumann   (N = n - 1): s = sin(pi k / (2N)),     k = 0..N
// The periodic index is the one that matches the spectrum of the printed
// circulant matrices (sin^2(k pi / N)); the Hartley basis pairs k and N-k,
// which share an eigenvalue.
//
// Coefficients of L = kappa tau Lambda^(alpha/2):
//   P13 (Section 4, Alg. 1):  R13, Q13 = R13(L/2), phi, phi1, phi2, phi3.
//   EXP (Cox-Matthews):      e^-L, e^-L/2, tau(1-e^-L/2)/L, and f1, 2 f2, f3
//   at z = -L. For L < 2 these are formed from Taylor series of
//   phi_k(z) = sum_j z^j / (j+k)!, where the closed forms cancel badly;
//   otherwise from the closed forms.
// Every function is templated on the scalar so that a forward-mode dual
// number gives d/dL for the adjoint's parameter gradients.
#pragma once

#include <cmath>

#ifndef SFRDE_HD
#if defined(__HIPCC__)
#define SFRDE_HD __host__ __device__
#else
#define SFRDE_HD
#endif
#endif

namespace sfrde {

struct Dual {
  double v, d;
  SFRDE_HD Dual() : v(0), d(0) {}
  SFRDE_HD Dual(double x) : v(x), d(0) {}
  SFRDE_HD Dual(double x, double dx) : v(x), d(dx) {}
};
SFRDE_HD inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
SFRDE_HD inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
SFRDE_HD inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
SFRDE_HD inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
SFRDE_HD inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
SFRDE_HD inline Dual operator+(double a, Dual b) { return Dual(a) + b; }
SFRDE_HD inline Dual operator-(double a, Dual b) { return Dual(a) - b; }
SFRDE_HD inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
SFRDE_HD inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
SFRDE_HD inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
SFRDE_HD inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
SFRDE_HD inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }

SFRDE_HD inline double val(double x) { return x; }
SFRDE_HD inline double val(Dual x) { return x.v; }
SFRDE_HD inline double xexp(double x) { return exp(x); }
SFRDE_HD inline Dual xexp(Dual x) {
  double e = exp(x.v);
  return Dual(e, e * x.d);
}

enum { C_R = 0, C_Q = 1, C_PHI = 2, C_PHI1 = 3, C_PHI2 = 4, C_PHI3 = 5, NCOEF = 6 };

// ETDRK4-P13: the six rational functions of the Alg. 1 precompute.
template <class R>
SFRDE_HD inline void p13_coefs(R L, double tau, R* out) {
  R L2 = L * L;
  R L3 = L2 * L;
  R D = 24.0 + 18.0 * L + 6.0 * L2 + L3;
  R Dh = 192.0 + 72.0 * L + 12.0 * L2 + L3;
  out[C_R] = (24.0 - 6.0 * L) / D;
  out[C_Q] = (192.0 - 24.0 * L) / Dh;
  out[C_PHI] = tau * (96.0 + 12.0 * L + L2) / Dh;
  out[C_PHI1] = tau * (4.0 - L) / D;
  out[C_PHI2] = tau * (8.0 + 2.0 * L) / D;
  out[C_PHI3] = tau * (4.0 + 3.0 * L + L2) / D;
}

// phi_1(z), phi_2(z), phi_3(z) by their Taylor series (|z| <= 2 here).
template <class R>
SFRDE_HD inline void phi123_series(R z, R* p) {
  // phi_k(z) = (1/k!) (1 + z/(k+1) (1 + z/(k+2) (1 + ...))), evaluated from
  // the innermost level out; 34 levels leave a remainder below 2^35/36! for
  // |z| <= 2.
  const int J = 34;
  R a1 = 1.0, a2 = 1.0, a3 = 1.0;
  for (int j = J; j >= 1; --j) {
    a1 = 1.0 + z * a1 / double(j + 1);
    a2 = 1.0 + z * a2 / double(j + 2);
    a3 = 1.0 + z * a3 / double(j + 3);
  }
  p[0] = a1;
  p[1] = a2 / 2.0;
  p[2] = a3 / 6.0;
}

template <class R>
SFRDE_HD inline void exp_coefs(R L, double tau, R* out) {
  if (val(L) < 2.0) {
    R z = -L;
    R p[3], ph[3];
    phi123_series(z, p);
    phi123_series(0.5 * z, ph);
    out[C_R] = xexp(z);
    out[C_Q] = xexp(0.5 * z);
    out[C_PHI] = 0.5 * tau * ph[0];
    out[C_PHI1] = tau * (p[0] - 3.0 * p[1] + 4.0 * p[2]);
    out[C_PHI2] = 2.0 * tau * (p[1] - 2.0 * p[2]);
    out[C_PHI3] = tau * (4.0 * p[2] - p[1]);
  } else {
    R E = xexp(-L);
    R E2 = xexp(-0.5 * L);
    R L2 = L * L;
    R L3 = L2 * L;
    out[C_R] = E;
    out[C_Q] = E2;
    out[C_PHI] = tau * (1.0 - E2) / L;
    out[C_PHI1] = tau * (4.0 - L - E * (4.0 + 3.0 * L + L2)) / L3;
    out[C_PHI2] = 2.0 * tau * (L - 2.0 + E * (L + 2.0)) / L3;
    out[C_PHI3] = tau * (4.0 - 3.0 * L + L2 - E * (4.0 + L)) / L3;
  }
}

template <class R>
SFRDE_HD inline void coefs(int scheme, R L, double tau, R* out) {
  if (scheme == 0)
    p13_coefs(L, tau, out);
  else
    exp_coefs(L, tau, out);
}

// d/dL of the six coefficients.
SFRDE_HD inline void coef_derivs(int scheme, double L, double tau, double* out) {
  Dual o[NCOEF];
  coefs(scheme, Dual(L, 1.0), tau, o);
  for (int i = 0; i < NCOEF; ++i) out[i] = o[i].d;
}

SFRDE_HD inline void coef_values(int scheme, double L, double tau, double* out) {
  coefs(scheme, L, tau, out);
}

// The plan's coefficient tables hold the decrements 1 - R and 1 - Q in the
// C_R and C_Q slots, the phi functions as they are. R and Q multiply the
// retained spectral state every step and lie within about L of 1 for the
// slowly decaying modes: stored as values, their rounding (half an ulp of 1,
// the same in every step) would change each such mode's decay rate by a
// relative 2^-25 / L. Stored as decrements they keep full relative
// precision, and the combine forms R x as x - (1 - R) x.
//   P13:  1 - R13 = L (24 + 6L + L^2) / D,  1 - Q13 = L (96 + 12L + L^2) / Dh
//         (L < 1; above, 1 - R13 and 1 - Q13 from the values, no cancellation)
//   EXP:  1 - e^-L = -expm1(-L),  1 - e^-L/2 = -expm1(-L/2)
SFRDE_HD inline void coef_table_values(int scheme, double L, double tau, double* out) {
  coefs(scheme, L, tau, out);
  if (scheme == 0) {
    if (L < 1.0) {
      const double D = 24.0 + L * (18.0 + L * (6.0 + L));
      const double Dh = 192.0 + L * (72.0 + L * (12.0 + L));
      out[C_R] = L * (24.0 + L * (6.0 + L)) / D;
      out[C_Q] = L * (96.0 + L * (12.0 + L)) / Dh;
    } else {
      out[C_R] = 1.0 - out[C_R];
      out[C_Q] = 1.0 - out[C_Q];
    }
  } else {
    out[C_R] = -expm1(-L);
    out[C_Q] = -expm1(-0.5 * L);
  }
}

// Per-axis eigenvalue at spectral index k (0-based, the library's order).
SFRDE_HD inline double axis_eigenvalue(int bc, long n, double h, long k) {
  const double pi = 3.14159265358979323846;
  double s;
  if (bc == 0) {  // periodic, N = n
    s = sin(pi * double(k) / double(n));
  } else if (bc == 1) {  // Dirichlet, N = n + 1, modes 1..N-1
    s = sin(pi * double(k + 1) / (2.0 * double(n + 1)));
  } else {  // Neumann, N = n - 1, modes 0..N
    s = sin(pi * double(k) / (2.0 * double(n - 1)));
  }
  double s2 = s * s;
  return 4.0 * s2 / (h * h * (1.0 - s2 / 3.0));
}

}  // namespace sfrde
