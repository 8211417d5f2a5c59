// Linear stability of the time stepping (Section 4.2.2, eq. Eq41).
//
// Test equation u' + c u = gamma u with y = -c tau (real, <= 0) and
// x = gamma tau (complex). One step of the four stages (eq. ETDRK4P13) with
// the scheme's coefficients at L = -y (tau = 1, f(u) = x u) multiplies u by
// r(x, y), a quartic in x. The |r| = 1 boundary for a fixed y is the set of
// x solving r(x, y) = e^{i theta}.
//
// One thread per evaluation point, FP64 throughout: these are analysis
// tools, not part of the time loop.
#pragma once

#include <hip/hip_runtime.h>

#include "coef.h"

namespace sfrde {

struct Cplx {
  double re, im;
};
__device__ __forceinline__ Cplx cadd(Cplx a, Cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cplx csub(Cplx a, Cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ Cplx cmul(Cplx a, Cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Cplx cscale(double s, Cplx a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ Cplx cdiv(Cplx a, Cplx b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// r(x, y): the stages on the scalar test equation from u = 1.
__global__ void k_amplification(int scheme, long long count, const double* __restrict__ x,
                                const double* __restrict__ y, double* __restrict__ r) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double yy = y[i];
  const Cplx X{x[2 * i], x[2 * i + 1]};
  if (!(yy <= 0.0) || !isfinite(yy) || !isfinite(X.re) || !isfinite(X.im)) {
    r[2 * i] = r[2 * i + 1] = __builtin_nan("");
    return;
  }
  double c[NCOEF];
  coefs(scheme, -yy, 1.0, c);
  const Cplx one{1.0, 0.0};
  const Cplx fu = X;
  const Cplx a = cadd(cscale(c[C_Q], one), cscale(c[C_PHI], fu));
  const Cplx fa = cmul(X, a);
  const Cplx b = cadd(cscale(c[C_Q], one), cscale(c[C_PHI], fa));
  const Cplx fb = cmul(X, b);
  const Cplx cc = cadd(cscale(c[C_Q], a), cscale(c[C_PHI], csub(cscale(2.0, fb), fu)));
  const Cplx fc = cmul(X, cc);
  const Cplx out = cadd(cadd(cscale(c[C_R], one), cscale(c[C_PHI1], fu)),
                        cadd(cscale(c[C_PHI2], cadd(fa, fb)), cscale(c[C_PHI3], fc)));
  r[2 * i] = out.re;
  r[2 * i + 1] = out.im;
}

// Polynomials in x of degree <= 4, lowest order first.
struct Poly4 {
  double c[5];
};
__device__ __forceinline__ Poly4 pmake(double c0, double c1) { return {{c0, c1, 0.0, 0.0, 0.0}}; }
__device__ __forceinline__ Poly4 paxpy(double s, const Poly4& p, double t, const Poly4& q) {
  Poly4 o;
  for (int k = 0; k < 5; ++k) o.c[k] = s * p.c[k] + t * q.c[k];
  return o;
}
__device__ __forceinline__ Poly4 pshift(const Poly4& p) {  // x * p (degree stays <= 4 here)
  return {{0.0, p.c[0], p.c[1], p.c[2], p.c[3]}};
}

// c_0..c_4 of r(., y): the stages run on polynomials in x.
__device__ inline Poly4 amplification_poly(int scheme, double y) {
  double c[NCOEF];
  coefs(scheme, -y, 1.0, c);
  const Poly4 one = pmake(1.0, 0.0);
  const Poly4 fu = pshift(one);
  const Poly4 a = paxpy(c[C_Q], one, c[C_PHI], fu);
  const Poly4 fa = pshift(a);
  const Poly4 b = paxpy(c[C_Q], one, c[C_PHI], fa);
  const Poly4 fb = pshift(b);
  const Poly4 cc = paxpy(c[C_Q], a, c[C_PHI], paxpy(2.0, fb, -1.0, fu));
  const Poly4 fc = pshift(cc);
  Poly4 r = paxpy(c[C_R], one, c[C_PHI1], fu);
  r = paxpy(1.0, r, c[C_PHI2], paxpy(1.0, fa, 1.0, fb));
  return paxpy(1.0, r, c[C_PHI3], fc);
}

constexpr int DK_ITERS = 200;  // Durand-Kerner sweeps (fixed count: every thread ends)

// Thread (i, k): the four x with r(x, y_i) = e^{i theta_k}, theta_k = 2 pi k / ntheta,
// by the Durand-Kerner (Weierstrass) simultaneous iteration on the monic
// quartic, started on the circle of Cauchy's root bound.
__global__ void k_stability_boundary(int scheme, long long ny, const double* __restrict__ y,
                                     long long ntheta, double* __restrict__ roots,
                                     double* __restrict__ poly) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ny * ntheta) return;
  const long long i = t / ntheta, k = t - i * ntheta;
  const double yy = y[i];
  double* out = roots + 8 * t;
  if (!(yy <= 0.0) || !isfinite(yy)) {
    for (int q = 0; q < 8; ++q) out[q] = __builtin_nan("");
    if (poly && k == 0)
      for (int q = 0; q < 5; ++q) poly[5 * i + q] = __builtin_nan("");
    return;
  }
  const Poly4 p = amplification_poly(scheme, yy);
  if (poly && k == 0)
    for (int q = 0; q < 5; ++q) poly[5 * i + q] = p.c[q];
  // monic coefficients of r(x) - e^{i theta}
  double sn, cs;
  sincospi(2.0 * double(k) / double(ntheta), &sn, &cs);
  Cplx m[4];
  const double inv4 = 1.0 / p.c[4];
  m[0] = {(p.c[0] - cs) * inv4, -sn * inv4};
  for (int q = 1; q < 4; ++q) m[q] = {p.c[q] * inv4, 0.0};
  double bound = 0.0;
  for (int q = 0; q < 4; ++q) bound = fmax(bound, sqrt(m[q].re * m[q].re + m[q].im * m[q].im));
  bound += 1.0;
  Cplx z[4];
  const Cplx w{0.4, 0.9};
  Cplx pw{bound, 0.0};
  for (int q = 0; q < 4; ++q) {
    z[q] = pw;
    pw = cmul(pw, w);
  }
  for (int it = 0; it < DK_ITERS; ++it) {
    for (int q = 0; q < 4; ++q) {
      // value of the monic quartic at z[q] (Horner)
      Cplx v{1.0, 0.0};
      for (int e = 3; e >= 0; --e) v = cadd(cmul(v, z[q]), m[e]);
      Cplx den{1.0, 0.0};
      for (int o = 0; o < 4; ++o)
        if (o != q) den = cmul(den, csub(z[q], z[o]));
      if (den.re != 0.0 || den.im != 0.0) z[q] = csub(z[q], cdiv(v, den));
    }
  }
  for (int q = 0; q < 4; ++q) {
    out[2 * q] = z[q].re;
    out[2 * q + 1] = z[q].im;
  }
}

}  // namespace sfrde
