// Pointwise reaction terms of the pattern models (Section 5.2), their
// transposed Jacobians and parameter partials, in the field precision T.
#pragma once

#include <hip/hip_runtime.h>

namespace sfrde {

enum {
  RXN_LINEAR = 0,
  RXN_FHN = 1,
  RXN_GRAY_SCOTT = 2,
  RXN_SCHNAKENBERG = 3,
  RXN_GM = 4,
  RXN_HUXLEY_MMS = 5,  // Example 2 of Section 5.1 (one species, 2D, with a source)
  RXN_FISHER_MMS = 6   // Example 1 of Section 5.1 (one species, 1D, with a source)
};
constexpr int MAX_SPECIES = 4;
constexpr int MAX_PARAMS = 16;
constexpr int RXN_NP_MAX = 5;  // parameters of any of the models (linear: one per species)
// Manufactured-source constants sit in p[MMS_P0..]: alpha, three source
// weights, the mesh widths (x, y); filled by the host, never user parameters.
constexpr int MMS_P0 = 8;

struct Rxn {
  int kind;
  int S;
  int np;
  double p[MAX_PARAMS];
};

// Reaction parameters converted to the field type once per kernel.
template <typename T>
struct RxnT {
  int kind, S;
  T p[5];
  T lin[MAX_SPECIES];
  __device__ __forceinline__ explicit RxnT(const Rxn& r) : kind(r.kind), S(r.S) {
    for (int k = 0; k < 5; ++k) p[k] = k < r.np ? T(r.p[k]) : T(0);
    for (int s = 0; s < MAX_SPECIES; ++s) lin[s] = s < r.np ? T(r.p[s]) : T(0);
  }
};

// f = f(u) for a reaction kind fixed at compile time (KIND), NS species.
template <typename T, int NS, int KIND>
__device__ __forceinline__ void rxn_eval_k(const RxnT<T>& r, const T* u, T* f) {
  if constexpr (KIND == RXN_LINEAR) {
#pragma unroll
    for (int s = 0; s < NS; ++s) f[s] = r.lin[s] * u[s];
  } else if constexpr (NS == 1) {
    // the pointwise parts of Examples 1 and 2 (the source is added by the
    // caller, which knows the point and the stage time)
    const T x = u[0];
    if constexpr (KIND == RXN_HUXLEY_MMS)
      f[0] = x * (T(1) - x) * (x - T(1));
    else
      f[0] = x - x * x;
  } else if constexpr (NS == 2) {
    const T x = u[0], v = u[1];
    if constexpr (KIND == RXN_FHN) {
      f[0] = x * (T(1) - x) * (x - r.p[0]) - v;
      f[1] = r.p[1] * (r.p[2] * x - r.p[3] * v - r.p[4]);
    } else if constexpr (KIND == RXN_GRAY_SCOTT) {
      const T xvv = x * v * v;
      f[0] = -xvv + r.p[0] * (T(1) - x);
      f[1] = xvv - (r.p[0] + r.p[1]) * v;
    } else if constexpr (KIND == RXN_SCHNAKENBERG) {
      const T xxv = x * x * v;
      f[0] = r.p[0] * (r.p[1] - x + xxv);
      f[1] = r.p[0] * (r.p[2] - xxv);
    } else {  // Gierer-Meinhardt
      f[0] = r.p[0] - r.p[1] * x + r.p[2] * x * x / v;
      f[1] = r.p[3] * x * x - r.p[4] * v;
    }
  }
}

// NS = number of species, fixed at compile time so that the per-point
// arrays stay in registers; the kind is taken at run time.
template <typename T, int NS>
__device__ __forceinline__ void rxn_eval_t(const RxnT<T>& r, const T* u, T* f) {
  switch (r.kind) {
    case RXN_LINEAR:
      rxn_eval_k<T, NS, RXN_LINEAR>(r, u, f);
      break;
    case RXN_FHN:
      rxn_eval_k<T, NS, RXN_FHN>(r, u, f);
      break;
    case RXN_GRAY_SCOTT:
      rxn_eval_k<T, NS, RXN_GRAY_SCOTT>(r, u, f);
      break;
    case RXN_SCHNAKENBERG:
      rxn_eval_k<T, NS, RXN_SCHNAKENBERG>(r, u, f);
      break;
    case RXN_GM:
      rxn_eval_k<T, NS, RXN_GM>(r, u, f);
      break;
    case RXN_HUXLEY_MMS:
      rxn_eval_k<T, NS, RXN_HUXLEY_MMS>(r, u, f);
      break;
    default:
      rxn_eval_k<T, NS, RXN_FISHER_MMS>(r, u, f);
      break;
  }
}

// out = J_f(u)^T g (out_r = sum_s g_s d f_s / d u_r), and
// pacc[k] += wgt * sum_s g_s d f_s / d p_k, for a kind fixed at compile time.
template <typename T, int NS, int KIND>
__device__ __forceinline__ void rxn_adjoint_k(const Rxn& r, const T* u, const T* g, T* out,
                                              double wgt, double* pacc, bool want_p) {
  if constexpr (KIND == RXN_LINEAR) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      out[s] = T(r.p[s]) * g[s];
      if (want_p) pacc[s] += wgt * double(g[s] * u[s]);
    }
  } else if constexpr (NS == 1) {
    // Examples 1 and 2: the sources do not depend on u
    const T x = u[0];
    if constexpr (KIND == RXN_HUXLEY_MMS)
      out[0] = -g[0] * (x - T(1)) * (T(3) * x - T(1));
    else
      out[0] = g[0] * (T(1) - T(2) * x);
  } else if constexpr (NS == 2) {
    const T x = u[0], v = u[1], gu = g[0], gv = g[1];
    if constexpr (KIND == RXN_FHN) {
      const T mu = T(r.p[0]), eps = T(r.p[1]), beta = T(r.p[2]), gam = T(r.p[3]), dlt = T(r.p[4]);
      const T dfu_du = -T(3) * x * x + T(2) * (T(1) + mu) * x - mu;
      out[0] = gu * dfu_du + gv * eps * beta;
      out[1] = -gu - gv * eps * gam;
      if (want_p) {
        pacc[0] += wgt * double(gu * (-x * (T(1) - x)));
        pacc[1] += wgt * double(gv * (beta * x - gam * v - dlt));
        pacc[2] += wgt * double(gv * eps * x);
        pacc[3] += wgt * double(-gv * eps * v);
        pacc[4] += wgt * double(-gv * eps);
      }
    } else if constexpr (KIND == RXN_GRAY_SCOTT) {
      const T F = T(r.p[0]), K = T(r.p[1]);
      const T xv2 = T(2) * x * v;
      out[0] = gu * (-v * v - F) + gv * v * v;
      out[1] = gu * (-xv2) + gv * (xv2 - F - K);
      if (want_p) {
        pacc[0] += wgt * double(gu * (T(1) - x) - gv * v);
        pacc[1] += wgt * double(-gv * v);
      }
    } else if constexpr (KIND == RXN_SCHNAKENBERG) {
      const T gm = T(r.p[0]), a = T(r.p[1]), b = T(r.p[2]);
      const T xv2 = T(2) * x * v, xx = x * x;
      out[0] = gm * (gu * (xv2 - T(1)) - gv * xv2);
      out[1] = gm * (gu - gv) * xx;
      if (want_p) {
        const T xxv = xx * v;
        pacc[0] += wgt * double(gu * (a - x + xxv) + gv * (b - xxv));
        pacc[1] += wgt * double(gu * gm);
        pacc[2] += wgt * double(gv * gm);
      }
    } else {  // Gierer-Meinhardt
      const T mu_u = T(r.p[1]), s_u = T(r.p[2]), s_v = T(r.p[3]), mu_v = T(r.p[4]);
      const T xv = x / v;
      out[0] = gu * (-mu_u + T(2) * s_u * xv) + gv * T(2) * s_v * x;
      out[1] = -gu * s_u * xv * xv - gv * mu_v;
      if (want_p) {
        pacc[0] += wgt * double(gu);
        pacc[1] += wgt * double(-gu * x);
        pacc[2] += wgt * double(gu * x * xv);
        pacc[3] += wgt * double(gv * x * x);
        pacc[4] += wgt * double(-gv * v);
      }
    }
  }
}

// The same with the kind taken at run time.
template <typename T, int NS>
__device__ __forceinline__ void rxn_adjoint(const Rxn& r, const T* u, const T* g, T* out,
                                            double wgt, double* pacc, bool want_p) {
  switch (r.kind) {
    case RXN_LINEAR: rxn_adjoint_k<T, NS, RXN_LINEAR>(r, u, g, out, wgt, pacc, want_p); break;
    case RXN_FHN: rxn_adjoint_k<T, NS, RXN_FHN>(r, u, g, out, wgt, pacc, want_p); break;
    case RXN_GRAY_SCOTT: rxn_adjoint_k<T, NS, RXN_GRAY_SCOTT>(r, u, g, out, wgt, pacc, want_p); break;
    case RXN_SCHNAKENBERG: rxn_adjoint_k<T, NS, RXN_SCHNAKENBERG>(r, u, g, out, wgt, pacc, want_p); break;
    case RXN_GM: rxn_adjoint_k<T, NS, RXN_GM>(r, u, g, out, wgt, pacc, want_p); break;
    case RXN_HUXLEY_MMS: rxn_adjoint_k<T, NS, RXN_HUXLEY_MMS>(r, u, g, out, wgt, pacc, want_p); break;
    default: rxn_adjoint_k<T, NS, RXN_FISHER_MMS>(r, u, g, out, wgt, pacc, want_p); break;
  }
}

}  // namespace sfrde
