// Device kernels of the ETDRK4 step.
//
// Every field is [S][total] with x fastest (ensembles: [member][S][total], the
// member taken from blockIdx.y). A kernel works on "line tiles":
// W lines along one axis (length n, stride `inner`), staged in LDS as
// buf[s][j][w] (j along the axis, w the line within the tile). Per-axis
// transforms are products with the axis matrix M (forward, unnormalised):
//   periodic  M[k][j] = cos(2 pi kj/N) + sin(2 pi kj/N)   (discrete Hartley)
//   Dirichlet M[k][j] = sin(pi (k+1)(j+1)/N)                (DST-I)
//   Neumann   M[k][j] = cos(pi kj/N) w_j, w = 1/2 at both ends (DCT-I)
// and the inverse along an axis is the same product scaled by 1/N, 2/N, 2/N;
// these scales are folded into the stage combine (one factor `cs` for all
// axes), so forward and inverse use identical arithmetic.
//
// One stage of eq. ETDRK4P13 in 3D is four kernels on one buffer P:
//   X: inverse-x, reaction f(stage value), forward-x
//   Y: forward-y
//   Z: forward-z, diagonal combine with the retained spectral arrays, inverse-z
//   Y: inverse-y
// (2D drops the Y passes). The combine keeps u_hat (spectral state), c_til
// and acc across the stages so that a and 2 f_b - f_u are never transformed
// again (linearity of the transforms):
//   st 0: a = Q u + phi f_u; c_til = Q a - phi f_u; acc = R u + phi1 f_u
//   st 1: b = Q u + phi f_a; acc += phi2 f_a
//   st 2: c = c_til + 2 phi f_b; acc += phi2 f_b
//   st 3: u_hat = acc + phi3 f_c
#pragma once

#include <hip/hip_runtime.h>

#include "coef.h"
#include "reactions.h"

namespace sfrde {

constexpr int NTHREADS = 256;
constexpr int KMAX = 32;  // outputs per thread in the dense transform: n*W <= KMAX*NTHREADS

struct Geom {
  int n;            // length of the transformed axis
  int spt;          // species per tile: all, or 1 (strided axes may split tiles by species,
                    // with the species index folded into the outer blocks)
  int fast;         // full tiles may use the 32-bit-offset vector paths of the FP32 engine
  int W;            // lines per tile (a power of two)
  int pitch;        // LDS row pitch (>= W)
  int wshift;       // log2(W)
  float inv_n;      // 1/n, for the element -> (line, row) split of x-axis tiles
  long long inner;  // stride of the axis (1 for x)
  long long outer;  // lines (inner == 1) or outer blocks of n*inner
  long long tpo;    // tiles per outer block (inner > 1)
  int tposh;        // log2(tpo) when tpo is a power of two, else -1
  long long ntiles;
  long long total;  // points per species
};

// Where a tile sits in the field, computed once per tile: element (j, w) is
// at base + j*rs + w*cs, and lanes w >= wvalid lie past the edge.
struct TileRef {
  long long base;
  int wvalid;
  int rs, cs;
};

// Outer block o of a strided-axis tile and the tile's index r within it: a
// shift when the tiles per outer block are a power of two, else a 32-bit
// division while the tile count allows (the 64-bit one costs several times
// as many instructions, each tile several times).
__device__ __forceinline__ void split_tile(const Geom& g, long long tile, long long& o,
                                           long long& r) {
  if (g.tposh >= 0) {
    o = tile >> g.tposh;
    r = tile & ((1LL << g.tposh) - 1);
  } else if (g.ntiles <= 0x7fffffffLL) {
    const unsigned q = (unsigned)tile / (unsigned)g.tpo;
    o = q;
    r = (long long)((unsigned)tile - q * (unsigned)g.tpo);
  } else {
    o = tile / g.tpo;
    r = tile - o * g.tpo;
  }
}

__device__ __forceinline__ TileRef tile_ref(const Geom& g, long long tile) {
  TileRef t;
  if (g.inner == 1) {
    const long long line0 = tile * g.W;
    t.base = line0 * g.n;
    const long long left = g.outer - line0;
    t.wvalid = left < g.W ? (int)left : g.W;
    t.rs = 1;
    t.cs = g.n;
  } else {
    long long o, r;
    split_tile(g, tile, o, r);
    const long long i0 = r * g.W;
    t.base = o * (long long)g.n * g.inner + i0;
    const long long left = g.inner - i0;
    t.wvalid = left < g.W ? (int)left : g.W;
    t.rs = (int)g.inner;
    t.cs = 1;
  }
  return t;
}

// Global index of element (j, w) of a tile; false for lanes past the edge.
__device__ __forceinline__ bool elem(const Geom& g, const TileRef& t, int j, int w, long long& idx) {
  idx = t.base + (long long)j * t.rs + (long long)w * t.cs;
  return w < t.wvalid;
}

// floor(e / n) for 0 <= e < 2^24 from a float reciprocal and one correction.
__device__ __forceinline__ int div_n(int e, int n, float inv_n) {
  int q = (int)((float)e * inv_n);
  if (q * n > e) --q;
  if ((q + 1) * n <= e) ++q;
  return q;
}

// Element e of the tile in coalescing order: consecutive threads touch
// consecutive global addresses.
__device__ __forceinline__ void unpack(const Geom& g, int e, int& j, int& w) {
  if (g.inner == 1) {
    w = div_n(e, g.n, g.inv_n);
    j = e - w * g.n;
  } else {
    j = e >> g.wshift;
    w = e & (g.W - 1);
  }
}

template <typename T>
__device__ __forceinline__ void load_tile(const Geom& g, long long tile, const T* __restrict__ src,
                                          T* buf, int S) {
  const TileRef tr = tile_ref(g, tile);
  const int ne = g.n * g.W;
  for (int s = 0; s < S; ++s) {
    const T* sp = src + (long long)s * g.total;
    T* b = buf + s * g.n * g.pitch;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      int j, w;
      unpack(g, e, j, w);
      long long idx;
      b[j * g.pitch + w] = elem(g, tr, j, w, idx) ? sp[idx] : T(0);
    }
  }
}

template <typename T>
__device__ __forceinline__ void store_tile(const Geom& g, long long tile, const T* buf,
                                           T* __restrict__ dst, int S) {
  const TileRef tr = tile_ref(g, tile);
  const int ne = g.n * g.W;
  for (int s = 0; s < S; ++s) {
    T* dp = dst + (long long)s * g.total;
    const T* b = buf + s * g.n * g.pitch;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      int j, w;
      unpack(g, e, j, w);
      long long idx;
      if (elem(g, tr, j, w, idx)) dp[idx] = b[j * g.pitch + w];
    }
  }
}

// 16-byte vectors of the field type.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int N = 4;
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int N = 2;
};
template <typename T>
__device__ __forceinline__ T vget(const typename Vec16<T>::type& v, int e);
template <>
__device__ __forceinline__ float vget<float>(const float4& v, int e) {
  return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}
template <>
__device__ __forceinline__ double vget<double>(const double2& v, int e) {
  return e == 0 ? v.x : v.y;
}
template <typename T>
__device__ __forceinline__ void vset(typename Vec16<T>::type& v, int e, T x);
template <>
__device__ __forceinline__ void vset<float>(float4& v, int e, float x) {
  if (e == 0) v.x = x; else if (e == 1) v.y = x; else if (e == 2) v.z = x; else v.w = x;
}
template <>
__device__ __forceinline__ void vset<double>(double2& v, int e, double x) {
  if (e == 0) v.x = x; else v.y = x;
}

// Whether a tile can move in 16-byte vectors: full tile, vector-aligned rows.
template <typename T>
__device__ __forceinline__ bool tile_vectorizable(const Geom& g, const TileRef& t, const void* p) {
  constexpr int VW = Vec16<T>::N;
  if (reinterpret_cast<unsigned long long>(p) & 15ull) return false;
  if (g.total % VW) return false;
  if (t.wvalid != g.W) return false;
  if (g.inner == 1) return (g.n % VW) == 0;
  return (g.inner % VW) == 0 && (g.W % VW) == 0;
}

// Vector v of one species' tile -> (global element, LDS row j, lane w): VW
// consecutive rows of one line (x axis) or VW consecutive lanes of one row.
template <typename T>
__device__ __forceinline__ void vec_coords(const Geom& g, const TileRef& t, int v, long long& gidx,
                                           int& j, int& w) {
  constexpr int VW = Vec16<T>::N;
  const int e = v * VW;
  unpack(g, e, j, w);
  gidx = t.base + (long long)j * t.rs + (long long)w * t.cs;
}

// Tile load with every vector load of a thread issued before any use.
template <typename T>
__device__ __forceinline__ void load_tile_fast(const Geom& g, long long tile,
                                               const T* __restrict__ src, T* buf, int S) {
  const TileRef tr = tile_ref(g, tile);
  if (!tile_vectorizable<T>(g, tr, src)) {
    load_tile(g, tile, src, buf, S);
    return;
  }
  using V = typename Vec16<T>::type;
  constexpr int VW = Vec16<T>::N;
  constexpr int CH = 4;
  const int per_s = g.n * g.W / VW;
  const int total_v = S * per_s;
  for (int base = 0; base < total_v; base += CH * blockDim.x) {
    V r[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int v = base + c * blockDim.x + threadIdx.x;
      if (v < total_v) {
        const int s = v >= per_s ? (v >= 2 * per_s ? (v >= 3 * per_s ? 3 : 2) : 1) : 0;
        long long gi;
        int j, w;
        vec_coords<T>(g, tr, v - s * per_s, gi, j, w);
        r[c] = *reinterpret_cast<const V*>(src + s * g.total + gi);
      }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int v = base + c * blockDim.x + threadIdx.x;
      if (v < total_v) {
        const int s = v >= per_s ? (v >= 2 * per_s ? (v >= 3 * per_s ? 3 : 2) : 1) : 0;
        long long gi;
        int j, w;
        vec_coords<T>(g, tr, v - s * per_s, gi, j, w);
        T* b = buf + s * g.n * g.pitch;
        for (int e = 0; e < VW; ++e) {
          if (g.inner == 1)
            b[(j + e) * g.pitch + w] = vget<T>(r[c], e);
          else
            b[j * g.pitch + w + e] = vget<T>(r[c], e);
        }
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void store_tile_fast(const Geom& g, long long tile, const T* buf,
                                                T* __restrict__ dst, int S) {
  const TileRef tr = tile_ref(g, tile);
  if (!tile_vectorizable<T>(g, tr, dst)) {
    store_tile(g, tile, buf, dst, S);
    return;
  }
  using V = typename Vec16<T>::type;
  constexpr int VW = Vec16<T>::N;
  const int per_s = g.n * g.W / VW;
  const int total_v = S * per_s;
  for (int v = threadIdx.x; v < total_v; v += blockDim.x) {
    const int s = v >= per_s ? (v >= 2 * per_s ? (v >= 3 * per_s ? 3 : 2) : 1) : 0;
    long long gi;
    int j, w;
    vec_coords<T>(g, tr, v - s * per_s, gi, j, w);
    const T* b = buf + s * g.n * g.pitch;
    V r;
    for (int e = 0; e < VW; ++e)
      vset<T>(r, e, g.inner == 1 ? b[(j + e) * g.pitch + w] : b[j * g.pitch + w + e]);
    *reinterpret_cast<V*>(dst + s * g.total + gi) = r;
  }
}

// In-place dense transform of every species' tile: b[k][w] <- sum_j M[k][j] b[j][w].
// Mt is the transposed matrix (Mt[j*n + k] = M[k][j]) so that the threads of
// a wave read consecutive k.
template <typename T>
__device__ __forceinline__ void dense_transform(T* buf, int S, const Geom& g,
                                                const T* __restrict__ Mt) {
  const int W = g.W, n = g.n, pitch = g.pitch;
  const int KG = blockDim.x / W;
  const int w = threadIdx.x % W, kg = threadIdx.x / W;
  for (int s = 0; s < S; ++s) {
    T* b = buf + s * n * pitch;
    T acc[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) acc[q] = T(0);
    for (int j = 0; j < n; ++j) {
      const T v = b[j * pitch + w];
      const T* mr = Mt + (long long)j * n + kg;
#pragma unroll
      for (int q = 0; q < KMAX; ++q) {
        if (kg + q * KG < n) acc[q] += mr[q * KG] * v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      const int k = kg + q * KG;
      if (k < n) b[k * pitch + w] = acc[q];
    }
    __syncthreads();
  }
}

// Per-point weight of the Neumann pencil (1/2 per axis at a boundary node).
__device__ __forceinline__ double point_weight(long long idx, long long n0, long long n1,
                                               long long n2) {
  long long i0 = idx % n0;
  long long r = idx / n0;
  long long i1 = r % n1;
  long long i2 = (r / n1) % n2;  // species-split tiles index past the first species
  double w = 1.0;
  if (i0 == 0 || i0 == n0 - 1) w *= 0.5;
  if (n1 > 1 && (i1 == 0 || i1 == n1 - 1)) w *= 0.5;  // n1 = 1: the padding axis of 1D
  if (n2 > 1 && (i2 == 0 || i2 == n2 - 1)) w *= 0.5;
  return w;
}

// --------------------------------------------------------------------------
enum { MODE_INIT = 4, MODE_RESTORE = 5 };

template <typename T>
struct StageArgs {
  Geom g;
  const T* Mt;
  T* P;             // in/out fields [S][total]
  const T* src;     // Z kernel: load from here and skip the forward transform
  const T* coef;    // [6][S][total]
  const T* ltab;    // [S][total] L values: P13 coefficients formed in the combine, or null
  const T* dcoef;   // [6][S][total] (adjoint parameter sensitivities)
  T* uhat;          // forward retained arrays
  T* ctil;
  T* acc;
  T* zh;            // adjoint retained arrays
  T* aacc;
  T* ahat;
  T* gu;
  double* G;        // [S][total] L-sensitivity accumulator
  T* st_phys;       // stored stage values of this step [4][S][total]
  T* st_uhat;       // stored spectral state of this step [S][total]
  T* st_fhat;       // stored transformed reactions [4][S][total]
  double* rp_acc;   // [np][gridDim.x] reaction-parameter accumulators
  int* flag;        // set to 1 on a non-finite value
  Rxn rxn;
  double t;
  T cs;             // product of the per-axis inverse scales
  T tau;            // time step
  // L formed in the kernel from the per-axis eigenvalues (FP32 vector Z
  // kernels): L = kt_s Lambda^ha_s, Lambda the sum of the axis eigenvalues.
  const double* lam[3];
  T kt[MAX_SPECIES];  // kappa_s tau
  T ha[MAX_SPECIES];  // alpha_s / 2
  int lfly;
  int lam_off;        // byte offset of the eigenvalue tables in dynamic LDS
  double* thp;        // adjoint Z kernels on L formed in the kernel: per-block kappa and
                      // alpha gradient partials [2 S][gridDim.x], accumulated (else G)
  int S;
  // Ensembles: nmem members of one grid, launched together with
  // blockIdx.y = member. Every per-member array is [member][...] with a
  // member stride of fsz (= S total) times its per-member field count;
  // rxm holds each member's reaction constants.
  int nmem;
  long long fsz;
  const Rxn* rxm;
  int mode;         // stage 0..3, or MODE_INIT / MODE_RESTORE
  int last;         // adjoint: this is step 0 (output u-bar, not phi3 u-bar)
  int neumann;
  long long n0, n1, n2;
};

// v[s] for a run-time species index by selects, so that the kernel argument
// block is never indexed dynamically (a modified copy of it would otherwise
// be placed in scratch memory).
template <typename T>
__device__ __forceinline__ T pick_species(const T (&v)[MAX_SPECIES], int s) {
  return s == 0 ? v[0] : s == 1 ? v[1] : s == 2 ? v[2] : v[3];
}

// Ensemble member of this block (blockIdx.y): offset every per-member array
// and take the member's reaction constants. No-op for a single problem.
template <typename T>
__device__ __forceinline__ void to_member(StageArgs<T>& a) {
  if (a.nmem <= 1) return;
  const long long b = blockIdx.y;
  const long long f = b * a.fsz;
  a.P += f;
  if (a.src) a.src += f;
  if (a.coef) a.coef += NCOEF * f;
  if (a.ltab) a.ltab += f;
  if (a.dcoef) a.dcoef += NCOEF * f;
  if (a.uhat) a.uhat += f;
  if (a.ctil) a.ctil += f;
  if (a.acc) a.acc += f;
  if (a.zh) a.zh += f;
  if (a.aacc) a.aacc += f;
  if (a.ahat) a.ahat += f;
  if (a.gu) a.gu += f;
  if (a.G) a.G += f;
  if (a.st_phys) a.st_phys += 4 * f;
  if (a.st_uhat) a.st_uhat += f;
  if (a.st_fhat) a.st_fhat += 4 * f;
  if (a.rp_acc) a.rp_acc += b * MAX_PARAMS * gridDim.x;
  if (a.thp) a.thp += b * 2 * a.S * gridDim.x;
  a.rxn = a.rxm[b];
}

// ---------------------------------------------------------------- pointwise
// Each phase walks the tile's elements in the coalescing order and works on
// the LDS buffer buf[s][j][w] in place.

// Manufactured sources of Examples 1 and 2 (Section 5.1) at node idx and time
// t, in FP64: s = u_t + kappa (-Delta)^(alpha/2) u - f(u) at the exact u, with
// the fractional Laplacian of the products of cosines (sines) taken from their
// eigenvalues on the continuous domain. Constants c = p[MMS_P0..]:
//   Example 2: (alpha, K1, K2, K3, hx, hy) with K1 = 9 kappa (8 pi^2)^(alpha/2)/16,
//              K2 = 3 kappa (40 pi^2)^(alpha/2)/16, K3 = kappa (72 pi^2)^(alpha/2)/16
//   Example 1: (alpha, K1, -, K3, h) with K1 = 3 kappa (2 pi)^alpha/4,
//              K3 = kappa (6 pi)^alpha/4
__device__ __forceinline__ double mms_source(const Rxn& r, double t, long long idx,
                                             long long n0, long long n1) {
  const double* c = r.p + MMS_P0;
  const long long i0 = idx % n0;
  if (r.kind == RXN_FISHER_MMS) {
    // u = e^-t sin^3(2 pi x), sin^3 = (3 sin(2 pi x) - sin(6 pi x))/4, interior nodes
    const double x = double(i0 + 1) * c[4];
    const double s1 = sinpi(2.0 * x), s3 = sinpi(6.0 * x);
    const double e = exp(-t), s13 = s1 * s1 * s1;
    return -2.0 * e * s13 + e * (c[1] * s1 - c[3] * s3) + e * e * s13 * s13;
  }
  // u = t^alpha C(x) C(y), C = cos^3(2 pi .) = (3 cos(2 pi .) + cos(6 pi .))/4
  const long long i1 = (idx / n0) % n1;
  const double x = double(i0) * c[4], y = double(i1) * c[5];
  const double c1x = cospi(2.0 * x), c3x = cospi(6.0 * x);
  const double c1y = cospi(2.0 * y), c3y = cospi(6.0 * y);
  const double cc = c1x * c1x * c1x * c1y * c1y * c1y;
  const double phi = c[1] * c1x * c1y + c[2] * (c3x * c1y + c1x * c3y) + c[3] * c3x * c3y;
  const double ta = t > 0.0 ? pow(t, c[0]) : 0.0;
  const double dta = t > 0.0 ? c[0] * ta / t : 0.0;
  const double w = ta * cc;
  return dta * cc + ta * phi - w * (1.0 - w) * (w - 1.0);
}

// Forward reaction: buf holds the stage value (physical); replaced by f.
// Walks the LDS tile row by row (lanes w fastest); the global index is only
// formed when stage values are stored.
template <typename T, int NS, int KIND>
__device__ __forceinline__ bool pw_reaction_n(const StageArgs<T>& a, T* buf, long long tile,
                                              bool record) {
  const Geom& g = a.g;
  const TileRef tr = tile_ref(g, tile);
  const RxnT<T> rx(a.rxn);
  const int sstride = g.n * g.pitch;
  bool bad = false;
  const int ne = g.n << g.wshift;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const int j = e >> g.wshift, w = e & (g.W - 1);
    if (w >= tr.wvalid) continue;
    T* cell = buf + j * g.pitch + w;
    T u[NS], f[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) u[s] = cell[s * sstride];
    if (record) {
      const long long idx = tr.base + (long long)j * tr.rs + (long long)w * tr.cs;
#pragma unroll
      for (int s = 0; s < NS; ++s) a.st_phys[((long long)a.mode * NS + s) * g.total + idx] = u[s];
    }
    rxn_eval_k<T, NS, KIND>(rx, u, f);
    if constexpr (NS == 1 && KIND >= RXN_HUXLEY_MMS) {
      const long long idx = tr.base + (long long)j * tr.rs + (long long)w * tr.cs;
      f[0] += T(mms_source(a.rxn, a.t, idx, a.n0, a.n1));
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      bad |= !isfinite(u[s]) || !isfinite(f[s]);
      cell[s * sstride] = f[s];
    }
  }
  return bad;
}

// record: also store the stage values (a.st_phys) from this pass.
template <typename T>
__device__ __forceinline__ bool pw_reaction(const StageArgs<T>& a, T* buf, long long tile,
                                            bool record = true) {
  record = record && a.st_phys != nullptr;
  // the kind is uniform: one loop per (species count, kind), no branch inside
  switch (a.S) {
    case 1:
      switch (a.rxn.kind) {
        case RXN_LINEAR: return pw_reaction_n<T, 1, RXN_LINEAR>(a, buf, tile, record);
        case RXN_HUXLEY_MMS: return pw_reaction_n<T, 1, RXN_HUXLEY_MMS>(a, buf, tile, record);
        default: return pw_reaction_n<T, 1, RXN_FISHER_MMS>(a, buf, tile, record);
      }
    case 2:
      switch (a.rxn.kind) {
        case RXN_LINEAR: return pw_reaction_n<T, 2, RXN_LINEAR>(a, buf, tile, record);
        case RXN_FHN: return pw_reaction_n<T, 2, RXN_FHN>(a, buf, tile, record);
        case RXN_GRAY_SCOTT: return pw_reaction_n<T, 2, RXN_GRAY_SCOTT>(a, buf, tile, record);
        case RXN_SCHNAKENBERG: return pw_reaction_n<T, 2, RXN_SCHNAKENBERG>(a, buf, tile, record);
        default: return pw_reaction_n<T, 2, RXN_GM>(a, buf, tile, record);
      }
    case 3:
      return pw_reaction_n<T, 3, RXN_LINEAR>(a, buf, tile, record);
    default:
      return pw_reaction_n<T, 4, RXN_LINEAR>(a, buf, tile, record);
  }
}

// Coefficients a forward stage needs, as c0..c3, with the decrements
// dQ = 1 - Q and dR = 1 - R in place of Q and R (the combine forms Q x as
// x - dQ x, which keeps the slow modes' decay exact to the rounding of dQ):
//   stage 0: dQ, phi, dR, phi1;  stage 1: dQ, phi, phi2;  stage 2: -, phi, phi2;
//   stage 3: -, -, phi3.
template <typename T>
__device__ __forceinline__ T recip(T x) {
  return T(1) / x;
}
template <>
__device__ __forceinline__ float recip<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// P13 coefficients (Section 4) of one L in the field precision. The
// denominators D = 24 + 18L + 6L^2 + L^3 and Dh = 192 + 72L + 12L^2 + L^3 are
// sums of positive terms for L >= 0. The decrements of R13 and Q13 are, for
// L < 1,
//   1 - R13 = L (24 + 6L + L^2) / D,   1 - Q13 = L (96 + 12L + L^2) / Dh,
// exactly 0 at L = 0 (the mean of a Neumann or periodic field is not damped)
// and accurate to their own relative rounding for small L; for L >= 1 they
// are 1 minus the values (no cancellation there). FP32 tables clamp L far
// below overflow of L^3.
template <typename T>
__device__ __forceinline__ void stage_coefs_L(int mode, T L, T tau, T& c0, T& c1, T& c2, T& c3) {
  const T iD = recip<T>(T(24) + L * (T(18) + L * (T(6) + L)));
  if (mode == 3) {
    c2 = tau * (T(4) + L * (T(3) + L)) * iD;
    return;
  }
  const bool small = L < T(1);
  const T iDh = recip<T>(T(192) + L * (T(72) + L * (T(12) + L)));
  const T ph = T(96) + L * (T(12) + L);
  c1 = tau * ph * iDh;
  if (mode <= 1) c0 = small ? L * ph * iDh : T(1) - T(24) * (T(8) - L) * iDh;
  if (mode != 0) {
    c2 = T(2) * tau * (T(4) + L) * iD;
    return;
  }
  c2 = small ? L * (T(24) + L * (T(6) + L)) * iD : T(1) - (T(24) - T(6) * L) * iD;
  c3 = tau * (T(4) - L) * iD;
}

// x - d x: a coefficient near 1 applied through its decrement d (one rounding).
template <typename T>
__device__ __forceinline__ T dec_mul(T d, T x) {
  return fma(-d, x, x);
}

template <typename T>
__device__ __forceinline__ void stage_coefs_tab(int mode, const T* cf, long long cst, T& c0, T& c1,
                                                T& c2, T& c3) {
  switch (mode) {
    case 0:
      c0 = cf[C_Q * cst];
      c1 = cf[C_PHI * cst];
      c2 = cf[C_R * cst];
      c3 = cf[C_PHI1 * cst];
      break;
    case 1:
      c0 = cf[C_Q * cst];
      c1 = cf[C_PHI * cst];
      c2 = cf[C_PHI2 * cst];
      break;
    case 2:
      c1 = cf[C_PHI * cst];
      c2 = cf[C_PHI2 * cst];
      break;
    default:
      c2 = cf[C_PHI3 * cst];
      break;
  }
}

// Forward stage combine: buf holds the transformed reaction (full spectral);
// replaced by cs times the next stage's spectral value.
template <typename T>
__device__ __forceinline__ void pw_combine(const StageArgs<T>& a, T* buf, long long tile) {
  const Geom& g = a.g;
  const TileRef tr = tile_ref(g, tile);
  const int S = a.S;
  const int ne = g.n * g.W;
  const long long tot = g.total;
  const long long cst = (long long)S * tot;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    int j, w;
    unpack(g, e, j, w);
    long long idx;
    if (!elem(g, tr, j, w, idx)) continue;
    for (int s = 0; s < g.spt; ++s) {
      T& cell = buf[(s * g.n + j) * g.pitch + w];
      const T fh = cell;
      const long long i = s * tot + idx;
      T out, c0 = T(0), c1 = T(0), c2 = T(0), c3 = T(0);
      if (a.mode <= 3) {
        if (a.ltab)
          stage_coefs_L<T>(a.mode, a.ltab[i], a.tau, c0, c1, c2, c3);
        else
          stage_coefs_tab<T>(a.mode, a.coef + i, cst, c0, c1, c2, c3);
      }
      switch (a.mode) {
        case 0: {
          const T uh = a.uhat[i];
          if (a.st_uhat) a.st_uhat[i] = uh;
          if (a.st_fhat) a.st_fhat[i] = fh;
          const T av = dec_mul(c0, uh) + c1 * fh;
          a.ctil[i] = dec_mul(c0, av) - c1 * fh;
          a.acc[i] = dec_mul(c2, uh) + c3 * fh;
          out = av;
          break;
        }
        case 1: {
          if (a.st_fhat) a.st_fhat[1 * cst + i] = fh;
          const T uh = a.uhat[i];
          out = dec_mul(c0, uh) + c1 * fh;
          a.acc[i] += c2 * fh;
          break;
        }
        case 2: {
          if (a.st_fhat) a.st_fhat[2 * cst + i] = fh;
          out = a.ctil[i] + T(2) * c1 * fh;
          a.acc[i] += c2 * fh;
          break;
        }
        case 3: {
          if (a.st_fhat) a.st_fhat[3 * cst + i] = fh;
          const T un = a.acc[i] + c2 * fh;
          a.uhat[i] = un;
          out = un;
          break;
        }
        case MODE_INIT:
          a.uhat[i] = fh;
          out = fh;
          break;
        default:  // MODE_RESTORE: the tile was loaded from the spectral state
          out = fh;
          break;
      }
      cell = a.cs * out;
    }
  }
}

// Vectorised forward combine for full tiles along a strided axis: each work
// item is VW consecutive lanes of one row of one species, with all of its
// global loads issued before the arithmetic. One instance per stage.
template <typename T, int MODE, bool LT>
__device__ __forceinline__ void combine_vec(const StageArgs<T>& a, T* buf, const TileRef& tr) {
  using V = typename Vec16<T>::type;
  constexpr int VW = Vec16<T>::N;
  const Geom& g = a.g;
  const int S = a.S;
  const long long tot = g.total;
  const long long cst = (long long)S * tot;
  const int ngroups = g.n * g.W / VW;
  const T cs = a.cs;
#pragma clang loop unroll(disable)
  for (int it = threadIdx.x; it < g.spt * ngroups; it += blockDim.x) {
    const int s = it >= ngroups ? (it >= 2 * ngroups ? (it >= 3 * ngroups ? 3 : 2) : 1) : 0;
    long long gi;
    int j, w;
    vec_coords<T>(g, tr, it - s * ngroups, gi, j, w);
    const long long i = s * tot + gi;
    T* cell = buf + (s * g.n + j) * g.pitch + w;
    // global loads first
    V Lv, t0, t1, t2, t3, uh, ac, ct;
    if (LT) {
      Lv = *reinterpret_cast<const V*>(a.ltab + i);
    } else {
      const T* cf = a.coef + i;
      if (MODE <= 1) t0 = *reinterpret_cast<const V*>(cf + C_Q * cst);
      if (MODE <= 2) t1 = *reinterpret_cast<const V*>(cf + C_PHI * cst);
      t2 = *reinterpret_cast<const V*>(cf + (MODE == 0 ? C_R : MODE == 3 ? C_PHI3 : C_PHI2) * cst);
      if (MODE == 0) t3 = *reinterpret_cast<const V*>(cf + C_PHI1 * cst);
    }
    if (MODE <= 1) uh = *reinterpret_cast<const V*>(a.uhat + i);
    if (MODE >= 1) ac = *reinterpret_cast<const V*>(a.acc + i);
    if (MODE == 2) ct = *reinterpret_cast<const V*>(a.ctil + i);
    V fh, o0, o1, out;
    for (int e = 0; e < VW; ++e) vset<T>(fh, e, cell[e]);
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      T c0 = T(0), c1 = T(0), c2 = T(0), c3 = T(0);
      if (LT) {
        stage_coefs_L<T>(MODE, vget<T>(Lv, e), a.tau, c0, c1, c2, c3);
      } else {
        if (MODE <= 1) c0 = vget<T>(t0, e);
        if (MODE <= 2) c1 = vget<T>(t1, e);
        c2 = vget<T>(t2, e);
        if (MODE == 0) c3 = vget<T>(t3, e);
      }
      const T f = vget<T>(fh, e);
      if (MODE == 0) {
        const T u = vget<T>(uh, e);
        const T av = dec_mul(c0, u) + c1 * f;
        vset<T>(o0, e, dec_mul(c0, av) - c1 * f);
        vset<T>(o1, e, dec_mul(c2, u) + c3 * f);
        vset<T>(out, e, cs * av);
      } else if (MODE == 1) {
        vset<T>(out, e, cs * (dec_mul(c0, vget<T>(uh, e)) + c1 * f));
        vset<T>(o1, e, vget<T>(ac, e) + c2 * f);
      } else if (MODE == 2) {
        vset<T>(out, e, cs * (vget<T>(ct, e) + T(2) * c1 * f));
        vset<T>(o1, e, vget<T>(ac, e) + c2 * f);
      } else {
        const T un = vget<T>(ac, e) + c2 * f;
        vset<T>(o0, e, un);
        vset<T>(out, e, cs * un);
      }
    }
    if (MODE == 0) {
      if (a.st_uhat) *reinterpret_cast<V*>(a.st_uhat + i) = uh;
      *reinterpret_cast<V*>(a.ctil + i) = o0;
    }
    if (a.st_fhat) *reinterpret_cast<V*>(a.st_fhat + MODE * cst + i) = fh;
    if (MODE <= 2) *reinterpret_cast<V*>(a.acc + i) = o1;
    if (MODE == 3) *reinterpret_cast<V*>(a.uhat + i) = o0;
    for (int e = 0; e < VW; ++e) cell[e] = vget<T>(out, e);
  }
}

// Forward combine of a tile; full tiles along strided axes move in vectors.
template <typename T>
__device__ __forceinline__ void pw_combine_fast(const StageArgs<T>& a, T* buf, long long tile) {
  const Geom& g = a.g;
  const TileRef tr = tile_ref(g, tile);
  if (g.inner == 1 || a.mode > 3 || !tile_vectorizable<T>(g, tr, a.uhat)) {
    pw_combine(a, buf, tile);
    return;
  }
  const bool lt = a.ltab != nullptr;
  switch (a.mode) {
    case 0:
      lt ? combine_vec<T, 0, true>(a, buf, tr) : combine_vec<T, 0, false>(a, buf, tr);
      break;
    case 1:
      lt ? combine_vec<T, 1, true>(a, buf, tr) : combine_vec<T, 1, false>(a, buf, tr);
      break;
    case 2:
      lt ? combine_vec<T, 2, true>(a, buf, tr) : combine_vec<T, 2, false>(a, buf, tr);
      break;
    default:
      lt ? combine_vec<T, 3, true>(a, buf, tr) : combine_vec<T, 3, false>(a, buf, tr);
      break;
  }
}

// Adjoint reaction: buf holds the cotangent of f(stage value) (physical);
// replaced by J^T of it at the stored stage value. Reaction-parameter
// partials are added to pacc (weighted by the Neumann point weights).
template <typename T, int NS, int KIND>
__device__ __forceinline__ void pw_adj_reaction_n(const StageArgs<T>& a, T* buf, long long tile,
                                                  double* pacc) {
  const Geom& g = a.g;
  const TileRef tr = tile_ref(g, tile);
  const bool want_p = a.rp_acc != nullptr;
  const int ne = g.n * g.W;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    int j, w;
    unpack(g, e, j, w);
    long long idx;
    if (!elem(g, tr, j, w, idx)) continue;
    T u[NS], gg[NS], o[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      gg[s] = buf[(s * g.n + j) * g.pitch + w];
      u[s] = a.st_phys[((long long)a.mode * NS + s) * g.total + idx];
    }
    const double wgt = a.neumann ? point_weight(idx, a.n0, a.n1, a.n2) : 1.0;
    rxn_adjoint_k<T, NS, KIND>(a.rxn, u, gg, o, wgt, pacc, want_p);
#pragma unroll
    for (int s = 0; s < NS; ++s) buf[(s * g.n + j) * g.pitch + w] = o[s];
  }
}

template <typename T>
__device__ __forceinline__ void pw_adj_reaction(const StageArgs<T>& a, T* buf, long long tile,
                                                double* pacc) {
  // the kind is uniform: one loop per (species count, kind)
  switch (a.S) {
    case 1:
      switch (a.rxn.kind) {
        case RXN_LINEAR: pw_adj_reaction_n<T, 1, RXN_LINEAR>(a, buf, tile, pacc); break;
        case RXN_HUXLEY_MMS: pw_adj_reaction_n<T, 1, RXN_HUXLEY_MMS>(a, buf, tile, pacc); break;
        default: pw_adj_reaction_n<T, 1, RXN_FISHER_MMS>(a, buf, tile, pacc); break;
      }
      break;
    case 2:
      switch (a.rxn.kind) {
        case RXN_LINEAR: pw_adj_reaction_n<T, 2, RXN_LINEAR>(a, buf, tile, pacc); break;
        case RXN_FHN: pw_adj_reaction_n<T, 2, RXN_FHN>(a, buf, tile, pacc); break;
        case RXN_GRAY_SCOTT: pw_adj_reaction_n<T, 2, RXN_GRAY_SCOTT>(a, buf, tile, pacc); break;
        case RXN_SCHNAKENBERG: pw_adj_reaction_n<T, 2, RXN_SCHNAKENBERG>(a, buf, tile, pacc); break;
        default: pw_adj_reaction_n<T, 2, RXN_GM>(a, buf, tile, pacc); break;
      }
      break;
    case 3:
      pw_adj_reaction_n<T, 3, RXN_LINEAR>(a, buf, tile, pacc);
      break;
    default:
      pw_adj_reaction_n<T, 4, RXN_LINEAR>(a, buf, tile, pacc);
      break;
  }
}

// Adjoint combine. Cotangents are carried in the variables for which the
// transposed transforms are the forward ones (physical cotangents divided by
// the Neumann point weights, spectral ones by the inverse scale and spectral
// weights). With z = cotangent of the step output and X the incoming term:
//   st 0 (c): aacc = R z; ahat = Q X; gu = phi1 z - phi X; out = phi2 z + 2 phi X
//   st 1 (b): aacc += Q X; out = phi2 z + phi X
//   st 2 (a): A = ahat + X; aacc += Q A; out = gu + phi A
//   st 3 (u): z <- aacc + X; out = phi3 z (or z itself at the first step)
// R and Q are applied through the tables' decrements 1 - R, 1 - Q as in the
// forward combine. G accumulates, per mode, y * g'(L) * x over every
// coefficient application y_out = g(L) x of the forward step, for the kappa
// and alpha gradients.
// The adjoint's coefficient table values from L in FP64 (P13, Section 4's
// rational forms; the C_R and C_Q slots hold the decrements 1 - R and 1 - Q,
// as the tables do) and the derivatives in L of the coefficients themselves
// (quotient rule, g' = (num' - g den') / den, D' = 18 + 12L + 3L^2,
// Dh' = 72 + 24L + 3L^2).
__device__ __forceinline__ void p13_table_derivs(double L, double tau, double* c, double* d) {
  const double D = 24.0 + L * (18.0 + L * (6.0 + L));
  const double Dh = 192.0 + L * (72.0 + L * (12.0 + L));
  const double iD = 1.0 / D, iDh = 1.0 / Dh;
  const double R = (24.0 - 6.0 * L) * iD, Q = (192.0 - 24.0 * L) * iDh;
  const bool small = L < 1.0;
  c[C_R] = small ? L * (24.0 + L * (6.0 + L)) * iD : 1.0 - R;
  c[C_Q] = small ? L * (96.0 + L * (12.0 + L)) * iDh : 1.0 - Q;
  c[C_PHI] = tau * (96.0 + L * (12.0 + L)) * iDh;
  c[C_PHI1] = tau * (4.0 - L) * iD;
  c[C_PHI2] = tau * (8.0 + 2.0 * L) * iD;
  c[C_PHI3] = tau * (4.0 + L * (3.0 + L)) * iD;
  const double dD = 18.0 + L * (12.0 + 3.0 * L), dDh = 72.0 + L * (24.0 + 3.0 * L);
  d[C_R] = (-6.0 - R * dD) * iD;
  d[C_Q] = (-24.0 - Q * dDh) * iDh;
  d[C_PHI] = (tau * (12.0 + 2.0 * L) - c[C_PHI] * dDh) * iDh;
  d[C_PHI1] = (-tau - c[C_PHI1] * dD) * iD;
  d[C_PHI2] = (2.0 * tau - c[C_PHI2] * dD) * iD;
  d[C_PHI3] = (tau * (3.0 + 2.0 * L) - c[C_PHI3] * dD) * iD;
}

template <typename T>
__device__ __forceinline__ void pw_adj_combine(const StageArgs<T>& a, T* buf, long long tile) {
  const Geom& g = a.g;
  const TileRef tr = tile_ref(g, tile);
  const int S = a.S;
  const int ne = g.n * g.W;
  const long long tot = g.total;
  const long long cst = (long long)S * tot;
  // FP64 P13 plans: the coefficients and their derivatives formed from L
  // (one table read per point instead of up to eleven)
  const bool from_l = std::is_same<T, double>::value && a.ltab != nullptr;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    int j, w;
    unpack(g, e, j, w);
    long long idx;
    if (!elem(g, tr, j, w, idx)) continue;
    for (int s = 0; s < g.spt; ++s) {
      T& cell = buf[(s * g.n + j) * g.pitch + w];
      const T X = cell;
      const long long i = s * tot + idx;
      const T* cf = a.coef + i;
      const T* dc = a.dcoef ? a.dcoef + i : nullptr;
      double cl[NCOEF], dl[NCOEF];
      if (from_l) p13_table_derivs(double(a.ltab[i]), double(a.tau), cl, dl);
      auto C = [&](int q) -> T { return from_l ? T(cl[q]) : cf[q * cst]; };
      auto Dq = [&](int q) -> T { return from_l ? T(dl[q]) : dc[q * cst]; };
      T out;
      switch (a.mode) {
        case 0: {
          const T z = a.zh[i];
          const T dQ = C(C_Q), cP = C(C_PHI);
          a.aacc[i] = dec_mul(C(C_R), z);
          a.ahat[i] = dec_mul(dQ, X);
          a.gu[i] = C(C_PHI1) * z - cP * X;
          out = C(C_PHI2) * z + T(2) * cP * X;
          if (a.G) {
            const T uh = a.st_uhat[i];
            const T fu = a.st_fhat[0 * cst + i], fa = a.st_fhat[1 * cst + i];
            const T fb = a.st_fhat[2 * cst + i], fc = a.st_fhat[3 * cst + i];
            const T ah = dec_mul(dQ, uh) + cP * fu;
            const T s1 = Dq(C_R) * uh + Dq(C_PHI1) * fu + Dq(C_PHI2) * (fa + fb) + Dq(C_PHI3) * fc;
            const T s2 = Dq(C_Q) * ah + Dq(C_PHI) * (T(2) * fb - fu);
            a.G[i] += double(z) * double(s1) + double(X) * double(s2);
          }
          break;
        }
        case 1: {
          const T z = a.zh[i];
          a.aacc[i] += dec_mul(C(C_Q), X);
          out = C(C_PHI2) * z + C(C_PHI) * X;
          if (a.G) {
            const T uh = a.st_uhat[i], fa = a.st_fhat[1 * cst + i];
            a.G[i] += double(X) * double(Dq(C_Q) * uh + Dq(C_PHI) * fa);
          }
          break;
        }
        case 2: {
          const T A = a.ahat[i] + X;
          a.aacc[i] += dec_mul(C(C_Q), A);
          out = a.gu[i] + C(C_PHI) * A;
          if (a.G) {
            const T uh = a.st_uhat[i], fu = a.st_fhat[0 * cst + i];
            a.G[i] += double(A) * double(Dq(C_Q) * uh + Dq(C_PHI) * fu);
          }
          break;
        }
        case 3: {
          const T zn = a.aacc[i] + X;
          a.zh[i] = zn;
          out = a.last ? zn : C(C_PHI3) * zn;
          break;
        }
        default:  // MODE_INIT: X is the transformed cotangent of u(T)
          a.zh[i] = X;
          out = C(C_PHI3) * X;
          break;
      }
      cell = a.cs * out;
    }
  }
}

// Block sums of the first m of v[0..M): out[k][blockIdx.x] (row stride
// gridDim.x) receives, or with `accumulate` gains, the sum of v[k] over the
// block. Each wave sums by lane exchanges (fixed order), then one thread per
// value adds the wave sums in wave order: two barriers in all, rather than one
// per halving step of an LDS tree. red: LDS of m * blockDim.x / 64 doubles,
// free for reuse (the caller's last LDS accesses precede the first barrier).
template <int M>
__device__ __forceinline__ void block_sums(double* red, const double (&v)[M], int m, double* out,
                                           bool accumulate) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < M; ++k) {
    if (k >= m) break;
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[k * nw + wid] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < m) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[threadIdx.x * nw + w];
    double* o = out + (long long)threadIdx.x * gridDim.x + blockIdx.x;
    *o = accumulate ? *o + t : t;
  }
}

// Block-wide sum of pacc[0..np) added to rp_acc[k][blockIdx.x] (fixed order).
__device__ __forceinline__ void block_add_partials(double* red, const double (&pacc)[RXN_NP_MAX],
                                                   int np, double* rp_acc) {
  block_sums(red, pacc, np, rp_acc, true);
}

// ---------------------------------------------------------------- tile bodies
// XF is the per-axis transform applied in place to every species' tile. FAST:
// full tiles move in 16-byte vectors with every load of a thread issued
// before its first use, and the combine runs on vectors of strided tiles.
template <bool FAST, typename T>
__device__ __forceinline__ void tile_in(const Geom& g, long long tile, const T* src, T* buf, int S) {
  if (FAST)
    load_tile_fast(g, tile, src, buf, S);
  else
    load_tile(g, tile, src, buf, S);
}

template <bool FAST, typename T>
__device__ __forceinline__ void tile_out(const Geom& g, long long tile, const T* buf, T* dst, int S) {
  if (FAST)
    store_tile_fast(g, tile, buf, dst, S);
  else
    store_tile(g, tile, buf, dst, S);
}

template <bool FAST, typename T, class XF>
__device__ __forceinline__ void body_x(const StageArgs<T>& a, T* buf, long long tile, XF& xf) {
  tile_in<FAST>(a.g, tile, a.P, buf, a.g.spt);
  __syncthreads();
  xf(buf, a.g.spt);
  const bool bad = pw_reaction(a, buf, tile);
  if (bad) a.flag[0] = 1;
  __syncthreads();
  xf(buf, a.g.spt);
  tile_out<FAST>(a.g, tile, buf, a.P, a.g.spt);
}

template <bool FAST, typename T, class XF>
__device__ __forceinline__ void body_z(const StageArgs<T>& a, T* buf, long long tile, XF& xf) {
  tile_in<FAST>(a.g, tile, a.src ? a.src : a.P, buf, a.g.spt);
  __syncthreads();
  if (!a.src) xf(buf, a.g.spt);
  if (FAST)
    pw_combine_fast(a, buf, tile);
  else
    pw_combine(a, buf, tile);
  __syncthreads();
  xf(buf, a.g.spt);
  tile_out<FAST>(a.g, tile, buf, a.P, a.g.spt);
}

template <bool FAST, typename T, class XF>
__device__ __forceinline__ void body_xadj(const StageArgs<T>& a, T* buf, long long tile, XF& xf,
                                          double* pacc) {
  tile_in<FAST>(a.g, tile, a.P, buf, a.g.spt);
  __syncthreads();
  xf(buf, a.g.spt);
  pw_adj_reaction(a, buf, tile, pacc);
  __syncthreads();
  xf(buf, a.g.spt);
  tile_out<FAST>(a.g, tile, buf, a.P, a.g.spt);
}

template <bool FAST, typename T, class XF>
__device__ __forceinline__ void body_zadj(const StageArgs<T>& a, T* buf, long long tile, XF& xf) {
  tile_in<FAST>(a.g, tile, a.P, buf, a.g.spt);
  __syncthreads();
  xf(buf, a.g.spt);
  pw_adj_combine(a, buf, tile);
  __syncthreads();
  xf(buf, a.g.spt);
  tile_out<FAST>(a.g, tile, buf, a.P, a.g.spt);
}

// Dense transform as a functor (one tile per block).
template <typename T>
struct DenseXf {
  const Geom* g;
  const T* Mt;
  __device__ __forceinline__ void operator()(T* buf, int S) { dense_transform(buf, S, *g, Mt); }
};

// X kernel, forward: inverse-x, reaction, forward-x (in place on P).
template <typename T, template <typename> class XFT = DenseXf, bool FAST = false>
__global__ __launch_bounds__(NTHREADS) void k_xstage(StageArgs<T> a) {
  to_member(a);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  XFT<T> xf{&a.g, a.Mt};
  body_x<FAST>(a, reinterpret_cast<T*>(smem_raw), blockIdx.x, xf);
}

// Z kernel, forward: forward transform along the last axis, stage combine,
// inverse transform (in place on P).
template <typename T, template <typename> class XFT = DenseXf, bool FAST = false>
__global__ __launch_bounds__(NTHREADS) void k_zstage(StageArgs<T> a) {
  to_member(a);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  XFT<T> xf{&a.g, a.Mt};
  body_z<FAST>(a, reinterpret_cast<T*>(smem_raw), blockIdx.x, xf);
}

// X kernel, adjoint: inverse-x of the spectral cotangent of f(stage value),
// transposed reaction Jacobian at the stored stage value, forward-x.
template <typename T, template <typename> class XFT = DenseXf, bool FAST = false>
__global__ __launch_bounds__(NTHREADS) void k_xadj(StageArgs<T> a) {
  to_member(a);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  XFT<T> xf{&a.g, a.Mt};
  double pacc[RXN_NP_MAX];
  for (int k = 0; k < RXN_NP_MAX; ++k) pacc[k] = 0.0;
  body_xadj<FAST>(a, reinterpret_cast<T*>(smem_raw), blockIdx.x, xf, pacc);
  if (a.rp_acc) {
    __syncthreads();
    block_add_partials(reinterpret_cast<double*>(smem_raw), pacc, a.rxn.np, a.rp_acc);
  }
}

// Z kernel, adjoint: forward-z, adjoint combine, inverse-z.
template <typename T, template <typename> class XFT = DenseXf, bool FAST = false>
__global__ __launch_bounds__(NTHREADS) void k_zadj(StageArgs<T> a) {
  to_member(a);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  XFT<T> xf{&a.g, a.Mt};
  body_zadj<FAST>(a, reinterpret_cast<T*>(smem_raw), blockIdx.x, xf);
}

// One transform along one axis, src -> dst (may alias), with optional
// Neumann point weights before (divide) or after (multiply).
template <typename T>
struct SingleArgs {
  Geom g;
  const T* Mt;
  const T* src;
  T* dst;
  int S;
  int pre_divide_w;
  int post_multiply_w;
  int nmem;         // ensemble members (blockIdx.y), fields [member][S][total]
  long long fsz;    // S total
  long long n0, n1, n2;
};

// Ensemble member of this block: offset the member's arrays (no-op for one).
template <typename T>
__device__ __forceinline__ void to_member(SingleArgs<T>& a) {
  if (a.nmem <= 1) return;
  const long long f = (long long)blockIdx.y * a.fsz;
  a.src += f;
  a.dst += f;
}

template <typename T, template <typename> class XFT = DenseXf, bool FAST = false>
__global__ __launch_bounds__(NTHREADS) void k_single(SingleArgs<T> a) {
  to_member(a);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  const Geom& g = a.g;
  const long long tile = blockIdx.x;
  const TileRef tr = tile_ref(g, tile);
  // tiles hold g.spt species (strided axes may hold one, with the species
  // index in the outer block)
  const int S = g.spt;
  tile_in<FAST>(g, tile, a.src, buf, S);
  __syncthreads();
  const int ne = g.n * g.W;
  if (a.pre_divide_w) {
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      int j, w;
      unpack(g, e, j, w);
      long long idx;
      if (!elem(g, tr, j, w, idx)) continue;
      const T wt = T(point_weight(idx, a.n0, a.n1, a.n2));
      for (int s = 0; s < S; ++s) buf[(s * g.n + j) * g.pitch + w] /= wt;
    }
    __syncthreads();
  }
  XFT<T>{&g, a.Mt}(buf, S);
  if (a.post_multiply_w) {
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      int j, w;
      unpack(g, e, j, w);
      long long idx;
      if (!elem(g, tr, j, w, idx)) continue;
      const T wt = T(point_weight(idx, a.n0, a.n1, a.n2));
      for (int s = 0; s < S; ++s) buf[(s * g.n + j) * g.pitch + w] *= wt;
    }
    __syncthreads();
  }
  tile_out<FAST>(g, tile, buf, a.dst, S);
}

// --------------------------------------------------------------------------
// Plan-time coefficient tables in FP64 (Alg. 1 precompute), stored in T:
// out[q][s][idx] for the six functions of L = kappa_s tau Lambda^(alpha_s/2),
// Lambda = lam0[i0] + lam1[i1] + lam2[i2], or their d/dL when deriv != 0.
struct CoefArgs {
  const double* lam0;
  const double* lam1;
  const double* lam2;
  long long n0, n1, n2, total;
  int S;
  int scheme;
  int deriv;
  int pad_;
  double tau;
  double alpha[MAX_SPECIES];
  double kappa[MAX_SPECIES];
};

__device__ __forceinline__ double lambda_at(const CoefArgs& c, long long idx) {
  long long i0 = idx % c.n0;
  long long r = idx / c.n0;
  long long i1 = r % c.n1;
  long long i2 = r / c.n1;
  double lam = c.lam0[i0] + c.lam1[i1];
  if (c.n2 > 1) lam += c.lam2[i2];
  return lam;
}

template <typename T>
__global__ void k_coefs(CoefArgs c, T* out) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < c.total;
       idx += (long long)gridDim.x * blockDim.x) {
    const double lam = lambda_at(c, idx);
    for (int s = 0; s < c.S; ++s) {
      const double L = lam > 0.0 ? c.kappa[s] * c.tau * pow(lam, 0.5 * c.alpha[s]) : 0.0;
      if (c.deriv == 2) {
        // L itself. FP32 tables clamp it at 1e12 so that L^3 stays finite;
        // there every P13 coefficient is at most about tau / L, far below
        // the FP32 resolution of the terms it is added to.
        const double Lc = sizeof(T) == 4 && L > 1e12 ? 1e12 : L;
        out[(long long)s * c.total + idx] = T(Lc);
        continue;
      }
      double v[NCOEF];
      if (c.deriv)
        coef_derivs(c.scheme, L, c.tau, v);
      else
        coef_table_values(c.scheme, L, c.tau, v);
      for (int q = 0; q < NCOEF; ++q) out[((long long)q * c.S + s) * c.total + idx] = T(v[q]);
    }
  }
}

// kappa/alpha gradients from the per-mode sensitivities G:
// part[q][block], q = 2s (kappa_s) and 2s+1 (alpha_s), of
// sum_k omega_k G_k dL_k/dtheta with dL/dkappa = tau Lambda^(alpha/2),
// dL/dalpha = L ln(Lambda)/2 and omega_k = cs * (Neumann spectral weights).
__global__ void k_greduce(CoefArgs c, const double* G, double cs, int neumann, double* part) {
  __shared__ double red[NTHREADS];
  double acc[2 * MAX_SPECIES];
  for (int q = 0; q < 2 * MAX_SPECIES; ++q) acc[q] = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < c.total;
       idx += (long long)gridDim.x * blockDim.x) {
    const double lam = lambda_at(c, idx);
    if (!(lam > 0.0)) continue;
    const double om = cs * (neumann ? point_weight(idx, c.n0, c.n1, c.n2) : 1.0);
    const double lnl = log(lam);
    for (int s = 0; s < c.S; ++s) {
      const double pw = pow(lam, 0.5 * c.alpha[s]);
      const double gk = om * G[(long long)s * c.total + idx];
      acc[2 * s] += gk * c.tau * pw;
      acc[2 * s + 1] += gk * 0.5 * c.kappa[s] * c.tau * pw * lnl;
    }
  }
  block_sums(red, acc, 2 * c.S, part, false);
}

// out[r] = sum over in[r][0..len) in a fixed order (one block per row).
__global__ void k_rowsum(const double* in, long long len, double* out) {
  __shared__ double red[NTHREADS];
  const double* row = in + blockIdx.x * len;
  double a = 0.0;
  for (long long i = threadIdx.x; i < len; i += blockDim.x) a += row[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

template <typename T>
__global__ void k_fill(T* p, long long n, T v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// Checkpoint header: CKPT_WORDS 64-bit words passed by value, lane i writes
// word i.
constexpr int CKPT_WORDS = 12;
struct CkptHeader {
  long long w[CKPT_WORDS];
};
__global__ void k_header(long long* h, CkptHeader v) {
  const int i = threadIdx.x;
  if (blockIdx.x == 0 && i < CKPT_WORDS) h[i] = v.w[i];
}

}  // namespace sfrde
