// Per-axis transforms on the matrix cores (gfx950 MFMA).
//
// Each axis matrix M (n x n, see kernels.h) has a reflection symmetry: with
// r(j) the mirrored index, M[k][r(j)] = +-M[k][j] (DCT-I, DST-I: sign (-1)^k),
// or M = C + S with C even and S odd under r (Hartley). Folding the input,
//   s_i = x[a_i] + x[b_i],  d_i = x[a_i] - x[b_i]   (pairs a_i, b_i = r(a_i)),
// splits the product into two half-size dense products E s and O d, and the
// outputs are recovered by an unfold: y_2m = (Es)_m, y_2m+1 = (Od)_m for
// DCT/DST, y_k = (Es)_k + (Od)_k and y_{N-k} = (Es)_k - (Od)_k for Hartley.
// That halves the multiply-adds of the dense product.
//
// The half-size matrices live in registers of a persistent block of 16
// waves: wave w owns 16 rows of E (w < RBe) or of O, for all K. Per tile of
// W lines the block folds the data in LDS, each wave runs its row block over
// all lines, results go back to LDS and are unfolded into the tile.
//
// FP32 fields: products on v_mfma_f32_16x16x32_f16 with both operands split
// into two binary16 terms after a per-column power-of-two scaling, three
// products accumulated in FP32: about the accuracy of an FP32 product.
// FP64 fields: v_mfma_f64_16x16x4_f64 on the unsplit values.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sfrde {

constexpr int MF_THREADS = 1024;  // 16 waves
constexpr int MF_WAVES = 16;
constexpr int MF_KSMAX_F32 = 4;   // K <= 128 in steps of 32
constexpr int MF_KSMAX_F64 = 32;  // K <= 128 in steps of 4

struct MfmaAxisDev {
  const void* Afrag;      // fragment-ordered half matrices
  int n;                  // axis length
  int ns;                 // folded entries (pairs and fixed points)
  int periodic;           // Hartley fold (else DCT-I / DST-I)
  int hK;                 // folded length (multiple of 32)
  int RBe;                // 16-row blocks of E
  int RB;                 // 16-row blocks of E and O (<= 16)
  int fb_pitch;           // row pitch of the fold buffer (elements)
  int r_pitch;            // row pitch of the result buffer (elements)
  int fb_off;             // byte offset of the fold/result area in LDS
  int direct;             // unfold is the even/odd row interleave (DCT-I, DST-I)
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Fold entry i: s_i = x[a] + x[b], d_i = x[a] - x[b]; b < 0 for a fixed point
// of the reflection (d_i = 0), a < 0 for padding (s_i = d_i = 0).
//   DCT-I / DST-I: pairs (i, n-1-i) for 2i+1 < n; the middle index when n is odd.
//   Hartley (N = n): 0 and N/2 are fixed; pairs (i, N-i) otherwise.
__device__ __forceinline__ void fold_pair(const MfmaAxisDev& ax, int i, int& a, int& b) {
  if (i >= ax.ns) {
    a = -1;
    b = -1;
    return;
  }
  a = i;
  if (!ax.periodic)
    b = 2 * i + 1 < ax.n ? ax.n - 1 - i : -1;
  else
    b = (i == 0 || 2 * i == ax.n) ? -1 : ax.n - i;
}

// Fold every line of one species' tile into fb: s rows then d rows, each
// [W][fb_pitch], eight consecutive i per work item.
template <typename T, int W>
__device__ __forceinline__ void mf_fold(const T* x, int pitch, const MfmaAxisDev& ax, T* fb) {
  const int items = W * (ax.hK / 8);
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int col = it % W;
    const int i0 = (it / W) * 8;
    T sv[8], dv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int a, b;
      fold_pair(ax, i0 + e, a, b);
      const T xa = a >= 0 ? x[a * pitch + col] : T(0);
      const T xb = b >= 0 ? x[b * pitch + col] : T(0);
      sv[e] = xa + xb;
      dv[e] = b >= 0 ? xa - xb : T(0);
    }
    T* ps = fb + col * ax.fb_pitch + i0;
    T* pd = fb + (W + col) * ax.fb_pitch + i0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      ps[e] = sv[e];
      pd[e] = dv[e];
    }
  }
}

// Hartley unfold of the result rows R[row][col] into the tile x[k][col]:
// y_k = E_k + O_k for k <= N/2, y_k = E_{N-k} - O_{N-k} above.
template <typename T, int W>
__device__ __forceinline__ void mf_unfold(const T* R, const MfmaAxisDev& ax, int n, T* x, int pitch) {
  const int ne = n * W;
  const int obase = 16 * ax.RBe;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const int k = e / W, col = e - k * W;
    const bool low = 2 * k <= n;
    const int kk = low ? k : n - k;
    const T ev = R[kk * ax.r_pitch + col], ov = R[(obase + kk) * ax.r_pitch + col];
    x[k * pitch + col] = low ? ev + ov : ev - ov;
  }
}

// ------------------------------------------------------------------ FP32
// Products on v_mfma_f32_16x16x32_f16. Both operands are split into two
// binary16 terms, v = v0 + v1 with v0 the rounding of v and v1 the rounding
// of what is left, and the three products A0 X0 + A0 X1 + A1 X0 are
// accumulated in FP32 (the dropped A1 X1 is below 2^-22 of the column
// scale). The matrices hold bounded entries (|a| <= sqrt 2); each folded data
// column is scaled by a power of two that puts its largest magnitude in
// [2^14, 2^15), so neither term leaves the binary16 range, and the results
// are scaled back exactly.
//
// Fold buffer (LDS, binary16 bits): [term][half s|d][col][F32_FBP], then the
// W inverse column scales as floats. F32_FBP = 136 leaves room for folded
// lengths up to 128 and keeps the 16-byte accesses free of bank conflicts.
constexpr int F32_FBP = 136;
constexpr int f32_fold_bytes(int W) { return 2 * 2 * W * F32_FBP * 2 + W * 4; }

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

// Two scaled floats -> packed binary16 head and tail terms.
__device__ __forceinline__ void split2_f16(float x0, float x1, float sc, unsigned& t0,
                                           unsigned& t1) {
  const f2v x = {x0 * sc, x1 * sc};
  const h2v a = __builtin_convertvector(x, h2v);
  const f2v r = x - __builtin_convertvector(a, f2v);
  const h2v b = __builtin_convertvector(r, h2v);
  t0 = __builtin_bit_cast(unsigned, a);
  t1 = __builtin_bit_cast(unsigned, b);
}

// Maximum over the 16 lanes of a DPP row (lanes 16r .. 16r+15).
__device__ __forceinline__ float row16_max(float m) {
  m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                             0, __builtin_bit_cast(int, m), 0x128, 0xf, 0xf, false)));
  m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                             0, __builtin_bit_cast(int, m), 0x124, 0xf, 0xf, false)));
  m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                             0, __builtin_bit_cast(int, m), 0x122, 0xf, 0xf, false)));
  m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                             0, __builtin_bit_cast(int, m), 0x121, 0xf, 0xf, false)));
  return m;
}

// Eight waves; wave w owns row blocks 2w and 2w + 1 (of E, then of O), so
// two 512-thread blocks share a CU and one block's memory waits overlap the
// other's arithmetic. W = 32 lines for strided axes (128-byte rows), 16 for
// the contiguous x axis (whose tiles hold every species).
template <int W_>
struct MfmaXfF32 {
  static constexpr int W = W_;
  static constexpr int THREADS = 512;
  static constexpr int P = W + 1;             // LDS row pitch of the tile
  static constexpr int FBP = F32_FBP;
  static constexpr int TS = 2 * W * F32_FBP;  // binary16 elements between the two terms
  static constexpr int FOLD_THREADS = 16 * W; // one 16-lane row per column
  static constexpr int CB = W / 16;           // 16-column blocks
  const MfmaAxisDev* ax;
  unsigned short* fb;
  float* scl;  // inverse column scales
  f16x8 A[2][MF_KSMAX_F32][2];
  int n, KS;
  int nrb;      // row blocks of this wave (0..2)
  bool shareB;  // both row blocks read the same fold half
  bool direct;
  int bofs[2];  // B-fragment offsets in fb per row block
  // fold work item of this thread: column col, entries i0 .. i0+7
  bool ffast;
  int i0, col, fa, fbb;
  // output rows of this lane's results (direct unfold), per row block
  int xrow[2], rmask[2];

  __device__ __forceinline__ MfmaXfF32(const Geom*, const MfmaAxisDev* ax_, float* fb_)
      : ax(ax_), fb(reinterpret_cast<unsigned short*>(fb_)) {
    scl = reinterpret_cast<float*>(fb + 2 * TS);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    n = ax->n;
    KS = ax->hK >> 5;
    direct = ax->direct != 0;
    const int rb0 = 2 * wave;
    nrb = ax->RB - rb0;
    nrb = nrb < 0 ? 0 : (nrb > 2 ? 2 : nrb);
    const uint4* src = reinterpret_cast<const uint4*>(ax->Afrag);
    bool isO[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rb = rb0 + h;
#pragma unroll
      for (int ks = 0; ks < MF_KSMAX_F32; ++ks)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          uint4 v = make_uint4(0, 0, 0, 0);
          if (h < nrb) v = src[((rb * MF_KSMAX_F32 + ks) * 2 + t) * 64 + lane];
          A[h][ks][t] = __builtin_bit_cast(f16x8, v);
        }
      isO[h] = rb >= ax->RBe;
      bofs[h] = ((isO[h] ? W : 0) + lane % 16) * FBP + 8 * (lane / 16);
      // direct unfold: E row m -> output 2m, O row m -> output 2m + 1
      const int mb = 16 * (isO[h] ? rb - ax->RBe : rb) + 4 * (lane / 16);
      const int row0 = 2 * mb + (isO[h] ? 1 : 0);
      xrow[h] = row0 * P + lane % 16;
      rmask[h] = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (h < nrb && row0 + 2 * r < n) rmask[h] |= 1 << r;
    }
    shareB = nrb < 2 || isO[0] == isO[1];
    // fold item; entries past the folded length come out as zeros
    col = (threadIdx.x >> 4) & (W - 1);
    i0 = (threadIdx.x & 15) << 3;
    const int bstart = ax->periodic ? n : n - 1;  // partner of entry i is bstart - i
    ffast = ax->periodic ? (i0 >= 1 && 2 * (i0 + 7) < n) : (2 * (i0 + 7) + 1 < n);
    fa = i0 * P + col;
    fbb = (bstart - i0) * P + col;
  }

  __device__ __forceinline__ void fold(const float* x) {
    if ((int)threadIdx.x >= FOLD_THREADS) return;
    float sv[8], dv[8];
    if (ffast) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float xa = x[fa + e * P], xb = x[fbb - e * P];
        sv[e] = xa + xb;
        dv[e] = xa - xb;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        int a, b;
        fold_pair(*ax, i0 + e, a, b);
        const float xa = a >= 0 ? x[a * P + col] : 0.f;
        const float xb = b >= 0 ? x[b * P + col] : 0.f;
        sv[e] = xa + xb;
        dv[e] = b >= 0 ? xa - xb : 0.f;
      }
    }
    float m = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) m = fmaxf(m, fmaxf(fabsf(sv[e]), fabsf(dv[e])));
    m = row16_max(m);
    int k = 15 - __builtin_amdgcn_frexp_expf(m);
    k = k < -126 ? -126 : (k > 126 ? 126 : k);
    const float sc = __builtin_amdgcn_ldexpf(1.f, k);
    if ((threadIdx.x & 15) == 0) scl[col] = __builtin_amdgcn_ldexpf(1.f, -k);
    unsigned s0[4], s1[4], d0[4], d1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      split2_f16(sv[2 * q], sv[2 * q + 1], sc, s0[q], s1[q]);
      split2_f16(dv[2 * q], dv[2 * q + 1], sc, d0[q], d1[q]);
    }
    unsigned short* ps = fb + col * FBP + i0;
    unsigned short* pd = ps + W * FBP;
    *reinterpret_cast<uint4*>(ps) = make_uint4(s0[0], s0[1], s0[2], s0[3]);
    *reinterpret_cast<uint4*>(ps + TS) = make_uint4(s1[0], s1[1], s1[2], s1[3]);
    *reinterpret_cast<uint4*>(pd) = make_uint4(d0[0], d0[1], d0[2], d0[3]);
    *reinterpret_cast<uint4*>(pd + TS) = make_uint4(d1[0], d1[1], d1[2], d1[3]);
  }

  __device__ __forceinline__ static f16x8 frag(const unsigned short* p) {
    return __builtin_bit_cast(f16x8, *reinterpret_cast<const uint4*>(p));
  }

  __device__ __forceinline__ void products(f32x4 (&acc)[2][CB]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[h][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (nrb == 0) return;
#pragma unroll
    for (int ks = 0; ks < MF_KSMAX_F32; ++ks) {
      if (ks >= KS) break;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int off = 16 * cb * FBP + 32 * ks;
        f16x8 b0 = frag(fb + bofs[0] + off), b1 = frag(fb + bofs[0] + off + TS);
        acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0][ks][1], b0, acc[0][cb], 0, 0, 0);
        acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0][ks][0], b1, acc[0][cb], 0, 0, 0);
        acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0][ks][0], b0, acc[0][cb], 0, 0, 0);
        if (nrb == 2) {
          if (!shareB) {
            b0 = frag(fb + bofs[1] + off);
            b1 = frag(fb + bofs[1] + off + TS);
          }
          acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[1][ks][1], b0, acc[1][cb], 0, 0, 0);
          acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[1][ks][0], b1, acc[1][cb], 0, 0, 0);
          acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[1][ks][0], b0, acc[1][cb], 0, 0, 0);
        }
      }
    }
    const int lane = threadIdx.x % 64;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const float inv = scl[16 * cb + lane % 16];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[h][cb][r] *= inv;
    }
  }

  __device__ __forceinline__ void operator()(float* buf, int S) {
    const int lane = threadIdx.x % 64;
    for (int s = 0; s < S; ++s) {
      float* x = buf + s * n * P;
      fold(x);
      __syncthreads();
      f32x4 acc[2][CB];
      products(acc);
      if (direct) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          float* xr = x + xrow[h];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (rmask[h] & (1 << r)) {
#pragma unroll
              for (int cb = 0; cb < CB; ++cb) xr[2 * r * P + 16 * cb] = acc[h][cb][r];
            }
          }
        }
        __syncthreads();
      } else {
        float* R = reinterpret_cast<float*>(fb);
        const int rb0 = 2 * (threadIdx.x / 64);
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h < nrb) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                R[(16 * (rb0 + h) + 4 * (lane / 16) + r) * ax->r_pitch + 16 * cb + lane % 16] =
                    acc[h][cb][r];
          }
        }
        __syncthreads();
        mf_unfold<float, W>(R, *ax, n, x, P);
        __syncthreads();
      }
    }
  }
};

// ------------------------------------------------------------------ FP64
struct MfmaXfF64 {
  static constexpr int W = 16;
  static constexpr int THREADS = MF_THREADS;
  const Geom* g;
  const MfmaAxisDev* ax;
  double* fb;
  double A[MF_KSMAX_F64];
  int wave, lane;

  __device__ __forceinline__ MfmaXfF64(const Geom* g_, const MfmaAxisDev* ax_, double* fb_)
      : g(g_), ax(ax_), fb(fb_) {
    wave = threadIdx.x / 64;
    lane = threadIdx.x % 64;
    const double* src = reinterpret_cast<const double*>(ax->Afrag);
#pragma unroll
    for (int ks = 0; ks < MF_KSMAX_F64; ++ks)
      A[ks] = wave < ax->RB ? src[(wave * MF_KSMAX_F64 + ks) * 64 + lane] : 0.0;
  }

  __device__ __forceinline__ void operator()(double* buf, int S) {
    const int n = g->n, pitch = g->pitch;
    const int KS = ax->hK / 4;
    for (int s = 0; s < S; ++s) {
      double* x = buf + s * n * pitch;
      mf_fold<double, W>(x, pitch, *ax, fb);
      __syncthreads();
      f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
      if (wave < ax->RB) {
        const int half = wave < ax->RBe ? 0 : 1;
        const double* bp = fb + (half * W + lane % 16) * ax->fb_pitch + lane / 16;
#pragma unroll
        for (int ks = 0; ks < MF_KSMAX_F64; ++ks) {
          if (ks < KS) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[ks], bp[4 * ks], acc, 0, 0, 0);
        }
      }
      // f64 16x16x4 result layout: lane l, register r holds row 4r + l/16, column l%16
      if (ax->direct) {
        // DCT-I / DST-I: E row m is output 2m, O row m is output 2m + 1.
        if (wave < ax->RB) {
          const bool isO = wave >= ax->RBe;
          const int mb = 16 * (isO ? wave - ax->RBe : wave) + lane / 16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = 2 * (mb + 4 * r) + (isO ? 1 : 0);
            if (k < n) x[k * pitch + lane % 16] = acc[r];
          }
        }
        __syncthreads();
      } else {
        __syncthreads();
        if (wave < ax->RB) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            fb[(16 * wave + 4 * r + lane / 16) * ax->r_pitch + lane % 16] = acc[r];
        }
        __syncthreads();
        mf_unfold<double, W>(fb, *ax, n, x, pitch);
        __syncthreads();
      }
    }
  }
};

// Engines per field type: the x axis (tiles of every species) and the
// strided axes.
template <typename T>
struct XfSel;
template <>
struct XfSel<float> {
  using X = MfmaXfF32<16>;
  using Z = MfmaXfF32<32>;
};
template <>
struct XfSel<double> {
  using X = MfmaXfF64;
  using Z = MfmaXfF64;
};
template <typename T>
using XfX = typename XfSel<T>::X;
template <typename T>
using XfZ = typename XfSel<T>::Z;

// ------------------------------------------------------------------ kernels
// Persistent: block b handles tiles b, b + gridDim.x, ... The global loads of
// the next tile are issued before the current tile is computed.
// Prefetch depth (16-byte vectors per thread) where the registers allow it:
// the FP32 forward, single-axis and adjoint-X kernels; 0 loads in place.
template <typename T>
struct MfPrefetch {
  static constexpr int fwd = 0;
};
template <>
struct MfPrefetch<float> {
  static constexpr int fwd = 0;
};

template <typename T, class XF>
__global__ __launch_bounds__(XF::THREADS, 4) void k_xstage_m(StageArgs<T> a, MfmaAxisDev ax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  XF xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  TilePrefetch<T, MfPrefetch<T>::fwd> pf;
  pf.issue(a.g, blockIdx.x, a.P, a.g.spt);
  for (long long tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
    pf.commit(a.g, tile, a.P, buf, a.g.spt);
    __syncthreads();
    pf.issue(a.g, tile + gridDim.x, a.P, a.g.spt);
    run_x(a, buf, tile, xf);
    __syncthreads();
  }
}

template <typename T, class XF>
__global__ __launch_bounds__(XF::THREADS, 4) void k_zstage_m(StageArgs<T> a, MfmaAxisDev ax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  XF xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  const T* src = a.src ? a.src : a.P;
  TilePrefetch<T, MfPrefetch<T>::fwd> pf;
  pf.issue(a.g, blockIdx.x, src, a.g.spt);
  for (long long tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
    pf.commit(a.g, tile, src, buf, a.g.spt);
    __syncthreads();
    pf.issue(a.g, tile + gridDim.x, src, a.g.spt);
    run_z(a, buf, tile, xf);
    __syncthreads();
  }
}

template <typename T, class XF>
__global__ __launch_bounds__(XF::THREADS, 4) void k_xadj_m(StageArgs<T> a, MfmaAxisDev ax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  XF xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  double pacc[MAX_PARAMS];
  for (int k = 0; k < MAX_PARAMS; ++k) pacc[k] = 0.0;
  TilePrefetch<T, MfPrefetch<T>::fwd> pf;
  pf.issue(a.g, blockIdx.x, a.P, a.g.spt);
  for (long long tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
    pf.commit(a.g, tile, a.P, buf, a.g.spt);
    __syncthreads();
    pf.issue(a.g, tile + gridDim.x, a.P, a.g.spt);
    run_xadj(a, buf, tile, xf, pacc);
    __syncthreads();
  }
  if (a.rp_acc) block_add_partials(reinterpret_cast<double*>(smem_raw), pacc, a.rxn.np, a.rp_acc);
}

template <typename T, class XF>
__global__ __launch_bounds__(XF::THREADS, 4) void k_zadj_m(StageArgs<T> a, MfmaAxisDev ax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  XF xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  TilePrefetch<T, 0> pf;
  pf.issue(a.g, blockIdx.x, a.P, a.g.spt);
  for (long long tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
    pf.commit(a.g, tile, a.P, buf, a.g.spt);
    __syncthreads();
    pf.issue(a.g, tile + gridDim.x, a.P, a.g.spt);
    run_zadj(a, buf, tile, xf);
    __syncthreads();
  }
}

// One transform along one axis, src -> dst (may alias), optional Neumann
// point weights before (divide) or after (multiply).
template <typename T, class XF>
__global__ __launch_bounds__(XF::THREADS, 4) void k_single_m(SingleArgs<T> a, MfmaAxisDev ax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  XF xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  const Geom& g = a.g;
  const int ne = g.n * g.W;
  TilePrefetch<T, MfPrefetch<T>::fwd> pf;
  pf.issue(g, blockIdx.x, a.src, g.spt);
  for (long long tile = blockIdx.x; tile < g.ntiles; tile += gridDim.x) {
    pf.commit(g, tile, a.src, buf, g.spt);
    __syncthreads();
    pf.issue(g, tile + gridDim.x, a.src, g.spt);
    const TileRef tr = tile_ref(g, tile);
    if (a.pre_divide_w) {
      for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        int j, w;
        unpack(g, e, j, w);
        long long idx;
        if (!elem(g, tr, j, w, idx)) continue;
        const T wt = T(point_weight(idx, a.n0, a.n1, a.n2));
        for (int s = 0; s < g.spt; ++s) buf[(s * g.n + j) * g.pitch + w] /= wt;
      }
      __syncthreads();
    }
    xf(buf, g.spt);
    if (a.post_multiply_w) {
      for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        int j, w;
        unpack(g, e, j, w);
        long long idx;
        if (!elem(g, tr, j, w, idx)) continue;
        const T wt = T(point_weight(idx, a.n0, a.n1, a.n2));
        for (int s = 0; s < g.spt; ++s) buf[(s * g.n + j) * g.pitch + w] *= wt;
      }
      __syncthreads();
    }
    store_tile_fast(g, tile, buf, a.dst, g.spt);
    __syncthreads();
  }
}

}  // namespace sfrde
